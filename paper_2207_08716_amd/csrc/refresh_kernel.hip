// Picard refresh with the stress invariant, as one z-marching tile kernel.
//
// The refresh of the lagged coefficients (thesis article 1, eqs (23)-(26))
// needs, when the viscosity depends on stress (power law, yield cap), the
// second invariant of the present deviatoric stress at every cell: the three
// normal stresses at the cell and the shear stresses of the twelve edges
// around it, averaged per component (eq (21) for the stresses, without the
// numerical compressibility term).  A 66 x H block owns a 64 x (H-2) column
// of cells plus a one-cell halo ring and marches upward through a chunk of
// planes, like the PT sweep: per plane it stages viscosities and velocities
// in LDS, computes each edge's shear stress once (xy edges of the plane, xz
// and yz edges of the level above, the level below carried from the previous
// plane), then updates k/mu_f, eta_phi and Mn of the tile cells in place.
// Edge stresses never touch memory.  The loads of the next plane are issued
// one step ahead from clamped (always in-bounds) addresses.
#include "pt_internal.h"

namespace ptk {

namespace {

constexpr int RW = 66;   // block width of both kernels (64 output columns)
constexpr int RH = 10;   // block height of the refresh (8 output rows)
constexpr int FH = 14;   // block height of the Fo kernel (72 registers: 15 waves fit)

template <int W, int H>
struct RefreshLds {
    double mu0[H][W], mu1[H][W];   // mu_s of planes p and p+1
    double vx[H][W], vy[H][W];     // velocities of plane p
    double vz1[H][W];              // vz of level p+1
    double txy[H][W];              // xy-edge stresses of plane p
    double txz[2][H][W], tyz[2][H][W];   // xz/yz-edge stresses by level parity
};

__device__ __forceinline__ double maxwell_a(double mu, double gdts_inv) {
    const double xi = mu * gdts_inv;
    return xi / (1.0 + xi);
}
__device__ __forceinline__ double maxwell_b(double mu, double gdts_inv) {
    const double xi = mu * gdts_inv;
    return 2.0 * mu / (1.0 + xi);
}

__global__ __launch_bounds__(RW * RH) void k_refresh_tiled(Geom g, Coef c, RefreshCoef r, AuxPtrs a) {
    constexpr int W = RW, H = RH;
    __shared__ RefreshLds<W, H> sh;

    const int gx = (g.nx + W - 3) / (W - 2);
    const int gy = (g.ny + H - 3) / (H - 2);
    const int64_t Tt = xcd_tile(blockIdx.x, (int64_t)gridDim.x);
    const int bx = (int)(Tt % gx);
    const int by = (int)((Tt / gx) % gy);
    const int bz = (int)(Tt / ((int64_t)gx * gy));
    int tx, ty;
    tile_thread<W, H>(tx, ty);
    const int i = bx * (W - 2) - 1 + tx;
    const int j = by * (H - 2) - 1 + ty;
    const int kz0 = bz * g.kz;
    const int kz1 = min(g.nz, kz0 + g.kz);

    const bool edge = tx >= 1 && ty >= 1;   // LDS neighbours at tx-1, ty-1 exist
    const bool outc = tx >= 1 && tx <= W - 2 && ty >= 1 && ty <= H - 2 && i < g.nx && j < g.ny;
    // edges computed by this thread (interior edges; boundary edges are zero
    // except for xy edges under the background shear of eq (32))
    const bool exy = edge && i >= 1 && i < g.nx && j >= 1 && j < g.ny;
    const bool bxy = edge && c.gbg_half != 0.0 && !exy && i >= 0 && i <= g.nx && j >= 0 && j <= g.ny;
    const bool exz = edge && i >= 1 && i < g.nx && j >= 0 && j < g.ny;
    const bool eyz = edge && j >= 1 && j < g.ny && i >= 0 && i < g.nx;

    const int ic = min(max(i, 0), g.nx), jc = min(max(j, 0), g.ny);
    const int64_t col = (int64_t)jc * g.P + ic;
    auto at = [&](int k) -> int64_t { return (int64_t)min(max(k, 0), g.nz) * g.S + col; };

    // values of level/plane q along the own column
    struct QSet { double mu, vx, vy, vz, sxz, syz; };
    // cell and xy-edge values of plane q
    struct CSet { double sxy, sxx, syy, szz, lp, k0, pt, pf, mn, eta; };
    auto load_q = [&](int q, QSet& v) {
        const int64_t o = at(q);
        v.mu = a.mus[o]; v.vx = a.vx[o]; v.vy = a.vy[o]; v.vz = a.vz[o];
        v.sxz = a.sxz[o]; v.syz = a.syz[o];
    };
    auto load_c = [&](int q, CSet& v) {
        const int64_t o = at(q);
        v.sxy = a.sxy[o];
        if (outc) {
            v.sxx = a.sxx[o]; v.syy = a.syy[o]; v.szz = a.szz[o];
            v.lp = a.lp[o]; v.pt = a.pt[o]; v.pf = a.pf[o]; v.mn = a.mn[o]; v.eta = a.eta[o];
            v.k0 = r.k0field ? a.k0[o] : r.kmuf0;
        }
    };

    // plane p = kz0 - 1 (the level below the first cells) and its successor
    QSet qc, qn;
    load_q(kz0 - 1, qc);
    load_q(kz0, qn);
    CSet cc{};   // plane p's cell set (the first step, below the chunk, has none)
    double txz_c = 0.0, tyz_c = 0.0;   // xz/yz-edge stresses of level p (own column)

    for (int pz = kz0 - 1; pz < kz1; ++pz) {
        const bool live = pz >= kz0;
        // prefetch the next step
        QSet qnn;
        CSet cn = cc;
        load_q(pz + 2, qnn);
        load_c(pz + 1, cn);

        sh.mu0[ty][tx] = qc.mu;
        sh.mu1[ty][tx] = qn.mu;
        sh.vx[ty][tx] = qc.vx;
        sh.vy[ty][tx] = qc.vy;
        sh.vz1[ty][tx] = qn.vz;
        __syncthreads();

        // edge stresses: xy edges of plane pz, xz/yz edges of level pz+1
        double txy = 0.0, txz_n = 0.0, tyz_n = 0.0;
        const int lv = pz + 1;
        if (live && exy) {
            const double mue = 0.25 * (sh.mu0[ty - 1][tx - 1] + sh.mu0[ty - 1][tx] + sh.mu0[ty][tx - 1] + qc.mu);
            const double e = 0.5 * ((qc.vx - sh.vx[ty - 1][tx]) * c.dyi + (qc.vy - sh.vy[ty][tx - 1]) * c.dxi) +
                             c.gbg_half;
            txy = maxwell_a(mue, c.gdts_inv) * cc.sxy + maxwell_b(mue, c.gdts_inv) * e;
        } else if (live && bxy) {
            // boundary edge: background strain rate only, viscosity averaged
            // over the cells inside
            double sum = 0.0;
            if (j >= 1) {
                if (i >= 1) sum += sh.mu0[ty - 1][tx - 1];
                if (i < g.nx) sum += sh.mu0[ty - 1][tx];
            }
            if (j < g.ny) {
                if (i >= 1) sum += sh.mu0[ty][tx - 1];
                if (i < g.nx) sum += qc.mu;
            }
            const double cnt = (double)(((i >= 1) + (i < g.nx)) * ((j >= 1) + (j < g.ny)));
            const double mue = sum / cnt;
            txy = maxwell_a(mue, c.gdts_inv) * cc.sxy + maxwell_b(mue, c.gdts_inv) * c.gbg_half;
        }
        if (exz && lv >= 1 && lv < g.nz) {
            const double mue = 0.25 * (sh.mu0[ty][tx - 1] + qc.mu + sh.mu1[ty][tx - 1] + qn.mu);
            const double e = 0.5 * ((qn.vx - qc.vx) * c.dzi + (qn.vz - sh.vz1[ty][tx - 1]) * c.dxi);
            txz_n = maxwell_a(mue, c.gdts_inv) * qn.sxz + maxwell_b(mue, c.gdts_inv) * e;
        }
        if (eyz && lv >= 1 && lv < g.nz) {
            const double mue = 0.25 * (sh.mu0[ty - 1][tx] + qc.mu + sh.mu1[ty - 1][tx] + qn.mu);
            const double e = 0.5 * ((qn.vy - qc.vy) * c.dzi + (qn.vz - sh.vz1[ty - 1][tx]) * c.dyi);
            tyz_n = maxwell_a(mue, c.gdts_inv) * qn.syz + maxwell_b(mue, c.gdts_inv) * e;
        }
        // neighbour velocities for the normal strain rates, taken before the
        // barrier (the next step's staging overwrites them)
        const double vx_e = (tx + 1 < W) ? sh.vx[ty][tx + 1] : 0.0;
        const double vy_n = (ty + 1 < H) ? sh.vy[ty + 1][tx] : 0.0;
        const int bn = lv & 1, bc = pz & 1;
        sh.txy[ty][tx] = txy;
        sh.txz[bn][ty][tx] = txz_n;
        sh.tyz[bn][ty][tx] = tyz_n;
        __syncthreads();

        if (live && outc) {
            const int64_t o = (int64_t)pz * g.S + col;
            const double s = exp(cc.lp);
            const double phi = 1.0 - s;
            const double rr = phi / r.phi0;
            const double kc = cc.k0 * rr * rr * rr;
            const double R = (cc.pf > cc.pt) ? 1.0 / r.R0 : 1.0;
            const double eta_new = r.eta0 * cc.mn * (r.phi0 / phi) * R;
            const double eta = r.first ? eta_new : exp(r.r_eta * log(eta_new) + (1.0 - r.r_eta) * log(cc.eta));

            // normal stresses at the cell
            const double mu = qc.mu;
            const double aa = maxwell_a(mu, c.gdts_inv), bb = maxwell_b(mu, c.gdts_inv);
            const double dxv = (vx_e - qc.vx) * c.dxi;
            const double dyv = (vy_n - qc.vy) * c.dyi;
            const double dzv = (qn.vz - qc.vz) * c.dzi;
            const double d3 = (dxv + dyv + dzv) * c.third;
            const double txx = aa * cc.sxx + bb * (dxv - d3);
            const double tyy = aa * cc.syy + bb * (dyv - d3);
            const double tzz = aa * cc.szz + bb * (dzv - d3);
            // edge stresses averaged to the cell
            const double axy = 0.25 * (sh.txy[ty][tx] + sh.txy[ty][tx + 1] + sh.txy[ty + 1][tx] + sh.txy[ty + 1][tx + 1]);
            const double axz = 0.25 * (txz_c + sh.txz[bc][ty][tx + 1] + txz_n + sh.txz[bn][ty][tx + 1]);
            const double ayz = 0.25 * (tyz_c + sh.tyz[bc][ty + 1][tx] + tyz_n + sh.tyz[bn][ty + 1][tx]);
            const double tii = sqrt(0.5 * (txx * txx + tyy * tyy + tzz * tzz) + axy * axy + axz * axz + ayz * ayz);

            double mn_new = r.mu0;
            if (r.powerlaw) {
                const double t = tii * r.tau0_inv;
                const double tp = (r.n_pow == 3.0) ? t * t : pow(t, r.n_pow - 1.0);
                mn_new = r.mu0 / (1.0 + tp);
            }
            if (r.dpcap) {
                const double tyl = fmax(r.coh_cos + (cc.pt - cc.pf) * r.sin_f, r.tau_y_min);
                // the viscosity that puts the present strain rate on the
                // yield surface, where it is below the viscous one
                if (tii > 0.0) mn_new = fmin(mn_new, cc.mn * tyl / tii);
            }
            const double mnr = r.first ? mn_new : exp(r.r_mu * log(mn_new) + (1.0 - r.r_mu) * log(cc.mn));
            a.kc[o] = kc;
            a.eta[o] = eta;
            a.mn[o] = mnr;
        }

        qc = qn;
        qn = qnn;
        cc = cn;
        txz_c = txz_n;
        tyz_c = tyz_n;
    }
}

// The stress-history divergence folded into face fields, after a refresh:
// mu_s = Mn phi0 cmu at the cells, then on every face owned by a tile cell
// (the x-, y- and z-faces at its low side) Fo = div(a So), with a = xi/(1+xi)
// at the cells and, for the shear components, at the edges from the mean of
// the four cells' mu_s; boundary faces carry zero.  Same tiling and march as
// the refresh: per plane the new mu_s and the normal history components are
// staged in LDS, each edge's a_e So_e is formed once (xy edges of the plane,
// xz/yz edges of the level above; the level below is carried over).
template <int W, int H>
struct FoLds {
    double mu0[H][W], mu1[H][W];   // new mu_s of planes p and p+1
    double sxx[H][W], syy[H][W];   // normal history of plane p
    double exy[H][W];              // a_e So_xy of the xy edges of plane p
    double exz[2][H][W], eyz[2][H][W];   // a_e So of the xz/yz edges by level parity
};

__global__ __launch_bounds__(RW * FH) void k_fo_tiled(Geom g, Coef c, RefreshCoef r, AuxPtrs a) {
    constexpr int W = RW, H = FH;
    __shared__ FoLds<W, H> sh;

    const int gx = (g.nx + W - 3) / (W - 2);
    const int gy = (g.ny + H - 3) / (H - 2);
    const int64_t Tt = xcd_tile(blockIdx.x, (int64_t)gridDim.x);
    const int bx = (int)(Tt % gx);
    const int by = (int)((Tt / gx) % gy);
    const int bz = (int)(Tt / ((int64_t)gx * gy));
    int tx, ty;
    tile_thread<W, H>(tx, ty);
    const int i = bx * (W - 2) - 1 + tx;
    const int j = by * (H - 2) - 1 + ty;
    const int kz0 = bz * g.kz;
    const int kz1 = min(g.nz, kz0 + g.kz);

    const bool edge = tx >= 1 && ty >= 1;
    const bool tcol = tx >= 1 && tx <= W - 2, trow = ty >= 1 && ty <= H - 2;
    const bool outc = tcol && trow && i < g.nx && j < g.ny;
    const bool exy = edge && i >= 1 && i < g.nx && j >= 1 && j < g.ny;
    const bool exz = edge && i >= 1 && i < g.nx && j >= 0 && j < g.ny;
    const bool eyz = edge && j >= 1 && j < g.ny && i >= 0 && i < g.nx;
    // boundary xy edges carry a history under the background shear of eq (32)
    const bool bxy = edge && c.gbg_half != 0.0 && !exy && i >= 0 && i <= g.nx && j >= 0 && j <= g.ny;
    // boundary faces at i = nx and j = ny belong to no cell: the halo thread
    // on them (in exactly one block) writes their zero
    const bool xbnd = trow && i == g.nx && j < g.ny;
    const bool ybnd = tcol && ty >= 1 && j == g.ny && i < g.nx;

    const int ic = min(max(i, 0), g.nx), jc = min(max(j, 0), g.ny);
    const int64_t col = (int64_t)jc * g.P + ic;
    auto at = [&](int k) -> int64_t { return (int64_t)min(max(k, 0), g.nz) * g.S + col; };
    auto mus_of = [&](double mn) { return mn * r.phi0 * r.cmu; };

    // plane/level q along the own column: Mn, szz (cells), sxz, syz (levels)
    struct QSet { double mn, szz, sxz, syz; };
    // plane q: sxx, syy (cells), sxy (xy edges)
    struct CSet { double sxx, syy, sxy; };
    auto load_q = [&](int q, QSet& v) {
        const int64_t o = at(q);
        v.mn = a.mn[o]; v.szz = a.szz[o]; v.sxz = a.sxz[o]; v.syz = a.syz[o];
    };
    auto load_c = [&](int q, CSet& v) {
        const int64_t o = at(q);
        v.sxx = a.sxx[o]; v.syy = a.syy[o]; v.sxy = a.sxy[o];
    };

    QSet qc, qn;
    load_q(kz0 - 1, qc);
    load_q(kz0, qn);
    CSet cc{};
    double mu_c = mus_of(qc.mn);
    double exz_c = 0.0, eyz_c = 0.0;   // a_e So of the xz/yz edges of level p (own column)
    double asz_p = 0.0;                // a * szz of plane p-1 (own column)

    for (int pz = kz0 - 1; pz < kz1; ++pz) {
        const bool live = pz >= kz0;
        QSet qnn;
        CSet cn = cc;
        load_q(pz + 2, qnn);
        load_c(pz + 1, cn);

        const double mu_n = mus_of(qn.mn);
        sh.mu0[ty][tx] = mu_c;
        sh.mu1[ty][tx] = mu_n;
        sh.sxx[ty][tx] = cc.sxx;
        sh.syy[ty][tx] = cc.syy;
        __syncthreads();

        const int lv = pz + 1;
        double e_xy = 0.0, e_xz = 0.0, e_yz = 0.0;
        if (live && exy) {
            const double mue = 0.25 * (sh.mu0[ty - 1][tx - 1] + sh.mu0[ty - 1][tx] + sh.mu0[ty][tx - 1] + mu_c);
            e_xy = maxwell_a(mue, c.gdts_inv) * cc.sxy;
        } else if (live && bxy) {
            double sum = 0.0;   // viscosity averaged over the cells inside
            if (j >= 1) {
                if (i >= 1) sum += sh.mu0[ty - 1][tx - 1];
                if (i < g.nx) sum += sh.mu0[ty - 1][tx];
            }
            if (j < g.ny) {
                if (i >= 1) sum += sh.mu0[ty][tx - 1];
                if (i < g.nx) sum += mu_c;
            }
            const double mue = sum / (double)(((i >= 1) + (i < g.nx)) * ((j >= 1) + (j < g.ny)));
            e_xy = maxwell_a(mue, c.gdts_inv) * cc.sxy;
        }
        if (exz && lv >= 1 && lv < g.nz) {
            const double mue = 0.25 * (sh.mu0[ty][tx - 1] + mu_c + sh.mu1[ty][tx - 1] + mu_n);
            e_xz = maxwell_a(mue, c.gdts_inv) * qn.sxz;
        }
        if (eyz && lv >= 1 && lv < g.nz) {
            const double mue = 0.25 * (sh.mu0[ty - 1][tx] + mu_c + sh.mu1[ty - 1][tx] + mu_n);
            e_yz = maxwell_a(mue, c.gdts_inv) * qn.syz;
        }
        // west and south neighbours' a * So, taken before the barrier (the
        // next step's staging overwrites them)
        const double a_c = maxwell_a(mu_c, c.gdts_inv);
        const double asx_w = (tx >= 1) ? maxwell_a(sh.mu0[ty][tx - 1], c.gdts_inv) * sh.sxx[ty][tx - 1] : 0.0;
        const double asy_s = (ty >= 1) ? maxwell_a(sh.mu0[ty - 1][tx], c.gdts_inv) * sh.syy[ty - 1][tx] : 0.0;
        const int bn = lv & 1, bc = pz & 1;
        sh.exy[ty][tx] = e_xy;
        sh.exz[bn][ty][tx] = e_xz;
        sh.eyz[bn][ty][tx] = e_yz;
        __syncthreads();

        const double asz = a_c * qc.szz;
        if (live && outc) {
            const int64_t o = (int64_t)pz * g.S + col;
            double fx = 0.0, fy = 0.0, fz = 0.0;
            if (i >= 1)
                fx = (a_c * cc.sxx - asx_w) * c.dxi + (sh.exy[ty + 1][tx] - e_xy) * c.dyi + (e_xz - exz_c) * c.dzi;
            if (j >= 1)
                fy = (sh.exy[ty][tx + 1] - e_xy) * c.dxi + (a_c * cc.syy - asy_s) * c.dyi + (e_yz - eyz_c) * c.dzi;
            if (pz >= 1)
                fz = (sh.exz[bc][ty][tx + 1] - exz_c) * c.dxi + (sh.eyz[bc][ty + 1][tx] - eyz_c) * c.dyi +
                     (asz - asz_p) * c.dzi;
            a.mus[o] = mu_c;
            a.fox[o] = fx;
            a.foy[o] = fy;
            a.foz[o] = fz;
            if (pz == g.nz - 1) a.foz[o + g.S] = 0.0;
        }
        if (live && xbnd) a.fox[(int64_t)pz * g.S + col] = 0.0;
        if (live && ybnd) a.foy[(int64_t)pz * g.S + col] = 0.0;

        qc = qn;
        qn = qnn;
        cc = cn;
        mu_c = mu_n;
        exz_c = e_xz;
        eyz_c = e_yz;
        asz_p = asz;
    }
}

}  // namespace

hipError_t launch_fo_tiled(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a, hipStream_t s) {
    const Geom v = sweep_geom(g, RW, FH);
    hipLaunchKernelGGL(k_fo_tiled, dim3((unsigned)iter_grid_blocks(g, RW, FH)), dim3(RW * FH), 0, s, v, c, r, a);
    return hipGetLastError();
}

hipError_t launch_refresh_tiled(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a,
                                hipStream_t s) {
    const Geom v = sweep_geom(g, RW, RH);
    hipLaunchKernelGGL(k_refresh_tiled, dim3((unsigned)iter_grid_blocks(g, RW, RH)), dim3(RW * RH), 0, s, v, c, r,
                       a);
    return hipGetLastError();
}

}  // namespace ptk
