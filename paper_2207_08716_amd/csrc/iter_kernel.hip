// Fused pseudo-transient iteration for gfx950.
//
// One launch performs a whole PT iteration (thesis article 1, section 2.2):
// total-pressure update (eq (17)), Darcy flux and fluid-pressure update
// (eqs (18), (20)), visco-elastic stresses (eq (21)), damped momentum update
// (eq (19)) and the porosity update in log space (eq (22)), all from the
// iteration-k state (Jacobi), with the boundary conditions of eqs (33)-(34).
//
// Work decomposition.  A BX x BY block owns a column of (BX-2) x (BY-2) cells
// plus a one-cell halo ring and marches upward through a chunk of KZ planes.
// Per plane the block
//   1. stages the plane's velocities, fluid pressure, permeability, solid
//      fraction and shear viscosity in LDS (values of plane p+1 that the
//      column needs again next plane stay in registers: a z register queue);
//   2. computes cell quantities (div V, Pt', stresses) on the cells and the
//      low halo, shear stresses on edges, and Pf', ln(1-phi)' on the tile;
//   3. after one more barrier, updates the three face velocities of every
//      tile cell.
// Stresses and Darcy fluxes never touch HBM.  Every field is read once and
// the iterated fields written once per iteration (plus halo re-reads, which
// mostly hit L2 because neighbouring tiles run together on one XCD).
#include "pt_internal.h"

namespace ptk {

namespace {

struct Lds {
    double vx[BY][BX], vy[BY][BX], vz1[BY][BX];
    double pf[BY][BX], kc[BY][BX], s[BY][BX], mu[BY][BX], mu1[BY][BX];
    double ptn[BY][BX], txx[BY][BX], tyy[BY][BX], txy[BY][BX], w[BY][BX];
    double txz[2][BY][BX], tyz[2][BY][BX];
};

__device__ __forceinline__ double nanmax(double m, double v) {
    // maximum that lets a NaN through (divergence must not be hidden)
    return (v > m || v != v) ? v : m;
}

// Tile order: consecutive tiles go to the same XCD (blocks are dealt to the
// eight XCDs round robin), so tiles that share halo planes share an L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t L, int64_t total) {
    const int64_t nx = 8;
    int64_t xcd = L % nx, idx = L / nx;
    int64_t q = total / nx, r = total % nx;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <bool UPD_LP, bool NORMS>
__global__ __launch_bounds__(BX * BY) void k_iter(Geom g, Coef c, IterPtrs p) {
    __shared__ Lds sh;

    const int gx = (g.nx + BX - 3) / (BX - 2);
    const int gy = (g.ny + BY - 3) / (BY - 2);
    const int64_t total = (int64_t)gridDim.x;
    const int64_t T = xcd_tile(blockIdx.x, total);
    const int bx = (int)(T % gx);
    const int by = (int)((T / gx) % gy);
    const int bz = (int)(T / ((int64_t)gx * gy));

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int i = bx * (BX - 2) - 1 + tx;
    const int j = by * (BY - 2) - 1 + ty;
    const int kz0 = bz * KZ;
    const int kz1 = min(g.nz, kz0 + KZ);

    const bool ci = (i >= 0) && (i < g.nx);
    const bool cj = (j >= 0) && (j < g.ny);
    const bool cell = ci && cj;
    const bool vxcol = (i >= 0) && (i <= g.nx) && cj;   // x-faces of this column
    const bool vycol = ci && (j >= 0) && (j <= g.ny);   // y-faces of this column
    const bool outc = cell && tx >= 1 && tx <= BX - 2 && ty >= 1 && ty <= BY - 2;
    const bool cellq = cell && tx <= BX - 2 && ty <= BY - 2;
    const bool edge = tx >= 1 && ty >= 1;
    // Every load is issued unconditionally from an address clamped into the
    // padded box (always inside the allocation); values of positions outside
    // a field's extent are replaced by zero where they are consumed.  This
    // keeps the loads branch-free so that a whole plane's worth is in flight
    // at once.
    const int ic = min(max(i, 0), g.nx), jc = min(max(j, 0), g.ny);
    const int64_t col = (int64_t)jc * g.P + ic;
    auto at = [&](int k) -> int64_t { return (int64_t)min(max(k, 0), g.nz) * g.S + col; };

    // queue set of a plane (own column): needed at planes p-1..p+1
    struct QSet { double vx, vy, vz, pf, kc, lp, mu; };
    // cell set of a plane: needed at plane p only
    struct CSet { double pt, pto, pfo, eta, lpo, rx, ry, rz, fox, foy, foz; };
    auto load_q = [&](int k, QSet& q) {
        const int64_t o = at(k);
        q.vx = p.vx[o]; q.vy = p.vy[o]; q.vz = p.vz[o]; q.pf = p.pf[o];
        q.kc = p.kc[o]; q.lp = p.lp[o]; q.mu = p.mus[o];
    };
    // The cell set is loaded only by the threads that use it (halo columns
    // would otherwise fetch tile-only fields from HBM a second time).
    auto load_c = [&](int k, CSet& c) {
        const int64_t o = at(k);
        if (cellq) {
            c.pt = p.pt[o]; c.pto = p.pto[o]; c.pfo = p.pfo[o]; c.eta = p.eta[o];
        }
        if (outc) {
            c.lpo = UPD_LP ? p.lpo[o] : 0.0;
            c.rx = p.rx[o]; c.ry = p.ry[o]; c.rz = p.rz[o];
            c.fox = p.fox[o]; c.foy = p.foy[o]; c.foz = p.foz[o];
        }
    };
    auto mask_q = [&](int k, QSet& q) {
        const bool pk = (k >= 0) && (k < g.nz);
        q.vx = (vxcol && pk) ? q.vx : 0.0;
        q.vy = (vycol && pk) ? q.vy : 0.0;
        q.vz = (cell && k >= 0 && k <= g.nz) ? q.vz : 0.0;
        q.pf = (cell && pk) ? q.pf : 0.0;
        q.kc = (cell && pk) ? q.kc : 0.0;
        q.lp = (cell && pk) ? q.lp : 0.0;
        q.mu = (cell && pk) ? q.mu : 0.0;
    };

    // register queue (own column): _p = plane p-1, _c = plane p, _n = plane p+1
    double vx_c, vy_c, vz_c, pf_p = 0.0, pf_c, kc_p = 0.0, kc_c, s_p = 0.0, s_c, mu_p = 0.0, mu_c, lp_c;
    double ptn_p = 0.0, tzz_p = 0.0, rg_p = 0.0, w_p = 0.0, txz_c = 0.0, tyz_c = 0.0;
    double nm[NNORM];
#pragma unroll
    for (int q = 0; q < NNORM; ++q) nm[q] = 0.0;

    QSet qn;     // plane p+1 (prefetched one step ahead)
    CSet cc{};   // cell set of plane p (prefetched one step ahead)
    {
        const int p0 = kz0 - 1;
        QSet q0;
        load_q(p0, q0);
        load_q(p0 + 1, qn);
        load_c(p0, cc);
        mask_q(p0, q0);
        vx_c = q0.vx; vy_c = q0.vy; vz_c = q0.vz; pf_c = q0.pf; kc_c = q0.kc; lp_c = q0.lp; mu_c = q0.mu;
        s_c = (cell && p0 >= 0) ? exp(lp_c) : 0.0;
    }

    for (int pz = kz0 - 1; pz < kz1; ++pz) {
        const bool plc = pz >= 0;                // plane pz is a real plane
        const bool pln = pz + 1 < g.nz;          // plane pz+1 is a real plane
        const bool live = pz >= kz0;             // outputs of this plane belong to the block

        // prefetch what the next step needs
        QSet qnn;
        CSet cn = cc;
        load_q(pz + 2, qnn);
        load_c(pz + 1, cn);

        // plane pz+1 for the queue (arrived during the previous step)
        mask_q(pz + 1, qn);
        const double vx_n = qn.vx, vy_n = qn.vy, vz_n = qn.vz, pf_n = qn.pf, kc_n = qn.kc;
        const double lp_n = qn.lp, mu_n = qn.mu;
        const double s_n = (cell && pln) ? exp(lp_n) : 0.0;

        // plane pz values needed for the cell quantities
        const bool cq = cellq && plc;
        const bool oc = outc && plc && live;
        const double pt = cc.pt, pto = cc.pto, pfo = cc.pfo, eta = cc.eta, lpo = cc.lpo;
        const double rx = cc.rx, ry = cc.ry, rz = cc.rz, fox = cc.fox, foy = cc.foy, foz = cc.foz;

        sh.vx[ty][tx] = vx_c;
        sh.vy[ty][tx] = vy_c;
        sh.vz1[ty][tx] = vz_n;
        sh.pf[ty][tx] = pf_c;
        sh.kc[ty][tx] = kc_c;
        sh.s[ty][tx] = s_c;
        sh.mu[ty][tx] = mu_c;
        sh.mu1[ty][tx] = mu_n;
        __syncthreads();

        // ---- cell quantities: div V, Pt' (eq (17)), stresses (eq (21)) ----
        double ptn = 0.0, txx = 0.0, tyy = 0.0, tzz = 0.0, rg = 0.0, w = 0.0, chi = 0.0;
        double rpt_k = 0.0;
        if (cq) {
            const double dxv = (sh.vx[ty][tx + 1] - vx_c) * c.dxi;
            const double dyv = (sh.vy[ty + 1][tx] - vy_c) * c.dyi;
            const double dzv = (vz_n - vz_c) * c.dzi;
            const double divv = dxv + dyv + dzv;
            chi = 1.0 / (eta * s_c);
            const double dtp = c.dtaupt_c * mu_c;
            if (c.mech_off) {
                ptn = pt;
            } else {
                ptn = (pt - dtp * (divv + c.beta_d * (-pto - c.alpha * (pf_c - pfo)) * c.dti - pf_c * chi)) /
                      (1.0 + dtp * (c.beta_d * c.dti + chi));
            }
            const double rimp = divv + c.beta_d * ((ptn - pto) - c.alpha * (pf_c - pfo)) * c.dti + (ptn - pf_c) * chi;
            const double xi = mu_c * c.gdts_inv;
            const double b = 2.0 * mu_c / (1.0 + xi);
            const double d3 = divv * c.third;
            const double comp = c.beta_n * rimp;
            txx = b * ((dxv - d3) + comp);
            tyy = b * ((dyv - d3) + comp);
            tzz = b * ((dzv - d3) + comp);
            rg = c.rhofg * (1.0 - s_c) + c.rhosg * s_c;
            if (NORMS) {
                w = b * comp - ptn + pt;
                rpt_k = divv + c.beta_d * ((pt - pto) - c.alpha * (pf_c - pfo)) * c.dti + (pt - pf_c) * chi;
            }
        }

        // ---- Darcy flux and fluid pressure (eqs (18), (20)); porosity (eq (22)) ----
        double pfn = 0.0, lpn = 0.0, rpf_k = 0.0;
        if (oc) {
            const double kw = sh.kc[ty][tx - 1], ke = sh.kc[ty][tx + 1];
            const double ks = sh.kc[ty - 1][tx], kn = sh.kc[ty + 1][tx];
            const double qxl = (i >= 1) ? -0.5 * (kw + kc_c) * (pf_c - sh.pf[ty][tx - 1]) * c.dxi : 0.0;
            const double qxh = (i + 1 < g.nx) ? -0.5 * (kc_c + ke) * (sh.pf[ty][tx + 1] - pf_c) * c.dxi : 0.0;
            const double qyl = (j >= 1) ? -0.5 * (ks + kc_c) * (pf_c - sh.pf[ty - 1][tx]) * c.dyi : 0.0;
            const double qyh = (j + 1 < g.ny) ? -0.5 * (kc_c + kn) * (sh.pf[ty + 1][tx] - pf_c) * c.dyi : 0.0;
            const double qzl = (pz >= 1) ? -0.5 * (kc_p + kc_c) * ((pf_c - pf_p) * c.dzi + c.buoy) : 0.0;
            const double qzh = pln ? -0.5 * (kc_c + kc_n) * ((pf_n - pf_c) * c.dzi + c.buoy) : 0.0;
            const double divq = (qxh - qxl) * c.dxi + (qyh - qyl) * c.dyi + (qzh - qzl) * c.dzi;
            double kl = kc_c;
            if (i >= 1) kl = fmax(kl, kw);
            if (i + 1 < g.nx) kl = fmax(kl, ke);
            if (j >= 1) kl = fmax(kl, ks);
            if (j + 1 < g.ny) kl = fmax(kl, kn);
            if (pz >= 1) kl = fmax(kl, kc_p);
            if (pln) kl = fmax(kl, kc_n);
            const double dtf = c.dtaupf_c / kl;
            pfn = (pf_c - dtf * (divq + c.beta_d * (-c.ab * pfo - c.alpha * (pt - pto)) * c.dti - pt * chi)) /
                  (1.0 + dtf * (c.beta_d * c.ab * c.dti + chi));
            if (NORMS)
                rpf_k = divq + c.beta_d * (c.ab * (pf_c - pfo) - c.alpha * (pt - pto)) * c.dti + (pf_c - pt) * chi;
            if (UPD_LP) {
                double adv = 0.5 * vx_c * (s_c - sh.s[ty][tx - 1]) * c.dxi;
                adv += 0.5 * sh.vx[ty][tx + 1] * (sh.s[ty][tx + 1] - s_c) * c.dxi;
                adv += 0.5 * vy_c * (s_c - sh.s[ty - 1][tx]) * c.dyi;
                adv += 0.5 * sh.vy[ty + 1][tx] * (sh.s[ty + 1][tx] - s_c) * c.dyi;
                adv += 0.5 * vz_c * (s_c - s_p) * c.dzi;
                adv += 0.5 * vz_n * (s_n - s_c) * c.dzi;
                const double dphidt = c.beta_phi * ((pfn - pfo) - (ptn - pto)) * c.dti + (pfn - ptn) / eta + adv;
                lpn = lpo - c.dt * dphidt;
            }
        }

        // ---- shear stresses on the xy-edges of plane pz and the xz/yz-edges of level pz+1 ----
        double txz_n = 0.0, tyz_n = 0.0, txy = 0.0;
        if (edge) {
            if (plc && i >= 1 && i < g.nx && j >= 1 && j < g.ny) {
                const double mue = 0.25 * (sh.mu[ty - 1][tx - 1] + sh.mu[ty - 1][tx] + sh.mu[ty][tx - 1] + mu_c);
                const double xie = mue * c.gdts_inv;
                const double be = 2.0 * mue / (1.0 + xie);
                const double exy = 0.5 * ((vx_c - sh.vx[ty - 1][tx]) * c.dyi + (vy_c - sh.vy[ty][tx - 1]) * c.dxi);
                txy = be * exy;
            }
            const bool lev = (pz + 1 >= 1) && (pz + 1 < g.nz);
            if (lev && i >= 1 && i < g.nx && cj) {
                const double mue = 0.25 * (sh.mu[ty][tx - 1] + mu_c + sh.mu1[ty][tx - 1] + mu_n);
                const double xie = mue * c.gdts_inv;
                const double be = 2.0 * mue / (1.0 + xie);
                const double exz = 0.5 * ((vx_n - vx_c) * c.dzi + (vz_n - sh.vz1[ty][tx - 1]) * c.dxi);
                txz_n = be * exz;
            }
            if (lev && j >= 1 && j < g.ny && ci) {
                const double mue = 0.25 * (sh.mu[ty - 1][tx] + mu_c + sh.mu1[ty - 1][tx] + mu_n);
                const double xie = mue * c.gdts_inv;
                const double be = 2.0 * mue / (1.0 + xie);
                const double eyz = 0.5 * ((vy_n - vy_c) * c.dzi + (vz_n - sh.vz1[ty - 1][tx]) * c.dyi);
                tyz_n = be * eyz;
            }
        }
        const int bn = (pz + 1) & 1, bc = pz & 1;
        sh.ptn[ty][tx] = ptn;
        sh.txx[ty][tx] = txx;
        sh.tyy[ty][tx] = tyy;
        sh.txy[ty][tx] = txy;
        if (NORMS) sh.w[ty][tx] = w;
        sh.txz[bn][ty][tx] = txz_n;
        sh.tyz[bn][ty][tx] = tyz_n;
        __syncthreads();

        // ---- momentum (eq (19)) and damped velocity update on the tile ----
        if (oc) {
            const int64_t o = (int64_t)pz * g.S + col;
            if (i >= 1) {
                const double f = (txx - sh.txx[ty][tx - 1]) * c.dxi + (sh.txy[ty + 1][tx] - txy) * c.dyi +
                                 (txz_n - txz_c) * c.dzi - (ptn - sh.ptn[ty][tx - 1]) * c.dxi + fox;
                double r = f * c.rho_i_inv + c.dampx * rx;
                double v = vx_c + (c.dtauv_c / fmax(mu_c, sh.mu[ty][tx - 1])) * r;
                if (c.mech_off) { r = rx; v = vx_c; }
                p.rx_o[o] = r;
                p.vx_o[o] = v;
                if (NORMS) {
                    nm[0] = nanmax(nm[0], fabs(f - (w - sh.w[ty][tx - 1]) * c.dxi));
                    nm[7] = nanmax(nm[7], fabs(v - vx_c));
                }
            }
            if (j >= 1) {
                const double f = (sh.txy[ty][tx + 1] - txy) * c.dxi + (tyy - sh.tyy[ty - 1][tx]) * c.dyi +
                                 (tyz_n - tyz_c) * c.dzi - (ptn - sh.ptn[ty - 1][tx]) * c.dyi + foy;
                double r = f * c.rho_i_inv + c.dampy * ry;
                double v = vy_c + (c.dtauv_c / fmax(mu_c, sh.mu[ty - 1][tx])) * r;
                if (c.mech_off) { r = ry; v = vy_c; }
                p.ry_o[o] = r;
                p.vy_o[o] = v;
                if (NORMS) {
                    nm[0] = nanmax(nm[0], fabs(f - (w - sh.w[ty - 1][tx]) * c.dyi));
                    nm[7] = nanmax(nm[7], fabs(v - vy_c));
                }
            }
            if (pz >= 1) {
                const double f = (sh.txz[bc][ty][tx + 1] - txz_c) * c.dxi + (sh.tyz[bc][ty + 1][tx] - tyz_c) * c.dyi +
                                 (tzz - tzz_p) * c.dzi - (ptn - ptn_p) * c.dzi - (0.5 * (rg_p + rg) - c.rhobg) + foz;
                double r = f * c.rho_i_inv + c.dampz * rz;
                double v = vz_c + (c.dtauv_c / fmax(mu_c, mu_p)) * r;
                if (c.mech_off) { r = rz; v = vz_c; }
                p.rz_o[o] = r;
                p.vz_o[o] = v;
                if (NORMS) {
                    nm[0] = nanmax(nm[0], fabs(f - (w - w_p) * c.dzi));
                    nm[6] = nanmax(nm[6], fabs(v - vz_c));
                    nm[7] = nanmax(nm[7], fabs(v - vz_c));
                }
            }
            p.pt_o[o] = ptn;
            p.pf_o[o] = pfn;
            if (UPD_LP) p.lp_o[o] = lpn;
            if (NORMS) {
                nm[1] = nanmax(nm[1], fabs(rpt_k));
                nm[2] = nanmax(nm[2], fabs(rpf_k));
                if (UPD_LP) nm[3] = nanmax(nm[3], fabs(lpn - lp_c));
                nm[4] = nanmax(nm[4], fabs(ptn - pt));
                nm[5] = nanmax(nm[5], fabs(pfn - pf_c));
            }
        }

        // advance the register queue
        vx_c = vx_n; vy_c = vy_n; vz_c = vz_n;
        pf_p = pf_c; pf_c = pf_n;
        kc_p = kc_c; kc_c = kc_n;
        s_p = s_c; s_c = s_n;
        mu_p = mu_c; mu_c = mu_n;
        lp_c = lp_n;
        ptn_p = ptn; tzz_p = tzz; rg_p = rg; w_p = w;
        txz_c = txz_n; tyz_c = tyz_n;
        qn = qnn;
        cc = cn;
    }

    if (NORMS) {
        // block maximum: wave64 butterfly, then across the waves through LDS
        __shared__ double red[(BX * BY) / 64][NNORM];
#pragma unroll
        for (int q = 0; q < NNORM; ++q) {
            double v = nm[q];
            for (int off = 32; off >= 1; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
            nm[q] = v;
        }
        const int lin = ty * BX + tx;
        const int wave = lin >> 6, lane = lin & 63;
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < NNORM; ++q) red[wave][q] = nm[q];
        }
        __syncthreads();
        if (lin < NNORM) {
            double v = 0.0;
            for (int wv = 0; wv < (BX * BY) / 64; ++wv) v = nanmax(v, red[wv][lin]);
            p.partials[(int64_t)blockIdx.x * NNORM + lin] = v;
        }
    }
}

__global__ __launch_bounds__(256) void k_reduce_max(const double* __restrict__ part, int64_t nb,
                                                    double* __restrict__ out) {
    __shared__ double red[4][NNORM];
    double m[NNORM];
#pragma unroll
    for (int q = 0; q < NNORM; ++q) m[q] = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
        for (int q = 0; q < NNORM; ++q) m[q] = nanmax(m[q], part[b * NNORM + q]);
    }
#pragma unroll
    for (int q = 0; q < NNORM; ++q) {
        double v = m[q];
        for (int off = 32; off >= 1; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
        m[q] = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NNORM; ++q) red[wave][q] = m[q];
    }
    __syncthreads();
    if (threadIdx.x < NNORM) {
        double v = 0.0;
        for (int wv = 0; wv < 4; ++wv) v = nanmax(v, red[wv][threadIdx.x]);
        out[threadIdx.x] = v;
    }
}

}  // namespace

hipError_t launch_iteration(const Geom& g, const Coef& c, const IterPtrs& p, int update_lp, int norms,
                            hipStream_t s) {
    const dim3 block(BX, BY, 1);
    const dim3 grid((unsigned)iter_grid_blocks(g), 1, 1);
    if (update_lp) {
        if (norms) hipLaunchKernelGGL((k_iter<true, true>), grid, block, 0, s, g, c, p);
        else hipLaunchKernelGGL((k_iter<true, false>), grid, block, 0, s, g, c, p);
    } else {
        if (norms) hipLaunchKernelGGL((k_iter<false, true>), grid, block, 0, s, g, c, p);
        else hipLaunchKernelGGL((k_iter<false, false>), grid, block, 0, s, g, c, p);
    }
    return hipGetLastError();
}

hipError_t launch_reduce_max(const double* partials, int64_t nblocks, double* out8, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(256), 0, s, partials, nblocks, out8);
    return hipGetLastError();
}

}  // namespace ptk
