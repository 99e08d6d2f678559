// Fused pseudo-transient sweep for gfx950.
//
// One launch performs a whole PT iteration (thesis article 1, section 2.2):
// total-pressure update (eq (17)), Darcy flux and fluid-pressure update
// (eqs (18), (20)), visco-elastic stresses (eq (21)), damped momentum update
// (eq (19)) and the porosity update in log space (eq (22)), all from the
// iteration-k state (Jacobi), with the boundary conditions of eqs (33)-(34).
//
// Modes of the same sweep:
//   THESIS  FP64, porosity updated every iteration (thesis schedule);
//   LINEAR  FP64, porosity frozen (one linear system of a Picard stage);
//   RESID   FP64, no update: writes the residuals f, r_Pt, r_Pf of the present
//           state (physical stress, current Pt) in FP32 for defect correction;
//   CORR    FP32 sweep on the correction system A(c) d = -r of a Picard stage:
//           the same iteration applied to x + d, with the FP64 residual of x as
//           right-hand side (no old values, no buoyancy, no history term).
//
// Work decomposition.  A BX x BY block owns a column of (BX-2) x (BY-2) cells
// plus a one-cell halo ring and marches upward through a chunk of g.kz planes.
// Per plane the block
//   1. stages the plane's velocities, fluid pressure, permeability, solid
//      fraction and shear viscosity in LDS (values of plane p+1 that the
//      column needs again next plane stay in registers: a z register queue);
//   2. computes cell quantities (div V, Pt', stresses) on the cells and the
//      low halo, shear stresses on edges, and Pf', ln(1-phi)' on the tile;
//   3. after one more barrier, updates the three face velocities of every
//      tile cell.
// The next plane's loads are issued one step ahead.  Stresses and Darcy
// fluxes never touch HBM; the iterated fields are written once.
//
// Damped velocity update of the FP64 sweeps (eq (19) with the script's
// damping): R' = f/rho_i + d R, V' = V + dtau_V R'.  Between checks the
// sweep does not store R: with dtau_V unchanged since the last iteration,
// d R = d (V - V_prev) / dtau_V, and V_prev is the other copy of V (the one
// this sweep overwrites), so V' = V + dtau_V f/rho_i + d (V - V_prev) needs
// no R stream (three fewer of 27).  The first sweep after the pseudo steps
// change (a refresh) reads the stored R instead (c.rform); sweeps that end a
// check interval store R' = (V' - V)/dtau_V (c.rwrite), so that it is there
// when the next refresh comes.  The FP32 correction sweeps do the same with
// the damped residual of the correction.
#include "pt_internal.h"

namespace ptk {

namespace {

template <typename T, int W, int H>
struct Lds {
    T vx[H][W], vy[H][W], vz1[H][W];
    T pf[H][W], kc[H][W], s[H][W], mu[H][W], mu1[H][W];
    T ptn[H][W], txx[H][W], tyy[H][W], txy[H][W], w[H][W];
    T txz[2][H][W], tyz[2][H][W];
};

// Block width of a sweep variant: the plain sweeps use BX, the variants that
// also reduce norms BX_NORMS (both give 64-column output tiles).
template <typename T, int MODE, bool NORMS>
constexpr int sweep_bx() {
    return (NORMS || MODE == MD_RESID) ? BX_NORMS : BX;
}
// Block height: taller tiles re-read fewer halo rows but need registers for
// more waves per CU, and the number of tiles sets how full the last round of
// blocks is; the heights below fit each variant's registers without spilling
// and were measured fastest at 511^3.
template <typename T, int MODE, bool NORMS>
constexpr int sweep_by() {
    if (NORMS || MODE == MD_RESID) return BY_NORMS;
    if (MODE == MD_THESIS) return BY;
    if (MODE == MD_CORR && sizeof(T) == 4) return BY_CORR32;
    return BY_LINEAR;
}

template <typename T>
__device__ __forceinline__ T nanmax(T m, T v) {
    // maximum that lets a NaN through (divergence must not be hidden)
    return (v > m || v != v) ? v : m;
}

// Constants in the working precision of the sweep.
template <typename T>
struct CT {
    T dxi, dyi, dzi, dt, dti, beta_d, alpha, beta_phi, rhofg, rhosg, rhobg, buoy, gdts_inv, beta_n,
        rho_i_inv, dtauv_c, dtaupt_c, dtaupf_c, dampx, dampy, dampz, ab, third, gbg_half;
    int mech_off, rform, rwrite;
    __device__ explicit CT(const Coef& c)
        : dxi(T(c.dxi)), dyi(T(c.dyi)), dzi(T(c.dzi)), dt(T(c.dt)), dti(T(c.dti)), beta_d(T(c.beta_d)),
          alpha(T(c.alpha)), beta_phi(T(c.beta_phi)), rhofg(T(c.rhofg)), rhosg(T(c.rhosg)),
          rhobg(T(c.rhobg)), buoy(T(c.buoy)), gdts_inv(T(c.gdts_inv)), beta_n(T(c.beta_n)),
          rho_i_inv(T(c.rho_i_inv)), dtauv_c(T(c.dtauv_c)), dtaupt_c(T(c.dtaupt_c)),
          dtaupf_c(T(c.dtaupf_c)), dampx(T(c.dampx)), dampy(T(c.dampy)), dampz(T(c.dampz)),
          ab(T(c.ab)), third(T(c.third)), gbg_half(T(c.gbg_half)), mech_off(c.mech_off), rform(c.rform),
          rwrite(c.rwrite) {}
};

// One face's damped velocity update (see the header): returns V', sets the
// damped residual R' in r.  q: the stored R (rform) or V_prev.
template <typename T, typename C>
__device__ __forceinline__ T damped_update(const C& c, T v_c, T q, T f, T damp, T dtv, T& r) {
    if (c.rform) {
        r = f * c.rho_i_inv + damp * q;
        return v_c + dtv * r;
    }
    const T v = v_c + dtv * (f * c.rho_i_inv) + damp * (v_c - q);
    r = (v - v_c) / dtv;
    return v;
}

// HV, if not 0, overrides the variant's block height.  BGS: the background
// shear of eq (32) is on (a variant of its own: the plain thesis sweep has no
// register to spare for it).
template <typename T, int MODE, bool NORMS, int HV = 0, bool BGS = false>
__global__ __launch_bounds__((sweep_bx<T, MODE, NORMS>() * (HV ? HV : sweep_by<T, MODE, NORMS>()))) void k_sweep(
    Geom g, Coef cd, SweepPtrs<T> p) {
    constexpr int W = sweep_bx<T, MODE, NORMS>();
    constexpr int H = HV ? HV : sweep_by<T, MODE, NORMS>();
    static_assert(W * H <= 1024, "a block holds at most 1024 threads");
    constexpr bool UPD_LP = (MODE == MD_THESIS);
    constexpr bool RESID = (MODE == MD_RESID);
    constexpr bool CORR = (MODE == MD_CORR);
    constexpr bool WNORM = NORMS || RESID;
    __shared__ Lds<T, W, H> sh;
    const CT<T> c(cd);
    const T zero = T(0), half = T(0.5), one = T(1), two = T(2), quarter = T(0.25);

    const int gx = (g.nx + W - 3) / (W - 2);
    const int gy = (g.ny + H - 3) / (H - 2);
    const int64_t total = (int64_t)gridDim.x;
    const int64_t Tt = xcd_tile(blockIdx.x, total);
    const int bx = (int)(Tt % gx);
    const int by = (int)((Tt / gx) % gy);
    const int bz = (int)(Tt / ((int64_t)gx * gy));

    int tx, ty;
    tile_thread<W, H>(tx, ty);
    const int i = bx * (W - 2) - 1 + tx;
    const int j = by * (H - 2) - 1 + ty;
    const int kz0 = bz * g.kz;
    const int kz1 = min(g.nz, kz0 + g.kz);

    const bool ci = (i >= 0) && (i < g.nx);
    const bool cj = (j >= 0) && (j < g.ny);
    const bool cell = ci && cj;
    const bool vxcol = (i >= 0) && (i <= g.nx) && cj;   // x-faces of this column
    const bool vycol = ci && (j >= 0) && (j <= g.ny);   // y-faces of this column
    const bool outc = cell && tx >= 1 && tx <= W - 2 && ty >= 1 && ty <= H - 2;
    const bool cellq = cell && tx <= W - 2 && ty <= H - 2;
    const bool edge = tx >= 1 && ty >= 1;

    // Every load is issued from an address clamped into the padded box
    // (always inside the allocation); values of positions outside a field's
    // extent are replaced by zero where they are consumed.  The loads are
    // branch-free so that a whole plane's worth is in flight at once.
    const int ic = min(max(i, 0), g.nx), jc = min(max(j, 0), g.ny);
    const int64_t col = (int64_t)jc * g.P + ic;
    auto at = [&](int k) -> int64_t { return (int64_t)min(max(k, 0), g.nz) * g.S + col; };

    // queue set of a plane (own column): needed at planes p-1..p+1
    struct QSet { T vx, vy, vz, pf, kc, lp, mu; };
    // cell set of a plane: needed at plane p only
    struct CSet { T pt, pto, pfo, eta, lpo, rx, ry, rz, fox, foy, foz; };
    auto load_q = [&](int k, QSet& q) {
        const int64_t o = at(k);
        q.vx = p.vx[o]; q.vy = p.vy[o]; q.vz = p.vz[o]; q.pf = p.pf[o];
        q.kc = p.kc[o]; q.mu = p.mus[o];
        q.lp = CORR ? zero : p.lp[o];
    };
    // The cell set is loaded only by the threads that use it (halo columns
    // would otherwise fetch tile-only fields from HBM a second time).  The
    // tile-only fields are read exactly once per launch: in FP64 they are
    // loaded non-temporally, which keeps them from displacing halo data in
    // the caches.  The FP32 sweep keeps ordinary loads: its whole working set
    // fits the last-level cache at 127^3, where non-temporal loads made the
    // mixed solve 8 % slower.
    auto once = [](const T* ptr) -> T {
        if constexpr (sizeof(T) == 8) return __builtin_nontemporal_load(ptr);
        else return *ptr;
    };
    auto load_c = [&](int k, CSet& cs) {
        const int64_t o = at(k);
        if (cellq) {
            cs.pt = p.pt[o]; cs.pto = p.pto[o]; cs.pfo = p.pfo[o]; cs.eta = p.eta[o];
        }
        if (outc) {
            cs.lpo = UPD_LP ? once(&p.lpo[o]) : zero;
            if (!RESID) {
                cs.rx = once(&p.rx[o]);
                cs.ry = once(&p.ry[o]);
                cs.rz = once(&p.rz[o]);
            }
            cs.fox = once(&p.fox[o]);
            cs.foy = once(&p.foy[o]);
            cs.foz = once(&p.foz[o]);
        }
    };
    auto mask_q = [&](int k, QSet& q) {
        const bool pk = (k >= 0) && (k < g.nz);
        q.vx = (vxcol && pk) ? q.vx : zero;
        q.vy = (vycol && pk) ? q.vy : zero;
        q.vz = (cell && k >= 0 && k <= g.nz) ? q.vz : zero;
        q.pf = (cell && pk) ? q.pf : zero;
        q.kc = (cell && pk) ? q.kc : zero;
        q.lp = (cell && pk) ? q.lp : zero;
        q.mu = (cell && pk) ? q.mu : zero;
    };
    auto solid = [&](bool ok, T lp) -> T { return CORR ? one : (ok ? T(exp(lp)) : zero); };

    // register queue (own column): _p = plane p-1, _c = plane p, _n = plane p+1
    T vx_c, vy_c, vz_c, pf_p = zero, pf_c, kc_p = zero, kc_c, s_p = zero, s_c, mu_p = zero, mu_c, lp_c;
    T ptn_p = zero, tzz_p = zero, rg_p = zero, w_p = zero, txz_c = zero, tyz_c = zero;
    T nm[NNORM];
#pragma unroll
    for (int q = 0; q < NNORM; ++q) nm[q] = zero;

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
        s_c = solid(cell && p0 >= 0, lp_c);
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
        const T vx_n = qn.vx, vy_n = qn.vy, vz_n = qn.vz, pf_n = qn.pf, kc_n = qn.kc;
        const T lp_n = qn.lp, mu_n = qn.mu;
        const T s_n = solid(cell && pln, lp_n);

        // plane pz values needed for the cell quantities
        const bool cq = cellq && plc;
        const bool oc = outc && plc && live;
        const T pt = cc.pt, pto = cc.pto, pfo = cc.pfo, eta = cc.eta, lpo = cc.lpo;
        const T rx = cc.rx, ry = cc.ry, rz = cc.rz, fox = cc.fox, foy = cc.foy, foz = cc.foz;

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
        T ptn = zero, txx = zero, tyy = zero, tzz = zero, rg = zero, w = zero, chi = zero;
        T rpt_k = zero;
        if (cq) {
            const T dxv = (sh.vx[ty][tx + 1] - vx_c) * c.dxi;
            const T dyv = (sh.vy[ty + 1][tx] - vy_c) * c.dyi;
            const T dzv = (vz_n - vz_c) * c.dzi;
            const T divv = dxv + dyv + dzv;
            const T dtp = c.dtaupt_c * mu_c;
            // r_Pt of iteration k: the numerical-compressibility term of the
            // stresses takes it before the pressure update
            if constexpr (CORR) {
                // d Pt' = [d Pt - dtau (div dV + r_Pt(x) - beta_d alpha dPf/dt - dPf chi)]
                //         / (1 + dtau (beta_d/dt + chi)); chi is a stored field here
                chi = eta;
                ptn = (pt - dtp * (divv + pto - c.beta_d * c.alpha * pf_c * c.dti - pf_c * chi)) /
                      (one + dtp * (c.beta_d * c.dti + chi));
                rpt_k = pto + divv + c.beta_d * (pt - c.alpha * pf_c) * c.dti + (pt - pf_c) * chi;
            } else {
                chi = one / (eta * s_c);
                if (RESID || c.mech_off) {
                    ptn = pt;
                } else {
                    ptn = (pt - dtp * (divv + c.beta_d * (-pto - c.alpha * (pf_c - pfo)) * c.dti - pf_c * chi)) /
                          (one + dtp * (c.beta_d * c.dti + chi));
                }
                rpt_k = divv + c.beta_d * ((pt - pto) - c.alpha * (pf_c - pfo)) * c.dti + (pt - pf_c) * chi;
                rg = c.rhofg * (one - s_c) + c.rhosg * s_c;
            }
            const T xi = mu_c * c.gdts_inv;
            const T b = two * mu_c / (one + xi);
            const T d3 = divv * c.third;
            const T comp = RESID ? zero : c.beta_n * rpt_k;
            txx = b * ((dxv - d3) + comp);
            tyy = b * ((dyv - d3) + comp);
            tzz = b * ((dzv - d3) + comp);
            if (NORMS) w = b * comp - ptn + pt;
        }

        // ---- Darcy flux and fluid pressure (eqs (18), (20)); porosity (eq (22)) ----
        T pfn = zero, lpn = zero, rpf_k = zero;
        if (oc) {
            const T buoy = CORR ? zero : c.buoy;
            const T kw = sh.kc[ty][tx - 1], ke = sh.kc[ty][tx + 1];
            const T ks = sh.kc[ty - 1][tx], kn = sh.kc[ty + 1][tx];
            const T qxl = (i >= 1) ? -half * (kw + kc_c) * (pf_c - sh.pf[ty][tx - 1]) * c.dxi : zero;
            const T qxh = (i + 1 < g.nx) ? -half * (kc_c + ke) * (sh.pf[ty][tx + 1] - pf_c) * c.dxi : zero;
            const T qyl = (j >= 1) ? -half * (ks + kc_c) * (pf_c - sh.pf[ty - 1][tx]) * c.dyi : zero;
            const T qyh = (j + 1 < g.ny) ? -half * (kc_c + kn) * (sh.pf[ty + 1][tx] - pf_c) * c.dyi : zero;
            const T qzl = (pz >= 1) ? -half * (kc_p + kc_c) * ((pf_c - pf_p) * c.dzi + buoy) : zero;
            const T qzh = pln ? -half * (kc_c + kc_n) * ((pf_n - pf_c) * c.dzi + buoy) : zero;
            const T divq = (qxh - qxl) * c.dxi + (qyh - qyl) * c.dyi + (qzh - qzl) * c.dzi;
            T kl = kc_c;
            if (i >= 1) kl = fmax(kl, kw);
            if (i + 1 < g.nx) kl = fmax(kl, ke);
            if (j >= 1) kl = fmax(kl, ks);
            if (j + 1 < g.ny) kl = fmax(kl, kn);
            if (pz >= 1) kl = fmax(kl, kc_p);
            if (pln) kl = fmax(kl, kc_n);
            const T dtf = c.dtaupf_c / kl;
            if constexpr (CORR) {
                pfn = (pf_c - dtf * (divq + pfo - c.beta_d * c.alpha * pt * c.dti - pt * chi)) /
                      (one + dtf * (c.beta_d * c.ab * c.dti + chi));
                if (WNORM) rpf_k = pfo + divq + c.beta_d * (c.ab * pf_c - c.alpha * pt) * c.dti + (pf_c - pt) * chi;
            } else if constexpr (RESID) {
                pfn = pf_c;
                rpf_k = divq + c.beta_d * (c.ab * (pf_c - pfo) - c.alpha * (pt - pto)) * c.dti + (pf_c - pt) * chi;
            } else {
                pfn = (pf_c - dtf * (divq + c.beta_d * (-c.ab * pfo - c.alpha * (pt - pto)) * c.dti - pt * chi)) /
                      (one + dtf * (c.beta_d * c.ab * c.dti + chi));
                if (WNORM)
                    rpf_k = divq + c.beta_d * (c.ab * (pf_c - pfo) - c.alpha * (pt - pto)) * c.dti + (pf_c - pt) * chi;
            }
            if constexpr (UPD_LP) {
                T adv = half * vx_c * (s_c - sh.s[ty][tx - 1]) * c.dxi;
                adv += half * sh.vx[ty][tx + 1] * (sh.s[ty][tx + 1] - s_c) * c.dxi;
                adv += half * vy_c * (s_c - sh.s[ty - 1][tx]) * c.dyi;
                adv += half * sh.vy[ty + 1][tx] * (sh.s[ty + 1][tx] - s_c) * c.dyi;
                adv += half * vz_c * (s_c - s_p) * c.dzi;
                adv += half * vz_n * (s_n - s_c) * c.dzi;
                const T dphidt = c.beta_phi * ((pfn - pfo) - (ptn - pto)) * c.dti + (pfn - ptn) / eta + adv;
                lpn = lpo - c.dt * dphidt;
            }
        }

        // ---- shear stresses on the xy-edges of plane pz and the xz/yz-edges of level pz+1 ----
        T txz_n = zero, tyz_n = zero, txy = zero;
        if (edge) {
            if (plc && i >= 1 && i < g.nx && j >= 1 && j < g.ny) {
                const T mue = quarter * (sh.mu[ty - 1][tx - 1] + sh.mu[ty - 1][tx] + sh.mu[ty][tx - 1] + mu_c);
                const T xie = mue * c.gdts_inv;
                const T be = two * mue / (one + xie);
                T exy = half * ((vx_c - sh.vx[ty - 1][tx]) * c.dyi + (vy_c - sh.vy[ty][tx - 1]) * c.dxi);
                if constexpr (BGS) exy += c.gbg_half;   // background shear (eq (32))
                txy = be * exy;
            } else if (BGS && plc && i >= 0 && i <= g.nx && j >= 0 && j <= g.ny) {
                // boundary edge: the perturbation slips freely, the background
                // strain rate remains; viscosity averaged over the cells inside
                // (the staged values outside the domain are zero)
                const T cnt = T(((i >= 1) + (i < g.nx)) * ((j >= 1) + (j < g.ny)));
                const T mue = (sh.mu[ty - 1][tx - 1] + sh.mu[ty - 1][tx] + sh.mu[ty][tx - 1] + mu_c) / cnt;
                const T xie = mue * c.gdts_inv;
                const T be = two * mue / (one + xie);
                txy = be * c.gbg_half;
            }
            const bool lev = (pz + 1 >= 1) && (pz + 1 < g.nz);
            if (lev && i >= 1 && i < g.nx && cj) {
                const T mue = quarter * (sh.mu[ty][tx - 1] + mu_c + sh.mu1[ty][tx - 1] + mu_n);
                const T xie = mue * c.gdts_inv;
                const T be = two * mue / (one + xie);
                const T exz = half * ((vx_n - vx_c) * c.dzi + (vz_n - sh.vz1[ty][tx - 1]) * c.dxi);
                txz_n = be * exz;
            }
            if (lev && j >= 1 && j < g.ny && ci) {
                const T mue = quarter * (sh.mu[ty - 1][tx] + mu_c + sh.mu1[ty - 1][tx] + mu_n);
                const T xie = mue * c.gdts_inv;
                const T be = two * mue / (one + xie);
                const T eyz = half * ((vy_n - vy_c) * c.dzi + (vz_n - sh.vz1[ty - 1][tx]) * c.dyi);
                tyz_n = be * eyz;
            }
        }
        // Neighbour viscosities for the velocity pseudo-steps are taken into
        // registers now: the input planes in LDS are overwritten by the next
        // step's staging, which faster waves may reach while the face updates
        // below are still running.
        const T mu_w = (tx >= 1) ? sh.mu[ty][tx - 1] : zero;
        const T mu_s = (ty >= 1) ? sh.mu[ty - 1][tx] : zero;
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
                const T f = (txx - sh.txx[ty][tx - 1]) * c.dxi + (sh.txy[ty + 1][tx] - txy) * c.dyi +
                            (txz_n - txz_c) * c.dzi - (ptn - sh.ptn[ty][tx - 1]) * c.dxi + fox;
                if constexpr (RESID) {
                    p.res_fx[o] = float(f);
                    nm[0] = nanmax(nm[0], T(fabs(f)));
                } else {
                    T r;
                    T v = damped_update<T>(c, vx_c, rx, f, T(c.dampx), T(c.dtauv_c / fmax(mu_c, mu_w)), r);
                    if (c.mech_off) { r = rx; v = vx_c; }
                    if (c.rwrite) p.rx_o[o] = r;
                    p.vx_o[o] = v;
                    if (NORMS) {
                        nm[0] = nanmax(nm[0], T(fabs(f - (w - sh.w[ty][tx - 1]) * c.dxi)));
                        nm[7] = nanmax(nm[7], T(fabs(v - vx_c)));
                    }
                }
            }
            if (j >= 1) {
                const T f = (sh.txy[ty][tx + 1] - txy) * c.dxi + (tyy - sh.tyy[ty - 1][tx]) * c.dyi +
                            (tyz_n - tyz_c) * c.dzi - (ptn - sh.ptn[ty - 1][tx]) * c.dyi + foy;
                if constexpr (RESID) {
                    p.res_fy[o] = float(f);
                    nm[0] = nanmax(nm[0], T(fabs(f)));
                } else {
                    T r;
                    T v = damped_update<T>(c, vy_c, ry, f, T(c.dampy), T(c.dtauv_c / fmax(mu_c, mu_s)), r);
                    if (c.mech_off) { r = ry; v = vy_c; }
                    if (c.rwrite) p.ry_o[o] = r;
                    p.vy_o[o] = v;
                    if (NORMS) {
                        nm[0] = nanmax(nm[0], T(fabs(f - (w - sh.w[ty - 1][tx]) * c.dyi)));
                        nm[7] = nanmax(nm[7], T(fabs(v - vy_c)));
                    }
                }
            }
            if (pz >= 1) {
                const T fs = (sh.txz[bc][ty][tx + 1] - txz_c) * c.dxi + (sh.tyz[bc][ty + 1][tx] - tyz_c) * c.dyi +
                             (tzz - tzz_p) * c.dzi - (ptn - ptn_p) * c.dzi;
                T f;
                if constexpr (CORR) {
                    f = fs + foz;
                } else {
                    f = fs - (half * (rg_p + rg) - c.rhobg) + foz;
                }
                if constexpr (RESID) {
                    p.res_fz[o] = float(f);
                    nm[0] = nanmax(nm[0], T(fabs(f)));
                } else {
                    T r;
                    T v = damped_update<T>(c, vz_c, rz, f, T(c.dampz), T(c.dtauv_c / fmax(mu_c, mu_p)), r);
                    if (c.mech_off) { r = rz; v = vz_c; }
                    if (c.rwrite) p.rz_o[o] = r;
                    p.vz_o[o] = v;
                    if (NORMS) {
                        nm[0] = nanmax(nm[0], T(fabs(f - (w - w_p) * c.dzi)));
                        nm[6] = nanmax(nm[6], T(fabs(v - vz_c)));
                        nm[7] = nanmax(nm[7], T(fabs(v - vz_c)));
                    }
                }
            }
            if constexpr (RESID) {
                p.res_rpt[o] = float(rpt_k);
                p.res_rpf[o] = float(rpf_k);
            } else {
                p.pt_o[o] = ptn;
                p.pf_o[o] = pfn;
                if constexpr (UPD_LP) {
                    p.lp_o[o] = lpn;
                    // phi' outside (0, 1): ln(1-phi)' not in (-inf, 0); checked
                    // with the norms (the plain sweep has no register to spare)
                    if (NORMS && !(lpn < zero && lpn > T(-1.0e300))) *p.domain = 1.0;
                }
            }
            if (WNORM) {
                nm[1] = nanmax(nm[1], T(fabs(rpt_k)));
                nm[2] = nanmax(nm[2], T(fabs(rpf_k)));
                if (UPD_LP) nm[3] = nanmax(nm[3], T(fabs(lpn - lp_c)));
                nm[4] = nanmax(nm[4], T(fabs(ptn - pt)));
                nm[5] = nanmax(nm[5], T(fabs(pfn - pf_c)));
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

    if constexpr (WNORM) {
        // Block maximum: wave64 butterfly in each of the H row waves (the
        // 66-wide layout's halo wave holds no tile cell and contributes
        // nothing), then across the row waves through LDS.
        __shared__ double red[H][NNORM];
        const int L = threadIdx.x;
        const int wave = L >> 6, lane = L & 63;
        if (wave < H) {
#pragma unroll
            for (int q = 0; q < NNORM; ++q) {
                T v = nm[q];
                for (int off = 32; off >= 1; off >>= 1) v = nanmax(v, T(__shfl_xor(v, off, 64)));
                nm[q] = v;
            }
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < NNORM; ++q) red[wave][q] = double(nm[q]);
            }
        }
        __syncthreads();
        if (L < NNORM) {
            double v = 0.0;
            for (int wv = 0; wv < H; ++wv) v = nanmax(v, red[wv][L]);
            p.partials[(int64_t)blockIdx.x * NNORM + L] = v;
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

template <typename T, int MODE, bool NORMS, int HV = 0>
void launch_sweep(const Geom& g, const Coef& c, const SweepPtrs<T>& p, hipStream_t s) {
    constexpr int W = sweep_bx<T, MODE, NORMS>(), H = HV ? HV : sweep_by<T, MODE, NORMS>();
    const Geom v = sweep_geom(g, W, H);
    // the correction system has no background term (it is in its right-hand side)
    if (MODE != MD_CORR && c.gbg_half != 0.0)
        hipLaunchKernelGGL((k_sweep<T, MODE, NORMS, HV, MODE != MD_CORR>), dim3((unsigned)iter_grid_blocks(g, W, H)),
                           dim3(W * H, 1, 1), 0, s, v, c, p);
    else
        hipLaunchKernelGGL((k_sweep<T, MODE, NORMS, HV, false>), dim3((unsigned)iter_grid_blocks(g, W, H)),
                           dim3(W * H, 1, 1), 0, s, v, c, p);
}

hipError_t launch_iteration(const Geom& g, const Coef& c, const SweepPtrs<double>& p, int mode, int norms,
                            hipStream_t s) {
    switch (mode) {
        case MD_THESIS:
            if (norms) launch_sweep<double, MD_THESIS, true>(g, c, p, s);
            else launch_sweep<double, MD_THESIS, false>(g, c, p, s);
            break;
        case MD_LINEAR:
            if (norms) launch_sweep<double, MD_LINEAR, true>(g, c, p, s);
            else launch_sweep<double, MD_LINEAR, false>(g, c, p, s);
            break;
        case MD_RESID:
            launch_sweep<double, MD_RESID, false>(g, c, p, s);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_correction(const Geom& g, const Coef& c, const SweepPtrs<float>& p, int norms, hipStream_t s) {
    if (norms) launch_sweep<float, MD_CORR, true>(g, c, p, s);
    else if (corr32_short(g)) launch_sweep<float, MD_CORR, false, BY_CORR32_SHORT>(g, c, p, s);
    else launch_sweep<float, MD_CORR, false>(g, c, p, s);
    return hipGetLastError();
}

hipError_t launch_correction64(const Geom& g, const Coef& c, const SweepPtrs<double>& p, int norms,
                               hipStream_t s) {
    if (norms) launch_sweep<double, MD_CORR, true>(g, c, p, s);
    else launch_sweep<double, MD_CORR, false>(g, c, p, s);
    return hipGetLastError();
}

hipError_t launch_reduce_max(const double* partials, int64_t nblocks, double* out8, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(256), 0, s, partials, nblocks, out8);
    return hipGetLastError();
}

}  // namespace ptk
