// Internal definitions shared by the kernels and the host side of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "ptporo.h"

namespace ptk {

// Compute units assumed when the device cannot be queried (MI355X: 256).
constexpr int DEFAULT_CUS = 256;

// Index layout common to every field: (k * (ny+1) + j) * P + i.
struct Geom {
    int nx, ny, nz;
    int64_t P;   // row pitch (elements)
    int64_t S;   // plane pitch = (ny + 1) * P
    int kz;      // planes per z chunk of a sweep (set per sweep variant at launch)
    int cus = DEFAULT_CUS;   // compute units of the device (one sweep block each)
    int tall32 = 0;          // FP32 correction sweep: always the 14-row tiles
};

// Physical and numerical constants, in the form the kernels use them.
struct Coef {
    double dxi, dyi, dzi;          // 1/dx, 1/dy, 1/dz
    double dt, dti;                // dt, 1/dt
    double beta_d, alpha, B, beta_phi;
    double rhofg, rhosg;           // fluid / solid density x g
    double rhobg;                  // background density x g
    double buoy;                   // rhofg - rhobg (Darcy flux term, z up)
    double gdts_inv;               // 1 / (G dtS)
    double beta_n;
    double rho_i_inv;
    double dtauv_c;                // rho_i h^2 / (c_v (1 + beta_n)):  dtau_V = dtauv_c / mu_s
    double dtaupt_c;               // (1 + beta_n) / n_max:          dtau_Pt = dtaupt_c * mu_s
    double dtaupf_c;               // h^2 (1 + beta_d B/alpha) / c_pf: dtau_Pf = dtaupf_c / k_loc
    double dampx, dampy, dampz;    // 1 - damp_c / n
    double ab;                     // alpha / B
    double third;                  // 1/3
    double gbg_half;               // half the background shear rate (xy strain rate of eq (32)), 0: none
    int mech_off;
    // FP64 sweeps: the rx..rz inputs hold the stored damped residual R
    // (rform) or the previous velocity iterate; rwrite: store R' (see the
    // sweep's header).  The correction sweeps always read and store R.
    int rform = 1;
    int rwrite = 1;
};

// Sweep modes (see iter_kernel.hip).
constexpr int MD_THESIS = 0;   // FP64, porosity updated
constexpr int MD_LINEAR = 1;   // FP64, porosity frozen
constexpr int MD_RESID = 2;    // FP64, residuals of the present state only
constexpr int MD_CORR = 3;     // FP32 correction sweep

// Pointers of one sweep (inputs at iteration k, outputs at k + 1).  In the
// correction mode the slots carry: vx..rz = correction d and its damped
// residual; pto = r_Pt(x), pfo = r_Pf(x), fox..foz = momentum residual f(x);
// eta = 1/((1-phi) eta_phi); kc, mus = FP32 copies of the coefficients.
template <typename T>
struct SweepPtrs {
    const T *vx, *vy, *vz, *pt, *pf, *lp, *rx, *ry, *rz;
    const T *fox, *foy, *foz, *pto, *pfo, *lpo, *kc, *eta, *mus;
    T *vx_o, *vy_o, *vz_o, *pt_o, *pf_o, *lp_o, *rx_o, *ry_o, *rz_o;
    float *res_fx, *res_fy, *res_fz, *res_rpt, *res_rpf;   // residual mode outputs
    double* partials;              // [n_blocks][8] maxima (norm variants)
    double* domain;                // set to 1 where ln(1-phi)' leaves (-inf, 0) (thesis mode)
};

constexpr int NNORM = 8;

// Tile of the fused sweep: a BX x BY thread block covers a (BX-2) x (BY-2)
// output tile plus one halo column/row on every side and marches in z.
// BX = 66 makes the output tile 64 columns wide: its rows start on 512-byte
// boundaries of the padded rows (whole cache lines written) and n = 2^k - 1
// grids fill their last tile; each row's 64 interior columns are one wave,
// the side halo columns of all rows one more (partial) wave.  The variants
// that also reduce norms need up to 196 registers, so at most 8 waves: 7
// rows.  Every cell's arithmetic is the same in every tiling.  Heights: the
// tallest tile whose
// waves fit the variant's registers is not always the fastest, since the
// number of tiles decides how full the last round of blocks is; measured
// at 511^3 (8-row tiles: 86 tile rows, 10-row tiles: 64).
constexpr int BX = 66;
constexpr int BY = 10;         // thesis sweep
constexpr int BY_LINEAR = 10;  // linear and FP64 correction sweeps
constexpr int BY_CORR32 = 14;  // FP32 correction sweep (large grids)
constexpr int BY_CORR32_SHORT = 10;   // FP32 correction sweep where its tiling costs less
constexpr int BX_NORMS = 66;     // sweeps with norms (up to 196 VGPRs: 8 waves)
constexpr int BY_NORMS = 7;
constexpr int KZ_MAX = 256;

constexpr int KZ_MIN = 4;

inline int64_t tiles_xy(const Geom& g, int bx = BX, int by = BY) {
    return (int64_t)((g.nx + bx - 3) / (bx - 2)) * ((g.ny + by - 3) / (by - 2));
}

// Planes per z chunk for a tiling: the sweep blocks occupy one CU each, so a
// launch takes ceil(blocks / CUs) rounds of (chunk + 2) plane steps (two
// planes of halo and prefetch per chunk); the chunk minimising that wins,
// the longer one on ties.
inline int choose_kz(const Geom& g, int bx, int by, int64_t* cost_out = nullptr) {
    const int64_t t = tiles_xy(g, bx, by);
    int best = KZ_MAX;
    int64_t best_cost = -1;
    for (int kz = KZ_MAX; kz >= KZ_MIN; kz /= 2) {
        const int64_t blocks = t * ((g.nz + kz - 1) / kz);
        const int64_t cus = g.cus > 0 ? g.cus : DEFAULT_CUS;
        const int64_t cost = ((blocks + cus - 1) / cus) * (std::min(kz, g.nz) + 2);
        if (best_cost < 0 || cost < best_cost) {
            best = kz;
            best_cost = cost;
        }
    }
    if (cost_out) *cost_out = best_cost;
    return best;
}

// Cost of a tiling in units of row-plane steps: a block's plane step is
// proportional to its rows, so the best chunk's cost times the block height.
inline int64_t tiling_cost(const Geom& g, int bx, int by) {
    int64_t c = 0;
    choose_kz(g, bx, by, &c);
    return c * by;
}

// Whether the FP32 correction sweep runs its shorter tiles on this grid
// (measured: 10 rows 19 % faster at 127^3 and 7 % at 255^3, 14 rows 12 %
// faster at 511^3; the cost model picks the same in all three).
inline bool corr32_short(const Geom& g) {
    if (g.tall32) return false;
    return tiling_cost(g, BX, BY_CORR32_SHORT) < tiling_cost(g, BX, BY_CORR32);
}

// The geometry of one sweep variant: its z chunk set.
inline Geom sweep_geom(const Geom& g, int bx, int by) {
    Geom v = g;
    v.kz = choose_kz(g, bx, by);
    return v;
}

inline int64_t iter_grid_blocks(const Geom& g, int bx, int by) {
    const Geom v = sweep_geom(g, bx, by);
    return tiles_xy(v, bx, by) * ((v.nz + v.kz - 1) / v.kz);
}

// Tile order of the z-marching kernels: consecutive tiles go to the same XCD
// (blocks are dealt to the eight XCDs round robin), so tiles that share halo
// planes share an L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t L, int64_t total) {
    const int64_t nx = 8;
    int64_t xcd = L % nx, idx = L / nx;
    int64_t q = total / nx, r = total % nx;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Thread layout of a W x H tile block (one-dimensional launch of W*H
// threads).  In 66-wide blocks wave r (r < H) takes the 64 interior columns
// of row r, so that every load and store of a row is one whole, aligned
// 512-byte segment, and the last wave takes the two side halo columns of all
// rows.  64-wide blocks map lanes to columns directly.
template <int W, int H>
__device__ __forceinline__ void tile_thread(int& tx, int& ty) {
    if constexpr (W == 64) {
        tx = (int)threadIdx.x & 63;
        ty = (int)threadIdx.x >> 6;
    } else {
        static_assert(W == 66, "tile blocks are 64 or 66 wide");
        const int L = threadIdx.x;
        if (L < 64 * H) {
            tx = 1 + (L & 63);
            ty = L >> 6;
        } else {
            const int r = L - 64 * H;
            tx = (r < H) ? 0 : W - 1;
            ty = (r < H) ? r : r - H;
        }
    }
}

// Blocks that write per-block norm maxima (size of the partials area).
inline int64_t norm_blocks(const Geom& g) { return iter_grid_blocks(g, BX_NORMS, BY_NORMS); }

// Launchers (defined in the .hip files).
hipError_t launch_iteration(const Geom& g, const Coef& c, const SweepPtrs<double>& p, int mode,
                            int norms, hipStream_t s);
hipError_t launch_correction(const Geom& g, const Coef& c, const SweepPtrs<float>& p, int norms,
                             hipStream_t s);
hipError_t launch_correction64(const Geom& g, const Coef& c, const SweepPtrs<double>& p, int norms,
                               hipStream_t s);
hipError_t launch_reduce_max(const double* partials, int64_t nblocks, double* out8, hipStream_t s);

struct AuxPtrs {
    // state (present copies)
    const double *vx, *vy, *vz, *pt, *pf, *lp;
    double *pto, *pfo, *lpo;
    double *sxx, *syy, *szz, *sxy, *sxz, *syz;
    double *fox, *foy, *foz;
    double *mn, *kc, *eta, *mus;
    const double* k0;
    double* lp_o;                  // porosity step output
    double* domain;                // set to 1 where ln(1-phi) leaves (-inf, 0)
};

struct RefreshCoef {
    double phi0, kmuf0, eta0, mu0, cmu, R0;
    double n_pow, tau0_inv, coh_cos, sin_f, tau_y_min;
    double r_eta, r_mu;
    int first, powerlaw, dpcap, k0field;
};

hipError_t launch_begin_step(const Geom& g, const Coef& c, const AuxPtrs& a, int update_history,
                             hipStream_t s);
hipError_t launch_refresh(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a,
                          hipStream_t s);
hipError_t launch_refresh_tiled(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a,
                                hipStream_t s);
hipError_t launch_fo_tiled(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a, hipStream_t s);
hipError_t launch_fo(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a,
                     hipStream_t s);
hipError_t launch_porosity_step(const Geom& g, const Coef& c, const AuxPtrs& a, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t s);
// ln(1-phi) and its old value from a porosity field; domain <- 1 where phi is
// not in (0, 1).
hipError_t launch_set_porosity(const Geom& g, const double* phi, double* lp, double* lpo, double* domain,
                               hipStream_t s);
// Damped residual R = (V - V_prev) / dtau_V on the interior faces (dtau_V =
// dtauv_c / the larger mu_s of the face's two cells).
hipError_t launch_damped_residual(const Geom& g, const Coef& c, const double* vx, const double* vy, const double* vz,
                                  const double* vx_p, const double* vy_p, const double* vz_p, const double* mus,
                                  double* rx, double* ry, double* rz, hipStream_t s);
// n doubles <- v (a kernel, so that the clear can sit in a captured graph).
hipError_t launch_fill(double* dst, double v, int64_t n, hipStream_t s);

// Mixed precision helpers.
struct MixedPtrs {
    // FP64 state (present copies) and coefficients
    double *vx, *vy, *vz, *pt, *pf;
    const double *lp, *kc, *eta, *mus;
    // FP32 correction (present copies) and coefficient copies
    const float *dvx, *dvy, *dvz, *dpt, *dpf;
    float *kc32, *mus32, *chi32;
};
hipError_t launch_prepare_mixed(const Geom& g, const MixedPtrs& m, hipStream_t s);

// Adjoint of a linear Picard stage.
hipError_t launch_gather(const double* src, const int64_t* offs, int n, double* out, hipStream_t s);
hipError_t launch_scatter(const double* vals, const int64_t* offs, int n, double* dst, hipStream_t s);
hipError_t launch_chi64(const Geom& g, const double* eta, const double* lp, double* chi, hipStream_t s);
hipError_t launch_adjoint_gradient(const Geom& g, const Coef& c, const double* kc, const double* pf,
                                   const double* lam_pf, double* grad, hipStream_t s);
hipError_t launch_exp_cells(const Geom& g, const double* src, double* dst, hipStream_t s);
hipError_t launch_apply_correction(const Geom& g, const MixedPtrs& m, hipStream_t s);

// Multigrid transfers between a fine grid gf and its coarse grid gc
// (mg_kernels.hip).  kind: 0 cells, 1/2/3 faces normal to x/y/z.
// Restriction of a cell field: averages (mean 0: arithmetic, 1: harmonic,
// 2: geometric) of the fine values around each coarse point, by the
// separable passes below (their scratch and rows).
hipError_t launch_mg_restrict(const Geom& gf, const Geom& gc, const double* src, double* dst, int mean, double* sa,
                              double* sb, const double* const tab[3], hipStream_t s);
// Normalised restriction rows of one axis (fine nf, coarse nc points; face:
// faces normal to the axis): MG_TAB doubles per coarse index (first fine
// index, count, MG_TAB - 2 weights), nc + face rows.
constexpr int MG_TAB = 10;
hipError_t launch_mg_taps(double* tab, int nf, int nc, int face, hipStream_t s);
// An FP32 fine field restricted by three separable passes through scratch
// sa ((nz_f + 1) (ny_f + 1) P_c doubles) and sb ((nz_f + 1) (ny_c + 1) P_c),
// with the rows of the x, y and z axes for its staggering.
hipError_t launch_mg_restrict32(const Geom& gf, const Geom& gc, int kind, const float* src, double* dst,
                                double* sa, double* sb, const double* const tab[3], hipStream_t s);
// Restricted r_Pt, r_Pf (a, b) -> pto = m[0] a + m[1] b, pfo = m[2] a + m[3] b.
hipError_t launch_mg_restrict_fold(const Geom& gf, const Geom& gc, const float* rpt, const float* rpf, double* pto,
                                   double* pfo, const double m[4], double* sa, double* sb, const double* const tab[3],
                                   hipStream_t s);
// dst (fine) += interpolated src (coarse); the walls' normal faces are kept.
hipError_t launch_mg_prolong_add(const Geom& gf, const Geom& gc, int kind, const double* src, double* dst,
                                 hipStream_t s);

// Krylov acceleration of the multigrid cycle (krylov_kernels.hip): the
// cycles' iterates recombined over a subspace of their own steps.
// Vectors are the fine grid's five unknowns or five residuals in their
// padded boxes; only entries that carry an equation are read or written.
constexpr int KRY_MAX = 8;         // stored directions at most
constexpr int KRY_SLOTS = 16;      // partial sums per block (>= 2 KRY_MAX)
constexpr int KRY_BLOCKS = 2048;
constexpr int KRY_VW = 4;          // columns per work item (the row pitch a multiple of it)   // blocks of the reduction kernels at most
struct KryVecs {
    const float* rk[5];            // residual of the iterate x_k
    const float* ry[5];            // residual of the cycle's result y
    double* x[5];                  // saved x_k (boxes of the fine geometry)
    double* y[5];                  // the fine fields' present copies
    const double* p[KRY_MAX][5];   // stored directions p_s and images A p_s, s < na
    const float* ap[KRY_MAX][5];
    double* p_new[5];              // the new direction and its image
    float* ap_new[5];
    double gamma[KRY_MAX];         // x' = y + sum gamma_s p_s
    double beta[KRY_MAX];          // p = (y - x) - sum beta_s p_s
    double wv2, wp2;               // squared weights of momentum and pressure rows
    int na;
};
// Partial sums go to part[0 .. KRY_BLOCKS * KRY_SLOTS), their totals to the
// KRY_SLOTS doubles after them.
// dots: totals s = <r_k, A p_s>_W, KRY_MAX + s = <r_y, A p_s>_W, s < na.
hipError_t launch_kry_dots(const Geom& g, const KryVecs& v, double* part, hipStream_t s);
// update: x, y <- y + sum gamma_s p_s; p_new = y - x - sum beta_s p_s,
// ap_new = r_k - r_y - sum beta_s A p_s; total 0 = <ap_new, ap_new>_W.
hipError_t launch_kry_update(const Geom& g, const KryVecs& v, double* part, hipStream_t s);
// save: x <- y.
hipError_t launch_kry_save(const Geom& g, const KryVecs& v, hipStream_t s);

// Adjoint of a Picard run (adjoint_kernels.hip).  rhs holds -xbar, the
// right-hand side of the transposed stage solve in the slots of the
// correction sweep (momentum rows on the faces, r_Pt and r_Pf in the cells).
struct AdjPtrs {
    // recorded stage (incoming ln(1-phi), coefficients, solution)
    const double *vx, *vy, *vz, *pt, *pf, *lp, *kc, *eta, *mus;
    // transposed-solve solution lambda
    const double *lvx, *lvy, *lvz, *lpt, *lpf;
    double *rvx, *rvy, *rvz, *rpt, *rpf;   // -xbar
    const double* lbar;                    // adjoint of the stage's outgoing ln(1-phi)
    double* lbar_out;                      // adjoint of its incoming ln(1-phi)
    double *eta_bar, *s_bar;               // porosity-step adjoints of eta and s
    double *pto_bar, *pfo_bar, *lo_bar;    // adjoints of the step's old values
    double *fbx, *fby, *fbz;               // adjoint of the history term div(a So)
    double *sbxx, *sbyy, *sbzz, *sbxy, *sbxz, *sbyz;   // adjoint of the history So
    double* grad;                          // dJ/d(ln k0), accumulated
};
hipError_t launch_adj_porosity(const Geom& g, const Coef& c, const AdjPtrs& a, hipStream_t s);
hipError_t launch_adj_coef(const Geom& g, const Coef& c, const AdjPtrs& a, hipStream_t s);
hipError_t launch_adj_step(const Geom& g, const Coef& c, const AdjPtrs& a, hipStream_t s);
hipError_t launch_adj_history(const Geom& g, const Coef& c, const AdjPtrs& a, hipStream_t s);
hipError_t launch_adj_oldvalues(const Geom& g, const Coef& c, const double* rpt, const double* rpf, double* pto,
                                double* pfo, hipStream_t s);
hipError_t launch_absmax5(const Geom& g, const double* const* f, double* partials, int64_t nblocks,
                          hipStream_t s);
// Per-block maxima of a cell field (its cell extent only) into partials[b * 8]
// (the other seven slots 0), nblocks blocks.
hipError_t launch_cell_max(const Geom& g, const double* f, double* partials, int64_t nblocks, hipStream_t s);

}  // namespace ptk
