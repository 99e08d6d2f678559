// Internal definitions shared by the kernels and the host side of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ptporo.h"

namespace ptk {

// Index layout common to every field: (k * (ny+1) + j) * P + i.
struct Geom {
    int nx, ny, nz;
    int64_t P;   // row pitch (elements)
    int64_t S;   // plane pitch = (ny + 1) * P
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
    int mech_off;
};

// Pointers of one PT sweep (inputs at iteration k, outputs at k + 1).
struct IterPtrs {
    const double *vx, *vy, *vz, *pt, *pf, *lp, *rx, *ry, *rz;
    const double *fox, *foy, *foz, *pto, *pfo, *lpo, *kc, *eta, *mus;
    double *vx_o, *vy_o, *vz_o, *pt_o, *pf_o, *lp_o, *rx_o, *ry_o, *rz_o;
    double* partials;              // [n_blocks][8] maxima (norm variant)
};

constexpr int NNORM = 8;

// Tile of the fused sweep: a BX x BY thread block covers a (BX-2) x (BY-2)
// output tile plus one halo column/row on every side and marches in z.
constexpr int BX = 64;
constexpr int BY = 8;
constexpr int KZ = 64;

inline int64_t iter_grid_blocks(const Geom& g) {
    int64_t gx = (g.nx + BX - 3) / (BX - 2);
    int64_t gy = (g.ny + BY - 3) / (BY - 2);
    int64_t gz = (g.nz + KZ - 1) / KZ;
    return gx * gy * gz;
}

// Launchers (defined in the .hip files).
hipError_t launch_iteration(const Geom& g, const Coef& c, const IterPtrs& p, int update_lp,
                            int norms, hipStream_t s);
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
    double *scr0, *scr1, *scr2;    // three padded-box scratch fields (workspace)
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
hipError_t launch_fo(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a,
                     hipStream_t s);
hipError_t launch_porosity_step(const Geom& g, const Coef& c, const AuxPtrs& a, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t s);

}  // namespace ptk
