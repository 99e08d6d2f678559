/*
 * ptwaves.h -- C ABI of the MI355X (gfx950) pseudo-transient solver for 3D
 * reactive porosity waves (thesis article 3; the appendix reactive script).
 *
 * The model: fluid pressure Pf, porosity phi and the volatile mass fraction
 * of the solid Xs (article 3, eqs (8)-(10)), effective pressure Pe = -Pf,
 * Darcy flux q = -k(phi)(grad Pf - rho_f g e_z) with k = k0/mu_f (phi/phi0)^3,
 * first-order reaction towards Xs_eq = clamp(beta_x Pf + Xs_max/2, 0, Xs_max)
 * (eq (4) in its nondimensional form, eq (10)), compressibilities
 * beta_P = phi beta_f + beta_d - (1 + phi) beta_s and
 * beta_phi = beta_d - beta_s/(1 - phi).  One implicit physical step dt is
 * found by pseudo-transient iterations on four cell fields (Xs, Pf, phi and
 * the fluid-pressure rate dPf/dt), every right-hand side at iteration k:
 *   Xs'     = Xs_old + dt (Xs_eq - Xs)/tau
 *   Pf'     = Pf + dtau (dPf/dt - (Pf - Pf_old)/dt)
 *   phi'    = clamp(phi_old + dt (1-phi)(beta_phi dPf/dt - Pe/(eta(1-phi))
 *             - (1+dX)/(1-Xs) dXs/dt), phi_min, phi_max)
 *   dPf/dt' = [-div q + Pe/(eta(1-phi)) + (1 - rho_s/(rho_f(1+dX)))(1-phi)
 *             (1+dX)/(1-Xs) dXs/dt] / beta_P
 * with the pseudo step dtau = h^2 / max(k/beta_P) / c_pf refreshed every
 * nup iterations, and the script's stopping quantity, the largest
 * one-iteration change of phi, Pf/10 and Xs, taken every nup iterations.
 * The pseudo steps after the first of a physical step take their maximum
 * from the check iteration just before (the same porosity), so a field the
 * caller writes in the middle of a step is seen by the pseudo step only
 * after the next pt_waves_begin_step.
 * Finite volumes on cells (dx = lx/nx), zero Darcy flux through the walls.
 *
 * Conventions as in ptporo.h: the caller owns every device buffer (the
 * library never allocates), one padded-box layout (element (i, j, k) at
 * (k (ny+1) + j) row_pitch + i, 256-byte aligned bases, row_pitch >= nx + 1;
 * only cells are used), calls only enqueue unless marked "synchronises",
 * status codes of ptporo.h, one handle per thread at a time.
 */
#ifndef PTWAVES_H
#define PTWAVES_H

#include "ptporo.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PT_WAVES_ABI_VERSION 1

typedef struct pt_waves pt_waves;

/* Fields; the first PT_W_NPING are double-buffered (Jacobi iteration). */
typedef enum {
    PT_W_XS = 0,      /* volatile mass fraction of the solid          */
    PT_W_PF,          /* fluid pressure                               */
    PT_W_PHI,         /* porosity                                     */
    PT_W_DPFDT,       /* fluid-pressure rate of the step              */
    PT_W_XSO, PT_W_PFO, PT_W_PHIO,   /* values at the previous step   */
    PT_W_NFIELDS
} pt_waves_field;
#define PT_W_NPING 4

/* Non-dimensional parameters (article 3, eqs (5)-(10): the scales of
 * eqs (5)-(7) are the units; the appendix reactive script's constants). */
typedef struct {
    int32_t version;                /* PT_WAVES_ABI_VERSION                     */
    int32_t nup;                    /* iterations between pseudo steps / checks */
    double lx, ly, lz;
    double phi0, k_muf0, eta;       /* background porosity, k0/mu_f, eta_phi    */
    double rho_f, rho_s, g;         /* densities and gravity (z up)             */
    double beta_d, beta_s, beta_f;  /* compressibilities                        */
    double tau;                     /* reaction time (1/Damkoehler)             */
    double beta_x, delta_x, xs_max; /* d Xs_eq/d Pf, solid density change, max  */
    double dt;                      /* physical step                            */
    double c_pf;                    /* pseudo-step safety factor                */
    double phi_min, phi_max;        /* porosity clamp                           */
} pt_waves_params;

pt_status pt_waves_create(int32_t nx, int32_t ny, int32_t nz, int64_t row_pitch, const pt_waves_params* params,
                          pt_waves** out);
pt_status pt_waves_destroy(pt_waves* w);
int64_t pt_waves_field_elems(const pt_waves* w);
/* copy 0 or 1 for the double-buffered fields, 0 otherwise. */
pt_status pt_waves_bind_field(pt_waves* w, int32_t field, int32_t copy, void* dev_ptr);
/* Per-block maxima, the reduced error and the pseudo step (a few MB). */
pt_status pt_waves_workspace_size(const pt_waves* w, size_t* bytes);
pt_status pt_waves_bind_workspace(pt_waves* w, void* dev_ptr, size_t bytes);
pt_status pt_waves_set_stream(pt_waves* w, void* hip_stream);
pt_status pt_waves_current(const pt_waves* w, int32_t field, int32_t* copy);

/* Start of a physical step: the old values Xs_old, Pf_old, phi_old <- the
 * present ones; resets the step's iteration count. */
pt_status pt_waves_begin_step(pt_waves* w);
/* n PT iterations continuing the step's count: the pseudo step before
 * iterations with (iter - 1) % nup == 0, the stopping quantity after
 * iterations with iter % nup == 0. */
pt_status pt_waves_iterate(pt_waves* w, int64_t n);
/* The stopping quantity of the last check.  Synchronises; PT_EDIVERGED if
 * it is not finite. */
pt_status pt_waves_last_error(pt_waves* w, double* err);
/* Iterate until the stopping quantity falls below eps (checked every nup
 * iterations) or the step's count reaches iter_max.  Synchronises.
 * PT_ENOTCONV at iter_max (the state is valid). */
pt_status pt_waves_solve_step(pt_waves* w, double eps, int64_t iter_max, int64_t* iters, double* err);
const char* pt_waves_last_message(const pt_waves* w);

#ifdef __cplusplus
}
#endif

#endif /* PTWAVES_H */
