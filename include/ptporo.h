/*
 * ptporo.h -- C ABI of the MI355X (gfx950) pseudo-transient solver for 3D
 * poro-visco-elastic two-phase flow.
 *
 * The method is the pseudo-transient (PT) iteration of thesis article 1,
 * section 2.2: the residual system of eqs (17)-(22) with the closures
 * (23)-(27), advanced by the explicit update of eq (16) with the pressures'
 * local terms implicit, damped solid velocities and porosity in log space,
 * on the staggered grid of Fig. 1, with the boundary conditions of
 * eqs (33)-(34) (zero normal velocity, zero normal Darcy flux, free slip).
 * Coefficients k(phi), eta_phi(phi, R) and mu_s are lagged and refreshed
 * (Picard); the solver stops on the one-iteration change of the thesis or on
 * a relative residual.
 *
 * Conventions (all entry points)
 * ------------------------------
 * Ownership.  The caller owns every device buffer and the stream; the library
 *   owns only the handle.  It never allocates device memory: the scratch it
 *   needs is in caller buffers bound with pt_bind_workspace (and, for the
 *   mixed-precision solves and the adjoints, pt_bind_mixed_workspace and
 *   pt_bind_adjoint_workspace; the run adjoint's tape is an argument).
 *   Bound pointers must stay valid while the handle uses them.
 * Layout.  Every field is an FP64 array in one common padded box layout:
 *   element (i, j, k) of any staggered field is at offset
 *   (k * (ny + 1) + j) * row_pitch + i, x fastest, so each field buffer holds
 *   pt_field_elems() doubles.  Cells use i < nx, j < ny, k < nz; x-faces
 *   i <= nx; y-faces j <= ny; z-faces k <= nz; xy-edges i <= nx, j <= ny;
 *   xz-edges i <= nx, k <= nz; yz-edges j <= ny, k <= nz.  Entries outside a
 *   field's extent are never written, except by pt_reset_state, which fills
 *   whole buffers; the kernels may read them (every load stays inside the
 *   buffer) and ignore their values.  Base pointers must be 256-byte aligned;
 *   row_pitch >= nx + 1.
 * State.  The nine iterated fields (PT_VX .. PT_RZ) are double-buffered
 *   (Jacobi iteration: no point reads a value written in the same sweep).
 *   Bind both copies (copy 0 and 1); pt_current() tells which copy holds the
 *   present state.  Boundary-normal faces of V and R must hold zero in both
 *   copies; the library never writes them.
 * Synchrony.  Calls that launch work only enqueue it on the bound stream
 *   (default: the null stream), except where marked "synchronises".
 * Errors.  Every call returns a pt_status and never throws.  PT_EINVAL: a
 *   bad argument (nothing was launched).  PT_EDEVICE: a HIP error.
 *   PT_EDIVERGED: a non-finite norm.  PT_EDOMAIN: the porosity left (0, 1)
 *   (ln(1-phi) not in (-inf, 0)); the porosity step and the iterations that
 *   compute norms flag it, and the next call that reads norms,
 *   pt_picard_step or pt_set_porosity reports it.  PT_EDIVERGED, PT_EDOMAIN and PT_EDEVICE put the handle in
 *   its error state: every call that launches work returns PT_ESTATE until
 *   pt_begin_step, pt_set_params, pt_reset_state or pt_set_porosity (the
 *   caller repairs or reloads the fields first).  PT_ENOTCONV: an iteration
 *   limit was hit (the state is valid).  pt_last_error() holds a message for
 *   the last failure on the handle.
 * Threads.  One handle must not be used by two threads at once; distinct
 *   handles are independent.
 */
#ifndef PTPORO_H
#define PTPORO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PT_ABI_VERSION 4

typedef struct pt_grid pt_grid;

typedef enum {
    PT_OK = 0,
    PT_ENOTCONV = 1,
    PT_EINVAL = -1,
    PT_EDEVICE = -2,
    PT_EDIVERGED = -3,
    PT_EDOMAIN = -4,
    PT_ESTATE = -5
} pt_status;

/* Field identifiers.  The first PT_NPING are double-buffered. */
typedef enum {
    PT_VX = 0, PT_VY, PT_VZ,        /* solid velocity, x/y/z-faces                    */
    PT_PT, PT_PF,                   /* total and fluid pressure (cells)               */
    PT_LP,                          /* ln(1 - phi) (cells)                            */
    PT_RX, PT_RY, PT_RZ,            /* damped momentum residual, faces (stored at
                                       checks only: pt_sync_damped_residual)        */
    PT_PTO, PT_PFO, PT_LPO,         /* previous-step Pt, Pf, ln(1-phi) (cells)        */
    PT_SXX, PT_SYY, PT_SZZ,         /* stress history, cells                          */
    PT_SXY, PT_SXZ, PT_SYZ,         /* stress history, xy/xz/yz-edges                 */
    PT_FOX, PT_FOY, PT_FOZ,         /* divergence of the relaxed stress history, faces */
    PT_MN,                          /* lagged shear-viscosity factor (cells)          */
    PT_K0,                          /* per-cell k0/mu_f (cells; only with PT_F_K0FIELD) */
    PT_KC,                          /* lagged k/mu_f (cells)                          */
    PT_ETA,                         /* lagged bulk viscosity eta_phi (cells)          */
    PT_MUS,                         /* lagged solid shear viscosity mu_s (cells)      */
    PT_NFIELDS
} pt_field;

#define PT_NPING 9

/* Flags of pt_params.flags */
#define PT_F_POWERLAW 1u   /* eq (24): mu_s = mu0 / (1 + (tau_II/tau0)^(n-1))        */
#define PT_F_DPCAP    2u   /* Drucker-Prager cap of the lagged viscosity: at a refresh,
                               Mn_new = min(Mn_visc, Mn tau_y / tau_II) with
                               tau_y = max(C cos f + (Pt - Pf) sin f, tau_y_min), the
                               viscosity that puts the present strain rate on the yield
                               surface where it is below the viscous one (the paper has
                               no cap; its plasticity is the power law of eq (24))  */
#define PT_F_K0FIELD  4u   /* k0 is the per-cell field PT_K0, else the scalar kmuf0   */
#define PT_F_MECHOFF  8u   /* freeze V and Pt (linear fluid-pressure diffusion limit) */
#define PT_F_FP32_TALL 16u /* launch shape only: the FP32 correction sweep always takes its
                              14-row tiles (else the launch cost model picks 10 or 14 rows);
                              every tiling gives bitwise the same fields                  */
#define PT_F_DTS_RULE 32u  /* stress-history step of the appendix two-phase script (per-step
                              block): each pt_begin_step sets dtS = max(mu_s) / (G xi_w) and
                              renews the history when the time accumulated since the last
                              renewal (dt per step) reaches it; the first step of a run keeps
                              the zero history.  The update_history arguments are ignored. */

/* Non-dimensional physical and numerical parameters (article 1, Table 2 and
 * the appendix two-phase script; the readings of ambiguous values are listed
 * in the design notes). */
typedef struct {
    int32_t version;                /* must be PT_ABI_VERSION                          */
    uint32_t flags;                 /* PT_F_*                                          */
    double lx, ly, lz;              /* domain size                                     */
    double phi0;                    /* background porosity                             */
    double kmuf0;                   /* k0 / mu_f (scalar)                              */
    double eta0, mu0, cmu;          /* bulk-viscosity factor, shear factor, mu_s = Mn phi0 cmu */
    double rhofg, rhosg;            /* fluid, solid density x gravity (z up)           */
    double beta_phi, beta_d;        /* 1/K_phi, 1/K_d                                  */
    double alpha, B;                /* Biot-Willis, Skempton                           */
    double G;                       /* shear modulus                                   */
    double R0;                      /* decompaction weakening factor (Pf > Pt)         */
    double n_pow, tau0;             /* power-law exponent and stress                   */
    double coh, fric_deg, tau_y_min;/* Drucker-Prager cohesion, friction angle, floor  */
    double dt, dtS;                 /* physical step, stress-history step              */
    double beta_n;                  /* numerical compressibility                       */
    double rho_i;                   /* inertial density of the velocity update         */
    double c_v, c_pf;               /* pseudo-step safety factors                      */
    double damp_c;                  /* velocity damping d = 1 - damp_c / n             */
    int32_t nup;                    /* iterations between refreshes / checks           */
    int32_t pad_;
    double r_eta, r_mu;             /* log-relaxation of the thesis schedule           */
    double shear_bg;                /* background simple shear rate d(Vx_bg)/dy = tau_bg/mu0
                                       (eq (32)); 0 = none.  It enters the xy strain rate on
                                       every xy edge; on boundary xy edges, where the solved
                                       (perturbation) velocity slips freely, it is the only
                                       strain rate, with the viscosity of the cells inside  */
    double xsi_w;                   /* wanted xi of the PT_F_DTS_RULE step (> 0 with it)   */
} pt_params;

/* Residual norms and one-iteration changes (all infinity norms).
 *   f    : max |momentum residual| (no numerical compressibility, current Pt)
 *   rpt  : max |r_Pt|      rpf : max |r_Pf|        (eqs (17), (18))
 *   dl, dpt, dpf, dvz, dv : max change of ln(1-phi), Pt, Pf, Vz, |V| over
 *          the last checked iteration (the thesis's stopping quantity). */
typedef struct {
    double f, rpt, rpf, dl, dpt, dpf, dvz, dv;
} pt_norms;

/* Create a handle for an nx x ny x nz cell grid (each >= 2) with the given
 * row pitch (>= nx + 1, in elements) and parameters (copied).  The launch
 * shapes use the compute-unit count of the current device (256 if none can
 * be queried). */
pt_status pt_create(int32_t nx, int32_t ny, int32_t nz, int64_t row_pitch,
                    const pt_params* params, pt_grid** out);
pt_status pt_destroy(pt_grid* g);

/* Elements per field buffer: (nz + 1) * (ny + 1) * row_pitch. */
int64_t pt_field_elems(const pt_grid* g);

/* Bind a device buffer of pt_field_elems() doubles to a field.  copy is 0 or
 * 1 for the double-buffered fields (PT_VX .. PT_RZ) and 0 otherwise. */
pt_status pt_bind_field(pt_grid* g, int32_t field, int32_t copy, void* dev_ptr);

/* Workspace of the solver: per-block partial maxima of the norms and the
 * eight reduced norms (a few MB at the largest grids).  Query the size, then
 * bind a device buffer of at least that many bytes (256-byte aligned). */
pt_status pt_workspace_size(const pt_grid* g, size_t* bytes);
pt_status pt_bind_workspace(pt_grid* g, void* dev_ptr, size_t bytes);

/* Stream for all launches (a hipStream_t; NULL = the null stream). */
pt_status pt_set_stream(pt_grid* g, void* hip_stream);

/* Progress report of long calls (pt_picard_step, pt_adjoint_run):
 * fn(user, phase, step, stage, sweeps) is called on the calling thread after
 * every stage, with phase PT_PROGRESS_STAGE (a stage of pt_picard_step),
 * PT_PROGRESS_FORWARD (recorded forward), PT_PROGRESS_RECOMPUTE (a
 * checkpointed step recomputed) or PT_PROGRESS_REVERSE (a transposed stage
 * solve), and the stage's sweep count.  fn = NULL: no reports. */
#define PT_PROGRESS_FORWARD 0
#define PT_PROGRESS_REVERSE 1
#define PT_PROGRESS_RECOMPUTE 2
#define PT_PROGRESS_STAGE 3
typedef void (*pt_progress_fn)(void* user, int32_t phase, int32_t step, int32_t stage, int64_t sweeps);
pt_status pt_set_progress(pt_grid* g, pt_progress_fn fn, void* user);
pt_status pt_set_params(pt_grid* g, const pt_params* params);

/* Which copy (0/1) of a double-buffered field holds the present state. */
pt_status pt_current(const pt_grid* g, int32_t field, int32_t* copy);

/* Start of a physical step (thesis script, per-step block): Pto <- Pt,
 * Pfo <- Pf, ln(1-phi)o <- ln(1-phi); if update_history, the stress
 * history becomes the deviatoric stress of the present state (eq (21)
 * without the numerical-compressibility term) and the folded history term
 * Fo is recomputed.  Resets the within-step iteration counter. */
pt_status pt_begin_step(pt_grid* g, int32_t update_history);

/* Picard refresh of the lagged coefficients from the present state
 * (eqs (23)-(26), decompaction switch of eq (25), optional power law and
 * Drucker-Prager cap), with log relaxation weights r_eta, r_mu (1 = none);
 * the first refresh of a handle never relaxes.  Recomputes mu_s and Fo. */
pt_status pt_refresh(pt_grid* g, double r_eta, double r_mu);

/* One fused PT iteration (eq (16) applied to eqs (17)-(22)).
 * update_porosity = 1 also advances ln(1-phi) (thesis schedule), 0 keeps
 * it frozen (linear Picard stage).  want_norms = 1 computes the residual
 * norms at the incoming state and the one-iteration changes (read them with
 * pt_last_norms). */
pt_status pt_iteration(pt_grid* g, int32_t update_porosity, int32_t want_norms);

/* n iterations of the thesis schedule, continuing the step's count: a
 * refresh with the relaxation of pt_params before iterations with
 * (iter - 1) % nup == 0, norms on iterations with iter % nup == 0. */
pt_status pt_iterate(pt_grid* g, int64_t n);

/* Norms of the last iteration that computed them.  Synchronises. */
pt_status pt_last_norms(pt_grid* g, pt_norms* out);

/* Linear PT solve with coefficients and porosity frozen, until
 * rho = max(g_V / g_V0, g_P / g_P0) <= rtol (g_V = max|f|,
 * g_P = max(|r_Pt|, |r_Pf|); groups with zero reference norm are dropped),
 * checked every nup iterations, or max_iter.  The reference (g_V0, g_P0) is
 * the residual of the step's first solve: set by the first solve after
 * pt_begin_step and kept for the step's later Picard stages (a later stage
 * starts from a residual that is already small, so a stage-local reference
 * would ask for a reduction below round-off).  Synchronises.  Returns
 * PT_ENOTCONV at max_iter (the state is valid; calling again continues). */
pt_status pt_solve_linear(pt_grid* g, double rtol, int64_t max_iter,
                          int64_t* iters, double* rho);

/* pt_solve_linear for callers that cannot allocate or bind device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same solve, bit for bit, with the per-block maxima, the
 * reduced norms and the domain flag in a static device scratch of the
 * library (1 MiB per GPU, a file-scope array kept until the process ends)
 * instead of the bound workspace, which it does not need.  The caller still
 * binds every field.  The device current at the call must hold the grid's
 * buffers.  Grids with more than 16382 norm blocks (about 1100^3 cells) are
 * refused with PT_EINVAL before any launch.  Calls on one GPU share its
 * scratch: calls that overlap on one GPU (other threads, other streams)
 * race.  Allocates nothing (no hipMalloc, no library allocation);
 * synchronises; the norms of its last check are not readable afterwards
 * (pt_last_norms reports none). */
pt_status pt_solve_linear_static(pt_grid* g, double rtol, int64_t max_iter,
                                 int64_t* iters, double* rho);

/* The residual reference of the current step (both -1 if not yet set), and
 * setting it explicitly (negative values unset it). */
pt_status pt_residual_reference(const pt_grid* g, double* gv, double* gp);
pt_status pt_set_residual_reference(pt_grid* g, double gv, double gp);

/* Porosity time step after a converged Picard stage: ln(1-phi) =
 * ln(1-phi)o - dt dphi/dt(V, Pt, Pf) (eq (22)) with the present solid
 * fraction.  A cell leaving (0, 1) is flagged (PT_EDOMAIN at the next norm
 * read or at the end of pt_picard_step). */
pt_status pt_porosity_step(pt_grid* g);

/* Initial state of a run (the zero state of article 1's set-ups): V, R, Pt,
 * Pf (both copies), old pressures, stress history and its divergence Fo
 * <- 0; Mn <- mu0; the lagged coefficients take their values before the
 * first refresh (k/mu_f <- kmuf0, eta_phi <- 1, mu_s <- mu0 phi0 cmu).
 * ln(1-phi), its old value and k0 keep their contents (the present copy of
 * ln(1-phi) becomes copy 0); set the porosity with pt_set_porosity.
 * Clears the counters (pt_counters), the error state and the domain flag;
 * the next refresh is a run's first (no relaxation), the mixed solve's FP32
 * damped residual restarts at zero.  Writes whole field buffers. */
pt_status pt_reset_state(pt_grid* g);

/* ln(1-phi) and its old value <- ln(1 - phi) on the cells (the log-space
 * porosity of eq (22)), from phi_dev: an FP64 device buffer in the field
 * layout (cells), 256-byte aligned, owned by the caller.  Synchronises.
 * PT_EDOMAIN if some phi is not in (0, 1) (the values are written anyway).
 * Clears the error state first. */
pt_status pt_set_porosity(pt_grid* g, const void* phi_dev);

/* Host-side counters of a handle, for resuming a run on a new handle that
 * binds the same buffers: get them, destroy the handle, create a new one,
 * bind the same field and workspace buffers, set them; the run then
 * continues bit for bit.  iter: iterations of the present step (decides the
 * thesis schedule's refreshes and checks); refreshed: a refresh has run
 * (later ones relax); ref_set, ref_v, ref_p: the step's residual reference
 * (pt_solve_linear); cur: the copy holding the present value of each
 * double-buffered field; mixed_copy, mixed_clean: the mixed workspace copy
 * that holds the FP32 damped residual and whether the workspace is
 * initialised (kept only if the mixed workspace is bound when set); steps,
 * dt_cum, dts: the stress-history step rule's state (PT_F_DTS_RULE);
 * r_stored, v_prev: where the damped residual R of the present iterate is
 * (the PT_RX..RZ copies, or the two copies of V; see
 * pt_sync_damped_residual). */
typedef struct {
    int32_t version;                /* PT_ABI_VERSION                                  */
    int32_t refreshed;
    int64_t iter;
    int32_t ref_set, mixed_copy;
    double ref_v, ref_p;
    int32_t cur[PT_NPING];
    int32_t mixed_clean;
    int64_t steps;                  /* pt_begin_step calls since creation or reset     */
    double dt_cum, dts;             /* PT_F_DTS_RULE: time since the last renewal; dtS */
    int32_t r_stored, v_prev;       /* R in PT_RX..RZ; V's other copy is V_prev       */
} pt_counters;
pt_status pt_get_counters(const pt_grid* g, pt_counters* out);
pt_status pt_set_counters(pt_grid* g, const pt_counters* in);

/* The damped momentum residual R of the PT velocity update (the script's
 * damping: R' = f/rho_i + d R, V' = V + dtau_V R') is stored in PT_RX..RZ
 * only by the sweeps that compute norms (the checks; every refresh of the
 * schedules follows one), by every sweep of pt_solve_linear (whose tight
 * tolerances need the stored R's digits), by every sweep with
 * PT_F_MECHOFF, and before any
 * call that changes the pseudo steps or V outside the sweeps (pt_refresh,
 * pt_set_params, pt_solve_mixed, pt_solve_mg, checkpoints).  In between,
 * the FP64 sweeps take d R from the two copies of V (d (V - V_prev) /
 * dtau_V), which saves three of the sweep's 27 field streams.  This call
 * stores R of the present iterate in the present copies of PT_RX..RZ (a
 * no-op if they hold it); call it before reading them.  Enqueued. */
pt_status pt_sync_damped_residual(pt_grid* g);

/* Stage solvers of pt_picard_step. */
#define PT_SOLVER_FP64 0    /* pt_solve_linear                               */
#define PT_SOLVER_MIXED 1   /* pt_solve_mixed (FP32 sweeps, FP64 correction) */
#define PT_SOLVER_MG 2      /* pt_solve_mg (geometric multigrid V-cycles)    */

/* One physical step of the Picard schedule (the thesis's M-P driver): the
 * step set-up of pt_begin_step(update_history), then n_picard stages of
 * { refresh without relaxation (eqs (23)-(26)); linear solve of the frozen
 * system to the relative residual rtol by the solver `mixed` (PT_SOLVER_*):
 * pt_solve_linear; pt_solve_mixed with inner tolerance eta_in and at most
 * 64 corrections, max_iter sweeps per correction; or pt_solve_mg with at
 * most max_iter V-cycles; porosity step of eq (22) }.  sweeps: PT sweeps of
 * all stages (FP64 or FP32), V-cycles for the multigrid solver; rho: the
 * largest final relative residual.  Synchronises.  PT_ENOTCONV: a stage
 * missed rtol within its limits; the step stops there with a valid state.
 * The mixed and multigrid forms need their workspaces. */
pt_status pt_picard_step(pt_grid* g, int32_t update_history, int32_t n_picard, double rtol, int64_t max_iter,
                         int32_t mixed, double eta_in, int64_t* sweeps, double* rho);

/* ---- Geometric multigrid for the linear Picard stage -------------------
 * The thesis's outlook (concluding chapter, future work): geometric
 * multigrid over the PT iteration, which without damping is a weighted
 * Jacobi iteration.  Correction scheme, V-cycles.  Each coarse grid has
 * ceil(n/2) cells per axis on the same domain (odd counts give grids that
 * are not nested); transfers interpolate linearly between the grids' cell
 * centres and faces per staggering, restriction being the transpose with
 * rows normalised.  Smoother: nu1 / nu2 linear PT sweeps before / after the
 * coarse correction, without damping and without the numerical
 * compressibility beta_n (neither changes the solution), with pseudo steps
 * rho_i h^2 / (c_v mu_s), mu_s / n_pt and h^2 (1 + beta_d B/alpha) /
 * (c_pf k_loc).  Coarsest grid: coarse_sweeps damped PT sweeps with the
 * handle's parameters.  Coarse operators: the same discretisation with
 * k/mu_f averaged harmonically, eta_phi by eta_mean and mu_s, ln(1-phi)
 * arithmetically over the finer grid; the coarse right-hand side sits in
 * the coarse grid's Fo and old-pressure fields.  Needs beta_d > 0 and
 * alpha B != 1. */
#define PT_MG_MAX_LEVELS 12
typedef struct {
    int32_t version;          /* PT_ABI_VERSION                                      */
    int32_t levels;           /* grids including the fine one, 2..PT_MG_MAX_LEVELS;
                                 0: coarsen until an axis has at most 8 cells        */
    int32_t nu1, nu2;         /* smoothing sweeps before (>= 1) and after (>= 0)     */
    int32_t coarse_sweeps;    /* damped PT sweeps on the coarsest grid (>= 1)        */
    int32_t n_pt;             /* the smoother's Pt pseudo step mu_s / n_pt (>= 1)    */
    double c_v, c_pf;         /* the smoother's pseudo-step factors                  */
    int32_t krylov;           /* 0: plain cycles; 1..PT_MG_MAX_KRYLOV: Krylov
                                 acceleration keeping that many directions         */
    int32_t eta_mean;         /* eta_phi averaged down the hierarchy: 0 arithmetic,
                                 1 harmonic, 2 geometric mean                      */
} pt_mg_params;
#define PT_MG_MAX_KRYLOV 8

/* Workspace of a hierarchy (the fine grid's FP32 residual, the
 * restriction's scratch of less than one fine FP64 box, and per coarse
 * grid 25 FP64 boxes plus, above the coarsest, 5 FP32 boxes: about a
 * quarter of the fine grid's fields; with krylov = m, a further 5 (m + 1)
 * FP64 and 5 (m + 1) FP32 fine boxes): query, then bind a device buffer
 * (256-byte aligned) of at least that size; binding clears it (enqueued).
 * PT_EINVAL if the grid cannot be coarsened to the requested levels, and
 * at binding with krylov > 0 if the row pitch is not a multiple of 4 (the
 * Krylov kernels move 4 columns as one vector). */
pt_status pt_mg_workspace_size(const pt_grid* g, const pt_mg_params* mg, size_t* bytes);
pt_status pt_bind_mg_workspace(pt_grid* g, const pt_mg_params* mg, void* dev_ptr, size_t bytes);
/* The bound hierarchy: levels (0 if none) and, if counts is not NULL, the
 * cell counts nx, ny, nz of each grid (3 * levels values). */
pt_status pt_mg_levels(const pt_grid* g, int32_t* levels, int32_t* counts);

/* One linear Picard stage (coefficients and porosity frozen, as
 * pt_solve_linear) by multigrid: repeat { nu1 smoothing sweeps; residual of
 * the state in FP64 and rho as in pt_solve_linear (same step reference; if
 * the step has none, the residual of the starting state sets it); stop when
 * rho <= rtol or after max_cycles coarse corrections; coarse-grid
 * correction; nu2 sweeps }.  cycles: coarse corrections done.
 * Synchronises once per cycle.  PT_ENOTCONV if rtol is not met (the state
 * is valid; calling again continues).
 *
 * With krylov = m > 0 the cycles are Krylov-accelerated (the stage
 * system and the cycle are linear): after nu1 sweeps, each step runs one
 * cycle from the iterate x (correction, nu2 + nu1 sweeps) to y, and moves
 * to x' = y + sum_s gamma_s p_s, gamma minimising the residual of x' in the
 * residual norm weighted by the step reference over the stored directions
 * p_s (at most m: the cycles' own steps y - x, made orthogonal in that
 * norm through their images A(y - x) = r(x) - r(y)).  The cycle's step
 * itself is never scaled down: single cycles can raise the residual norm
 * before the following ones reduce it.  Directions are FP64, their images
 * FP32.  The stop is rho of x' or of y (then y is kept), <= rtol; each
 * step costs one cycle, two residuals and two vector passes (four
 * synchronisations).  A call starts without stored directions. */
pt_status pt_solve_mg(pt_grid* g, double rtol, int64_t max_cycles, int64_t* cycles, double* rho);

/* ---- Mixed precision (FP32 sweeps inside FP64 defect correction) --------
 * FP32 workspace for the correction system: query the size (24 FP32 padded
 * boxes, each pt_field_elems() + 64 floats apart), then bind a device buffer
 * (256-byte aligned) of at least that many bytes.  The library clears it
 * before first use.  Boxes 16..20 hold the FP64 residual of pt_residual
 * (f_x, f_y, f_z, r_Pt, r_Pf) in FP32, in the field layout. */
pt_status pt_mixed_workspace_size(const pt_grid* g, size_t* bytes);
pt_status pt_bind_mixed_workspace(pt_grid* g, void* dev_ptr, size_t bytes);

/* FP64 residuals f, r_Pt, r_Pf of the present state with the present
 * coefficients (the quantities whose infinity norms pt_solve_linear tests),
 * written to the mixed workspace in FP32; norms via pt_last_norms.  Needs the
 * mixed workspace. */
pt_status pt_residual(pt_grid* g);

/* One linear Picard stage solved by defect correction (coefficients and
 * porosity frozen, as pt_solve_linear): repeat { r = residual of x in FP64;
 * stop when rho (as in pt_solve_linear, same step reference) <= rtol; solve
 * A d = -r by FP32 PT sweeps from d = 0 (the damped residual of d carried
 * over from the previous correction) until the correction residual falls
 * to eta_in times r or to rtol/2 on the scale of rho (so that the last
 * correction solves only the gap left to rtol), stops improving (no new 1 %
 * minimum in 40 checks: the FP32 round-off floor) or max_inner sweeps,
 * checked every nup sweeps;
 * x += d in FP64 }.  At most max_outer corrections.  Synchronises.
 * PT_ENOTCONV if rtol is not met (calling again continues). */
pt_status pt_solve_mixed(pt_grid* g, double rtol, double eta_in, int64_t max_inner, int32_t max_outer,
                         int64_t* inner_iters, int32_t* outer_iters, double* rho);

/* ---- Adjoint of a linear Picard stage (gradient of a misfit) -------------
 * Misfit J = 1/2 sum_s (Pf(cell_s) - d_s)^2 over ns distinct sensor cells,
 * given as linear indices over the nx*ny*nz cells (x fastest).  FP64
 * workspace (40 boxes, each pt_field_elems() + 32 doubles apart, and a
 * sensor tail): query the size for a sensor capacity, then bind. */
pt_status pt_adjoint_workspace_size(const pt_grid* g, int32_t max_sensors, size_t* bytes);
pt_status pt_bind_adjoint_workspace(pt_grid* g, void* dev_ptr, size_t bytes, int32_t max_sensors);

/* k0 <- exp(logk0) on the cells (logk0: FP64 device buffer in the field
 * layout).  Needs PT_F_K0FIELD. */
pt_status pt_set_log_k0(pt_grid* g, const void* logk0_dev);

/* J of the present state (host arrays sensors[ns], d_obs[ns]).  Synchronises. */
pt_status pt_misfit(pt_grid* g, const int64_t* sensors, int32_t ns, const double* d_obs, double* J);

/* Gradient dJ/d(ln k0) for the present linear Picard stage, whose solution
 * the present state must be (coefficients and porosity as frozen for the
 * stage).  The stage's residual Jacobian J_F is symmetric on this grid, so
 * the adjoint J_F^T lambda = dJ/dx is solved by the stage's own PT sweep (FP64)
 * with right-hand side dJ/dx, until its residual falls to rtol times
 * max|dJ/dPf| (checked every nup sweeps) or max_iter; then
 * dJ/d(ln k0_c) = -lambda^T dF/d(ln k0_c), from the Darcy flux of eq (20)
 * (k = k0 (phi/phi0)^3), into grad_dev (FP64, field layout, cells).
 * Synchronises.  PT_ENOTCONV if rtol is not met (gradient still written). */
pt_status pt_adjoint_stage(pt_grid* g, const int64_t* sensors, int32_t ns, const double* d_obs, double rtol,
                           int64_t max_iter, void* grad_dev, double* J, int64_t* iters, double* rho);

/* ---- Adjoint of a recorded Picard run ------------------------------------
 * The run: from the present state, n_steps physical steps (the first without
 * a stress-history update, the later ones with it, eq (21)), each of
 * n_picard stages: refresh without relaxation (eqs (23)-(26)), linear solve
 * to rtol (as pt_solve_linear, reference of the step), porosity step
 * (eq (22)).  J = 1/2 sum_s (Pf_s - d_s)^2 at the end of the run.
 * The gradient dJ/d(ln k0) is the discrete adjoint of the converged run:
 * per stage in reverse order, the adjoint of the porosity step, the
 * transposed stage solve (the stage Jacobian is symmetric: FP64 PT sweeps
 * to adj_rtol times the right-hand side's max norm), the adjoints of k/mu_f,
 * 1/((1-phi) eta_phi), the buoyancy and the old values, and the chain of the
 * refresh k = k0 (phi/phi0)^3, eta_phi ~ phi0/phi back to the stage's
 * incoming ln(1-phi); per step boundary, the old values and the stress
 * history (So = a So_prev + b E(V), with history term div(a So)) carry the
 * adjoint to the previous step.  The decompaction switch R is piecewise
 * constant (no derivative).  Needs PT_F_K0FIELD and the Newtonian law (no
 * PT_F_POWERLAW, PT_F_DPCAP, PT_F_MECHOFF), and the adjoint workspace.
 *
 * options: PT_ADJ_CHECKPOINT (tape below) and PT_ADJ_MIXED: the forward
 * stages by pt_solve_mixed and the transposed solves by defect correction
 * too (FP32 sweeps; the FP64 residual of the transposed system is the stage
 * residual with gravity off and the right-hand side put in the history and
 * old-pressure terms; inner tolerance 1e-4, at most 64 corrections per
 * solve; needs the mixed workspace and beta_d > 0).
 * The tape is a caller-owned device buffer, 256-byte aligned, of at least
 * pt_adjoint_tape_size(options) bytes.  Without PT_ADJ_CHECKPOINT it receives every stage's V,
 * Pt, Pf, incoming ln(1-phi), k/mu_f and eta_phi (8 padded boxes per stage;
 * n_steps * n_picard * 8 boxes).  With PT_ADJ_CHECKPOINT it keeps each step's start
 * state (V, Pt, Pf, ln(1-phi), R, stress history: 15 boxes per step) plus
 * one step's stages (n_picard * 8 boxes); the reverse sweep recomputes each
 * step from its checkpoint, bitwise the recorded run, at the cost of a
 * second forward pass.  grad_dev: one FP64 padded box, overwritten (cells).
 * On return the grid holds the end state of the run (without
 * PT_ADJ_CHECKPOINT) or of its first step (with it).  Synchronises.  PT_ENOTCONV if a forward
 * or transposed solve misses its tolerance within max_iter (nothing after
 * it is computed). */
#define PT_ADJ_CHECKPOINT 1
#define PT_ADJ_MIXED 2
pt_status pt_adjoint_tape_size(const pt_grid* g, int32_t n_steps, int32_t n_picard, int32_t options,
                               size_t* bytes);
pt_status pt_adjoint_run(pt_grid* g, int32_t n_steps, int32_t n_picard, int32_t options, double rtol,
                         double adj_rtol, int64_t max_iter, const int64_t* sensors, int32_t ns, const double* d_obs,
                         void* tape, size_t tape_bytes, void* grad_dev, double* J, int64_t* fwd_iters,
                         int64_t* adj_iters);

/* Streaming copy of n doubles (achievable-bandwidth reference). */
pt_status pt_copy(pt_grid* g, const void* src, void* dst, int64_t n);

const char* pt_status_str(pt_status s);
const char* pt_last_error(const pt_grid* g);
int32_t pt_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PTPORO_H */
