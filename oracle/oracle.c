/*
 * oracle.c -- plain, slow FP64 CPU reference of the pseudo-transient (PT)
 * iteration for 3D poro-visco-elastic two-phase flow.
 *
 * TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no source with the GPU path.
 *
 * What it computes (thesis article 1, section 2.2):
 *   - the PT residual system, eqs (17)-(22), with the closures (23)-(27);
 *   - the explicit PT update of eq (16): pressures with their local terms
 *     taken implicitly, damped solid velocities, porosity in log space
 *     (the paragraph after Table 1);
 *   - the Picard refresh of the lagged coefficients k(phi), eta_phi(phi, R)
 *     and mu_s (eqs (23)-(26)) with log relaxation;
 *   - residual norms and the one-iteration change used by the thesis's
 *     stopping rule max|U_{tau+dtau} - U_tau| < eps (after eq (16)).
 *
 * Discretisation: finite volumes on a staggered grid (Fig. 1).  Pressures,
 * porosity and coefficients live in cell centres, velocities on faces,
 * normal stresses in cells and shear stresses on edges.  dx = lx/nx; faces
 * and edges on the domain boundary carry the boundary conditions of
 * eqs (33)-(34): zero normal velocity, zero normal Darcy flux and zero shear
 * stress (free slip).  z points up.
 *
 * Each stage is written as its own loop over the points it defines, with
 * every intermediate stored in a full array, in the order the equations are
 * stated.  Compile with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_ABI_VERSION 1

typedef struct {
    int32_t nx, ny, nz;
    double lx, ly, lz;
    double phi0, kmuf0, eta0, mu0, cmu, rhofg, rhosg;
    double beta_phi, beta_d, alpha, B, G, R0;
    double n_pow, tau0, coh, fric_deg, tau_y_min;
    double dt, dtS;
    double beta_n, rho_i, c_v, c_pf, damp_c;
    int32_t powerlaw, dpcap, mech_off, k0field;
    /* Grid counts used by the damping (1 - damp_c/n) and the Pt pseudo-step
     * (n_max) when the arrays cover only a window of a larger grid; 0 means
     * the arrays' own counts. */
    int32_t ngx, ngy, ngz;
    /* Grid spacings of the full grid for such a window (0: l/n). */
    double hx, hy, hz;
    /* Alternative readings of the iteration (OR_V_*), 0 for the readings
     * the solver implements.  They change the pseudo-time path only, never
     * the converged solution; tests use them to show why a reading was
     * taken. */
    int32_t variant;
    /* Background simple shear (article 1, eq (32)): the shear rate
     * d(Vx_bg)/dy of a background velocity Vx_bg(y) that enters the xy
     * strain rate on every xy-edge (0: none).  The solved velocity is the
     * perturbation; on boundary xy-edges its own strain rate is zero (free
     * slip), so they carry the background part alone. */
    double shear_bg;
} or_params;

/* beta_n r_Pt in the normal stresses evaluated at the updated Pt' instead of
 * the iteration-k values the script uses. */
#define OR_V_BETAN_UPDATED 1
/* velocity pseudo-step as printed in the script, rho_i h^2 (1+beta_n)/(c_v mu_s),
 * instead of dividing by (1+beta_n). */
#define OR_V_DTV_PRINTED 2
/* fluid-pressure pseudo-step from the cell's own k/mu_f, as printed, instead
 * of the largest of the cell and its face neighbours. */
#define OR_V_DTPF_CELL 4

/* Solver state: every pointer is a dense FP64 array, x fastest.
 *   cells:    nx*ny*nz
 *   x-faces:  (nx+1)*ny*nz     y-faces: nx*(ny+1)*nz   z-faces: nx*ny*(nz+1)
 *   xy-edges: (nx+1)*(ny+1)*nz  xz-edges: (nx+1)*ny*(nz+1)
 *   yz-edges: nx*(ny+1)*(nz+1) */
typedef struct {
    double *vx, *vy, *vz;          /* solid velocity (faces)                 */
    double *pt, *pf, *lp;          /* total, fluid pressure; lp = ln(1-phi)  */
    double *rx, *ry, *rz;          /* damped momentum residual (faces)       */
    double *pto, *pfo, *lpo;       /* values at the previous physical step   */
    double *sxx, *syy, *szz;       /* stress history (cells)                 */
    double *sxy, *sxz, *syz;       /* stress history (edges)                 */
    double *mn;                    /* lagged shear-viscosity factor (cells)  */
    double *k0;                    /* per-cell k0/mu_f, used if k0field      */
    double *kc, *eta, *mus;        /* lagged k/mu_f, eta_phi, mu_s (cells)   */
    /* Optional additive momentum source on the faces (NULL: none).  Only the
     * adjoint's transposed solves set it, to impose a right-hand side on the
     * momentum rows; the method itself has no such term.                    */
    double *fsx, *fsy, *fsz;
} or_state;

typedef struct {
    or_params p;
    int nx, ny, nz;
    double dx, dy, dz, h;
    int nmax;
    size_t nc, nfx, nfy, nfz, nexy, nexz, neyz;
    /* scratch */
    double *s, *divv, *rpt, *rpf, *ptn, *pfn, *lpn, *rhog;
    double *txx, *tyy, *tzz, *txy, *txz, *tyz;
    double *qx, *qy, *qz, *divq;
    double *fx, *fy, *fz;
    double *vxn, *vyn, *vzn, *rxn, *ryn, *rzn;
} or_ctx;

/* ---- index maps (x fastest) ---------------------------------------------- */
#define NX (c->nx)
#define NY (c->ny)
#define NZ (c->nz)
#define IC(i, j, k)   ((((size_t)(k)) * NY + (size_t)(j)) * NX + (size_t)(i))
#define IFX(i, j, k)  ((((size_t)(k)) * NY + (size_t)(j)) * (NX + 1) + (size_t)(i))
#define IFY(i, j, k)  ((((size_t)(k)) * (NY + 1) + (size_t)(j)) * NX + (size_t)(i))
#define IFZ(i, j, k)  ((((size_t)(k)) * NY + (size_t)(j)) * NX + (size_t)(i))
#define IEXY(i, j, k) ((((size_t)(k)) * (NY + 1) + (size_t)(j)) * (NX + 1) + (size_t)(i))
#define IEXZ(i, j, k) ((((size_t)(k)) * NY + (size_t)(j)) * (NX + 1) + (size_t)(i))
#define IEYZ(i, j, k) ((((size_t)(k)) * (NY + 1) + (size_t)(j)) * NX + (size_t)(i))

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

or_ctx *or_create(const or_params *p)
{
    if (!p || p->nx < 2 || p->ny < 2 || p->nz < 2) return NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->p = *p;
    c->nx = p->nx; c->ny = p->ny; c->nz = p->nz;
    c->dx = p->hx > 0.0 ? p->hx : p->lx / p->nx;
    c->dy = p->hy > 0.0 ? p->hy : p->ly / p->ny;
    c->dz = p->hz > 0.0 ? p->hz : p->lz / p->nz;
    c->h = dmin(c->dx, dmin(c->dy, c->dz));
    {
        int gx = p->ngx > 0 ? p->ngx : p->nx, gy = p->ngy > 0 ? p->ngy : p->ny, gz = p->ngz > 0 ? p->ngz : p->nz;
        c->nmax = gx > gy ? gx : gy;
        if (gz > c->nmax) c->nmax = gz;
    }
    size_t nx = p->nx, ny = p->ny, nz = p->nz;
    c->nc = nx * ny * nz;
    c->nfx = (nx + 1) * ny * nz; c->nfy = nx * (ny + 1) * nz; c->nfz = nx * ny * (nz + 1);
    c->nexy = (nx + 1) * (ny + 1) * nz; c->nexz = (nx + 1) * ny * (nz + 1);
    c->neyz = nx * (ny + 1) * (nz + 1);
    c->s = zalloc(c->nc); c->divv = zalloc(c->nc); c->rpt = zalloc(c->nc);
    c->rpf = zalloc(c->nc); c->ptn = zalloc(c->nc); c->pfn = zalloc(c->nc);
    c->lpn = zalloc(c->nc); c->rhog = zalloc(c->nc);
    c->txx = zalloc(c->nc); c->tyy = zalloc(c->nc); c->tzz = zalloc(c->nc);
    c->txy = zalloc(c->nexy); c->txz = zalloc(c->nexz); c->tyz = zalloc(c->neyz);
    c->qx = zalloc(c->nfx); c->qy = zalloc(c->nfy); c->qz = zalloc(c->nfz);
    c->divq = zalloc(c->nc);
    c->fx = zalloc(c->nfx); c->fy = zalloc(c->nfy); c->fz = zalloc(c->nfz);
    c->vxn = zalloc(c->nfx); c->vyn = zalloc(c->nfy); c->vzn = zalloc(c->nfz);
    c->rxn = zalloc(c->nfx); c->ryn = zalloc(c->nfy); c->rzn = zalloc(c->nfz);
    return c;
}

void or_destroy(or_ctx *c)
{
    if (!c) return;
    double *all[] = {c->s, c->divv, c->rpt, c->rpf, c->ptn, c->pfn, c->lpn, c->rhog,
                     c->txx, c->tyy, c->tzz, c->txy, c->txz, c->tyz, c->qx, c->qy,
                     c->qz, c->divq, c->fx, c->fy, c->fz, c->vxn, c->vyn, c->vzn,
                     c->rxn, c->ryn, c->rzn};
    for (size_t n = 0; n < sizeof(all) / sizeof(all[0]); ++n) free(all[n]);
    free(c);
}

int or_abi_version(void) { return OR_ABI_VERSION; }

#ifdef _OPENMP
#include <omp.h>
#endif
/* Number of threads the OpenMP loops use. */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the following OpenMP loops (timing only). */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Background density x gravity: rho_bg g = phi0 rho_f g + (1-phi0) rho_s g
 * (the script's rogBG).  Pressures are perturbations from the lithostatic
 * state of this density. */
static double rhobg_g(const or_ctx *c)
{
    return c->p.rhofg * c->p.phi0 + (1.0 - c->p.phi0) * c->p.rhosg;
}

/* ---- stage 0: solid fraction and density from ln(1-phi) (eq (27)) ---------- */
static void solid_fraction(or_ctx *c, const or_state *st)
{
    const or_params *p = &c->p;
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                size_t q = IC(i, j, k);
                double s = exp(st->lp[q]);
                double phi = 1.0 - s;
                c->s[q] = s;
                c->rhog[q] = p->rhofg * phi + p->rhosg * s;
            }
}

/* ---- stage 1: divergence of the solid velocity (cells) -------------------- */
static void divergence(or_ctx *c, const double *vx, const double *vy, const double *vz)
{
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i)
                c->divv[IC(i, j, k)] = (vx[IFX(i + 1, j, k)] - vx[IFX(i, j, k)]) / c->dx
                                     + (vy[IFY(i, j + 1, k)] - vy[IFY(i, j, k)]) / c->dy
                                     + (vz[IFZ(i, j, k + 1)] - vz[IFZ(i, j, k)]) / c->dz;
}

/* chi = 1/((1-phi) eta_phi), the bulk-viscous coupling of eqs (17)-(18). */
static double chi_at(const or_ctx *c, const or_state *st, size_t q)
{
    return 1.0 / (st->eta[q] * c->s[q]);
}

/* ---- stage 2: total-pressure residual of eq (17) (cells) ------------------ */
/* r_Pt = div V + beta_d((Pt-Pto) - alpha(Pf-Pfo))/dt + (Pt-Pf) chi, evaluated
 * with the total pressure ptv (the current Pt, or the updated Pt').          */
static void total_pressure_residual(or_ctx *c, const or_state *st, const double *ptv)
{
    const or_params *p = &c->p;
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                size_t q = IC(i, j, k);
                double chi = chi_at(c, st, q);
                c->rpt[q] = c->divv[q]
                          + p->beta_d * ((ptv[q] - st->pto[q]) - p->alpha * (st->pf[q] - st->pfo[q])) / p->dt
                          + (ptv[q] - st->pf[q]) * chi;
            }
}

/* ---- stage 3: Darcy flux, eq (20), and fluid-pressure residual, eq (18) ---- */
/* q = -k/mu_f (grad Pf + (rho_f g - rho_bg g) e_z) on interior faces,
 * q.n = 0 on boundary faces (eq (34)); face k/mu_f is the mean of the two
 * cells.  r_Pf = div q + beta_d((alpha/B)(Pf-Pfo) - alpha(Pt-Pto))/dt
 *              + (Pf-Pt) chi.                                               */
static void fluid_pressure_residual(or_ctx *c, const or_state *st)
{
    const or_params *p = &c->p;
    const double buoy = p->rhofg - rhobg_g(c);
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i <= NX; ++i) {
                double q = 0.0;
                if (i > 0 && i < NX) {
                    double kf = 0.5 * (st->kc[IC(i - 1, j, k)] + st->kc[IC(i, j, k)]);
                    q = -kf * (st->pf[IC(i, j, k)] - st->pf[IC(i - 1, j, k)]) / c->dx;
                }
                c->qx[IFX(i, j, k)] = q;
            }
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j <= NY; ++j)
            for (int i = 0; i < NX; ++i) {
                double q = 0.0;
                if (j > 0 && j < NY) {
                    double kf = 0.5 * (st->kc[IC(i, j - 1, k)] + st->kc[IC(i, j, k)]);
                    q = -kf * (st->pf[IC(i, j, k)] - st->pf[IC(i, j - 1, k)]) / c->dy;
                }
                c->qy[IFY(i, j, k)] = q;
            }
#pragma omp parallel for
    for (int k = 0; k <= NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                double q = 0.0;
                if (k > 0 && k < NZ) {
                    double kf = 0.5 * (st->kc[IC(i, j, k - 1)] + st->kc[IC(i, j, k)]);
                    q = -kf * ((st->pf[IC(i, j, k)] - st->pf[IC(i, j, k - 1)]) / c->dz + buoy);
                }
                c->qz[IFZ(i, j, k)] = q;
            }
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                size_t q = IC(i, j, k);
                c->divq[q] = (c->qx[IFX(i + 1, j, k)] - c->qx[IFX(i, j, k)]) / c->dx
                           + (c->qy[IFY(i, j + 1, k)] - c->qy[IFY(i, j, k)]) / c->dy
                           + (c->qz[IFZ(i, j, k + 1)] - c->qz[IFZ(i, j, k)]) / c->dz;
                double chi = chi_at(c, st, q);
                c->rpf[q] = c->divq[q]
                          + p->beta_d * ((p->alpha / p->B) * (st->pf[q] - st->pfo[q])
                                         - p->alpha * (st->pt[q] - st->pto[q])) / p->dt
                          + (st->pf[q] - st->pt[q]) * chi;
            }
}

/* ---- stage 4: visco-elastic deviatoric stresses, eq (21) ------------------ */
/* Backward-Euler Maxwell: tau = a*So + b*(edot + beta_n r_Pt [normal only]),
 * xi = mu_s/(G dtS), a = xi/(1+xi), b = 2 mu_s/(1+xi).  On edges xi and mu_s
 * are the means of the four neighbouring cells.  Boundary edges carry zero
 * shear stress.  with_betan = 0 drops the numerical-compressibility term.  */
static void stresses(or_ctx *c, const or_state *st, int with_betan)
{
    const or_params *p = &c->p;
    const double bn = with_betan ? p->beta_n : 0.0;
    const double gdt = p->G * p->dtS;
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                size_t q = IC(i, j, k);
                double mu = st->mus[q];
                double xi = mu / gdt;
                double a = xi / (1.0 + xi);
                double b = 2.0 * mu / (1.0 + xi);
                double dv3 = c->divv[q] / 3.0;
                double exx = (st->vx[IFX(i + 1, j, k)] - st->vx[IFX(i, j, k)]) / c->dx - dv3;
                double eyy = (st->vy[IFY(i, j + 1, k)] - st->vy[IFY(i, j, k)]) / c->dy - dv3;
                double ezz = (st->vz[IFZ(i, j, k + 1)] - st->vz[IFZ(i, j, k)]) / c->dz - dv3;
                double comp = bn * c->rpt[q];
                c->txx[q] = a * st->sxx[q] + b * (exx + comp);
                c->tyy[q] = a * st->syy[q] + b * (eyy + comp);
                c->tzz[q] = a * st->szz[q] + b * (ezz + comp);
            }
    const double gbg = p->shear_bg;
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j <= NY; ++j)
            for (int i = 0; i <= NX; ++i) {
                double t = 0.0;
                if (i > 0 && i < NX && j > 0 && j < NY) {
                    double mue = 0.25 * (st->mus[IC(i - 1, j - 1, k)] + st->mus[IC(i, j - 1, k)]
                                       + st->mus[IC(i - 1, j, k)] + st->mus[IC(i, j, k)]);
                    double xie = mue / gdt;
                    double a = xie / (1.0 + xie);
                    double b = 2.0 * mue / (1.0 + xie);
                    double exy = 0.5 * ((st->vx[IFX(i, j, k)] - st->vx[IFX(i, j - 1, k)]) / c->dy
                                      + (st->vy[IFY(i, j, k)] - st->vy[IFY(i - 1, j, k)]) / c->dx);
                    if (gbg != 0.0) exy += 0.5 * gbg;
                    t = a * st->sxy[IEXY(i, j, k)] + b * exy;
                } else if (gbg != 0.0) {
                    /* boundary edge: the background strain rate only, with
                     * the viscosity averaged over the cells inside */
                    double sum = 0.0;
                    int cnt = 0;
                    for (int jj = j - 1; jj <= j; ++jj)
                        for (int ii = i - 1; ii <= i; ++ii)
                            if (ii >= 0 && ii < NX && jj >= 0 && jj < NY) {
                                sum += st->mus[IC(ii, jj, k)];
                                ++cnt;
                            }
                    double mue = sum / cnt;
                    double xie = mue / gdt;
                    double a = xie / (1.0 + xie);
                    double b = 2.0 * mue / (1.0 + xie);
                    t = a * st->sxy[IEXY(i, j, k)] + b * (0.5 * gbg);
                }
                c->txy[IEXY(i, j, k)] = t;
            }
#pragma omp parallel for
    for (int k = 0; k <= NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i <= NX; ++i) {
                double t = 0.0;
                if (i > 0 && i < NX && k > 0 && k < NZ) {
                    double mue = 0.25 * (st->mus[IC(i - 1, j, k - 1)] + st->mus[IC(i, j, k - 1)]
                                       + st->mus[IC(i - 1, j, k)] + st->mus[IC(i, j, k)]);
                    double xie = mue / gdt;
                    double a = xie / (1.0 + xie);
                    double b = 2.0 * mue / (1.0 + xie);
                    double exz = 0.5 * ((st->vx[IFX(i, j, k)] - st->vx[IFX(i, j, k - 1)]) / c->dz
                                      + (st->vz[IFZ(i, j, k)] - st->vz[IFZ(i - 1, j, k)]) / c->dx);
                    t = a * st->sxz[IEXZ(i, j, k)] + b * exz;
                }
                c->txz[IEXZ(i, j, k)] = t;
            }
#pragma omp parallel for
    for (int k = 0; k <= NZ; ++k)
        for (int j = 0; j <= NY; ++j)
            for (int i = 0; i < NX; ++i) {
                double t = 0.0;
                if (j > 0 && j < NY && k > 0 && k < NZ) {
                    double mue = 0.25 * (st->mus[IC(i, j - 1, k - 1)] + st->mus[IC(i, j, k - 1)]
                                       + st->mus[IC(i, j - 1, k)] + st->mus[IC(i, j, k)]);
                    double xie = mue / gdt;
                    double a = xie / (1.0 + xie);
                    double b = 2.0 * mue / (1.0 + xie);
                    double eyz = 0.5 * ((st->vy[IFY(i, j, k)] - st->vy[IFY(i, j, k - 1)]) / c->dz
                                      + (st->vz[IFZ(i, j, k)] - st->vz[IFZ(i, j - 1, k)]) / c->dy);
                    t = a * st->syz[IEYZ(i, j, k)] + b * eyz;
                }
                c->tyz[IEYZ(i, j, k)] = t;
            }
}

/* ---- stage 5: total momentum balance, eq (19) (interior faces) ------------- */
/* f = div(tau) - grad P - (rho g - rho_bg g) e_z, with P the pressure given
 * (the updated Pt in the PT iteration, the current Pt for the residual),
 * plus the optional source of the state.
 * Boundary faces: f = 0 (not updated, normal velocity fixed at zero).        */
static void momentum(or_ctx *c, const or_state *st, const double *ptp)
{
    const double rbg = rhobg_g(c);
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i <= NX; ++i) {
                double f = 0.0;
                if (i > 0 && i < NX)
                    f = (c->txx[IC(i, j, k)] - c->txx[IC(i - 1, j, k)]) / c->dx
                      + (c->txy[IEXY(i, j + 1, k)] - c->txy[IEXY(i, j, k)]) / c->dy
                      + (c->txz[IEXZ(i, j, k + 1)] - c->txz[IEXZ(i, j, k)]) / c->dz
                      - (ptp[IC(i, j, k)] - ptp[IC(i - 1, j, k)]) / c->dx;
                if (st->fsx && i > 0 && i < NX) f += st->fsx[IFX(i, j, k)];
                c->fx[IFX(i, j, k)] = f;
            }
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j <= NY; ++j)
            for (int i = 0; i < NX; ++i) {
                double f = 0.0;
                if (j > 0 && j < NY)
                    f = (c->txy[IEXY(i + 1, j, k)] - c->txy[IEXY(i, j, k)]) / c->dx
                      + (c->tyy[IC(i, j, k)] - c->tyy[IC(i, j - 1, k)]) / c->dy
                      + (c->tyz[IEYZ(i, j, k + 1)] - c->tyz[IEYZ(i, j, k)]) / c->dz
                      - (ptp[IC(i, j, k)] - ptp[IC(i, j - 1, k)]) / c->dy;
                if (st->fsy && j > 0 && j < NY) f += st->fsy[IFY(i, j, k)];
                c->fy[IFY(i, j, k)] = f;
            }
#pragma omp parallel for
    for (int k = 0; k <= NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                double f = 0.0;
                if (k > 0 && k < NZ)
                    f = (c->txz[IEXZ(i + 1, j, k)] - c->txz[IEXZ(i, j, k)]) / c->dx
                      + (c->tyz[IEYZ(i, j + 1, k)] - c->tyz[IEYZ(i, j, k)]) / c->dy
                      + (c->tzz[IC(i, j, k)] - c->tzz[IC(i, j, k - 1)]) / c->dz
                      - (ptp[IC(i, j, k)] - ptp[IC(i, j, k - 1)]) / c->dz
                      - (0.5 * (c->rhog[IC(i, j, k - 1)] + c->rhog[IC(i, j, k)]) - rbg);
                if (st->fsz && k > 0 && k < NZ) f += st->fsz[IFZ(i, j, k)];
                c->fz[IFZ(i, j, k)] = f;
            }
}

/* ---- stage 6: porosity rate in log space, eq (22) --------------------------- */
/* d phi/dt = beta_phi((Pf-Pfo) - (Pt-Pto))/dt + (Pf-Pt)/eta_phi + V.grad(1-phi)
 * with the advection term averaged from the faces to the cell centre and the
 * boundary faces contributing nothing (V.n = 0 there).  The new log solid
 * fraction is L = Lo - dt * dphi/dt.                                          */
static void porosity_update(or_ctx *c, const or_state *st, const double *ptn,
                            const double *pfn, double *lpn)
{
    const or_params *p = &c->p;
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                size_t q = IC(i, j, k);
                double s = c->s[q];
                double adv = 0.0;
                if (i > 0)      adv += 0.5 * st->vx[IFX(i, j, k)] * (s - c->s[IC(i - 1, j, k)]) / c->dx;
                if (i < NX - 1) adv += 0.5 * st->vx[IFX(i + 1, j, k)] * (c->s[IC(i + 1, j, k)] - s) / c->dx;
                if (j > 0)      adv += 0.5 * st->vy[IFY(i, j, k)] * (s - c->s[IC(i, j - 1, k)]) / c->dy;
                if (j < NY - 1) adv += 0.5 * st->vy[IFY(i, j + 1, k)] * (c->s[IC(i, j + 1, k)] - s) / c->dy;
                if (k > 0)      adv += 0.5 * st->vz[IFZ(i, j, k)] * (s - c->s[IC(i, j, k - 1)]) / c->dz;
                if (k < NZ - 1) adv += 0.5 * st->vz[IFZ(i, j, k + 1)] * (c->s[IC(i, j, k + 1)] - s) / c->dz;
                double dphidt = p->beta_phi * ((pfn[q] - st->pfo[q]) - (ptn[q] - st->pto[q])) / p->dt
                              + (pfn[q] - ptn[q]) / st->eta[q]
                              + adv;
                lpn[q] = st->lpo[q] - p->dt * dphidt;
            }
}

/* ---- pseudo-time steps ------------------------------------------------------ */
/* dtau_V  = rho_i h^2 / (c_v mu_s (1+beta_n))            at cells, and on a
 *           face the smaller of its two cells' values;
 * dtau_Pt = mu_s (1+beta_n) / n_max;
 * dtau_Pf = h^2 (1 + beta_d B/alpha) / (c_pf k_loc), k_loc the largest k/mu_f
 *           of the cell and its face neighbours.                              */
static double dtau_v_cell(const or_ctx *c, double mus)
{
    const or_params *p = &c->p;
    if (p->variant & OR_V_DTV_PRINTED)
        return p->rho_i * c->h * c->h * (1.0 + p->beta_n) / (p->c_v * mus);
    return p->rho_i * c->h * c->h / (p->c_v * mus * (1.0 + p->beta_n));
}

static double dtau_pf_cell(const or_ctx *c, const or_state *st, int i, int j, int k)
{
    const or_params *p = &c->p;
    double km = st->kc[IC(i, j, k)];
    if (p->variant & OR_V_DTPF_CELL)
        return c->h * c->h * (1.0 + p->beta_d * p->B / p->alpha) / (p->c_pf * km);
    if (i > 0)      km = dmax(km, st->kc[IC(i - 1, j, k)]);
    if (i < NX - 1) km = dmax(km, st->kc[IC(i + 1, j, k)]);
    if (j > 0)      km = dmax(km, st->kc[IC(i, j - 1, k)]);
    if (j < NY - 1) km = dmax(km, st->kc[IC(i, j + 1, k)]);
    if (k > 0)      km = dmax(km, st->kc[IC(i, j, k - 1)]);
    if (k < NZ - 1) km = dmax(km, st->kc[IC(i, j, k + 1)]);
    return c->h * c->h * (1.0 + p->beta_d * p->B / p->alpha) / (p->c_pf * km);
}

/* norms[] layout shared with the Python driver:
 *   0: max |f| (momentum residual, no beta_n term, current Pt)
 *   1: max |r_Pt|      2: max |r_Pf|
 *   3: max |dL|        4: max |dPt|     5: max |dPf|     6: max |dVz|
 *   7: max |dV| over all three components                                   */
#define OR_NNORMS 8

/* Maxima that keep a NaN (a diverged iterate must not look converged). */
static double nmax(double a, double b)
{
    if (a != a || b != b) return NAN;
    return a > b ? a : b;
}

static double amax_diff(const double *a, const double *b, size_t n)
{
    double m = 0.0;
    for (size_t q = 0; q < n; ++q) m = nmax(m, fabs(a[q] - b[q]));
    return m;
}

static double amax(const double *a, size_t n)
{
    double m = 0.0;
    for (size_t q = 0; q < n; ++q) m = nmax(m, fabs(a[q]));
    return m;
}

/* Residuals of the discrete system at the current state with the current
 * (frozen) coefficients: momentum f (no numerical compressibility, current
 * Pt), r_Pt and r_Pf.  Written to the caller's arrays (any may be NULL).     */
void or_residual(or_ctx *c, const or_state *st, double *fx, double *fy, double *fz,
                 double *rpt, double *rpf)
{
    solid_fraction(c, st);
    divergence(c, st->vx, st->vy, st->vz);
    total_pressure_residual(c, st, st->pt);
    fluid_pressure_residual(c, st);
    stresses(c, st, 0);
    momentum(c, st, st->pt);
    if (fx) memcpy(fx, c->fx, c->nfx * sizeof(double));
    if (fy) memcpy(fy, c->fy, c->nfy * sizeof(double));
    if (fz) memcpy(fz, c->fz, c->nfz * sizeof(double));
    if (rpt) memcpy(rpt, c->rpt, c->nc * sizeof(double));
    if (rpf) memcpy(rpf, c->rpf, c->nc * sizeof(double));
}

/* One PT iteration (Jacobi: every right-hand side uses iteration-k values).
 * update_lp = 1: porosity is updated every iteration (thesis schedule);
 * update_lp = 0: porosity is frozen (linear Picard stage).
 * norms (may be NULL): residuals at the incoming state and the change.       */
void or_iteration(or_ctx *c, or_state *st, int update_lp, double *norms)
{
    const or_params *p = &c->p;
    const int nx = NX, ny = NY, nz = NZ;

    if (norms) {
        or_residual(c, st, NULL, NULL, NULL, NULL, NULL);
        norms[0] = nmax(amax(c->fx, c->nfx), nmax(amax(c->fy, c->nfy), amax(c->fz, c->nfz)));
        norms[1] = amax(c->rpt, c->nc);
        norms[2] = amax(c->rpf, c->nc);
    }

    solid_fraction(c, st);
    divergence(c, st->vx, st->vy, st->vz);
    total_pressure_residual(c, st, st->pt);
    fluid_pressure_residual(c, st);

    /* Pressures: P' = P - dtau * r(P') with the terms local in P implicit
     * (eq (16) applied to eqs (17), (18)); Pt' uses Pf^k and Pf' uses Pt^k. */
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t q = IC(i, j, k);
                double chi = chi_at(c, st, q);
                if (p->mech_off) {
                    c->ptn[q] = st->pt[q];
                } else {
                    double dtp = st->mus[q] * (1.0 + p->beta_n) / c->nmax;
                    double num = st->pt[q] - dtp * (c->divv[q]
                                 + p->beta_d * (-st->pto[q] - p->alpha * (st->pf[q] - st->pfo[q])) / p->dt
                                 - st->pf[q] * chi);
                    double den = 1.0 + dtp * (p->beta_d / p->dt + chi);
                    c->ptn[q] = num / den;
                }
                double dtf = dtau_pf_cell(c, st, i, j, k);
                double num = st->pf[q] - dtf * (c->divq[q]
                             + p->beta_d * (-(p->alpha / p->B) * st->pfo[q] - p->alpha * (st->pt[q] - st->pto[q])) / p->dt
                             - st->pt[q] * chi);
                double den = 1.0 + dtf * (p->beta_d * p->alpha / (p->B * p->dt) + chi);
                c->pfn[q] = num / den;
            }

    /* Stresses from V^k with the numerical-compressibility term beta_n r_Pt
     * of iteration k (r_Pt above, formed before the pressure update, as the
     * script forms it); momentum with the updated Pt'. */
    if (p->variant & OR_V_BETAN_UPDATED)
        total_pressure_residual(c, st, c->ptn);
    stresses(c, st, 1);
    momentum(c, st, c->ptn);

    /* Damped velocity update: R' = f/rho_i + d R, V' = V + dtau_V R'. */
    const double dmx = 1.0 - p->damp_c / (p->ngx > 0 ? p->ngx : nx);
    const double dmy = 1.0 - p->damp_c / (p->ngy > 0 ? p->ngy : ny);
    const double dmz = 1.0 - p->damp_c / (p->ngz > 0 ? p->ngz : nz);
    memcpy(c->vxn, st->vx, c->nfx * sizeof(double));
    memcpy(c->vyn, st->vy, c->nfy * sizeof(double));
    memcpy(c->vzn, st->vz, c->nfz * sizeof(double));
    memcpy(c->rxn, st->rx, c->nfx * sizeof(double));
    memcpy(c->ryn, st->ry, c->nfy * sizeof(double));
    memcpy(c->rzn, st->rz, c->nfz * sizeof(double));
    if (!p->mech_off) {
#pragma omp parallel for
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 1; i < nx; ++i) {
                    size_t q = IFX(i, j, k);
                    double r = c->fx[q] / p->rho_i + dmx * st->rx[q];
                    double dtv = dmin(dtau_v_cell(c, st->mus[IC(i - 1, j, k)]), dtau_v_cell(c, st->mus[IC(i, j, k)]));
                    c->rxn[q] = r;
                    c->vxn[q] = st->vx[q] + dtv * r;
                }
#pragma omp parallel for
        for (int k = 0; k < nz; ++k)
            for (int j = 1; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t q = IFY(i, j, k);
                    double r = c->fy[q] / p->rho_i + dmy * st->ry[q];
                    double dtv = dmin(dtau_v_cell(c, st->mus[IC(i, j - 1, k)]), dtau_v_cell(c, st->mus[IC(i, j, k)]));
                    c->ryn[q] = r;
                    c->vyn[q] = st->vy[q] + dtv * r;
                }
#pragma omp parallel for
        for (int k = 1; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t q = IFZ(i, j, k);
                    double r = c->fz[q] / p->rho_i + dmz * st->rz[q];
                    double dtv = dmin(dtau_v_cell(c, st->mus[IC(i, j, k - 1)]), dtau_v_cell(c, st->mus[IC(i, j, k)]));
                    c->rzn[q] = r;
                    c->vzn[q] = st->vz[q] + dtv * r;
                }
    }

    if (update_lp)
        porosity_update(c, st, c->ptn, c->pfn, c->lpn);
    else
        memcpy(c->lpn, st->lp, c->nc * sizeof(double));

    if (norms) {
        norms[3] = amax_diff(c->lpn, st->lp, c->nc);
        norms[4] = amax_diff(c->ptn, st->pt, c->nc);
        norms[5] = amax_diff(c->pfn, st->pf, c->nc);
        norms[6] = amax_diff(c->vzn, st->vz, c->nfz);
        norms[7] = nmax(norms[6], nmax(amax_diff(c->vxn, st->vx, c->nfx), amax_diff(c->vyn, st->vy, c->nfy)));
    }

    memcpy(st->pt, c->ptn, c->nc * sizeof(double));
    memcpy(st->pf, c->pfn, c->nc * sizeof(double));
    memcpy(st->lp, c->lpn, c->nc * sizeof(double));
    memcpy(st->vx, c->vxn, c->nfx * sizeof(double));
    memcpy(st->vy, c->vyn, c->nfy * sizeof(double));
    memcpy(st->vz, c->vzn, c->nfz * sizeof(double));
    memcpy(st->rx, c->rxn, c->nfx * sizeof(double));
    memcpy(st->ry, c->ryn, c->nfy * sizeof(double));
    memcpy(st->rz, c->rzn, c->nfz * sizeof(double));
}

/* Porosity time update after a converged Picard stage: L = Lo - dt dphi/dt
 * evaluated at the solved V, Pt, Pf with the current solid fraction.       */
void or_porosity_step(or_ctx *c, or_state *st)
{
    solid_fraction(c, st);
    porosity_update(c, st, st->pt, st->pf, c->lpn);
    memcpy(st->lp, c->lpn, c->nc * sizeof(double));
}

/* Start of a physical time step: store the old pressures and porosity; if
 * update_history, store the deviatoric stress of the current state (without
 * the numerical-compressibility term) as the new stress history.            */
void or_begin_step(or_ctx *c, or_state *st, int update_history)
{
    if (update_history) {
        solid_fraction(c, st);
        divergence(c, st->vx, st->vy, st->vz);
        total_pressure_residual(c, st, st->pt);
        stresses(c, st, 0);
        memcpy(st->sxx, c->txx, c->nc * sizeof(double));
        memcpy(st->syy, c->tyy, c->nc * sizeof(double));
        memcpy(st->szz, c->tzz, c->nc * sizeof(double));
        memcpy(st->sxy, c->txy, c->nexy * sizeof(double));
        memcpy(st->sxz, c->txz, c->nexz * sizeof(double));
        memcpy(st->syz, c->tyz, c->neyz * sizeof(double));
    }
    memcpy(st->pto, st->pt, c->nc * sizeof(double));
    memcpy(st->pfo, st->pf, c->nc * sizeof(double));
    memcpy(st->lpo, st->lp, c->nc * sizeof(double));
}

/* Picard refresh of the lagged coefficients from the current state
 * (eqs (23)-(26)):
 *   k/mu_f   = k0 (phi/phi0)^3 / mu_f                          (eq (23))
 *   R        = 1/R0 if Pf > Pt, else 1                          (eq (25))
 *   eta_new  = eta0 Mn (phi0/phi) R; eta = exp(r_eta ln eta_new + (1-r_eta) ln eta)
 *   tau_II   from the deviatoric stress of the current state without the
 *            numerical-compressibility term (edges averaged to centres)
 *   Mn_visc  = mu0 / (1 + (tau_II/tau0)^(n-1))  (power law, eq (24)) or mu0
 *   cap      : tau_y = max(C cos(f) + (Pt-Pf) sin(f), tau_y_min);
 *              Mn_new = min(Mn_visc, Mn tau_y/tau_II) where tau_II > 0, i.e.
 *              the viscosity that would put the present strain rate on the
 *              yield surface, where that is below the viscous one (a cell
 *              at the yield surface keeps its Mn: yielded fixed points)
 *   Mn       = exp(r_mu ln Mn_new + (1-r_mu) ln Mn);  mu_s = Mn phi0 cmu
 * first = 1 takes the new values without relaxation.  The stress invariant
 * uses the coefficients in force before this refresh.                       */
void or_refresh(or_ctx *c, or_state *st, int first, double r_eta, double r_mu)
{
    const or_params *p = &c->p;
    const int need_tau = p->powerlaw || p->dpcap;
    solid_fraction(c, st);
    if (need_tau) {
        divergence(c, st->vx, st->vy, st->vz);
        total_pressure_residual(c, st, st->pt);
        stresses(c, st, 0);
    }
    const double cosf = cos(p->fric_deg * M_PI / 180.0);
    const double sinf = sin(p->fric_deg * M_PI / 180.0);
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                size_t q = IC(i, j, k);
                double phi = 1.0 - c->s[q];
                double r = phi / p->phi0;
                double k0 = p->k0field ? st->k0[q] : p->kmuf0;
                st->kc[q] = k0 * r * r * r;

                double R = (st->pf[q] > st->pt[q]) ? 1.0 / p->R0 : 1.0;
                double eta_new = p->eta0 * st->mn[q] * (p->phi0 / phi) * R;
                double eta = first ? eta_new : exp(r_eta * log(eta_new) + (1.0 - r_eta) * log(st->eta[q]));

                double mn_new = p->mu0;
                if (need_tau) {
                    double axy = 0.25 * (c->txy[IEXY(i, j, k)] + c->txy[IEXY(i + 1, j, k)]
                                       + c->txy[IEXY(i, j + 1, k)] + c->txy[IEXY(i + 1, j + 1, k)]);
                    double axz = 0.25 * (c->txz[IEXZ(i, j, k)] + c->txz[IEXZ(i + 1, j, k)]
                                       + c->txz[IEXZ(i, j, k + 1)] + c->txz[IEXZ(i + 1, j, k + 1)]);
                    double ayz = 0.25 * (c->tyz[IEYZ(i, j, k)] + c->tyz[IEYZ(i, j + 1, k)]
                                       + c->tyz[IEYZ(i, j, k + 1)] + c->tyz[IEYZ(i, j + 1, k + 1)]);
                    double tii = sqrt(0.5 * (c->txx[q] * c->txx[q] + c->tyy[q] * c->tyy[q] + c->tzz[q] * c->tzz[q])
                                      + axy * axy + axz * axz + ayz * ayz);
                    if (p->powerlaw) {
                        double t = tii / p->tau0;
                        double tp = (p->n_pow == 3.0) ? t * t : pow(t, p->n_pow - 1.0);
                        mn_new = p->mu0 / (1.0 + tp);
                    }
                    if (p->dpcap) {
                        double ty = dmax(p->coh * cosf + (st->pt[q] - st->pf[q]) * sinf, p->tau_y_min);
                        if (tii > 0.0) mn_new = dmin(mn_new, st->mn[q] * ty / tii);
                    }
                }
                double mn = first ? mn_new : exp(r_mu * log(mn_new) + (1.0 - r_mu) * log(st->mn[q]));
                st->eta[q] = eta;
                st->mn[q] = mn;
                st->mus[q] = mn * p->phi0 * p->cmu;
            }
}

/* Stress invariant tau_II at the cells for the current state and
 * coefficients (as the refresh computes it); out has nx*ny*nz entries.     */
void or_tau_ii(or_ctx *c, const or_state *st, double *out)
{
    solid_fraction(c, st);
    divergence(c, st->vx, st->vy, st->vz);
    total_pressure_residual(c, st, st->pt);
    stresses(c, st, 0);
#pragma omp parallel for
    for (int k = 0; k < NZ; ++k)
        for (int j = 0; j < NY; ++j)
            for (int i = 0; i < NX; ++i) {
                size_t q = IC(i, j, k);
                double axy = 0.25 * (c->txy[IEXY(i, j, k)] + c->txy[IEXY(i + 1, j, k)]
                                   + c->txy[IEXY(i, j + 1, k)] + c->txy[IEXY(i + 1, j + 1, k)]);
                double axz = 0.25 * (c->txz[IEXZ(i, j, k)] + c->txz[IEXZ(i + 1, j, k)]
                                   + c->txz[IEXZ(i, j, k + 1)] + c->txz[IEXZ(i + 1, j, k + 1)]);
                double ayz = 0.25 * (c->tyz[IEYZ(i, j, k)] + c->tyz[IEYZ(i, j + 1, k)]
                                   + c->tyz[IEYZ(i, j, k + 1)] + c->tyz[IEYZ(i, j + 1, k + 1)]);
                out[q] = sqrt(0.5 * (c->txx[q] * c->txx[q] + c->tyy[q] * c->tyy[q] + c->tzz[q] * c->tzz[q])
                              + axy * axy + axz * axz + ayz * ayz);
            }
}

/* Stress-history time step (the script recomputes it every physical step). */
void or_set_dts(or_ctx *c, double dts)
{
    c->p.dtS = dts;
}

/* Largest lagged shear viscosity mu_s over the cells. */
double or_max_mus(const or_ctx *c, const or_state *st)
{
    double m = 0.0;
    for (size_t q = 0; q < c->nc; ++q) m = nmax(m, st->mus[q]);
    return m;
}

/* Copies of the last computed stresses and Darcy fluxes, for tests. */
void or_last_stresses(const or_ctx *c, double *txx, double *tyy, double *tzz,
                      double *txy, double *txz, double *tyz)
{
    memcpy(txx, c->txx, c->nc * sizeof(double));
    memcpy(tyy, c->tyy, c->nc * sizeof(double));
    memcpy(tzz, c->tzz, c->nc * sizeof(double));
    memcpy(txy, c->txy, c->nexy * sizeof(double));
    memcpy(txz, c->txz, c->nexz * sizeof(double));
    memcpy(tyz, c->tyz, c->neyz * sizeof(double));
}

void or_last_fluxes(const or_ctx *c, double *qx, double *qy, double *qz)
{
    memcpy(qx, c->qx, c->nfx * sizeof(double));
    memcpy(qy, c->qy, c->nfy * sizeof(double));
    memcpy(qz, c->qz, c->nfz * sizeof(double));
}

/* ---- 1D heat-diffusion PT example (article 1, Fig. 2) ----------------------
 * U_t: values at the previous time step; U: initial guess, overwritten with
 * the PT result.  The two end points keep their values (no update there,
 * f = 0), as in the printed program.  Returns the number of iterations.      */
int or_heat1d_step(int n, double dx, double dt, double lam_rho_cp, double eps,
                   const double *Ut, double *U, int max_iter)
{
    double *Utau = (double *)malloc((size_t)n * sizeof(double));
    double dtau = 1.0 / (2.0 * lam_rho_cp / (dx * dx) + 1.0 / dt);
    int it = 0;
    double err = 2.0 * eps;
    while (err > eps && it < max_iter) {
        memcpy(Utau, U, (size_t)n * sizeof(double));
        err = 0.0;
        for (int i = 0; i < n; ++i) {
            double f = 0.0;
            if (i > 0 && i < n - 1) f = lam_rho_cp * (Utau[i + 1] - 2.0 * Utau[i] + Utau[i - 1]) / (dx * dx);
            U[i] = Utau[i] + dtau * f - dtau * (Utau[i] - Ut[i]) / dt;
            err = dmax(err, fabs(U[i] - Utau[i]));
        }
        ++it;
    }
    free(Utau);
    return it;
}
