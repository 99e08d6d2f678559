/*
 * reactive.c -- plain, slow FP64 CPU reference of the pseudo-transient
 * iteration for 3D reactive porosity waves (thesis article 3).
 *
 * TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no source with the GPU path.
 *
 * The model (article 3, eqs (8)-(10), in the form of the appendix reactive
 * script): fluid pressure Pf, porosity phi and the volatile mass fraction of
 * the solid Xs, with effective pressure Pe = -Pf, Darcy flux
 *   q = -k(phi) (grad Pf - rho_f g e_z),  k = k0/mu_f (phi/phi0)^3,
 * first-order reaction kinetics towards Xs_eq = clamp(beta_x Pf + Xs_max/2,
 * 0, Xs_max) with time constant tau, and the compressibilities
 *   beta_P   = phi beta_f + beta_d - (1 + phi) beta_s,
 *   beta_phi = beta_d - beta_s / (1 - phi).
 * One implicit physical step of dt is found by pseudo-transient iterations
 * on four cell fields (Xs, Pf, phi and the fluid-pressure rate dPf/dt):
 *   dXs/dt   = (Xs_eq - Xs) / tau
 *   Xs'      = Xs_old + dt dXs/dt
 *   Pf'      = Pf + dtau (dPf/dt - (Pf - Pf_old)/dt)
 *   dphi/dt  = (1 - phi)(beta_phi dPf/dt - Pe/(eta (1-phi))
 *              - (1 + dX)/(1 - Xs) dXs/dt)
 *   phi'     = clamp(phi_old + dt dphi/dt, phi_min, phi_max)
 *   dPf/dt'  = [-div q + Pe/(eta (1-phi))
 *              + (1 - rho_s/(rho_f (1+dX))) (1-phi)(1+dX)/(1-Xs) dXs/dt] / beta_P
 * with every right-hand side at iteration k (Jacobi), and the pseudo step
 * dtau = h^2 / max(k/beta_P) / c_pf taken every nup iterations.
 *
 * Discretisation: finite volumes on cells (dx = lx/nx), Darcy flux on the
 * faces with the face permeability the mean of the two cells', zero normal
 * flux on boundary faces; every cell is updated.  Compile with
 * -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nx, ny, nz;
    double lx, ly, lz;
    double phi0, k_muf0, eta;
    double rho_f, rho_s, g;
    double beta_d, beta_s, beta_f;
    double tau, beta_x, delta_x, xs_max;
    double dt, c_pf, phi_min, phi_max;
} rw_params;

typedef struct {
    double *xs, *pf, *phi, *dpfdt;          /* iterated (cells)          */
    double *xs_old, *pf_old, *phi_old;      /* previous physical step    */
} rw_state;

typedef struct {
    rw_params p;
    int nx, ny, nz;
    double dx, dy, dz, h;
    size_t nc;
    double *k, *divq, *xsn, *pfn, *phin, *dpn;
} rw_ctx;

#define RNX (c->nx)
#define RNY (c->ny)
#define RNZ (c->nz)
#define RIC(i, j, k) ((((size_t)(k)) * RNY + (size_t)(j)) * RNX + (size_t)(i))

static double rw_dmax(double a, double b) { return a > b ? a : b; }
static double rw_dmin(double a, double b) { return a < b ? a : b; }
static double rw_nmax(double a, double b)
{
    if (a != a || b != b) return NAN;
    return a > b ? a : b;
}

rw_ctx *rw_create(const rw_params *p)
{
    if (!p || p->nx < 2 || p->ny < 2 || p->nz < 2) return NULL;
    rw_ctx *c = (rw_ctx *)calloc(1, sizeof(rw_ctx));
    c->p = *p;
    c->nx = p->nx; c->ny = p->ny; c->nz = p->nz;
    c->dx = p->lx / p->nx; c->dy = p->ly / p->ny; c->dz = p->lz / p->nz;
    c->h = rw_dmin(c->dx, rw_dmin(c->dy, c->dz));
    c->nc = (size_t)p->nx * p->ny * p->nz;
    c->k = (double *)calloc(c->nc, sizeof(double));
    c->divq = (double *)calloc(c->nc, sizeof(double));
    c->xsn = (double *)calloc(c->nc, sizeof(double));
    c->pfn = (double *)calloc(c->nc, sizeof(double));
    c->phin = (double *)calloc(c->nc, sizeof(double));
    c->dpn = (double *)calloc(c->nc, sizeof(double));
    return c;
}

void rw_destroy(rw_ctx *c)
{
    if (!c) return;
    free(c->k); free(c->divq); free(c->xsn); free(c->pfn); free(c->phin); free(c->dpn);
    free(c);
}

/* Permeability over fluid viscosity, k0/mu_f (phi/phi0)^3 (a product, not pow). */
static void permeability(rw_ctx *c, const double *phi)
{
    const rw_params *p = &c->p;
#pragma omp parallel for
    for (int k = 0; k < RNZ; ++k)
        for (int j = 0; j < RNY; ++j)
            for (int i = 0; i < RNX; ++i) {
                size_t q = RIC(i, j, k);
                double r = phi[q] / p->phi0;
                c->k[q] = p->k_muf0 * r * r * r;
            }
}

static double beta_p(const rw_params *p, double phi)
{
    return phi * p->beta_f + p->beta_d - (1.0 + phi) * p->beta_s;
}

/* Pseudo step of the fluid pressure: h^2 / max over cells of k/beta_P / c_pf. */
double rw_dtau(rw_ctx *c, const rw_state *st)
{
    permeability(c, st->phi);
    double m = 0.0;
    for (size_t q = 0; q < c->nc; ++q) m = rw_nmax(m, c->k[q] / beta_p(&c->p, st->phi[q]));
    return c->h * c->h / m / c->p.c_pf;
}

/* div q at every cell, q = -k_f (grad Pf - rho_f g e_z) on interior faces, 0
 * on boundary faces; k_f the mean of the two cells' k. */
static void darcy_divergence(rw_ctx *c, const double *pf)
{
    const rw_params *p = &c->p;
    const double rfg = p->rho_f * p->g;
#pragma omp parallel for
    for (int k = 0; k < RNZ; ++k)
        for (int j = 0; j < RNY; ++j)
            for (int i = 0; i < RNX; ++i) {
                size_t q = RIC(i, j, k);
                double qxl = 0.0, qxh = 0.0, qyl = 0.0, qyh = 0.0, qzl = 0.0, qzh = 0.0;
                if (i > 0)       qxl = -0.5 * (c->k[RIC(i - 1, j, k)] + c->k[q]) * (pf[q] - pf[RIC(i - 1, j, k)]) / c->dx;
                if (i < RNX - 1) qxh = -0.5 * (c->k[q] + c->k[RIC(i + 1, j, k)]) * (pf[RIC(i + 1, j, k)] - pf[q]) / c->dx;
                if (j > 0)       qyl = -0.5 * (c->k[RIC(i, j - 1, k)] + c->k[q]) * (pf[q] - pf[RIC(i, j - 1, k)]) / c->dy;
                if (j < RNY - 1) qyh = -0.5 * (c->k[q] + c->k[RIC(i, j + 1, k)]) * (pf[RIC(i, j + 1, k)] - pf[q]) / c->dy;
                if (k > 0)       qzl = -0.5 * (c->k[RIC(i, j, k - 1)] + c->k[q]) * ((pf[q] - pf[RIC(i, j, k - 1)]) / c->dz - rfg);
                if (k < RNZ - 1) qzh = -0.5 * (c->k[q] + c->k[RIC(i, j, k + 1)]) * ((pf[RIC(i, j, k + 1)] - pf[q]) / c->dz - rfg);
                c->divq[q] = (qxh - qxl) / c->dx + (qyh - qyl) / c->dy + (qzh - qzl) / c->dz;
            }
}

/* One PT iteration from iteration-k values (Jacobi).  err (may be NULL):
 * the script's stopping quantity, the largest of |dphi|, |dPf|/10, |dXs|
 * over the iteration. */
void rw_iteration(rw_ctx *c, rw_state *st, double dtau, double *err)
{
    const rw_params *p = &c->p;
    permeability(c, st->phi);
    darcy_divergence(c, st->pf);
    const double rho_term = 1.0 - p->rho_s / (p->rho_f * (1.0 + p->delta_x));
#pragma omp parallel for
    for (int k = 0; k < RNZ; ++k)
        for (int j = 0; j < RNY; ++j)
            for (int i = 0; i < RNX; ++i) {
                size_t q = RIC(i, j, k);
                double pf = st->pf[q], phi = st->phi[q], xs = st->xs[q], dp = st->dpfdt[q];
                double pe = -pf;
                double xseq = rw_dmin(rw_dmax(p->beta_x * pf + 0.5 * p->xs_max, 0.0), p->xs_max);
                double bp = beta_p(p, phi);
                double bphi = p->beta_d - p->beta_s / (1.0 - phi);
                double dxsdt = (xseq - xs) / p->tau;
                double compaction = pe / (p->eta * (1.0 - phi));
                c->xsn[q] = st->xs_old[q] + p->dt * dxsdt;
                c->pfn[q] = pf + dtau * dp - dtau * (pf - st->pf_old[q]) / p->dt;
                double dphidt = (1.0 - phi) * (bphi * dp - compaction - (1.0 + p->delta_x) / (1.0 - xs) * dxsdt);
                c->phin[q] = rw_dmin(rw_dmax(st->phi_old[q] + p->dt * dphidt, p->phi_min), p->phi_max);
                c->dpn[q] = (-c->divq[q] + compaction
                             + rho_term * (1.0 - phi) * (1.0 + p->delta_x) / (1.0 - xs) * dxsdt) / bp;
            }
    if (err) {
        double e = 0.0;
        for (size_t q = 0; q < c->nc; ++q) {
            e = rw_nmax(e, fabs(c->phin[q] - st->phi[q]));
            e = rw_nmax(e, fabs(c->pfn[q] - st->pf[q]) / 10.0);
            e = rw_nmax(e, fabs(c->xsn[q] - st->xs[q]));
        }
        *err = e;
    }
    memcpy(st->xs, c->xsn, c->nc * sizeof(double));
    memcpy(st->pf, c->pfn, c->nc * sizeof(double));
    memcpy(st->phi, c->phin, c->nc * sizeof(double));
    memcpy(st->dpfdt, c->dpn, c->nc * sizeof(double));
}

/* Start of a physical step: the old values. */
void rw_begin_step(rw_ctx *c, rw_state *st)
{
    memcpy(st->xs_old, st->xs, c->nc * sizeof(double));
    memcpy(st->pf_old, st->pf, c->nc * sizeof(double));
    memcpy(st->phi_old, st->phi, c->nc * sizeof(double));
}
