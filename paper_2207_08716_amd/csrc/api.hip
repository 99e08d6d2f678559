// Host side of the C ABI declared in include/ptporo.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "pt_internal.h"

using namespace ptk;

struct pt_grid {
    Geom geom;
    pt_params prm;
    Coef coef;
    double* f[PT_NFIELDS][2];
    int cur[PT_NPING];
    void* ws = nullptr;
    size_t ws_bytes = 0;
    double* aws = nullptr;     // FP64 workspace of the stage adjoint
    size_t aws_bytes = 0;
    int32_t aws_sensors = 0;   // sensor capacity of the adjoint workspace
    float* mws = nullptr;      // FP32 workspace of the mixed-precision solve
    size_t mws_bytes = 0;
    bool mws_clean = false;    // both correction copies zeroed once
    int mx_copy = 0;           // correction copy holding the present R_d
    hipStream_t stream = nullptr;
    int64_t iter = 0;          // iteration count within the current step
    double ref_v = 0.0, ref_p = 0.0;   // residual reference of the step (g_V0, g_P0)
    bool ref_set = false;
    bool refreshed = false;    // any refresh done on this handle
    bool norms_pending = false;
    bool broken = false;       // PT_ESTATE: a divergence, domain or device error occurred
    double* nw = nullptr;      // norm area in place of the workspace (pt_solve_linear_static)
    int64_t steps = 0;         // pt_begin_step calls since creation or reset
    double dt_cum = 0.0;       // PT_F_DTS_RULE: time accumulated since the last history renewal
    double dts = 0.0;          // PT_F_DTS_RULE: the present stress-history step
    pt_progress_fn progress = nullptr;   // per-stage report of long calls
    void* progress_user = nullptr;
    // The FP64 sweeps store the damped residual R only at checks (see the
    // sweep): r_ok: the present copies of PT_RX..RZ hold R of the present
    // iterate; vp_ok: the other copies of V hold the previous iterate under
    // the present velocity pseudo steps (so that R = (V - V_prev) / dtau_V).
    bool r_ok = true;
    bool vp_ok = false;
    double* gws = nullptr;     // multigrid workspace
    size_t gws_bytes = 0;
    pt_mg_params mgp{};        // multigrid parameters of the bound workspace
    int mg_levels = 0;         // grids of the hierarchy, the fine one included
    Geom mg_geom[PT_MG_MAX_LEVELS];
    int mg_cur[PT_MG_MAX_LEVELS] = {};   // present copy of the coarse grids' iterated fields
    std::string err;
};

namespace {

// Failures that leave the state unusable put the handle in its error state
// (PT_ESTATE) until pt_set_params, pt_begin_step, pt_reset_state or
// pt_set_porosity.
pt_status fail(pt_grid* g, pt_status s, const char* msg) {
    if (g) {
        g->err = msg;
        if (s == PT_EDIVERGED || s == PT_EDOMAIN || s == PT_EDEVICE) g->broken = true;
    }
    return s;
}

pt_status hip_fail(pt_grid* g, hipError_t e, const char* where) {
    if (g) {
        g->err = std::string(where) + ": " + hipGetErrorString(e);
        g->broken = true;
    }
    return PT_EDEVICE;
}

bool valid_params(const pt_params* p) {
    if (!p || p->version != PT_ABI_VERSION) return false;
    const double pos[] = {p->lx, p->ly, p->lz, p->phi0, p->kmuf0, p->eta0, p->mu0, p->cmu, p->alpha,
                          p->B, p->G, p->R0, p->dt, p->dtS, p->rho_i, p->c_v, p->c_pf};
    for (double v : pos)
        if (!(v > 0.0) || !std::isfinite(v)) return false;
    if (!(p->phi0 < 1.0) || p->nup < 1 || p->beta_d < 0.0 || p->beta_phi < 0.0 || p->beta_n < 0.0) return false;
    if (!std::isfinite(p->shear_bg)) return false;
    if ((p->flags & PT_F_DTS_RULE) && !(p->xsi_w > 0.0 && std::isfinite(p->xsi_w))) return false;
    return true;
}

void make_coef(pt_grid* g) {
    const pt_params& p = g->prm;
    Coef& c = g->coef;
    const double dx = p.lx / g->geom.nx, dy = p.ly / g->geom.ny, dz = p.lz / g->geom.nz;
    const double h = std::fmin(dx, std::fmin(dy, dz));
    const int nmax = std::max(g->geom.nx, std::max(g->geom.ny, g->geom.nz));
    c.dxi = 1.0 / dx;
    c.dyi = 1.0 / dy;
    c.dzi = 1.0 / dz;
    c.dt = p.dt;
    c.dti = 1.0 / p.dt;
    c.beta_d = p.beta_d;
    c.alpha = p.alpha;
    c.B = p.B;
    c.beta_phi = p.beta_phi;
    c.rhofg = p.rhofg;
    c.rhosg = p.rhosg;
    c.rhobg = p.rhofg * p.phi0 + (1.0 - p.phi0) * p.rhosg;
    c.buoy = p.rhofg - c.rhobg;
    // the stress-history step: the parameter, or the rule's present value
    const double dts = ((p.flags & PT_F_DTS_RULE) && g->dts > 0.0) ? g->dts : p.dtS;
    c.gdts_inv = 1.0 / (p.G * dts);
    c.gbg_half = 0.5 * p.shear_bg;
    c.beta_n = p.beta_n;
    c.rho_i_inv = 1.0 / p.rho_i;
    c.dtauv_c = p.rho_i * h * h / (p.c_v * (1.0 + p.beta_n));
    c.dtaupt_c = (1.0 + p.beta_n) / nmax;
    c.dtaupf_c = h * h * (1.0 + p.beta_d * p.B / p.alpha) / p.c_pf;
    c.dampx = 1.0 - p.damp_c / g->geom.nx;
    c.dampy = 1.0 - p.damp_c / g->geom.ny;
    c.dampz = 1.0 - p.damp_c / g->geom.nz;
    c.ab = p.alpha / p.B;
    c.third = 1.0 / 3.0;
    c.mech_off = (p.flags & PT_F_MECHOFF) ? 1 : 0;
    g->geom.tall32 = (p.flags & PT_F_FP32_TALL) ? 1 : 0;
}

RefreshCoef make_refresh(const pt_grid* g, double r_eta, double r_mu) {
    const pt_params& p = g->prm;
    RefreshCoef r{};
    r.phi0 = p.phi0;
    r.kmuf0 = p.kmuf0;
    r.eta0 = p.eta0;
    r.mu0 = p.mu0;
    r.cmu = p.cmu;
    r.R0 = p.R0;
    r.n_pow = p.n_pow;
    r.tau0_inv = 1.0 / p.tau0;
    const double fr = p.fric_deg * M_PI / 180.0;
    r.coh_cos = p.coh * std::cos(fr);
    r.sin_f = std::sin(fr);
    r.tau_y_min = p.tau_y_min;
    r.r_eta = r_eta;
    r.r_mu = r_mu;
    r.first = g->refreshed ? 0 : 1;
    r.powerlaw = (p.flags & PT_F_POWERLAW) ? 1 : 0;
    r.dpcap = (p.flags & PT_F_DPCAP) ? 1 : 0;
    r.k0field = (p.flags & PT_F_K0FIELD) ? 1 : 0;
    return r;
}

size_t ws_needed(const pt_grid* g);
double* domain_flag(pt_grid* g);

// Where the sweeps put their per-block maxima, the reduced norms and the
// domain flag: the bound workspace, or the static scratch during
// pt_solve_linear_static.
double* norm_area(pt_grid* g) { return g->nw ? g->nw : static_cast<double*>(g->ws); }
bool norm_area_ready(const pt_grid* g) { return g->nw || (g->ws && g->ws_bytes >= ws_needed(g)); }

double* cur(pt_grid* g, int f) { return f < PT_NPING ? g->f[f][g->cur[f]] : g->f[f][0]; }
double* alt(pt_grid* g, int f) { return g->f[f][1 - g->cur[f]]; }

bool bound(pt_grid* g, std::initializer_list<int> fields, bool both) {
    for (int f : fields) {
        if (!g->f[f][0]) return false;
        if (both && f < PT_NPING && !g->f[f][1]) return false;
    }
    return true;
}

AuxPtrs aux(pt_grid* g) {
    AuxPtrs a{};
    a.vx = cur(g, PT_VX);
    a.vy = cur(g, PT_VY);
    a.vz = cur(g, PT_VZ);
    a.pt = cur(g, PT_PT);
    a.pf = cur(g, PT_PF);
    a.lp = cur(g, PT_LP);
    a.pto = cur(g, PT_PTO);
    a.pfo = cur(g, PT_PFO);
    a.lpo = cur(g, PT_LPO);
    a.sxx = cur(g, PT_SXX);
    a.syy = cur(g, PT_SYY);
    a.szz = cur(g, PT_SZZ);
    a.sxy = cur(g, PT_SXY);
    a.sxz = cur(g, PT_SXZ);
    a.syz = cur(g, PT_SYZ);
    a.fox = cur(g, PT_FOX);
    a.foy = cur(g, PT_FOY);
    a.foz = cur(g, PT_FOZ);
    a.mn = cur(g, PT_MN);
    a.kc = cur(g, PT_KC);
    a.eta = cur(g, PT_ETA);
    a.mus = cur(g, PT_MUS);
    a.k0 = g->f[PT_K0][0];
    a.lp_o = alt(g, PT_LP);
    a.domain = domain_flag(g);
    return a;
}

const std::initializer_list<int> kAllCore = {PT_VX, PT_VY, PT_VZ, PT_PT, PT_PF, PT_LP, PT_RX, PT_RY,
                                            PT_RZ, PT_PTO, PT_PFO, PT_LPO, PT_SXX, PT_SYY, PT_SZZ,
                                            PT_SXY, PT_SXZ, PT_SYZ, PT_FOX, PT_FOY, PT_FOZ, PT_MN,
                                            PT_KC, PT_ETA, PT_MUS};

pt_status check_ready(pt_grid* g) {
    if (g->broken) {
        const std::string why = g->err;
        g->err = "handle in error state (" + why + "); call pt_begin_step, pt_set_params, pt_reset_state or pt_set_porosity";
        g->err.resize(std::min<size_t>(g->err.size(), 400));
        return PT_ESTATE;
    }
    if (!bound(g, kAllCore, true)) return fail(g, PT_EINVAL, "not every field (both copies of the iterated ones) is bound");
    if ((g->prm.flags & PT_F_K0FIELD) && !g->f[PT_K0][0]) return fail(g, PT_EINVAL, "PT_F_K0FIELD set but PT_K0 not bound");
    if (!norm_area_ready(g)) return fail(g, PT_EINVAL, "workspace not bound or too small");
    return PT_OK;
}

// Workspace layout (doubles): [partials: n_blocks * 8][norms: 8][domain
// flag: 1], padded to a multiple of 256 bytes.  The flag is set (to 1) by the
// kernels that write ln(1-phi) where phi leaves (0, 1).
size_t ws_needed(const pt_grid* g) {
    const int64_t head = norm_blocks(g->geom) * NNORM + NNORM + 1;
    return (size_t)((head + 31) / 32 * 32) * sizeof(double);
}

double* domain_flag(pt_grid* g) {
    double* a = norm_area(g);
    return a ? a + norm_blocks(g->geom) * NNORM + NNORM : nullptr;
}

pt_status clear_domain(pt_grid* g) {
    hipError_t e = launch_fill(domain_flag(g), 0.0, 1, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "domain flag clear");
    return PT_OK;
}

pt_status sync_r(pt_grid* g);

pt_status refresh_impl(pt_grid* g, double r_eta, double r_mu) {
    // the pseudo steps change with mu_s: R must be stored, V_prev no longer serves
    pt_status sst = sync_r(g);
    if (sst != PT_OK) return sst;
    g->vp_ok = false;
    const RefreshCoef r = make_refresh(g, r_eta, r_mu);
    const AuxPtrs a = aux(g);
    hipError_t e = launch_refresh(g->geom, g->coef, r, a, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "refresh");
    e = launch_fo(g->geom, g->coef, r, a, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "fo");
    g->refreshed = true;
    return PT_OK;
}

SweepPtrs<double> sweep_ptrs(pt_grid* g) {
    SweepPtrs<double> p{};
    p.vx = cur(g, PT_VX); p.vy = cur(g, PT_VY); p.vz = cur(g, PT_VZ);
    p.pt = cur(g, PT_PT); p.pf = cur(g, PT_PF); p.lp = cur(g, PT_LP);
    p.rx = cur(g, PT_RX); p.ry = cur(g, PT_RY); p.rz = cur(g, PT_RZ);
    p.fox = cur(g, PT_FOX); p.foy = cur(g, PT_FOY); p.foz = cur(g, PT_FOZ);
    p.pto = cur(g, PT_PTO); p.pfo = cur(g, PT_PFO); p.lpo = cur(g, PT_LPO);
    p.kc = cur(g, PT_KC); p.eta = cur(g, PT_ETA); p.mus = cur(g, PT_MUS);
    p.vx_o = alt(g, PT_VX); p.vy_o = alt(g, PT_VY); p.vz_o = alt(g, PT_VZ);
    p.pt_o = alt(g, PT_PT); p.pf_o = alt(g, PT_PF); p.lp_o = alt(g, PT_LP);
    p.rx_o = alt(g, PT_RX); p.ry_o = alt(g, PT_RY); p.rz_o = alt(g, PT_RZ);
    p.partials = norm_area(g);
    p.domain = domain_flag(g);
    return p;
}

pt_status reduce_norms(pt_grid* g) {
    const int64_t nb = norm_blocks(g->geom);
    double* out = norm_area(g) + nb * NNORM;
    hipError_t e = launch_reduce_max(norm_area(g), nb, out, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "reduce");
    g->norms_pending = true;
    return PT_OK;
}

pt_status iteration_impl(pt_grid* g, int update_lp, int norms, bool keep_r = false) {
    SweepPtrs<double> p = sweep_ptrs(g);
    Coef c = g->coef;
    // the damping memory: V - V_prev when the other copy of V is the previous
    // iterate under these pseudo steps, the stored R otherwise; R is stored
    // by the sweeps with norms (the checks, which precede every refresh of
    // the schedules), by every sweep with the mechanics frozen, and by every
    // sweep of a solve to a relative residual (keep_r: near convergence
    // V - V_prev loses the digits that a stored R keeps, which would put the
    // attainable residual above the tightest tolerances)
    const bool vp = g->vp_ok && !c.mech_off && !keep_r;
    if (vp) {
        p.rx = alt(g, PT_VX);
        p.ry = alt(g, PT_VY);
        p.rz = alt(g, PT_VZ);
    }
    c.rform = vp ? 0 : 1;
    c.rwrite = (norms || c.mech_off || keep_r) ? 1 : 0;
    hipError_t e = launch_iteration(g->geom, c, p, update_lp ? MD_THESIS : MD_LINEAR, norms, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "iteration");
    if (norms) {
        pt_status st = reduce_norms(g);
        if (st != PT_OK) return st;
    }
    for (int f = 0; f < PT_NPING; ++f) {
        if (f == PT_LP && !update_lp) continue;
        if ((f == PT_RX || f == PT_RY || f == PT_RZ) && !c.rwrite) continue;
        g->cur[f] ^= 1;
    }
    g->r_ok = c.rwrite != 0;
    g->vp_ok = true;
    g->iter += 1;
    return PT_OK;
}

// Store the damped residual of the present iterate in the present copies of
// PT_RX..RZ when the sweeps carry it only in the two copies of V.
pt_status sync_r(pt_grid* g) {
    if (g->r_ok || !g->vp_ok) return PT_OK;
    hipError_t e = launch_damped_residual(g->geom, g->coef, cur(g, PT_VX), cur(g, PT_VY), cur(g, PT_VZ),
                                          alt(g, PT_VX), alt(g, PT_VY), alt(g, PT_VZ), cur(g, PT_MUS),
                                          cur(g, PT_RX), cur(g, PT_RY), cur(g, PT_RZ), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "damped residual");
    g->r_ok = true;
    return PT_OK;
}

// ---- mixed precision workspace --------------------------------------------
// FP32 padded boxes: [0..7] correction copy 0 (dvx dvy dvz dpt dpf drx dry drz),
// [8..15] copy 1, [16..20] residual of x (fx fy fz rpt rpf), [21] k, [22] mu_s,
// [23] chi.
constexpr int MX_NBOX = 24;
constexpr int MX_RES = 16;

int64_t mx_box(const pt_grid* g) { return g->geom.S * (int64_t)(g->geom.nz + 1); }
// Workspace boxes follow each other at a stride of one box plus 256 bytes:
// boxes a power of two apart (2^27 elements at 511^3) put the sweeps' many
// streams on the same memory channels at the same moment (measured: the
// fields of one skewed allocation sweep ~5 % faster than unskewed ones).
int64_t mx_stride(const pt_grid* g) { return mx_box(g) + 64; }   // floats
size_t mx_needed(const pt_grid* g) { return (size_t)(MX_NBOX * mx_stride(g)) * sizeof(float); }
float* mx(pt_grid* g, int b) { return g->mws + (int64_t)b * mx_stride(g); }

// The eight reduced norms and the domain flag (copied together).
pt_status read_norms(pt_grid* g, pt_norms* out) {
    double host[NNORM + 1];
    hipError_t e = hipMemcpyAsync(host, norm_area(g) + norm_blocks(g->geom) * NNORM, sizeof(host),
                                  hipMemcpyDeviceToHost, g->stream);
    const hipError_t es = hipStreamSynchronize(g->stream);   // also on a failed copy: host is local
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return hip_fail(g, e, "norms copy");
    out->f = host[0]; out->rpt = host[1]; out->rpf = host[2]; out->dl = host[3];
    out->dpt = host[4]; out->dpf = host[5]; out->dvz = host[6]; out->dv = host[7];
    for (int q = 0; q < NNORM; ++q)
        if (!std::isfinite(host[q])) return fail(g, PT_EDIVERGED, "non-finite residual norm");
    if (host[NNORM] != 0.0) return fail(g, PT_EDOMAIN, "porosity left (0, 1): ln(1-phi) not in (-inf, 0)");
    return PT_OK;
}

// Largest value of a cell field (synchronises; uses the norm area, so the
// last norms are no longer readable).
pt_status cells_max(pt_grid* g, const double* f, double* out) {
    const int64_t nb = norm_blocks(g->geom);
    double* area = norm_area(g);
    hipError_t e = launch_cell_max(g->geom, f, area, nb, g->stream);
    if (e == hipSuccess) e = launch_reduce_max(area, nb, area + nb * NNORM, g->stream);
    double host = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&host, area + nb * NNORM, sizeof(double), hipMemcpyDeviceToHost, g->stream);
    const hipError_t es = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return hip_fail(g, e, "cell maximum");
    g->norms_pending = false;
    if (!std::isfinite(host)) return fail(g, PT_EDIVERGED, "non-finite viscosity");
    *out = host;
    return PT_OK;
}

// The domain flag alone (synchronises).
pt_status read_domain(pt_grid* g) {
    double flag = 0.0;
    hipError_t e = hipMemcpyAsync(&flag, domain_flag(g), sizeof(double), hipMemcpyDeviceToHost, g->stream);
    const hipError_t es = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return hip_fail(g, e, "domain flag copy");
    if (flag != 0.0) return fail(g, PT_EDOMAIN, "porosity left (0, 1): ln(1-phi) not in (-inf, 0)");
    return PT_OK;
}

}  // namespace

extern "C" {

int32_t pt_abi_version(void) { return PT_ABI_VERSION; }

const char* pt_status_str(pt_status s) {
    switch (s) {
        case PT_OK: return "ok";
        case PT_ENOTCONV: return "iteration limit reached";
        case PT_EINVAL: return "invalid argument";
        case PT_EDEVICE: return "device error";
        case PT_EDIVERGED: return "diverged (non-finite norm)";
        case PT_EDOMAIN: return "porosity out of (0,1)";
        case PT_ESTATE: return "handle in error state";
    }
    return "unknown status";
}

const char* pt_last_error(const pt_grid* g) { return g ? g->err.c_str() : "null handle"; }

pt_status pt_create(int32_t nx, int32_t ny, int32_t nz, int64_t row_pitch, const pt_params* params,
                    pt_grid** out) {
    if (!out) return PT_EINVAL;
    *out = nullptr;
    if (nx < 2 || ny < 2 || nz < 2 || row_pitch < (int64_t)nx + 1) return PT_EINVAL;
    if (!valid_params(params)) return PT_EINVAL;
    pt_grid* g = new (std::nothrow) pt_grid();
    if (!g) return PT_EINVAL;
    g->geom.nx = nx;
    g->geom.ny = ny;
    g->geom.nz = nz;
    g->geom.P = row_pitch;
    g->geom.S = row_pitch * (int64_t)(ny + 1);
    g->geom.kz = KZ_MAX;   // each sweep variant sets its own chunk at launch
    g->prm = *params;
    g->dt_cum = params->dt;
    g->dts = params->dtS;
    std::memset(g->f, 0, sizeof(g->f));
    std::memset(g->cur, 0, sizeof(g->cur));
    // compute units of the current device for the launch cost model (the
    // default where no device can be queried; no error is left behind)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        g->geom.cus = cus;
    (void)hipGetLastError();
    make_coef(g);
    *out = g;
    return PT_OK;
}

pt_status pt_destroy(pt_grid* g) {
    delete g;
    return PT_OK;
}

int64_t pt_field_elems(const pt_grid* g) { return g ? g->geom.S * (int64_t)(g->geom.nz + 1) : 0; }

pt_status pt_bind_field(pt_grid* g, int32_t field, int32_t copy, void* dev_ptr) {
    if (!g) return PT_EINVAL;
    if (field < 0 || field >= PT_NFIELDS) return fail(g, PT_EINVAL, "bad field id");
    if (copy < 0 || copy > 1 || (copy == 1 && field >= PT_NPING)) return fail(g, PT_EINVAL, "bad copy index");
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u)) return fail(g, PT_EINVAL, "null or unaligned pointer");
    g->f[field][copy] = static_cast<double*>(dev_ptr);
    return PT_OK;
}

pt_status pt_workspace_size(const pt_grid* g, size_t* bytes) {
    if (!g || !bytes) return PT_EINVAL;
    *bytes = ws_needed(g);
    return PT_OK;
}

pt_status pt_bind_workspace(pt_grid* g, void* dev_ptr, size_t bytes) {
    if (!g) return PT_EINVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) || bytes < ws_needed(g))
        return fail(g, PT_EINVAL, "workspace missing, unaligned or too small");
    g->ws = dev_ptr;
    g->ws_bytes = bytes;
    return PT_OK;
}

pt_status pt_set_progress(pt_grid* g, pt_progress_fn fn, void* user) {
    if (!g) return PT_EINVAL;
    g->progress = fn;
    g->progress_user = user;
    return PT_OK;
}

pt_status pt_set_stream(pt_grid* g, void* hip_stream) {
    if (!g) return PT_EINVAL;
    g->stream = static_cast<hipStream_t>(hip_stream);
    return PT_OK;
}

pt_status pt_set_params(pt_grid* g, const pt_params* params) {
    if (!g) return PT_EINVAL;
    if (!valid_params(params)) return fail(g, PT_EINVAL, "invalid parameters");
    // the velocity pseudo steps may change: store R under the old ones
    if (!g->broken && g->ws && bound(g, kAllCore, true)) {
        pt_status st = sync_r(g);
        if (st != PT_OK) return st;
    }
    g->vp_ok = false;
    g->prm = *params;
    make_coef(g);
    g->broken = false;
    return PT_OK;
}

pt_status pt_current(const pt_grid* g, int32_t field, int32_t* copy) {
    if (!g || !copy || field < 0 || field >= PT_NFIELDS) return PT_EINVAL;
    *copy = field < PT_NPING ? g->cur[field] : 0;
    return PT_OK;
}

pt_status pt_begin_step(pt_grid* g, int32_t update_history) {
    if (!g) return PT_EINVAL;
    g->broken = false;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    st = clear_domain(g);
    if (st != PT_OK) return st;
    // the FP32 damped residual of the mixed solves restarts with the step, so
    // that a mixed step depends only on the state it starts from
    g->mws_clean = false;
    g->mx_copy = 0;
    const bool rule = (g->prm.flags & PT_F_DTS_RULE) != 0;
    double dts_new = 0.0;
    if (rule) {
        // the script's per-step block: dtS = max(mu_s) / (G xi_w); the history
        // is renewed (with the stresses of the previous dtS) when the time
        // accumulated since the last renewal reaches it
        if (g->steps >= 1) g->dt_cum += g->prm.dt;
        double mx = 0.0;
        st = cells_max(g, cur(g, PT_MUS), &mx);
        if (st != PT_OK) return st;
        dts_new = mx / (g->prm.G * g->prm.xsi_w);
        update_history = (g->steps >= 1 && g->dt_cum >= dts_new) ? 1 : 0;
    }
    const AuxPtrs a = aux(g);
    hipError_t e = launch_begin_step(g->geom, g->coef, a, update_history, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "begin_step");
    if (rule) {
        if (update_history || g->steps == 0) g->dt_cum = 0.0;
        g->dts = dts_new;
        make_coef(g);
    }
    if (update_history || rule) {
        // the folded history term with this step's Maxwell coefficients
        const RefreshCoef r = make_refresh(g, 1.0, 1.0);
        e = launch_fo(g->geom, g->coef, r, a, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "fo");
    }
    g->steps += 1;
    g->iter = 0;
    g->ref_set = false;
    return PT_OK;
}

pt_status pt_residual_reference(const pt_grid* g, double* gv, double* gp) {
    if (!g || !gv || !gp) return PT_EINVAL;
    *gv = g->ref_set ? g->ref_v : -1.0;
    *gp = g->ref_set ? g->ref_p : -1.0;
    return PT_OK;
}

pt_status pt_set_residual_reference(pt_grid* g, double gv, double gp) {
    if (!g) return PT_EINVAL;
    if (gv < 0.0 || gp < 0.0) {
        g->ref_set = false;
        return PT_OK;
    }
    g->ref_v = gv;
    g->ref_p = gp;
    g->ref_set = true;
    return PT_OK;
}

pt_status pt_refresh(pt_grid* g, double r_eta, double r_mu) {
    if (!g) return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    if (!(r_eta >= 0.0 && r_eta <= 1.0 && r_mu >= 0.0 && r_mu <= 1.0)) return fail(g, PT_EINVAL, "relaxation weight outside [0,1]");
    return refresh_impl(g, r_eta, r_mu);
}

pt_status pt_iteration(pt_grid* g, int32_t update_porosity, int32_t want_norms) {
    if (!g) return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    if (want_norms && !norm_area_ready(g)) return fail(g, PT_EINVAL, "norms need a bound workspace");
    return iteration_impl(g, update_porosity ? 1 : 0, want_norms ? 1 : 0);
}

pt_status pt_iterate(pt_grid* g, int64_t n) {
    if (!g || n < 0) return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    if (!g->ws || g->ws_bytes < ws_needed(g)) return fail(g, PT_EINVAL, "workspace not bound");
    const int64_t nup = g->prm.nup;
    for (int64_t m = 0; m < n; ++m) {
        const int64_t it = g->iter + 1;
        if ((it - 1) % nup == 0) {
            st = refresh_impl(g, g->prm.r_eta, g->prm.r_mu);
            if (st != PT_OK) return st;
        }
        st = iteration_impl(g, 1, (it % nup == 0) ? 1 : 0);
        if (st != PT_OK) return st;
    }
    return PT_OK;
}

pt_status pt_last_norms(pt_grid* g, pt_norms* out) {
    if (!g || !out) return PT_EINVAL;
    if (!g->norms_pending) return fail(g, PT_EINVAL, "no norms computed yet");
    return read_norms(g, out);
}

}  // extern "C"

namespace {
// The linear solve of pt_solve_linear on whatever norm area is in force.
pt_status solve_linear_core(pt_grid* g, double rtol, int64_t max_iter, int64_t* iters, double* rho) {
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    const int64_t nup = g->prm.nup;
    double r = INFINITY;
    int64_t it = 0;
    while (it < max_iter) {
        ++it;
        const bool want = (it == 1 && !g->ref_set) || (it % nup == 0);
        st = iteration_impl(g, 0, want ? 1 : 0, true);
        if (st != PT_OK) return st;
        if (!want) continue;
        pt_norms nm;
        st = read_norms(g, &nm);
        if (st != PT_OK) {
            if (iters) *iters = it;
            return st;
        }
        const double gv = nm.f, gp = std::fmax(nm.rpt, nm.rpf);
        if (!g->ref_set) {
            g->ref_v = gv;
            g->ref_p = gp;
            g->ref_set = true;
        }
        r = 0.0;
        if (g->ref_v > 0.0) r = std::fmax(r, gv / g->ref_v);
        if (g->ref_p > 0.0) r = std::fmax(r, gp / g->ref_p);
        if (it % nup == 0 && r <= rtol) break;
    }
    if (iters) *iters = it;
    if (rho) *rho = r;
    return (r <= rtol) ? PT_OK : PT_ENOTCONV;
}

// ---- the static scratch of pt_solve_linear_static -------------------------
// File-scope device array: each GPU the library runs on holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): the address
// is looked up once per device with hipGetSymbolAddress, with that device
// current, and kept here.
constexpr int64_t STATIC_SCRATCH_DOUBLES = 131072;   // 1 MiB
__device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
double* scratch_ptr[MAX_DEVICES] = {};

pt_status static_scratch(pt_grid* g, double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(g, e, "static scratch: current device");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(g, PT_EINVAL, "static scratch: device index out of range");
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(g, e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch: symbol address");
        scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = scratch_ptr[dev];
    return PT_OK;
}
}  // namespace

extern "C" {

pt_status pt_solve_linear(pt_grid* g, double rtol, int64_t max_iter, int64_t* iters, double* rho) {
    if (!g || !(rtol > 0.0) || max_iter < 1) return PT_EINVAL;
    if (!g->ws || g->ws_bytes < ws_needed(g)) return fail(g, PT_EINVAL, "workspace not bound");
    return solve_linear_core(g, rtol, max_iter, iters, rho);
}

pt_status pt_solve_linear_static(pt_grid* g, double rtol, int64_t max_iter, int64_t* iters, double* rho) {
    if (!g || !(rtol > 0.0) || max_iter < 1) return PT_EINVAL;
    const int64_t need = norm_blocks(g->geom) * NNORM + NNORM + 1;
    if (need > STATIC_SCRATCH_DOUBLES)
        return fail(g, PT_EINVAL, "grid too large for the static scratch of pt_solve_linear_static "
                                  "(more than 16382 norm blocks); use pt_solve_linear with a bound workspace");
    double* sp = nullptr;
    pt_status st = static_scratch(g, &sp);
    if (st != PT_OK) return st;
    g->nw = sp;
    // the domain flag must start at zero (the linear sweep never sets it);
    // a fill kernel, so that the call can sit in a captured graph
    hipError_t e = launch_fill(domain_flag(g), 0.0, 1, g->stream);
    if (e != hipSuccess) st = hip_fail(g, e, "static scratch clear");
    if (st == PT_OK) st = solve_linear_core(g, rtol, max_iter, iters, rho);
    // the norms of the last check stay readable only until the next call
    // that computes norms into the bound workspace
    g->nw = nullptr;
    g->norms_pending = false;
    return st;
}

pt_status pt_porosity_step(pt_grid* g) {
    if (!g) return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    const AuxPtrs a = aux(g);
    hipError_t e = launch_porosity_step(g->geom, g->coef, a, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "porosity_step");
    g->cur[PT_LP] ^= 1;
    return PT_OK;
}

pt_status pt_set_porosity(pt_grid* g, const void* phi_dev) {
    if (!g || !phi_dev) return PT_EINVAL;
    if (reinterpret_cast<uintptr_t>(phi_dev) & 255u) return fail(g, PT_EINVAL, "porosity buffer unaligned");
    g->broken = false;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    st = clear_domain(g);
    if (st != PT_OK) return st;
    hipError_t e = launch_set_porosity(g->geom, static_cast<const double*>(phi_dev), cur(g, PT_LP), cur(g, PT_LPO),
                                       domain_flag(g), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "set porosity");
    return read_domain(g);
}

pt_status pt_reset_state(pt_grid* g) {
    if (!g) return PT_EINVAL;
    g->broken = false;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    const int64_t n = g->geom.S * (int64_t)(g->geom.nz + 1);
    const pt_params& p = g->prm;
    const int zero_fields[] = {PT_VX, PT_VY, PT_VZ, PT_PT, PT_PF, PT_RX, PT_RY, PT_RZ, PT_PTO, PT_PFO,
                               PT_SXX, PT_SYY, PT_SZZ, PT_SXY, PT_SXZ, PT_SYZ, PT_FOX, PT_FOY, PT_FOZ};
    hipError_t e = hipSuccess;
    for (int f : zero_fields)
        for (int c = 0; c < (f < PT_NPING ? 2 : 1) && e == hipSuccess; ++c) e = launch_fill(g->f[f][c], 0.0, n, g->stream);
    // coefficients before the first refresh (which overwrites them)
    if (e == hipSuccess) e = launch_fill(g->f[PT_MN][0], p.mu0, n, g->stream);
    if (e == hipSuccess) e = launch_fill(g->f[PT_KC][0], p.kmuf0, n, g->stream);
    if (e == hipSuccess) e = launch_fill(g->f[PT_ETA][0], 1.0, n, g->stream);
    if (e == hipSuccess) e = launch_fill(g->f[PT_MUS][0], p.mu0 * p.phi0 * p.cmu, n, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "reset state");
    g->r_ok = true;     // R = 0 and V = V_prev = 0
    g->vp_ok = true;
    // ln(1-phi) keeps its buffers: the present copy becomes copy 0 with the rest
    if (g->cur[PT_LP] != 0) {
        e = launch_copy(g->f[PT_LP][1], g->f[PT_LP][0], n, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "reset state");
    }
    std::memset(g->cur, 0, sizeof(g->cur));
    g->iter = 0;
    g->steps = 0;
    g->dt_cum = g->prm.dt;
    g->dts = g->prm.dtS;
    make_coef(g);
    g->ref_set = false;
    g->refreshed = false;
    g->norms_pending = false;
    g->mws_clean = false;
    g->mx_copy = 0;
    return clear_domain(g);
}

pt_status pt_get_counters(const pt_grid* g, pt_counters* out) {
    if (!g || !out) return PT_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->version = PT_ABI_VERSION;
    out->iter = g->iter;
    out->refreshed = g->refreshed ? 1 : 0;
    out->ref_set = g->ref_set ? 1 : 0;
    out->ref_v = g->ref_v;
    out->ref_p = g->ref_p;
    for (int f = 0; f < PT_NPING; ++f) out->cur[f] = g->cur[f];
    out->mixed_copy = g->mx_copy;
    out->mixed_clean = g->mws_clean ? 1 : 0;
    out->steps = g->steps;
    out->dt_cum = g->dt_cum;
    out->dts = g->dts;
    out->r_stored = g->r_ok ? 1 : 0;
    out->v_prev = g->vp_ok ? 1 : 0;
    return PT_OK;
}

pt_status pt_set_counters(pt_grid* g, const pt_counters* in) {
    if (!g || !in) return PT_EINVAL;
    if (in->version != PT_ABI_VERSION || in->iter < 0 || (in->mixed_copy & ~1) || (in->mixed_clean & ~1) ||
        (in->refreshed & ~1) || (in->ref_set & ~1) || in->steps < 0 || !std::isfinite(in->dt_cum) ||
        !(in->dts > 0.0 && std::isfinite(in->dts)) || (in->r_stored & ~1) || (in->v_prev & ~1) ||
        !(in->r_stored || in->v_prev))
        return fail(g, PT_EINVAL, "bad counters");
    for (int f = 0; f < PT_NPING; ++f)
        if (in->cur[f] & ~1) return fail(g, PT_EINVAL, "bad copy index in counters");
    g->iter = in->iter;
    g->refreshed = in->refreshed != 0;
    g->ref_set = in->ref_set != 0;
    g->ref_v = in->ref_v;
    g->ref_p = in->ref_p;
    for (int f = 0; f < PT_NPING; ++f) g->cur[f] = in->cur[f];
    // the mixed workspace's contents count as kept only if it is bound
    g->mx_copy = in->mixed_copy;
    g->mws_clean = g->mws && in->mixed_clean != 0;
    g->steps = in->steps;
    g->dt_cum = in->dt_cum;
    g->dts = in->dts;
    g->r_ok = in->r_stored != 0;
    g->vp_ok = in->v_prev != 0;
    make_coef(g);
    return PT_OK;
}

pt_status pt_sync_damped_residual(pt_grid* g) {
    if (!g) return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    return sync_r(g);
}

pt_status pt_mixed_workspace_size(const pt_grid* g, size_t* bytes) {
    if (!g || !bytes) return PT_EINVAL;
    *bytes = mx_needed(g);
    return PT_OK;
}

pt_status pt_bind_mixed_workspace(pt_grid* g, void* dev_ptr, size_t bytes) {
    if (!g) return PT_EINVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) || bytes < mx_needed(g))
        return fail(g, PT_EINVAL, "mixed workspace missing, unaligned or too small");
    g->mws = static_cast<float*>(dev_ptr);
    g->mws_bytes = bytes;
    g->mws_clean = false;
    g->mx_copy = 0;
    return PT_OK;
}

pt_status pt_residual(pt_grid* g) {
    if (!g) return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    if (!g->mws) return fail(g, PT_EINVAL, "mixed workspace not bound");
    SweepPtrs<double> p = sweep_ptrs(g);
    p.res_fx = mx(g, MX_RES + 0);
    p.res_fy = mx(g, MX_RES + 1);
    p.res_fz = mx(g, MX_RES + 2);
    p.res_rpt = mx(g, MX_RES + 3);
    p.res_rpf = mx(g, MX_RES + 4);
    hipError_t e = launch_iteration(g->geom, g->coef, p, MD_RESID, 1, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "residual");
    return reduce_norms(g);
}

namespace {

// One FP32 correction sweep: the correction d in copy cp, its damped
// residual R_d in copy cr.  As in the FP64 sweeps, R_d is read only by the
// first sweep of a correction (rform; d restarts at zero, so d - d_prev says
// nothing) and stored only by the sweeps that end a check interval or the
// correction (rwrite); in between the sweep takes it from the two copies of
// d, three streams fewer.
pt_status correction_sweep(pt_grid* g, int cp, int cr, int norms, bool rform, bool rwrite) {
    SweepPtrs<float> p{};
    const int src = cp ? 8 : 0, dst = cp ? 0 : 8;
    const int rsrc = cr ? 8 : 0, rdst = cr ? 0 : 8;
    p.vx = mx(g, src + 0); p.vy = mx(g, src + 1); p.vz = mx(g, src + 2);
    p.pt = mx(g, src + 3); p.pf = mx(g, src + 4);
    if (rform) {
        p.rx = mx(g, rsrc + 5); p.ry = mx(g, rsrc + 6); p.rz = mx(g, rsrc + 7);
    } else {
        p.rx = mx(g, dst + 0); p.ry = mx(g, dst + 1); p.rz = mx(g, dst + 2);
    }
    p.vx_o = mx(g, dst + 0); p.vy_o = mx(g, dst + 1); p.vz_o = mx(g, dst + 2);
    p.pt_o = mx(g, dst + 3); p.pf_o = mx(g, dst + 4);
    p.rx_o = mx(g, rdst + 5); p.ry_o = mx(g, rdst + 6); p.rz_o = mx(g, rdst + 7);
    p.fox = mx(g, MX_RES + 0); p.foy = mx(g, MX_RES + 1); p.foz = mx(g, MX_RES + 2);
    p.pto = mx(g, MX_RES + 3); p.pfo = mx(g, MX_RES + 4);
    p.kc = mx(g, 21); p.mus = mx(g, 22); p.eta = mx(g, 23);
    p.partials = norm_area(g);
    Coef c = g->coef;
    c.rform = rform ? 1 : 0;
    c.rwrite = rwrite ? 1 : 0;
    hipError_t e = launch_correction(g->geom, c, p, norms, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "correction sweep");
    if (norms) return reduce_norms(g);
    return PT_OK;
}

MixedPtrs mixed_ptrs(pt_grid* g, int cp) {
    MixedPtrs m{};
    m.vx = cur(g, PT_VX); m.vy = cur(g, PT_VY); m.vz = cur(g, PT_VZ);
    m.pt = cur(g, PT_PT); m.pf = cur(g, PT_PF);
    m.lp = cur(g, PT_LP); m.kc = cur(g, PT_KC); m.eta = cur(g, PT_ETA); m.mus = cur(g, PT_MUS);
    const int b = cp ? 8 : 0;
    m.dvx = mx(g, b + 0); m.dvy = mx(g, b + 1); m.dvz = mx(g, b + 2);
    m.dpt = mx(g, b + 3); m.dpf = mx(g, b + 4);
    m.kc32 = mx(g, 21); m.mus32 = mx(g, 22); m.chi32 = mx(g, 23);
    return m;
}

// Corrections per stage of a mixed Picard step (each gains about 1e-3).
constexpr int32_t PICARD_MAX_CORRECTIONS = 64;

double group_rho(const pt_norms& nm, double g0v, double g0p) {
    double r = 0.0;
    if (g0v > 0.0) r = std::fmax(r, nm.f / g0v);
    if (g0p > 0.0) r = std::fmax(r, std::fmax(nm.rpt, nm.rpf) / g0p);
    return r;
}

}  // namespace

}  // extern "C"

namespace {

// What a defect-correction solve works on: the FP64 residual sweep's inputs
// (x, coefficients, old values or right-hand side), the FP64 fields the
// correction is added to, and the residual's constants.
struct MixedTarget {
    SweepPtrs<double> resid;
    MixedPtrs m;
    Coef coef;
};

// Defect correction: repeat { r = FP64 residual of x; stop when rho <= rtol
// (reference: ref_v/ref_p, set from the first residual if !ref_set); FP32
// PT sweeps on A d = -r from d = 0, the damped residual of d carried over in
// correction copy `copy`, until the residual of d is eta_in times r, or
// rtol/2 on the outer scale, or stalls; x += d }.
pt_status mixed_core(pt_grid* g, const MixedTarget& t, double rtol, double eta_in, int64_t max_inner,
                     int32_t max_outer, double& ref_v, double& ref_p, bool& ref_set, int& copy,
                     int64_t* inner_iters, int32_t* outer_iters, double* rho) {
    const int64_t box_bytes = mx_stride(g) * (int64_t)sizeof(float);
    MixedPtrs m = t.m;
    m.kc32 = mx(g, 21); m.mus32 = mx(g, 22); m.chi32 = mx(g, 23);
    hipError_t e = launch_prepare_mixed(g->geom, m, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "prepare mixed");
    SweepPtrs<double> rp = t.resid;
    rp.res_fx = mx(g, MX_RES + 0);
    rp.res_fy = mx(g, MX_RES + 1);
    rp.res_fz = mx(g, MX_RES + 2);
    rp.res_rpt = mx(g, MX_RES + 3);
    rp.res_rpf = mx(g, MX_RES + 4);
    rp.partials = norm_area(g);
    const int64_t nup = g->prm.nup;
    // the inner solve stops when its residual has not reached a new minimum
    // (by 1 %) for this many checks: FP32 cannot go below its round-off level
    const int stall_checks = 40;
    // ... and once x + d would meet the outer tolerance with this margin: the
    // last correction of a solve needs only the gap left to rtol, not a full
    // eta_in reduction
    const double target_margin = 0.5;
    double r = INFINITY;
    int64_t inner_total = 0;
    int32_t outer = 0;
    pt_status st;
    for (;;) {
        e = launch_iteration(g->geom, t.coef, rp, MD_RESID, 1, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "residual");
        st = reduce_norms(g);
        if (st != PT_OK) return st;
        pt_norms nm;
        st = read_norms(g, &nm);
        if (st != PT_OK) return st;
        if (!ref_set) {
            ref_v = nm.f;
            ref_p = std::fmax(nm.rpt, nm.rpf);
            ref_set = true;
        }
        r = group_rho(nm, ref_v, ref_p);
        if (r <= rtol || outer >= max_outer) break;
        const double gv = nm.f, gp = std::fmax(nm.rpt, nm.rpf);
        // correction d = 0; the damped residual R_d carries over from the
        // previous correction: with it, the PT iteration on A d = -r(x) is
        // the continuation of the PT iteration on x itself (same operator,
        // same pseudo-steps), so a restart costs no convergence
        int cp = copy, cr = copy;
        e = hipMemsetAsync(mx(g, cp ? 8 : 0), 0, 5 * box_bytes, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "correction clear");
        double best = INFINITY;
        int since_best = 0;
        for (int64_t it = 1; it <= max_inner; ++it) {
            const bool chk = (it % nup == 0);
            // every exit of this loop follows a check or the last sweep: R_d stored there
            const bool rwrite = chk || it == max_inner;
            st = correction_sweep(g, cp, cr, chk ? 1 : 0, it == 1, rwrite);
            if (st != PT_OK) return st;
            cp ^= 1;
            if (rwrite) cr ^= 1;
            ++inner_total;
            if (chk) {
                pt_norms ni;
                st = read_norms(g, &ni);
                if (st != PT_OK) return st;
                const double ri = group_rho(ni, gv, gp);
                if (ri <= eta_in || group_rho(ni, ref_v, ref_p) <= target_margin * rtol) break;
                if (ri < 0.99 * best) {
                    best = ri;
                    since_best = 0;
                } else if (++since_best >= stall_checks) {
                    break;
                }
            }
        }
        const int b = cp ? 8 : 0;
        m.dvx = mx(g, b + 0); m.dvy = mx(g, b + 1); m.dvz = mx(g, b + 2);
        m.dpt = mx(g, b + 3); m.dpf = mx(g, b + 4);
        e = launch_apply_correction(g->geom, m, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "apply correction");
        // the next correction's d starts in the copy that holds R_d (either
        // copy serves: d is cleared, R_d lives in boxes of its own)
        copy = cr;
        ++outer;
    }
    if (inner_iters) *inner_iters += inner_total;
    if (outer_iters) *outer_iters += outer;
    if (rho) *rho = r;
    return (r <= rtol) ? PT_OK : PT_ENOTCONV;
}

pt_status mixed_ready(pt_grid* g) {
    if (!g->mws) return fail(g, PT_EINVAL, "mixed workspace not bound");
    if (g->prm.flags & PT_F_MECHOFF) return fail(g, PT_EINVAL, "mixed precision does not support PT_F_MECHOFF");
    if (!g->mws_clean) {
        hipError_t e = hipMemsetAsync(g->mws, 0, 16 * mx_stride(g) * (int64_t)sizeof(float), g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "mixed workspace clear");
        g->mws_clean = true;
    }
    return PT_OK;
}

}  // namespace

extern "C" {

pt_status pt_solve_mixed(pt_grid* g, double rtol, double eta_in, int64_t max_inner, int32_t max_outer,
                         int64_t* inner_iters, int32_t* outer_iters, double* rho) {
    if (!g || !(rtol > 0.0) || !(eta_in > 0.0 && eta_in < 1.0) || max_inner < 1 || max_outer < 1)
        return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    st = mixed_ready(g);
    if (st != PT_OK) return st;
    // the corrections change V outside the sweeps: keep R stored
    st = sync_r(g);
    if (st != PT_OK) return st;
    g->vp_ok = false;
    MixedTarget t;
    t.resid = sweep_ptrs(g);
    t.m = mixed_ptrs(g, 0);
    t.coef = g->coef;
    if (inner_iters) *inner_iters = 0;
    if (outer_iters) *outer_iters = 0;
    return mixed_core(g, t, rtol, eta_in, max_inner, max_outer, g->ref_v, g->ref_p, g->ref_set, g->mx_copy,
                      inner_iters, outer_iters, rho);
}

// ---- adjoint of a linear Picard stage ---------------------------------------
namespace {
// FP64 boxes: [0..7] lambda copy 0 (V, Pt, Pf, damped residual), [8..15] copy 1,
// [16..20] right-hand side (f, r_Pt, r_Pf), [21] chi; for the run adjoint
// [22], [23] L_bar in/out, [24] eta_bar, [25] s_bar, [26..28] Pto/Pfo/Lo
// adjoints, [29..31] history-term adjoint, [32..37] So adjoint (xx yy zz xy xz
// yz), [38..39] old pressures of a mixed transposed solve; then the sensor
// tail: offsets (int64), gathered values, seeds.
constexpr int AD_NBOX = 40;
constexpr int AD_RHS = 16, AD_CHI = 21, AD_LBAR = 22, AD_ETAB = 24, AD_SB = 25, AD_OLD = 26, AD_FB = 29,
              AD_SO = 32, AD_MXOLD = 38;
// per recorded stage: V (3), Pt, Pf, incoming ln(1-phi), k/mu_f, eta_phi
constexpr int TAPE_NBOX = 8;
int64_t ad_stride(const pt_grid* g) { return mx_box(g) + 32; }   // doubles: one box + 256 bytes
size_t ad_needed(const pt_grid* g, int32_t max_sensors) {
    return (size_t)(AD_NBOX * ad_stride(g) + 3 * (int64_t)max_sensors) * sizeof(double);
}
double* ad(pt_grid* g, int b) { return g->aws + (int64_t)b * ad_stride(g); }
int64_t* ad_offs(pt_grid* g) { return reinterpret_cast<int64_t*>(g->aws + AD_NBOX * ad_stride(g)); }
double* ad_vals(pt_grid* g) { return g->aws + AD_NBOX * ad_stride(g) + g->aws_sensors; }
double* ad_seed(pt_grid* g) { return g->aws + AD_NBOX * ad_stride(g) + 2 * (int64_t)g->aws_sensors; }

// Sensor cells (linear indices over the nx*ny*nz cells, x fastest) to
// padded-box offsets, with range and distinctness checks.
pt_status sensor_offsets(pt_grid* g, const int64_t* sensors, int32_t ns, std::vector<int64_t>& offs) {
    const int64_t nc = (int64_t)g->geom.nx * g->geom.ny * g->geom.nz;
    offs.resize(ns);
    std::vector<int64_t> sorted(sensors, sensors + ns);
    std::sort(sorted.begin(), sorted.end());
    for (int32_t s = 0; s < ns; ++s) {
        if (sorted[s] < 0 || sorted[s] >= nc) return fail(g, PT_EINVAL, "sensor cell out of range");
        if (s > 0 && sorted[s] == sorted[s - 1]) return fail(g, PT_EINVAL, "duplicate sensor cell");
        const int64_t c = sensors[s];
        const int64_t i = c % g->geom.nx, j = (c / g->geom.nx) % g->geom.ny, k = c / ((int64_t)g->geom.nx * g->geom.ny);
        offs[s] = k * g->geom.S + j * g->geom.P + i;
    }
    return PT_OK;
}

// Small host-to-device copy from caller-side or temporary host memory: the
// stream is synchronised before returning, so the source may be freed at once
// (also on error paths).
static hipError_t upload_sync(void* dst, const void* src, size_t bytes, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    return e != hipSuccess ? e : e2;
}

// J = 1/2 sum (Pf_s - d_s)^2 of the present state; leaves the gathered Pf in vals.
pt_status misfit_impl(pt_grid* g, const int64_t* sensors, int32_t ns, const double* d_obs, double* J,
                      std::vector<double>& resid) {
    std::vector<int64_t> offs;
    pt_status st = sensor_offsets(g, sensors, ns, offs);
    if (st != PT_OK) return st;
    hipError_t e = upload_sync(ad_offs(g), offs.data(), ns * sizeof(int64_t), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "sensor upload");
    e = launch_gather(cur(g, PT_PF), ad_offs(g), ns, ad_vals(g), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "gather");
    std::vector<double> vals(ns);
    e = hipMemcpyAsync(vals.data(), ad_vals(g), ns * sizeof(double), hipMemcpyDeviceToHost, g->stream);
    const hipError_t es = hipStreamSynchronize(g->stream);   // also on a failed copy: vals is local
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return hip_fail(g, e, "gather download");
    resid.resize(ns);
    double acc = 0.0;
    for (int32_t s = 0; s < ns; ++s) {
        resid[s] = vals[s] - d_obs[s];
        acc += resid[s] * resid[s];
    }
    *J = 0.5 * acc;
    return PT_OK;
}
// Transposed stage solve J_F lambda = xbar with -xbar in boxes AD_RHS..+4,
// the coefficients k/mu_f = kc, mu_s = mus and chi in box AD_CHI, by the FP64
// correction sweep (J_F is symmetric).  lambda starts at zero; convergence
// when both residual groups fall to rtol times max|xbar|.  Returns the copy
// (0 or 1) holding lambda.
pt_status transposed_solve(pt_grid* g, const double* kc, const double* mus, double rtol, int64_t max_iter,
                           int* lam_copy, int64_t* iters, double* rho) {
    const int64_t box_bytes = ad_stride(g) * (int64_t)sizeof(double);
    hipError_t e = hipMemsetAsync(ad(g, 0), 0, 16 * box_bytes, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "adjoint clear");
    const int64_t nb = norm_blocks(g->geom);
    const double* rhs[5] = {ad(g, AD_RHS), ad(g, AD_RHS + 1), ad(g, AD_RHS + 2), ad(g, AD_RHS + 3), ad(g, AD_RHS + 4)};
    e = launch_absmax5(g->geom, rhs, norm_area(g), nb, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "rhs norm");
    pt_status st = reduce_norms(g);
    if (st != PT_OK) return st;
    pt_norms n0;
    st = read_norms(g, &n0);
    if (st != PT_OK) return st;
    const double ref = n0.f;
    int cp = 0;
    int64_t it = 0;
    double r = 0.0;
    if (ref > 0.0) {
        const int64_t nup = g->prm.nup;
        r = INFINITY;
        while (it < max_iter) {
            ++it;
            const bool chk = (it % nup == 0);
            SweepPtrs<double> p{};
            const int src = cp ? 8 : 0, dst = cp ? 0 : 8;
            p.vx = ad(g, src + 0); p.vy = ad(g, src + 1); p.vz = ad(g, src + 2);
            p.pt = ad(g, src + 3); p.pf = ad(g, src + 4);
            p.rx = ad(g, src + 5); p.ry = ad(g, src + 6); p.rz = ad(g, src + 7);
            p.vx_o = ad(g, dst + 0); p.vy_o = ad(g, dst + 1); p.vz_o = ad(g, dst + 2);
            p.pt_o = ad(g, dst + 3); p.pf_o = ad(g, dst + 4);
            p.rx_o = ad(g, dst + 5); p.ry_o = ad(g, dst + 6); p.rz_o = ad(g, dst + 7);
            p.fox = ad(g, AD_RHS); p.foy = ad(g, AD_RHS + 1); p.foz = ad(g, AD_RHS + 2);
            p.pto = ad(g, AD_RHS + 3); p.pfo = ad(g, AD_RHS + 4);
            p.eta = ad(g, AD_CHI); p.kc = kc; p.mus = mus;
            p.partials = norm_area(g);
            e = launch_correction64(g->geom, g->coef, p, chk ? 1 : 0, g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "adjoint sweep");
            cp ^= 1;
            if (chk) {
                st = reduce_norms(g);
                if (st != PT_OK) return st;
                pt_norms nm;
                st = read_norms(g, &nm);
                if (st != PT_OK) return st;
                r = group_rho(nm, ref, ref);
                if (r <= rtol) break;
            }
        }
    }
    *lam_copy = cp;
    if (iters) *iters += it;
    if (rho) *rho = std::fmax(*rho, r);
    return (r <= rtol) ? PT_OK : PT_ENOTCONV;
}
// The same transposed solve by defect correction: FP64 residual F(lambda) =
// J_F lambda - xbar (the stage residual with gravity off, the history term
// -xbar_V and old pressures from k_adj_oldvalues), FP32 PT sweeps on the
// correction (their own right-hand side is the residual), lambda += d in
// FP64.  lambda ends in copy 0.  Needs beta_d > 0 and the mixed workspace.
pt_status mixed_transposed_solve(pt_grid* g, const double* lp, const double* kc, const double* eta,
                                 const double* mus, double rtol, double eta_in, int64_t max_iter, int64_t* iters) {
    const int64_t box_bytes = ad_stride(g) * (int64_t)sizeof(double);
    hipError_t e = hipMemsetAsync(ad(g, 0), 0, 8 * box_bytes, g->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(g->mws, 0, 16 * mx_stride(g) * (int64_t)sizeof(float), g->stream);
    if (e == hipSuccess)
        e = launch_adj_oldvalues(g->geom, g->coef, ad(g, AD_RHS + 3), ad(g, AD_RHS + 4), ad(g, AD_MXOLD),
                                 ad(g, AD_MXOLD + 1), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "mixed adjoint set-up");
    MixedTarget t;
    t.resid = SweepPtrs<double>{};
    SweepPtrs<double>& p = t.resid;
    p.vx = ad(g, 0); p.vy = ad(g, 1); p.vz = ad(g, 2); p.pt = ad(g, 3); p.pf = ad(g, 4);
    p.lp = lp; p.kc = kc; p.eta = eta; p.mus = mus;
    p.pto = ad(g, AD_MXOLD); p.pfo = ad(g, AD_MXOLD + 1);
    p.fox = ad(g, AD_RHS); p.foy = ad(g, AD_RHS + 1); p.foz = ad(g, AD_RHS + 2);
    t.m = MixedPtrs{};
    t.m.vx = ad(g, 0); t.m.vy = ad(g, 1); t.m.vz = ad(g, 2); t.m.pt = ad(g, 3); t.m.pf = ad(g, 4);
    t.m.lp = lp; t.m.kc = kc; t.m.eta = eta; t.m.mus = mus;
    t.coef = g->coef;
    t.coef.rhofg = 0.0;
    t.coef.rhosg = 0.0;
    t.coef.rhobg = 0.0;
    t.coef.buoy = 0.0;
    t.coef.gbg_half = 0.0;
    double rv = 0.0, rp = 0.0, rho = 0.0;
    bool ref_set = false;
    int copy = 0;
    int32_t outer = 0;
    return mixed_core(g, t, rtol, eta_in, max_iter, PICARD_MAX_CORRECTIONS, rv, rp, ref_set, copy, iters, &outer,
                      &rho);
}
}  // namespace
}  // extern "C"

namespace {

// ---- geometric multigrid for the linear Picard stage ------------------------
// Correction scheme with V-cycles.  Every grid runs the library's own sweeps:
// the smoother is the linear PT sweep without damping and without the
// numerical compressibility (a weighted Jacobi iteration; neither term
// changes the solution), with the Pt pseudo step mu_s / n_pt; the coarsest
// grid runs the damped PT sweep.  A coarse grid (ceil(n/2) cells per axis,
// same domain) holds the correction e of its finer grid and solves
// A e = -R r, the restricted residual of the finer grid, written into the
// grid's constant terms: the face fields Fo (momentum) and the old pressures
// (whose terms in r_Pt and r_Pf are linear), with the physical constants
// (buoyancy, background shear) set to zero so that the residual at e = 0 is
// exactly R r.  Coefficients (k/mu_f harmonically, eta_phi by the chosen
// mean, mu_s and ln(1-phi) arithmetically) are averaged down at each solve.
//
// Workspace (doubles, boxes a box plus 256 bytes apart): the fine grid's FP32
// residual (5 boxes); per-block maxima of the coarse residual sweeps (sized
// for the first coarse grid, plus a flag slot); per coarse grid l: 25 FP64
// boxes (the 8 iterated fields in two copies, ln(1-phi), Fo, the old
// pressures, k/mu_f, eta_phi, mu_s) and, above the coarsest grid, its FP32
// residual (5 boxes); the restriction's scratch (less than one fine FP64 box).
constexpr int MG_NB = 25;
constexpr int MG_LP = 16, MG_FOX = 17, MG_PTO = 20, MG_PFO = 21, MG_KC = 22, MG_ETA = 23, MG_MUS = 24;

int64_t box_of(const Geom& g) { return g.S * (int64_t)(g.nz + 1); }
int64_t mg_stride(const Geom& g) { return box_of(g) + 32; }                       // doubles
int64_t mg_res_doubles(const Geom& g) { return ((5 * (box_of(g) + 64) + 1) / 2 + 31) / 32 * 32; }

Geom mg_coarse_geom(const Geom& f) {
    Geom c = f;
    c.nx = (f.nx + 1) / 2;
    c.ny = (f.ny + 1) / 2;
    c.nz = (f.nz + 1) / 2;
    c.P = ((int64_t)c.nx + 1 + 31) / 32 * 32;
    c.S = c.P * (int64_t)(c.ny + 1);
    c.kz = KZ_MAX;
    c.tall32 = 0;
    return c;
}

bool mg_valid(const pt_mg_params* m) {
    if (!m || m->version != PT_ABI_VERSION) return false;
    if (m->levels != 0 && (m->levels < 2 || m->levels > PT_MG_MAX_LEVELS)) return false;
    if (m->nu1 < 1 || m->nu2 < 0 || m->nu1 > 1000 || m->nu2 > 1000) return false;
    if (m->coarse_sweeps < 1 || m->coarse_sweeps > 1000000 || m->n_pt < 1) return false;
    if (!(m->c_v > 0.0 && std::isfinite(m->c_v)) || !(m->c_pf > 0.0 && std::isfinite(m->c_pf))) return false;
    if (m->krylov < 0 || m->krylov > PT_MG_MAX_KRYLOV || m->eta_mean < 0 || m->eta_mean > 2) return false;
    return true;
}

// Level geometries of a hierarchy; 0 levels if the grid cannot be coarsened.
int mg_plan(const pt_grid* g, const pt_mg_params& m, Geom* out) {
    out[0] = g->geom;
    int L = 1;
    while (L < PT_MG_MAX_LEVELS) {
        const Geom& f = out[L - 1];
        const int nmin = std::min(f.nx, std::min(f.ny, f.nz));
        if (m.levels == 0 ? nmin <= 8 : L >= m.levels) break;
        if (nmin < 4) break;                       // a coarse grid needs at least 2 cells per axis
        out[L] = mg_coarse_geom(f);
        ++L;
    }
    if (m.levels != 0 && L != m.levels) return 0;
    return L >= 2 ? L : 0;
}

// Per-block maxima of the coarse grids' residual sweeps: the most blocks
// of any coarse grid (the chunking can give a smaller grid more blocks).
int64_t mg_part_blocks(const Geom* geo, int L) {
    int64_t nb = 0;
    for (int l = 1; l < L; ++l) nb = std::max(nb, norm_blocks(geo[l]));
    return nb;
}
int64_t mg_part_doubles(const Geom* geo, int L) { return (mg_part_blocks(geo, L) * NNORM + NNORM + 1 + 31) / 32 * 32; }

// Doubles of the grids' pieces.
int64_t mg_levels_doubles(const Geom* geo, int L) {
    int64_t n = mg_res_doubles(geo[0]) + mg_part_doubles(geo, L);
    for (int l = 1; l < L; ++l) {
        n += MG_NB * mg_stride(geo[l]);
        if (l < L - 1) n += mg_res_doubles(geo[l]);
    }
    return n;
}

// Scratch of the separable restriction, sized for the fine grid's (the
// largest): the x-restricted field and the x- and y-restricted field.
int64_t mg_scr_a(const Geom* geo) { return ((int64_t)(geo[0].nz + 1) * (geo[0].ny + 1) * geo[1].P + 31) / 32 * 32; }
int64_t mg_scr_b(const Geom* geo) { return ((int64_t)(geo[0].nz + 1) * (geo[1].ny + 1) * geo[1].P + 31) / 32 * 32; }

// The restriction rows of every grid transfer l -> l + 1: per axis, the rows
// for cells and for faces normal to it.
int64_t mg_tab_rows(const Geom& c, int axis) { return (axis == 0 ? c.nx : axis == 1 ? c.ny : c.nz) + 1; }
int64_t mg_tab_doubles(const Geom* geo, int L) {
    int64_t n = 0;
    for (int l = 1; l < L; ++l)
        for (int a = 0; a < 3; ++a) n += 2 * mg_tab_rows(geo[l], a) * MG_TAB;
    return (n + 31) / 32 * 32;
}

// Doubles of the hierarchy's pieces (without the Krylov vectors).
int64_t mg_core_doubles(const Geom* geo, int L) {
    return mg_levels_doubles(geo, L) + mg_scr_a(geo) + mg_scr_b(geo) + mg_tab_doubles(geo, L);
}

// Krylov vectors after them: the saved iterate and m directions p (5 FP64
// fine boxes each), the residual of the cycle's result and m images A p (5
// FP32 fine boxes each), and the partial sums of the inner products.
int64_t kry_part_doubles() { return ((int64_t)KRY_BLOCKS * KRY_SLOTS + KRY_SLOTS + 31) / 32 * 32; }
int64_t kry_doubles(const Geom& f, int m) {
    return 5 * (1 + (int64_t)m) * mg_stride(f) + (1 + (int64_t)m) * mg_res_doubles(f) + kry_part_doubles();
}

size_t mg_needed(const pt_grid* g, const pt_mg_params& m) {
    Geom geo[PT_MG_MAX_LEVELS];
    const int L = mg_plan(g, m, geo);
    if (!L) return 0;
    int64_t n = mg_core_doubles(geo, L);
    if (m.krylov > 0) n += kry_doubles(geo[0], m.krylov);
    return (size_t)n * sizeof(double);
}

// Workspace pieces.
float* mg_res(pt_grid* g, int l, int q) {
    double* base = g->gws;
    if (l > 0) {
        base += mg_res_doubles(g->mg_geom[0]) + mg_part_doubles(g->mg_geom, g->mg_levels);
        for (int k = 1; k < l; ++k) base += MG_NB * mg_stride(g->mg_geom[k]) + mg_res_doubles(g->mg_geom[k]);
        base += MG_NB * mg_stride(g->mg_geom[l]);
    }
    return reinterpret_cast<float*>(base) + (int64_t)q * (box_of(g->mg_geom[l]) + 64);
}
double* mg_partials(pt_grid* g) { return g->gws + mg_res_doubles(g->mg_geom[0]); }
double* mg_scr(pt_grid* g, int b) {
    double* base = g->gws + mg_levels_doubles(g->mg_geom, g->mg_levels);
    return b == 0 ? base : base + mg_scr_a(g->mg_geom);
}
// Rows of the transfer from grid l to l + 1 along `axis` (face: for faces
// normal to it).
double* mg_tab(pt_grid* g, int l, int axis, int face) {
    double* p = mg_scr(g, 1) + mg_scr_b(g->mg_geom);
    for (int k = 1; k <= l; ++k)
        for (int a = 0; a < 3; ++a) p += 2 * mg_tab_rows(g->mg_geom[k], a) * MG_TAB;
    for (int a = 0; a < axis; ++a) p += 2 * mg_tab_rows(g->mg_geom[l + 1], a) * MG_TAB;
    return p + (face ? mg_tab_rows(g->mg_geom[l + 1], axis) * MG_TAB : 0);
}
double* kry_base(pt_grid* g) { return g->gws + mg_core_doubles(g->mg_geom, g->mg_levels); }
double* kry_x(pt_grid* g, int q) { return kry_base(g) + (int64_t)q * mg_stride(g->mg_geom[0]); }
double* kry_p(pt_grid* g, int s, int q) { return kry_base(g) + (5 + 5 * (int64_t)s + q) * mg_stride(g->mg_geom[0]); }
// v = 0: residual of the cycle's result; 1 + s: A p_s.
float* kry_vec(pt_grid* g, int v, int q) {
    const Geom& f = g->mg_geom[0];
    double* b = kry_base(g) + 5 * (1 + (int64_t)g->mgp.krylov) * mg_stride(f) + (int64_t)v * mg_res_doubles(f);
    return reinterpret_cast<float*>(b) + (int64_t)q * (box_of(f) + 64);
}
double* kry_part(pt_grid* g) {
    const Geom& f = g->mg_geom[0];
    const int64_t m = g->mgp.krylov;
    return kry_base(g) + 5 * (1 + m) * mg_stride(f) + (1 + m) * mg_res_doubles(f);
}
double* mg_box(pt_grid* g, int l, int b) {
    double* base = g->gws + mg_res_doubles(g->mg_geom[0]) + mg_part_doubles(g->mg_geom, g->mg_levels);
    for (int k = 1; k < l; ++k) base += MG_NB * mg_stride(g->mg_geom[k]) + mg_res_doubles(g->mg_geom[k]);
    return base + (int64_t)b * mg_stride(g->mg_geom[l]);
}

// Sweep constants of grid l: the smoother's (or, for the coarsest grid, the
// damped PT's) pseudo steps; on coarse grids no physical constant terms.
Coef mg_coef(const pt_grid* g, int l, bool coarsest) {
    const pt_params& p = g->prm;
    const pt_mg_params& m = g->mgp;
    const Geom& gl = g->mg_geom[l];
    Coef c = g->coef;
    const double dx = p.lx / gl.nx, dy = p.ly / gl.ny, dz = p.lz / gl.nz;
    const double h = std::fmin(dx, std::fmin(dy, dz));
    c.dxi = 1.0 / dx;
    c.dyi = 1.0 / dy;
    c.dzi = 1.0 / dz;
    if (coarsest) {
        const int nmax = std::max(gl.nx, std::max(gl.ny, gl.nz));
        c.beta_n = p.beta_n;
        c.dtauv_c = p.rho_i * h * h / (p.c_v * (1.0 + p.beta_n));
        c.dtaupt_c = (1.0 + p.beta_n) / nmax;
        c.dtaupf_c = h * h * (1.0 + p.beta_d * p.B / p.alpha) / p.c_pf;
        c.dampx = 1.0 - p.damp_c / gl.nx;
        c.dampy = 1.0 - p.damp_c / gl.ny;
        c.dampz = 1.0 - p.damp_c / gl.nz;
    } else {
        c.beta_n = 0.0;
        c.dtauv_c = p.rho_i * h * h / m.c_v;
        c.dtaupt_c = 1.0 / m.n_pt;
        c.dtaupf_c = h * h * (1.0 + p.beta_d * p.B / p.alpha) / m.c_pf;
        c.dampx = c.dampy = c.dampz = 0.0;
    }
    if (l > 0) {
        c.rhofg = c.rhosg = c.rhobg = c.buoy = 0.0;
        c.gbg_half = 0.0;
    }
    return c;
}

SweepPtrs<double> mg_ptrs(pt_grid* g, int l) {
    if (l == 0) {
        SweepPtrs<double> p = sweep_ptrs(g);
        p.res_fx = mg_res(g, 0, 0); p.res_fy = mg_res(g, 0, 1); p.res_fz = mg_res(g, 0, 2);
        p.res_rpt = mg_res(g, 0, 3); p.res_rpf = mg_res(g, 0, 4);
        return p;
    }
    SweepPtrs<double> p{};
    const int src = g->mg_cur[l] ? 8 : 0, dst = g->mg_cur[l] ? 0 : 8;
    p.vx = mg_box(g, l, src + 0); p.vy = mg_box(g, l, src + 1); p.vz = mg_box(g, l, src + 2);
    p.pt = mg_box(g, l, src + 3); p.pf = mg_box(g, l, src + 4);
    p.rx = mg_box(g, l, src + 5); p.ry = mg_box(g, l, src + 6); p.rz = mg_box(g, l, src + 7);
    p.vx_o = mg_box(g, l, dst + 0); p.vy_o = mg_box(g, l, dst + 1); p.vz_o = mg_box(g, l, dst + 2);
    p.pt_o = mg_box(g, l, dst + 3); p.pf_o = mg_box(g, l, dst + 4);
    p.rx_o = mg_box(g, l, dst + 5); p.ry_o = mg_box(g, l, dst + 6); p.rz_o = mg_box(g, l, dst + 7);
    p.lp = p.lpo = p.lp_o = mg_box(g, l, MG_LP);
    p.fox = mg_box(g, l, MG_FOX); p.foy = mg_box(g, l, MG_FOX + 1); p.foz = mg_box(g, l, MG_FOX + 2);
    p.pto = mg_box(g, l, MG_PTO); p.pfo = mg_box(g, l, MG_PFO);
    p.kc = mg_box(g, l, MG_KC); p.eta = mg_box(g, l, MG_ETA); p.mus = mg_box(g, l, MG_MUS);
    p.partials = mg_partials(g);
    p.domain = mg_partials(g) + mg_part_blocks(g->mg_geom, g->mg_levels) * NNORM + NNORM;
    if (l < g->mg_levels - 1) {
        p.res_fx = mg_res(g, l, 0); p.res_fy = mg_res(g, l, 1); p.res_fz = mg_res(g, l, 2);
        p.res_rpt = mg_res(g, l, 3); p.res_rpf = mg_res(g, l, 4);
    }
    return p;
}

// n linear sweeps on grid l with the smoother's (or the coarsest grid's) constants.
pt_status mg_smooth(pt_grid* g, int l, int n) {
    const bool coarsest = l == g->mg_levels - 1;
    Coef c = mg_coef(g, l, coarsest);
    // the smoother has no damping: R is neither needed nor stored, and its
    // input slots take the present V (a cache hit instead of three streams);
    // the coarsest grid's damped sweeps run the stored-R form on its own R
    c.rform = 1;
    c.rwrite = coarsest ? 1 : 0;
    for (int k = 0; k < n; ++k) {
        SweepPtrs<double> p = mg_ptrs(g, l);
        if (!coarsest) {
            p.rx = p.vx;
            p.ry = p.vy;
            p.rz = p.vz;
        }
        hipError_t e = launch_iteration(g->mg_geom[l], c, p, MD_LINEAR, 0, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "multigrid sweep");
        if (l == 0) {
            for (int f = 0; f < PT_NPING; ++f)
                if (f != PT_LP && f != PT_RX && f != PT_RY && f != PT_RZ) g->cur[f] ^= 1;
            g->iter += 1;
        } else {
            g->mg_cur[l] ^= 1;
        }
    }
    return PT_OK;
}

// Residual of grid l into its FP32 boxes (grid 0: with the norms reduced).
pt_status mg_residual(pt_grid* g, int l) {
    const SweepPtrs<double> p = mg_ptrs(g, l);
    const Coef c = l == 0 ? g->coef : mg_coef(g, l, false);
    hipError_t e = launch_iteration(g->mg_geom[l], c, p, MD_RESID, 1, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "multigrid residual");
    return l == 0 ? reduce_norms(g) : PT_OK;
}

// Coarse-grid correction of grid l (its residual is in its FP32 boxes).
pt_status mg_correct(pt_grid* g, int l) {
    const int c = l + 1;
    const Geom& gf = g->mg_geom[l];
    const Geom& gc = g->mg_geom[c];
    const int64_t nbox = box_of(gc);
    hipError_t e = hipSuccess;
    // the correction starts at zero (the present copies of V, Pt, Pf, R)
    const int cp = g->mg_cur[c] ? 8 : 0;
    for (int b = 0; b < 8 && e == hipSuccess; ++b) e = launch_fill(mg_box(g, c, cp + b), 0.0, nbox, g->stream);
    // right-hand side: the restricted residual in the constant terms
    for (int a = 0; a < 3 && e == hipSuccess; ++a) {
        const double* tab[3] = {mg_tab(g, l, 0, a == 0), mg_tab(g, l, 1, a == 1), mg_tab(g, l, 2, a == 2)};
        e = launch_mg_restrict32(gf, gc, a + 1, mg_res(g, l, a), mg_box(g, c, MG_FOX + a), mg_scr(g, 0), mg_scr(g, 1),
                                 tab, g->stream);
    }
    if (e == hipSuccess) {
        const pt_params& p = g->prm;
        // c(-pto + alpha pfo) = a, c(alpha pto - (alpha/B) pfo) = b, c = beta_d/dt
        const double k = p.beta_d / p.dt, al = p.alpha, ab = p.alpha / p.B;
        const double det = k * k * (ab - al * al);
        const double m[4] = {-k * ab / det, -k * al / det, -k * al / det, -k / det};
        const double* tab[3] = {mg_tab(g, l, 0, 0), mg_tab(g, l, 1, 0), mg_tab(g, l, 2, 0)};
        e = launch_mg_restrict_fold(gf, gc, mg_res(g, l, 3), mg_res(g, l, 4), mg_box(g, c, MG_PTO),
                                    mg_box(g, c, MG_PFO), m, mg_scr(g, 0), mg_scr(g, 1), tab, g->stream);
    }
    if (e != hipSuccess) return hip_fail(g, e, "multigrid restriction");
    pt_status st;
    if (c == g->mg_levels - 1) {
        st = mg_smooth(g, c, g->mgp.coarse_sweeps);
    } else {
        st = mg_smooth(g, c, g->mgp.nu1);
        if (st == PT_OK) st = mg_residual(g, c);
        if (st == PT_OK) st = mg_correct(g, c);
        if (st == PT_OK) st = mg_smooth(g, c, g->mgp.nu2);
    }
    if (st != PT_OK) return st;
    // add the interpolated correction to grid l's present copies
    const int cc = g->mg_cur[c] ? 8 : 0;
    for (int q = 0; q < 5 && e == hipSuccess; ++q) {
        double* dst;
        if (l == 0) {
            const int fl[5] = {PT_VX, PT_VY, PT_VZ, PT_PT, PT_PF};
            dst = cur(g, fl[q]);
        } else {
            dst = mg_box(g, l, (g->mg_cur[l] ? 8 : 0) + q);
        }
        e = launch_mg_prolong_add(gf, gc, q < 3 ? q + 1 : 0, mg_box(g, c, cc + q), dst, g->stream);
    }
    if (e != hipSuccess) return hip_fail(g, e, "multigrid prolongation");
    return PT_OK;
}

// Coefficients of every coarse grid from its finer one.
pt_status mg_coefficients(pt_grid* g) {
    hipError_t e = hipSuccess;
    for (int l = 1; l < g->mg_levels && e == hipSuccess; ++l) {
        const Geom& gf = g->mg_geom[l - 1];
        const Geom& gc = g->mg_geom[l];
        const double* kc = l == 1 ? cur(g, PT_KC) : mg_box(g, l - 1, MG_KC);
        const double* eta = l == 1 ? cur(g, PT_ETA) : mg_box(g, l - 1, MG_ETA);
        const double* mus = l == 1 ? cur(g, PT_MUS) : mg_box(g, l - 1, MG_MUS);
        const double* lp = l == 1 ? cur(g, PT_LP) : mg_box(g, l - 1, MG_LP);
        const double* tab[3] = {mg_tab(g, l - 1, 0, 0), mg_tab(g, l - 1, 1, 0), mg_tab(g, l - 1, 2, 0)};
        double *sa = mg_scr(g, 0), *sb = mg_scr(g, 1);
        e = launch_mg_restrict(gf, gc, kc, mg_box(g, l, MG_KC), 1, sa, sb, tab, g->stream);
        if (e == hipSuccess)
            e = launch_mg_restrict(gf, gc, eta, mg_box(g, l, MG_ETA), g->mgp.eta_mean, sa, sb, tab, g->stream);
        if (e == hipSuccess) e = launch_mg_restrict(gf, gc, mus, mg_box(g, l, MG_MUS), 0, sa, sb, tab, g->stream);
        if (e == hipSuccess) e = launch_mg_restrict(gf, gc, lp, mg_box(g, l, MG_LP), 0, sa, sb, tab, g->stream);
    }
    if (e != hipSuccess) return hip_fail(g, e, "multigrid coefficients");
    return PT_OK;
}

pt_status mg_rho(pt_grid* g, double* r) {
    pt_norms nm;
    pt_status st = read_norms(g, &nm);
    if (st != PT_OK) return st;
    const double gv = nm.f, gp = std::fmax(nm.rpt, nm.rpf);
    if (!g->ref_set) {
        g->ref_v = gv;
        g->ref_p = gp;
        g->ref_set = true;
    }
    double v = 0.0;
    if (g->ref_v > 0.0) v = std::fmax(v, gv / g->ref_v);
    if (g->ref_p > 0.0) v = std::fmax(v, gp / g->ref_p);
    *r = v;
    return PT_OK;
}

// The Krylov vectors of the fine grid with its present copies.
KryVecs kry_vecs(pt_grid* g) {
    KryVecs v{};
    const int fl[5] = {PT_VX, PT_VY, PT_VZ, PT_PT, PT_PF};
    for (int q = 0; q < 5; ++q) {
        v.rk[q] = mg_res(g, 0, q);
        v.ry[q] = kry_vec(g, 0, q);
        v.x[q] = kry_x(g, q);
        v.y[q] = cur(g, fl[q]);
    }
    // the stopping norm's scales: momentum rows by the velocity reference,
    // pressure rows by the pressure reference (the other one if one is 0)
    const double rv = g->ref_v > 0.0 ? g->ref_v : (g->ref_p > 0.0 ? g->ref_p : 1.0);
    const double rp = g->ref_p > 0.0 ? g->ref_p : rv;
    v.wv2 = 1.0 / (rv * rv);
    v.wp2 = 1.0 / (rp * rp);
    return v;
}

// The first n totals of the last reduction (synchronises).
pt_status kry_read(pt_grid* g, double* out, int n) {
    hipError_t e = hipMemcpyAsync(out, kry_part(g) + (int64_t)KRY_BLOCKS * KRY_SLOTS, n * sizeof(double),
                                  hipMemcpyDeviceToHost, g->stream);
    const hipError_t es = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return hip_fail(g, e, "Krylov sums copy");
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(out[k])) return fail(g, PT_EDIVERGED, "non-finite Krylov inner product");
    return PT_OK;
}

// Krylov acceleration of the cycle (pt_solve_mg with krylov > 0): the
// recombination of multigrid iterates over earlier corrections known as
// Krylov subspace acceleration.  The fine residual boxes hold r(x) of the
// iterate x; the cycle's result y is formed in the fine fields from x, its
// residual goes to the Krylov residual boxes.  The step keeps the whole
// cycle, x' = y + sum gamma_s p_s, with gamma minimising
// |r(y) - sum gamma_s A p_s|_W over the stored directions (W-orthogonal
// images, so one inner product each); the cycle's own step z = y - x,
// made W-orthogonal to the directions that stay, is stored for the
// following steps.  Minimising along z as well (GCR) stagnates: single
// cycles raise the residual norm transiently on the stage systems, where
// the minimiser then takes no step at all; so z is never scaled down.
pt_status solve_mg_krylov(pt_grid* g, double rtol, int64_t max_cycles, int64_t* cycles, double* rho) {
    const int m = g->mgp.krylov;
    const Geom& f = g->mg_geom[0];
    double app[KRY_MAX] = {};   // <A p_s, A p_s>_W of the stored slots
    int nd = 0, head = 0;       // slots in use; the oldest once all are
    int64_t c = 0;
    double r = INFINITY;
    pt_status st = mg_smooth(g, 0, g->mgp.nu1);
    if (st == PT_OK) st = mg_residual(g, 0);
    if (st == PT_OK) st = mg_rho(g, &r);
    bool saved = false;
    while (st == PT_OK && !(r <= rtol) && c < max_cycles) {
        hipError_t e = hipSuccess;
        if (!saved) {
            e = launch_kry_save(f, kry_vecs(g), g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "Krylov save");
            saved = true;
        }
        // y: one cycle from x
        st = mg_correct(g, 0);
        if (st == PT_OK) st = mg_smooth(g, 0, g->mgp.nu2 + g->mgp.nu1);
        if (st != PT_OK) break;
        {
            SweepPtrs<double> p = mg_ptrs(g, 0);
            p.res_fx = kry_vec(g, 0, 0); p.res_fy = kry_vec(g, 0, 1); p.res_fz = kry_vec(g, 0, 2);
            p.res_rpt = kry_vec(g, 0, 3); p.res_rpf = kry_vec(g, 0, 4);
            e = launch_iteration(f, g->coef, p, MD_RESID, 1, g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "multigrid residual");
        }
        st = reduce_norms(g);
        double ry = INFINITY;
        if (st == PT_OK) st = mg_rho(g, &ry);
        if (st != PT_OK) break;
        ++c;
        if (ry <= rtol) {   // y meets the tolerance: keep it
            r = ry;
            break;
        }
        // the new direction replaces the oldest once all slots are in use
        const int slot = nd < m ? nd : head;
        KryVecs v = kry_vecs(g);
        v.na = nd;
        for (int s = 0; s < nd; ++s)
            for (int q = 0; q < 5; ++q) {
                v.p[s][q] = kry_p(g, s, q);
                v.ap[s][q] = kry_vec(g, 1 + s, q);
            }
        for (int q = 0; q < 5; ++q) {
            v.p_new[q] = kry_p(g, slot, q);
            v.ap_new[q] = kry_vec(g, 1 + slot, q);
        }
        if (nd > 0) {
            e = launch_kry_dots(f, v, kry_part(g), g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "Krylov inner products");
            double d[KRY_SLOTS];
            st = kry_read(g, d, KRY_SLOTS);
            if (st != PT_OK) break;
            for (int s = 0; s < nd; ++s) {
                // r(y + gamma p_s) = r(y) - gamma A p_s
                v.gamma[s] = d[KRY_MAX + s] / app[s];
                v.beta[s] = s == slot ? 0.0 : (d[s] - d[KRY_MAX + s]) / app[s];
            }
        }
        e = launch_kry_update(f, v, kry_part(g), g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "Krylov step");
        double t[1];
        st = kry_read(g, t, 1);
        if (st != PT_OK) break;
        if (t[0] > 0.0) {
            app[slot] = t[0];
            if (nd < m) ++nd; else head = (head + 1) % m;
        } else {
            // z lies in the span of the stored directions: start afresh
            nd = 0;
            head = 0;
        }
        st = mg_residual(g, 0);
        if (st == PT_OK) st = mg_rho(g, &r);
    }
    if (cycles) *cycles = c;
    if (rho) *rho = r;
    if (st != PT_OK) return st;
    return (r <= rtol) ? PT_OK : PT_ENOTCONV;
}

pt_status solve_mg_core(pt_grid* g, double rtol, int64_t max_cycles, int64_t* cycles, double* rho) {
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    if (!g->gws) return fail(g, PT_EINVAL, "multigrid workspace not bound");
    if (!(g->prm.beta_d > 0.0) || g->prm.alpha * g->prm.alpha * g->prm.B == g->prm.alpha)
        return fail(g, PT_EINVAL, "multigrid needs beta_d > 0 and alpha B != 1 (the pressure terms carry the "
                                  "coarse right-hand side)");
    // the cycles change V outside the damped sweeps: keep R stored
    st = sync_r(g);
    if (st != PT_OK) return st;
    g->vp_ok = false;
    st = mg_coefficients(g);
    if (st != PT_OK) return st;
    double r = INFINITY;
    if (!g->ref_set) {
        // the reference is the residual of the state the solve starts from
        st = mg_residual(g, 0);
        if (st == PT_OK) st = mg_rho(g, &r);
        if (st != PT_OK) return st;
    }
    if (g->mgp.krylov > 0) return solve_mg_krylov(g, rtol, max_cycles, cycles, rho);
    int64_t c = 0;
    for (;;) {
        st = mg_smooth(g, 0, g->mgp.nu1);
        if (st == PT_OK) st = mg_residual(g, 0);
        if (st == PT_OK) st = mg_rho(g, &r);
        if (st != PT_OK) break;
        if (r <= rtol || c >= max_cycles) break;
        st = mg_correct(g, 0);
        if (st == PT_OK) st = mg_smooth(g, 0, g->mgp.nu2);
        if (st != PT_OK) break;
        ++c;
    }
    if (cycles) *cycles = c;
    if (rho) *rho = r;
    if (st != PT_OK) return st;
    return (r <= rtol) ? PT_OK : PT_ENOTCONV;
}

}  // namespace

extern "C" {

pt_status pt_mg_workspace_size(const pt_grid* g, const pt_mg_params* mg, size_t* bytes) {
    if (!g || !bytes || !mg_valid(mg)) return PT_EINVAL;
    const size_t n = mg_needed(g, *mg);
    if (!n) return PT_EINVAL;
    *bytes = n;
    return PT_OK;
}

pt_status pt_bind_mg_workspace(pt_grid* g, const pt_mg_params* mg, void* dev_ptr, size_t bytes) {
    if (!g) return PT_EINVAL;
    if (!mg_valid(mg)) return fail(g, PT_EINVAL, "bad multigrid parameters");
    const size_t need = mg_needed(g, *mg);
    if (!need) return fail(g, PT_EINVAL, "grid too small to coarsen to the requested levels");
    if (mg->krylov > 0 && g->geom.P % KRY_VW != 0)
        return fail(g, PT_EINVAL, "Krylov acceleration needs a row pitch that is a multiple of 4");
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) || bytes < need)
        return fail(g, PT_EINVAL, "multigrid workspace missing, unaligned or too small");
    g->mgp = *mg;
    g->mg_levels = mg_plan(g, *mg, g->mg_geom);
    g->gws = static_cast<double*>(dev_ptr);
    g->gws_bytes = bytes;
    for (int l = 0; l < PT_MG_MAX_LEVELS; ++l) g->mg_cur[l] = 0;
    // the walls' normal faces of the coarse corrections are never written:
    // clear the whole workspace once
    hipError_t e = launch_fill(g->gws, 0.0, (int64_t)(need / sizeof(double)), g->stream);
    // the restriction rows of every transfer, once per hierarchy
    for (int l = 0; l + 1 < g->mg_levels && e == hipSuccess; ++l) {
        const Geom& f = g->mg_geom[l];
        const Geom& c = g->mg_geom[l + 1];
        const int nf[3] = {f.nx, f.ny, f.nz}, nc[3] = {c.nx, c.ny, c.nz};
        for (int a = 0; a < 3 && e == hipSuccess; ++a)
            for (int face = 0; face < 2 && e == hipSuccess; ++face)
                e = launch_mg_taps(mg_tab(g, l, a, face), nf[a], nc[a], face, g->stream);
    }
    if (e != hipSuccess) return hip_fail(g, e, "multigrid workspace clear");
    return PT_OK;
}

pt_status pt_mg_levels(const pt_grid* g, int32_t* levels, int32_t* counts) {
    if (!g || !levels) return PT_EINVAL;
    *levels = g->gws ? g->mg_levels : 0;
    if (counts)
        for (int l = 0; l < *levels; ++l) {
            counts[3 * l] = g->mg_geom[l].nx;
            counts[3 * l + 1] = g->mg_geom[l].ny;
            counts[3 * l + 2] = g->mg_geom[l].nz;
        }
    return PT_OK;
}

pt_status pt_solve_mg(pt_grid* g, double rtol, int64_t max_cycles, int64_t* cycles, double* rho) {
    if (!g || !(rtol > 0.0) || max_cycles < 0) return PT_EINVAL;
    return solve_mg_core(g, rtol, max_cycles, cycles, rho);
}

pt_status pt_picard_step(pt_grid* g, int32_t update_history, int32_t n_picard, double rtol, int64_t max_iter,
                         int32_t mixed, double eta_in, int64_t* sweeps, double* rho) {
    if (!g || n_picard < 1 || !(rtol > 0.0) || max_iter < 1) return PT_EINVAL;
    if (mixed < PT_SOLVER_FP64 || mixed > PT_SOLVER_MG) return PT_EINVAL;
    if (mixed == PT_SOLVER_MIXED && !(eta_in > 0.0 && eta_in < 1.0)) return PT_EINVAL;
    if (mixed == PT_SOLVER_MG && !g->gws) return fail(g, PT_EINVAL, "multigrid workspace not bound");
    pt_status st = pt_begin_step(g, update_history ? 1 : 0);
    if (st != PT_OK) return st;
    int64_t total = 0;
    double rmax = 0.0;
    for (int p = 0; p < n_picard; ++p) {
        st = pt_refresh(g, 1.0, 1.0);
        if (st != PT_OK) return st;
        int64_t it = 0;
        double r = 0.0;
        if (mixed == PT_SOLVER_MG) {
            st = pt_solve_mg(g, rtol, max_iter, &it, &r);
        } else if (mixed == PT_SOLVER_MIXED) {
            int32_t outer = 0;
            st = pt_solve_mixed(g, rtol, eta_in, max_iter, PICARD_MAX_CORRECTIONS, &it, &outer, &r);
        } else {
            st = pt_solve_linear(g, rtol, max_iter, &it, &r);
        }
        total += it;
        rmax = std::fmax(rmax, r);
        if (sweeps) *sweeps = total;
        if (rho) *rho = rmax;
        if (st != PT_OK) return st;   // PT_ENOTCONV: the step stops at this stage
        st = pt_porosity_step(g);
        if (st != PT_OK) return st;
        if (g->progress) g->progress(g->progress_user, PT_PROGRESS_STAGE, 0, p, it);
    }
    // a porosity step that left (0, 1) would surface only at the next norm read
    return read_domain(g);
}

pt_status pt_adjoint_workspace_size(const pt_grid* g, int32_t max_sensors, size_t* bytes) {
    if (!g || !bytes || max_sensors < 1) return PT_EINVAL;
    *bytes = ad_needed(g, max_sensors);
    return PT_OK;
}

pt_status pt_bind_adjoint_workspace(pt_grid* g, void* dev_ptr, size_t bytes, int32_t max_sensors) {
    if (!g) return PT_EINVAL;
    if (max_sensors < 1 || !dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) ||
        bytes < ad_needed(g, max_sensors))
        return fail(g, PT_EINVAL, "adjoint workspace missing, unaligned or too small");
    g->aws = static_cast<double*>(dev_ptr);
    g->aws_bytes = bytes;
    g->aws_sensors = max_sensors;
    return PT_OK;
}

pt_status pt_set_log_k0(pt_grid* g, const void* logk0_dev) {
    if (!g || !logk0_dev) return PT_EINVAL;
    if (!(g->prm.flags & PT_F_K0FIELD) || !g->f[PT_K0][0]) return fail(g, PT_EINVAL, "no k0 field bound");
    hipError_t e = launch_exp_cells(g->geom, static_cast<const double*>(logk0_dev), g->f[PT_K0][0], g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "exp");
    return PT_OK;
}

pt_status pt_misfit(pt_grid* g, const int64_t* sensors, int32_t ns, const double* d_obs, double* J) {
    if (!g || !sensors || !d_obs || !J) return PT_EINVAL;
    if (!g->aws) return fail(g, PT_EINVAL, "adjoint workspace not bound");
    if (ns < 1 || ns > g->aws_sensors) return fail(g, PT_EINVAL, "sensor count outside the workspace capacity");
    std::vector<double> resid;
    return misfit_impl(g, sensors, ns, d_obs, J, resid);
}

pt_status pt_adjoint_stage(pt_grid* g, const int64_t* sensors, int32_t ns, const double* d_obs, double rtol,
                           int64_t max_iter, void* grad_dev, double* J, int64_t* iters, double* rho) {
    if (!g || !sensors || !d_obs || !grad_dev || !(rtol > 0.0) || max_iter < 1) return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    if (!g->aws) return fail(g, PT_EINVAL, "adjoint workspace not bound");
    if (ns < 1 || ns > g->aws_sensors) return fail(g, PT_EINVAL, "sensor count outside the workspace capacity");
    if (reinterpret_cast<uintptr_t>(grad_dev) & 255u) return fail(g, PT_EINVAL, "gradient buffer unaligned");
    double Jv = 0.0;
    std::vector<double> resid;
    st = misfit_impl(g, sensors, ns, d_obs, &Jv, resid);
    if (st != PT_OK) return st;
    std::vector<double> seed(ns);
    for (int32_t s = 0; s < ns; ++s) seed[s] = -resid[s];   // -xbar, xbar = dJ/dPf
    const int64_t box_bytes = ad_stride(g) * (int64_t)sizeof(double);
    hipError_t e = hipMemsetAsync(ad(g, AD_RHS), 0, 5 * box_bytes, g->stream);
    if (e == hipSuccess) e = upload_sync(ad_seed(g), seed.data(), ns * sizeof(double), g->stream);
    if (e == hipSuccess) e = launch_scatter(ad_seed(g), ad_offs(g), ns, ad(g, AD_RHS + 4), g->stream);
    if (e == hipSuccess) e = launch_chi64(g->geom, cur(g, PT_ETA), cur(g, PT_LP), ad(g, AD_CHI), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "adjoint set-up");
    int cp = 0;
    int64_t it = 0;
    double r = 0.0;
    st = transposed_solve(g, cur(g, PT_KC), cur(g, PT_MUS), rtol, max_iter, &cp, &it, &r);
    if (st != PT_OK && st != PT_ENOTCONV) return st;
    e = launch_adjoint_gradient(g->geom, g->coef, cur(g, PT_KC), cur(g, PT_PF), ad(g, (cp ? 8 : 0) + 4),
                                static_cast<double*>(grad_dev), g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "adjoint gradient");
    if (J) *J = Jv;
    if (iters) *iters = it;
    if (rho) *rho = r;
    return (r <= rtol) ? PT_OK : PT_ENOTCONV;
}

}  // extern "C"

namespace {
// Fields that restart a step exactly: V, Pt, Pf, ln(1-phi), damped residual
// R, stress history.  Old values, Fo and the coefficients are recomputed by
// the step set-up and the refresh (no relaxation, Newtonian law).
constexpr int CKPT_FIELDS[] = {PT_VX, PT_VY, PT_VZ, PT_PT, PT_PF, PT_LP, PT_RX, PT_RY, PT_RZ,
                               PT_SXX, PT_SYY, PT_SZZ, PT_SXY, PT_SXZ, PT_SYZ};
constexpr int CKPT_NBOX = sizeof(CKPT_FIELDS) / sizeof(CKPT_FIELDS[0]);
// Inner tolerance of the mixed solves of a run adjoint.
constexpr double ADJ_MIXED_ETA_IN = 1e-4;

size_t tape_boxes(int32_t n_steps, int32_t n_picard, int32_t options) {
    return (options & PT_ADJ_CHECKPOINT) ? (size_t)n_steps * CKPT_NBOX + (size_t)n_picard * TAPE_NBOX
                      : (size_t)n_steps * n_picard * TAPE_NBOX;
}

// One Picard step from the present state, recording its stages at rec(p, b).
template <typename Rec>
pt_status recorded_step(pt_grid* g, int n, int32_t n_picard, double rtol, int64_t max_iter, Rec rec,
                        int64_t* fit, int32_t phase, bool mixed) {
    const int64_t box = mx_box(g);
    // pt_begin_step restarts the FP32 damped residual of the mixed solves, so
    // that a step recomputed from its checkpoint repeats the recorded one bit
    // for bit
    pt_status st = pt_begin_step(g, n >= 1 ? 1 : 0);
    if (st != PT_OK) return st;
    (void)mixed;
    for (int p = 0; p < n_picard; ++p) {
        st = refresh_impl(g, 1.0, 1.0);
        if (st != PT_OK) return st;
        const int rec_in[3] = {PT_LP, PT_KC, PT_ETA};
        for (int b = 0; b < 3; ++b) {
            hipError_t e = launch_copy(cur(g, rec_in[b]), rec(p, 5 + b), box, g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "tape record");
        }
        int64_t it = 0;
        double rho = 0.0;
        if (mixed) {
            int32_t outer = 0;
            st = pt_solve_mixed(g, rtol, ADJ_MIXED_ETA_IN, max_iter, PICARD_MAX_CORRECTIONS, &it, &outer, &rho);
        } else {
            st = pt_solve_linear(g, rtol, max_iter, &it, &rho);
        }
        *fit += it;
        if (st == PT_ENOTCONV) return fail(g, PT_ENOTCONV, "a forward stage did not reach rtol");
        if (st != PT_OK) return st;
        const int rec_out[5] = {PT_VX, PT_VY, PT_VZ, PT_PT, PT_PF};
        for (int b = 0; b < 5; ++b) {
            hipError_t e = launch_copy(cur(g, rec_out[b]), rec(p, b), box, g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "tape record");
        }
        st = pt_porosity_step(g);
        if (st != PT_OK) return st;
        if (g->progress) g->progress(g->progress_user, phase, n, p, it);
    }
    return PT_OK;
}

// Copy the present state into (save) or out of (restore) a step checkpoint.
pt_status checkpoint_copy(pt_grid* g, double* ck, bool save) {
    const int64_t box = mx_box(g);
    if (save) {
        pt_status st = sync_r(g);
        if (st != PT_OK) return st;
    } else {
        g->r_ok = true;
        g->vp_ok = false;
    }
    for (int b = 0; b < CKPT_NBOX; ++b) {
        double* f = cur(g, CKPT_FIELDS[b]);
        hipError_t e = save ? launch_copy(f, ck + b * box, box, g->stream) : launch_copy(ck + b * box, f, box, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "checkpoint");
    }
    return PT_OK;
}
}  // namespace

extern "C" {

pt_status pt_adjoint_tape_size(const pt_grid* g, int32_t n_steps, int32_t n_picard, int32_t options,
                               size_t* bytes) {
    if (!g || !bytes || n_steps < 1 || n_picard < 1) return PT_EINVAL;
    *bytes = tape_boxes(n_steps, n_picard, options) * (size_t)mx_box(g) * sizeof(double);
    return PT_OK;
}

pt_status pt_adjoint_run(pt_grid* g, int32_t n_steps, int32_t n_picard, int32_t options, double rtol,
                         double adj_rtol, int64_t max_iter, const int64_t* sensors, int32_t ns, const double* d_obs,
                         void* tape, size_t tape_bytes, void* grad_dev, double* J, int64_t* fwd_iters,
                         int64_t* adj_iters) {
    if (!g || !sensors || !d_obs || !tape || !grad_dev || n_steps < 1 || n_picard < 1 || !(rtol > 0.0) ||
        !(adj_rtol > 0.0) || max_iter < 1)
        return PT_EINVAL;
    pt_status st = check_ready(g);
    if (st != PT_OK) return st;
    if (g->prm.flags & (PT_F_POWERLAW | PT_F_DPCAP | PT_F_MECHOFF))
        return fail(g, PT_EINVAL, "the run adjoint needs the Newtonian viscosity law with mechanics on");
    if (g->prm.shear_bg != 0.0 || (g->prm.flags & PT_F_DTS_RULE))
        return fail(g, PT_EINVAL, "the run adjoint does not cover the background shear or the dtS rule");
    if (!(g->prm.flags & PT_F_K0FIELD)) return fail(g, PT_EINVAL, "the run adjoint needs a k0 field");
    if (options & ~(PT_ADJ_CHECKPOINT | PT_ADJ_MIXED)) return fail(g, PT_EINVAL, "unknown run-adjoint option");
    const bool checkpoint = (options & PT_ADJ_CHECKPOINT) != 0;
    const bool mixed = (options & PT_ADJ_MIXED) != 0;
    if (mixed) {
        if (!(g->prm.beta_d > 0.0)) return fail(g, PT_EINVAL, "the mixed run adjoint needs beta_d > 0");
        st = mixed_ready(g);
        if (st != PT_OK) return st;
    }
    if (!g->aws) return fail(g, PT_EINVAL, "adjoint workspace not bound");
    if (ns < 1 || ns > g->aws_sensors) return fail(g, PT_EINVAL, "sensor count outside the workspace capacity");
    size_t need = 0;
    pt_adjoint_tape_size(g, n_steps, n_picard, options, &need);
    if (tape_bytes < need) return fail(g, PT_EINVAL, "tape too small");
    if ((reinterpret_cast<uintptr_t>(tape) | reinterpret_cast<uintptr_t>(grad_dev)) & 255u)
        return fail(g, PT_EINVAL, "tape or gradient buffer unaligned");
    const int64_t box = mx_box(g);
    double* T = static_cast<double*>(tape);
    // all stages: stage (n, p) at T[(n P + p) 8 boxes]; checkpoints: step n's
    // start state at T[n 15 boxes], then one step's stages after them
    double* step_tape = T + (int64_t)n_steps * CKPT_NBOX * box;
    auto tp = [&](int n, int p, int b) {
        if (checkpoint) return step_tape + ((int64_t)p * TAPE_NBOX + b) * box;
        return T + (((int64_t)n * n_picard + p) * TAPE_NBOX + b) * box;
    };
    hipError_t e;

    // ---- recorded forward: n_steps Picard steps of n_picard stages ----------
    int64_t fit = 0;
    // whether a refresh preceded each step (the first refresh of a handle
    // takes the new coefficients without the relaxation formula)
    std::vector<char> refreshed_at(n_steps, 0);
    for (int n = 0; n < n_steps; ++n) {
        if (checkpoint) {
            st = checkpoint_copy(g, T + (int64_t)n * CKPT_NBOX * box, true);
            if (st != PT_OK) return st;
            refreshed_at[n] = g->refreshed ? 1 : 0;
        }
        st = recorded_step(g, n, n_picard, rtol, max_iter, [&](int p, int b) { return tp(n, p, b); }, &fit,
                           PT_PROGRESS_FORWARD, mixed);
        if (st != PT_OK) return st;
    }
    double Jv = 0.0;
    std::vector<double> resid;
    st = misfit_impl(g, sensors, ns, d_obs, &Jv, resid);
    if (st != PT_OK) return st;

    // ---- reverse sweep ---------------------------------------------------------
    const int64_t box_bytes = box * (int64_t)sizeof(double);
    e = hipMemsetAsync(ad(g, AD_RHS), 0, (AD_NBOX - AD_RHS) * ad_stride(g) * (int64_t)sizeof(double), g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(grad_dev, 0, box_bytes, g->stream);
    std::vector<double> seed(ns);
    for (int32_t s = 0; s < ns; ++s) seed[s] = -resid[s];
    if (e == hipSuccess) e = upload_sync(ad_seed(g), seed.data(), ns * sizeof(double), g->stream);
    if (e == hipSuccess) e = launch_scatter(ad_seed(g), ad_offs(g), ns, ad(g, AD_RHS + 4), g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "run adjoint set-up");
    AdjPtrs a{};
    a.mus = cur(g, PT_MUS);
    a.rvx = ad(g, AD_RHS); a.rvy = ad(g, AD_RHS + 1); a.rvz = ad(g, AD_RHS + 2);
    a.rpt = ad(g, AD_RHS + 3); a.rpf = ad(g, AD_RHS + 4);
    double* lb[2] = {ad(g, AD_LBAR), ad(g, AD_LBAR + 1)};
    int lin = 0;
    a.eta_bar = ad(g, AD_ETAB); a.s_bar = ad(g, AD_SB);
    a.pto_bar = ad(g, AD_OLD); a.pfo_bar = ad(g, AD_OLD + 1); a.lo_bar = ad(g, AD_OLD + 2);
    a.fbx = ad(g, AD_FB); a.fby = ad(g, AD_FB + 1); a.fbz = ad(g, AD_FB + 2);
    a.sbxx = ad(g, AD_SO); a.sbyy = ad(g, AD_SO + 1); a.sbzz = ad(g, AD_SO + 2);
    a.sbxy = ad(g, AD_SO + 3); a.sbxz = ad(g, AD_SO + 4); a.sbyz = ad(g, AD_SO + 5);
    a.grad = static_cast<double*>(grad_dev);
    int64_t ait = 0;
    double arho = 0.0;
    for (int n = n_steps - 1; n >= 0; --n) {
        if (checkpoint && n < n_steps - 1) {
            // recompute step n from its checkpoint (bitwise the recorded run)
            st = checkpoint_copy(g, T + (int64_t)n * CKPT_NBOX * box, false);
            if (st != PT_OK) return st;
            g->refreshed = refreshed_at[n] != 0;
            int64_t rit = 0;
            st = recorded_step(g, n, n_picard, rtol, max_iter, [&](int p, int b) { return tp(n, p, b); }, &rit,
                               PT_PROGRESS_RECOMPUTE, mixed);
            if (st != PT_OK) return st;
        }
        for (int p = n_picard - 1; p >= 0; --p) {
            a.vx = tp(n, p, 0); a.vy = tp(n, p, 1); a.vz = tp(n, p, 2);
            a.pt = tp(n, p, 3); a.pf = tp(n, p, 4);
            a.lp = tp(n, p, 5); a.kc = tp(n, p, 6); a.eta = tp(n, p, 7);
            a.lbar = lb[lin];
            a.lbar_out = lb[1 - lin];
            e = launch_adj_porosity(g->geom, g->coef, a, g->stream);
            if (e == hipSuccess) e = launch_chi64(g->geom, a.eta, a.lp, ad(g, AD_CHI), g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "run adjoint porosity");
            int cp = 0;
            const int64_t ait0 = ait;
            if (mixed)
                st = mixed_transposed_solve(g, a.lp, a.kc, a.eta, a.mus, adj_rtol, ADJ_MIXED_ETA_IN, max_iter, &ait);
            else
                st = transposed_solve(g, a.kc, a.mus, adj_rtol, max_iter, &cp, &ait, &arho);
            if (st == PT_ENOTCONV) return fail(g, PT_ENOTCONV, "a transposed stage solve did not reach adj_rtol");
            if (st != PT_OK) return st;
            const int lb0 = cp ? 8 : 0;
            a.lvx = ad(g, lb0); a.lvy = ad(g, lb0 + 1); a.lvz = ad(g, lb0 + 2);
            a.lpt = ad(g, lb0 + 3); a.lpf = ad(g, lb0 + 4);
            e = launch_adj_coef(g->geom, g->coef, a, g->stream);
            if (e != hipSuccess) return hip_fail(g, e, "run adjoint coefficients");
            lin = 1 - lin;
            if (g->progress) g->progress(g->progress_user, PT_PROGRESS_REVERSE, n, p, ait - ait0);
        }
        if (n == 0) break;
        a.lbar = lb[lin];
        a.lbar_out = lb[1 - lin];
        e = launch_adj_step(g->geom, g->coef, a, g->stream);
        if (e == hipSuccess) e = launch_adj_history(g->geom, g->coef, a, g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "run adjoint step boundary");
        lin = 1 - lin;
    }
    e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "run adjoint");
    if (J) *J = Jv;
    if (fwd_iters) *fwd_iters = fit;
    if (adj_iters) *adj_iters = ait;
    return PT_OK;
}

pt_status pt_copy(pt_grid* g, const void* src, void* dst, int64_t n) {
    if (!g || !src || !dst || n < 0) return PT_EINVAL;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u)
        return fail(g, PT_EINVAL, "copy buffers must be 16-byte aligned");
    hipError_t e = launch_copy(static_cast<const double*>(src), static_cast<double*>(dst), n, g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "copy");
    return PT_OK;
}

}  // extern "C"
