// Per-step and per-refresh kernels: old values and stress history, Picard
// refresh of the lagged coefficients, the folded stress-history divergence Fo,
// the porosity time step of a Picard stage, and a streaming copy.
//
// These run once per physical step or once every nup PT iterations, so they
// are plain one-thread-per-point stencils that read neighbours through the
// caches.
#include "pt_internal.h"

namespace ptk {

namespace {

constexpr int AB = 256;

struct Idx {
    int i, j, k;
};

__device__ __forceinline__ bool box_index(const Geom& g, int64_t t, Idx& q) {
    // one thread per point of the (nx+1) x (ny+1) x (nz+1) box
    const int64_t nxp = g.nx + 1, nyp = g.ny + 1;
    const int64_t n = nxp * nyp * (g.nz + 1);
    if (t >= n) return false;
    q.i = (int)(t % nxp);
    q.j = (int)((t / nxp) % nyp);
    q.k = (int)(t / (nxp * nyp));
    return true;
}

__device__ __forceinline__ int64_t at(const Geom& g, int i, int j, int k) {
    return (int64_t)k * g.S + (int64_t)j * g.P + i;
}

// Maxwell coefficients of eq (21) (backward Euler): xi = mu/(G dtS),
// a = xi/(1+xi) multiplies the stress history, b = 2 mu/(1+xi) the strain rate.
__device__ __forceinline__ double coef_a(double mu, double gdts_inv) {
    const double xi = mu * gdts_inv;
    return xi / (1.0 + xi);
}
__device__ __forceinline__ double coef_b(double mu, double gdts_inv) {
    const double xi = mu * gdts_inv;
    return 2.0 * mu / (1.0 + xi);
}

// Deviatoric stresses at the current state without the numerical
// compressibility term: tau = a * So + b * edot.  Boundary edges carry zero.
struct StressEval {
    const Geom& g;
    const Coef& c;
    const AuxPtrs& a;
    __device__ double mus(int i, int j, int k) const { return a.mus[at(g, i, j, k)]; }
    __device__ double divv(int i, int j, int k) const {
        return (a.vx[at(g, i + 1, j, k)] - a.vx[at(g, i, j, k)]) * c.dxi +
               (a.vy[at(g, i, j + 1, k)] - a.vy[at(g, i, j, k)]) * c.dyi +
               (a.vz[at(g, i, j, k + 1)] - a.vz[at(g, i, j, k)]) * c.dzi;
    }
    __device__ void normal(int i, int j, int k, double& txx, double& tyy, double& tzz) const {
        const int64_t o = at(g, i, j, k);
        const double mu = a.mus[o];
        const double aa = coef_a(mu, c.gdts_inv), bb = coef_b(mu, c.gdts_inv);
        const double dxv = (a.vx[at(g, i + 1, j, k)] - a.vx[o]) * c.dxi;
        const double dyv = (a.vy[at(g, i, j + 1, k)] - a.vy[o]) * c.dyi;
        const double dzv = (a.vz[at(g, i, j, k + 1)] - a.vz[o]) * c.dzi;
        const double d3 = (dxv + dyv + dzv) * c.third;
        txx = aa * a.sxx[o] + bb * (dxv - d3);
        tyy = aa * a.syy[o] + bb * (dyv - d3);
        tzz = aa * a.szz[o] + bb * (dzv - d3);
    }
    __device__ double xy(int i, int j, int k) const {
        if (i < 1 || i >= g.nx || j < 1 || j >= g.ny) {
            if (c.gbg_half == 0.0) return 0.0;
            // boundary edge under the background shear of eq (32): the
            // background strain rate alone, viscosity of the cells inside
            double sum = 0.0;
            for (int jj = j - 1; jj <= j; ++jj)
                for (int ii = i - 1; ii <= i; ++ii)
                    if (ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny) sum += mus(ii, jj, k);
            const double mue = sum / (double)(((i >= 1) + (i < g.nx)) * ((j >= 1) + (j < g.ny)));
            return coef_a(mue, c.gdts_inv) * a.sxy[at(g, i, j, k)] + coef_b(mue, c.gdts_inv) * c.gbg_half;
        }
        const double mue = 0.25 * (mus(i - 1, j - 1, k) + mus(i, j - 1, k) + mus(i - 1, j, k) + mus(i, j, k));
        const int64_t o = at(g, i, j, k);
        const double e = 0.5 * ((a.vx[o] - a.vx[at(g, i, j - 1, k)]) * c.dyi + (a.vy[o] - a.vy[at(g, i - 1, j, k)]) * c.dxi) +
                         c.gbg_half;
        return coef_a(mue, c.gdts_inv) * a.sxy[o] + coef_b(mue, c.gdts_inv) * e;
    }
    __device__ double xz(int i, int j, int k) const {
        if (i < 1 || i >= g.nx || k < 1 || k >= g.nz) return 0.0;
        const double mue = 0.25 * (mus(i - 1, j, k - 1) + mus(i, j, k - 1) + mus(i - 1, j, k) + mus(i, j, k));
        const int64_t o = at(g, i, j, k);
        const double e = 0.5 * ((a.vx[o] - a.vx[at(g, i, j, k - 1)]) * c.dzi + (a.vz[o] - a.vz[at(g, i - 1, j, k)]) * c.dxi);
        return coef_a(mue, c.gdts_inv) * a.sxz[o] + coef_b(mue, c.gdts_inv) * e;
    }
    __device__ double yz(int i, int j, int k) const {
        if (j < 1 || j >= g.ny || k < 1 || k >= g.nz) return 0.0;
        const double mue = 0.25 * (mus(i, j - 1, k - 1) + mus(i, j, k - 1) + mus(i, j - 1, k) + mus(i, j, k));
        const int64_t o = at(g, i, j, k);
        const double e = 0.5 * ((a.vy[o] - a.vy[at(g, i, j, k - 1)]) * c.dzi + (a.vz[o] - a.vz[at(g, i, j - 1, k)]) * c.dyi);
        return coef_a(mue, c.gdts_inv) * a.syz[o] + coef_b(mue, c.gdts_inv) * e;
    }
};

// Start of a physical step: old pressures and porosity; optionally the new
// stress history (computed into registers first, written after a grid-wide
// separation: the history write happens in a second kernel).
__global__ __launch_bounds__(AB) void k_old_values(Geom g, AuxPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    if (q.i >= g.nx || q.j >= g.ny || q.k >= g.nz) return;
    const int64_t o = at(g, q.i, q.j, q.k);
    a.pto[o] = a.pt[o];
    a.pfo[o] = a.pf[o];
    a.lpo[o] = a.lp[o];
}

// Stress history <- tau(present state).  Each point reads only its own
// history value and the (read-only) velocities and viscosities, so the
// update can be done in place.
__global__ __launch_bounds__(AB) void k_history(Geom g, Coef c, AuxPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const StressEval se{g, c, a};
    const int i = q.i, j = q.j, k = q.k;
    const int64_t o = at(g, i, j, k);
    if (i < g.nx && j < g.ny && k < g.nz) {
        double txx, tyy, tzz;
        se.normal(i, j, k, txx, tyy, tzz);
        a.sxx[o] = txx;
        a.syy[o] = tyy;
        a.szz[o] = tzz;
    }
    if (k < g.nz) a.sxy[o] = se.xy(i, j, k);
    if (j < g.ny) a.sxz[o] = se.xz(i, j, k);
    if (i < g.nx) a.syz[o] = se.yz(i, j, k);
}

// Refresh of the lagged coefficients (eqs (23)-(26)) when the viscosity does
// not depend on stress: k/mu_f, eta_phi and Mn at the cells from cell values
// alone.  (With a power law or yield cap the tiled refresh kernel computes
// the stress invariant and does the same updates.)
__global__ __launch_bounds__(AB) void k_refresh(Geom g, Coef c, RefreshCoef r, AuxPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    const int64_t o = at(g, i, j, k);
    const double s = exp(a.lp[o]);
    const double phi = 1.0 - s;
    const double rr = phi / r.phi0;
    const double k0 = r.k0field ? a.k0[o] : r.kmuf0;
    const double kc = k0 * rr * rr * rr;

    const double pt = a.pt[o], pf = a.pf[o], mn = a.mn[o];
    const double R = (pf > pt) ? 1.0 / r.R0 : 1.0;
    const double eta_new = r.eta0 * mn * (r.phi0 / phi) * R;
    const double eta = r.first ? eta_new : exp(r.r_eta * log(eta_new) + (1.0 - r.r_eta) * log(a.eta[o]));
    const double mnr = r.first ? r.mu0 : exp(r.r_mu * log(r.mu0) + (1.0 - r.r_mu) * log(mn));
    a.kc[o] = kc;
    a.eta[o] = eta;
    a.mn[o] = mnr;
}

// Porosity time step of a Picard stage (eq (22)):
//   ln(1-phi) = ln(1-phi)o - dt [beta_phi((Pf-Pfo) - (Pt-Pto))/dt + (Pf-Pt)/eta + V.grad(1-phi)]
__global__ __launch_bounds__(AB) void k_porosity(Geom g, Coef c, AuxPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    const int64_t o = at(g, i, j, k);
    auto sf = [&](int ii, int jj, int kk) { return exp(a.lp[at(g, ii, jj, kk)]); };
    const double s = sf(i, j, k);
    double adv = 0.0;
    if (i > 0) adv += 0.5 * a.vx[o] * (s - sf(i - 1, j, k)) * c.dxi;
    if (i < g.nx - 1) adv += 0.5 * a.vx[at(g, i + 1, j, k)] * (sf(i + 1, j, k) - s) * c.dxi;
    if (j > 0) adv += 0.5 * a.vy[o] * (s - sf(i, j - 1, k)) * c.dyi;
    if (j < g.ny - 1) adv += 0.5 * a.vy[at(g, i, j + 1, k)] * (sf(i, j + 1, k) - s) * c.dyi;
    if (k > 0) adv += 0.5 * a.vz[o] * (s - sf(i, j, k - 1)) * c.dzi;
    if (k < g.nz - 1) adv += 0.5 * a.vz[at(g, i, j, k + 1)] * (sf(i, j, k + 1) - s) * c.dzi;
    const double pt = a.pt[o], pf = a.pf[o];
    const double dphidt = c.beta_phi * ((pf - a.pfo[o]) - (pt - a.pto[o])) * c.dti + (pf - pt) / a.eta[o] + adv;
    const double lpn = a.lpo[o] - c.dt * dphidt;
    a.lp_o[o] = lpn;
    if (!(lpn < 0.0 && lpn > -1.0e300)) *a.domain = 1.0;   // phi outside (0, 1)
}

// ln(1-phi) (and its old value) from the porosity on the cells; the domain
// flag is set where phi is not in (0, 1).
__global__ __launch_bounds__(AB) void k_set_porosity(Geom g, const double* __restrict__ phi, double* __restrict__ lp,
                                                     double* __restrict__ lpo, double* __restrict__ domain) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    if (q.i >= g.nx || q.j >= g.ny || q.k >= g.nz) return;
    const int64_t o = at(g, q.i, q.j, q.k);
    const double p = phi[o];
    if (!(p > 0.0 && p < 1.0)) *domain = 1.0;
    const double l = log(1.0 - p);
    lp[o] = l;
    lpo[o] = l;
}

// Per-block maxima of a cell field over its cell extent (grid-stride over
// the cells); partials[b * 8] gets the block's maximum, the other slots 0.
__global__ __launch_bounds__(AB) void k_cell_max(Geom g, const double* __restrict__ f, double* __restrict__ partials) {
    __shared__ double red[AB / 64];
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    double m = -1.0e300;
    for (int64_t t = (int64_t)blockIdx.x * AB + threadIdx.x; t < ncell; t += (int64_t)gridDim.x * AB) {
        const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny), k = (int)(t / ((int64_t)g.nx * g.ny));
        const double v = f[at(g, i, j, k)];
        m = (v > m || v != v) ? v : m;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double v = __shfl_xor(m, off, 64);
        m = (v > m || v != v) ? v : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x < NNORM) {
        double r = 0.0;
        if (threadIdx.x == 0) {
            r = red[0];
            for (int w = 1; w < AB / 64; ++w) r = (red[w] > r || red[w] != red[w]) ? red[w] : r;
        }
        partials[(int64_t)blockIdx.x * NNORM + threadIdx.x] = r;
    }
}

__global__ __launch_bounds__(AB) void k_fill(double* __restrict__ dst, double v, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * AB + threadIdx.x; t < n; t += (int64_t)gridDim.x * AB) dst[t] = v;
}

// Streaming copy: each thread moves CU_UNROLL 16-byte vectors per pass, all
// loads issued before the stores.
constexpr int CU_UNROLL = 4;
typedef double dvec2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(AB) void k_copy(const dvec2* __restrict__ src, dvec2* __restrict__ dst, int64_t n2) {
    const int64_t chunk = (int64_t)AB * CU_UNROLL;
    for (int64_t base = (int64_t)blockIdx.x * chunk; base < n2; base += (int64_t)gridDim.x * chunk) {
        dvec2 v[CU_UNROLL];
#pragma unroll
        for (int u = 0; u < CU_UNROLL; ++u) {
            const int64_t t = base + u * AB + threadIdx.x;
            if (t < n2) v[u] = __builtin_nontemporal_load(src + t);
        }
#pragma unroll
        for (int u = 0; u < CU_UNROLL; ++u) {
            const int64_t t = base + u * AB + threadIdx.x;
            if (t < n2) __builtin_nontemporal_store(v[u], dst + t);
        }
    }
}

__global__ void k_copy_tail(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
    if (threadIdx.x == 0 && n % 2 == 1) dst[n - 1] = src[n - 1];
}

// Mixed precision, once per Picard stage: FP32 copies of k/mu_f and mu_s,
// and chi = 1/((1-phi) eta_phi) with the porosity frozen for the stage.
__global__ __launch_bounds__(AB) void k_prepare_mixed(Geom g, MixedPtrs m) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    if (q.i >= g.nx || q.j >= g.ny || q.k >= g.nz) return;
    const int64_t o = at(g, q.i, q.j, q.k);
    m.kc32[o] = float(m.kc[o]);
    m.mus32[o] = float(m.mus[o]);
    m.chi32[o] = float(1.0 / (m.eta[o] * exp(m.lp[o])));
}

// Damped residual of the present iterate from the two copies of V: R =
// (V - V_prev) / dtau_V on the interior faces, dtau_V = dtauv_c / the larger
// mu_s of the face's two cells (the velocity pseudo step of the sweep).
__global__ __launch_bounds__(AB) void k_damped_residual(Geom g, double dtauv_c, const double* __restrict__ vx,
                                                        const double* __restrict__ vy, const double* __restrict__ vz,
                                                        const double* __restrict__ vxp,
                                                        const double* __restrict__ vyp,
                                                        const double* __restrict__ vzp,
                                                        const double* __restrict__ mus, double* __restrict__ rx,
                                                        double* __restrict__ ry, double* __restrict__ rz) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    if (q.i >= g.nx || q.j >= g.ny || q.k >= g.nz) return;
    const int64_t o = at(g, q.i, q.j, q.k);
    const double mu = mus[o];
    // the same operations as the sweep's stored R' = (V' - V) / dtau_V
    if (q.i >= 1) rx[o] = (vx[o] - vxp[o]) / (dtauv_c / fmax(mu, mus[at(g, q.i - 1, q.j, q.k)]));
    if (q.j >= 1) ry[o] = (vy[o] - vyp[o]) / (dtauv_c / fmax(mu, mus[at(g, q.i, q.j - 1, q.k)]));
    if (q.k >= 1) rz[o] = (vz[o] - vzp[o]) / (dtauv_c / fmax(mu, mus[at(g, q.i, q.j, q.k - 1)]));
}

// Defect correction x <- x + d in FP64 (velocity faces, pressures).  The
// correction is zero on boundary faces and outside every extent.
__global__ __launch_bounds__(AB) void k_apply_correction(Geom g, MixedPtrs m) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    const int64_t o = at(g, i, j, k);
    if (j < g.ny && k < g.nz && i >= 1 && i < g.nx) m.vx[o] += double(m.dvx[o]);
    if (i < g.nx && k < g.nz && j >= 1 && j < g.ny) m.vy[o] += double(m.dvy[o]);
    if (i < g.nx && j < g.ny && k >= 1 && k < g.nz) m.vz[o] += double(m.dvz[o]);
    if (i < g.nx && j < g.ny && k < g.nz) {
        m.pt[o] += double(m.dpt[o]);
        m.pf[o] += double(m.dpf[o]);
    }
}

// ---- adjoint of a linear Picard stage -------------------------------------
__global__ void k_gather(const double* __restrict__ src, const int64_t* __restrict__ offs, int n,
                         double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = src[offs[t]];
}

__global__ void k_scatter(const double* __restrict__ vals, const int64_t* __restrict__ offs, int n,
                          double* __restrict__ dst) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[offs[t]] = vals[t];
}

// chi = 1/((1-phi) eta_phi) with the porosity frozen for the stage.
__global__ __launch_bounds__(AB) void k_chi64(Geom g, const double* __restrict__ eta,
                                              const double* __restrict__ lp, double* __restrict__ chi) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    if (q.i >= g.nx || q.j >= g.ny || q.k >= g.nz) return;
    const int64_t o = at(g, q.i, q.j, q.k);
    chi[o] = 1.0 / (eta[o] * exp(lp[o]));
}

// dJ/d(ln k0) at cell c = -K_c * sum over c's interior faces of
// -(1/2) ((Pf_H - Pf_L)/h + b) (lam_L - lam_H)/h, from the Darcy flux
// q = -(K_L + K_H)/2 ((Pf_H - Pf_L)/h + b) that r_Pf carries as +q/h in the
// lower cell L and -q/h in the upper cell H (b: buoyancy term, z only).
__global__ __launch_bounds__(AB) void k_adjoint_gradient(Geom g, Coef c, const double* __restrict__ kc,
                                                         const double* __restrict__ pf,
                                                         const double* __restrict__ lam,
                                                         double* __restrict__ grad) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    const int64_t o = at(g, i, j, k);
    double acc = 0.0;
    auto face = [&](int64_t lo, int64_t hi, double hinv, double b) {
        const double gf = (pf[hi] - pf[lo]) * hinv + b;
        acc += -0.5 * gf * (lam[lo] - lam[hi]) * hinv;
    };
    if (i > 0) face(at(g, i - 1, j, k), o, c.dxi, 0.0);
    if (i < g.nx - 1) face(o, at(g, i + 1, j, k), c.dxi, 0.0);
    if (j > 0) face(at(g, i, j - 1, k), o, c.dyi, 0.0);
    if (j < g.ny - 1) face(o, at(g, i, j + 1, k), c.dyi, 0.0);
    if (k > 0) face(at(g, i, j, k - 1), o, c.dzi, c.buoy);
    if (k < g.nz - 1) face(o, at(g, i, j, k + 1), c.dzi, c.buoy);
    grad[o] = -kc[o] * acc;
}

__global__ __launch_bounds__(AB) void k_exp_cells(Geom g, const double* __restrict__ src, double* __restrict__ dst) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    if (q.i >= g.nx || q.j >= g.ny || q.k >= g.nz) return;
    const int64_t o = at(g, q.i, q.j, q.k);
    dst[o] = exp(src[o]);
}

inline dim3 box_grid(const Geom& g) {
    const int64_t n = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    return dim3((unsigned)((n + AB - 1) / AB));
}

}  // namespace

hipError_t launch_begin_step(const Geom& g, const Coef& c, const AuxPtrs& a, int update_history,
                             hipStream_t s) {
    if (update_history) hipLaunchKernelGGL(k_history, box_grid(g), dim3(AB), 0, s, g, c, a);
    hipLaunchKernelGGL(k_old_values, box_grid(g), dim3(AB), 0, s, g, a);
    return hipGetLastError();
}

hipError_t launch_refresh(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a, hipStream_t s) {
    if (r.powerlaw || r.dpcap) return launch_refresh_tiled(g, c, r, a, s);
    hipLaunchKernelGGL(k_refresh, box_grid(g), dim3(AB), 0, s, g, c, r, a);
    return hipGetLastError();
}

hipError_t launch_fo(const Geom& g, const Coef& c, const RefreshCoef& r, const AuxPtrs& a, hipStream_t s) {
    return launch_fo_tiled(g, c, r, a, s);
}

hipError_t launch_porosity_step(const Geom& g, const Coef& c, const AuxPtrs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_porosity, box_grid(g), dim3(AB), 0, s, g, c, a);
    return hipGetLastError();
}

hipError_t launch_set_porosity(const Geom& g, const double* phi, double* lp, double* lpo, double* domain,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_set_porosity, box_grid(g), dim3(AB), 0, s, g, phi, lp, lpo, domain);
    return hipGetLastError();
}

hipError_t launch_cell_max(const Geom& g, const double* f, double* partials, int64_t nblocks, hipStream_t s) {
    if (nblocks > 0) hipLaunchKernelGGL(k_cell_max, dim3((unsigned)nblocks), dim3(AB), 0, s, g, f, partials);
    return hipGetLastError();
}

hipError_t launch_fill(double* dst, double v, int64_t n, hipStream_t s) {
    if (n > 0) {
        int64_t blocks = (n + AB - 1) / AB;
        if (blocks > 256 * 16) blocks = 256 * 16;
        hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(AB), 0, s, dst, v, n);
    }
    return hipGetLastError();
}

hipError_t launch_damped_residual(const Geom& g, const Coef& c, const double* vx, const double* vy, const double* vz,
                                  const double* vx_p, const double* vy_p, const double* vz_p, const double* mus,
                                  double* rx, double* ry, double* rz, hipStream_t s) {
    hipLaunchKernelGGL(k_damped_residual, box_grid(g), dim3(AB), 0, s, g, c.dtauv_c, vx, vy, vz, vx_p, vy_p, vz_p,
                       mus, rx, ry, rz);
    return hipGetLastError();
}

hipError_t launch_prepare_mixed(const Geom& g, const MixedPtrs& m, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare_mixed, box_grid(g), dim3(AB), 0, s, g, m);
    return hipGetLastError();
}

hipError_t launch_apply_correction(const Geom& g, const MixedPtrs& m, hipStream_t s) {
    hipLaunchKernelGGL(k_apply_correction, box_grid(g), dim3(AB), 0, s, g, m);
    return hipGetLastError();
}

hipError_t launch_gather(const double* src, const int64_t* offs, int n, double* out, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, s, src, offs, n, out);
    return hipGetLastError();
}

hipError_t launch_scatter(const double* vals, const int64_t* offs, int n, double* dst, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, vals, offs, n, dst);
    return hipGetLastError();
}

hipError_t launch_chi64(const Geom& g, const double* eta, const double* lp, double* chi, hipStream_t s) {
    hipLaunchKernelGGL(k_chi64, box_grid(g), dim3(AB), 0, s, g, eta, lp, chi);
    return hipGetLastError();
}

hipError_t launch_adjoint_gradient(const Geom& g, const Coef& c, const double* kc, const double* pf,
                                   const double* lam_pf, double* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_adjoint_gradient, box_grid(g), dim3(AB), 0, s, g, c, kc, pf, lam_pf, grad);
    return hipGetLastError();
}

hipError_t launch_exp_cells(const Geom& g, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_exp_cells, box_grid(g), dim3(AB), 0, s, g, src, dst);
    return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t s) {
    const int64_t n2 = n / 2;
    if (n2 > 0) {
        int64_t blocks = (n2 + (int64_t)AB * CU_UNROLL - 1) / ((int64_t)AB * CU_UNROLL);
        if (blocks > 256 * 32) blocks = 256 * 32;
        hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(AB), 0, s,
                           reinterpret_cast<const dvec2*>(src), reinterpret_cast<dvec2*>(dst), n2);
    }
    if (n % 2 == 1) hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace ptk
