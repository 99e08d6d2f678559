// Reactive porosity waves (thesis article 3; the appendix reactive script):
// the fused pseudo-transient sweep, the pseudo-step reduction and the host
// side of the C ABI declared in include/ptwaves.h.
//
// One launch is one PT iteration on the four iterated cell fields (Xs, Pf,
// phi, dPf/dt) from iteration-k values.  The only neighbour data are Pf and
// the permeability k(phi) of the six face neighbours (the Darcy flux of each
// face), so a 66 x 12 block owns a 64 x 10 column of cells plus a one-cell
// halo ring and marches up a chunk of planes: per plane it stages Pf and k
// in LDS (double-buffered: one barrier per plane), keeps the planes below
// and above of its own column in registers, and updates its tile cells.
// The check variant (every nup-th iteration) also takes the maximum of
// k/beta_P over its output porosity, which the next pseudo step needs, so
// that only the first pseudo step of a physical step reads the porosity
// in a pass of its own.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "pt_internal.h"
#include "ptwaves.h"

namespace ptk {
namespace {

// Block shape: 66 x 12 (64 x 10 output cells; 13 waves of <= 74 VGPRs, two
// blocks per CU).  Measured at 506 x 506 x 2042, PT iteration with its
// pseudo-step and check kernels amortised: 8 rows 10.19 ms, 10 rows 10.26,
// 11 rows 9.74, 12 rows 9.38, 13 rows 9.39, 14 rows 9.47, 15 rows 9.51; the
// 10-row tiles at one block per CU 9.39; chunks of 64, 128 and 512 planes
// instead of the cost model's 256: 9.62, 9.48, 9.89; non-temporal loads of
// the tile-only fields 1-2 % slower at every height.
constexpr int WW = 66;   // block width (64 output columns)
constexpr int WH = 12;   // block height (10 output rows)
constexpr int RB = 256;  // threads of the reduction kernels

struct WavesCoef {
    double dxi, dyi, dzi, rfg;           // 1/dx, ..., rho_f g
    double phi0_inv, k_muf0, eta;
    double beta_d, beta_s, beta_f;
    double tau_inv, beta_x, xs_half, xs_max;
    double dt, dti, phi_min, phi_max;
    double onepdx, rho_term;             // 1 + dX, 1 - rho_s/(rho_f (1 + dX))
    double h2_cpf;                       // h^2 / c_pf
};

struct WavesPtrs {
    const double *xs, *pf, *phi, *dp, *xso, *pfo, *phio;
    double *xs_o, *pf_o, *phi_o, *dp_o;
    const double* dtau;                  // pseudo step (device scalar)
    double* partials;                    // [blocks][8]: the block's error, max k/beta_P of its output
};

__device__ __forceinline__ double perm(const WavesCoef& c, double phi) {
    const double r = phi * c.phi0_inv;
    return c.k_muf0 * r * r * r;
}
__device__ __forceinline__ double beta_p(const WavesCoef& c, double phi) {
    return phi * c.beta_f + c.beta_d - (1.0 + phi) * c.beta_s;
}
__device__ __forceinline__ double nanmax(double m, double v) { return (v > m || v != v) ? v : m; }

template <bool NORMS>
__global__ __launch_bounds__(WW * WH) void k_waves_sweep(Geom g, WavesCoef c, WavesPtrs p) {
    constexpr int W = WW, H = WH;
    __shared__ double spf[2][H][W], skc[2][H][W];
    const int gx = (g.nx + W - 3) / (W - 2);
    const int gy = (g.ny + H - 3) / (H - 2);
    const int64_t Tt = xcd_tile(blockIdx.x, (int64_t)gridDim.x);
    const int bx = (int)(Tt % gx), by = (int)((Tt / gx) % gy), bz = (int)(Tt / ((int64_t)gx * gy));
    int tx, ty;
    tile_thread<W, H>(tx, ty);
    const int i = bx * (W - 2) - 1 + tx;
    const int j = by * (H - 2) - 1 + ty;
    const int kz0 = bz * g.kz, kz1 = min(g.nz, kz0 + g.kz);
    const bool cell = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    const bool tile = cell && tx >= 1 && tx <= W - 2 && ty >= 1 && ty <= H - 2;
    const int ic = min(max(i, 0), g.nx), jc = min(max(j, 0), g.ny);
    const int64_t col = (int64_t)jc * g.P + ic;
    auto at = [&](int k) -> int64_t { return (int64_t)min(max(k, 0), g.nz) * g.S + col; };
    const double dtau = *p.dtau;

    // own column: Pf and k of planes p-1, p, p+1 (zero outside the domain)
    auto qload = [&](int k, double& pf, double& kc, double& phi) {
        const int64_t o = at(k);
        pf = p.pf[o];
        phi = p.phi[o];
        const bool ok = cell && k >= 0 && k < g.nz;
        kc = ok ? perm(c, phi) : 0.0;
        pf = ok ? pf : 0.0;
    };
    double pf_p, kc_p, phi_p, pf_c, kc_c, phi_c, pf_n, kc_n, phi_n;
    qload(kz0 - 1, pf_p, kc_p, phi_p);
    qload(kz0, pf_c, kc_c, phi_c);
    qload(kz0 + 1, pf_n, kc_n, phi_n);
    // tile-only values of plane p, loaded one plane ahead
    double xs = 0.0, dp = 0.0, xso = 0.0, pfo = 0.0, phio = 0.0;
    auto tload = [&](int k, double& a, double& b, double& d, double& e, double& f) {
        if (tile) {
            const int64_t o = at(k);
            a = p.xs[o]; b = p.dp[o]; d = p.xso[o]; e = p.pfo[o]; f = p.phio[o];
        }
    };
    tload(kz0, xs, dp, xso, pfo, phio);
    double err = 0.0, kmax = 0.0;

    for (int pz = kz0; pz < kz1; ++pz) {
        const int buf = pz & 1;
        // prefetch the next step
        double pf_nn, kc_nn, phi_nn, xs2 = 0.0, dp2 = 0.0, xso2 = 0.0, pfo2 = 0.0, phio2 = 0.0;
        qload(pz + 2, pf_nn, kc_nn, phi_nn);
        tload(pz + 1, xs2, dp2, xso2, pfo2, phio2);

        spf[buf][ty][tx] = pf_c;
        skc[buf][ty][tx] = kc_c;
        __syncthreads();

        if (tile) {
            // Darcy flux of the six faces (zero through the walls), eq (8)'s divergence
            const double kw = skc[buf][ty][tx - 1], ke = skc[buf][ty][tx + 1];
            const double ks = skc[buf][ty - 1][tx], kn = skc[buf][ty + 1][tx];
            const double qxl = (i > 0) ? -0.5 * (kw + kc_c) * (pf_c - spf[buf][ty][tx - 1]) * c.dxi : 0.0;
            const double qxh = (i < g.nx - 1) ? -0.5 * (kc_c + ke) * (spf[buf][ty][tx + 1] - pf_c) * c.dxi : 0.0;
            const double qyl = (j > 0) ? -0.5 * (ks + kc_c) * (pf_c - spf[buf][ty - 1][tx]) * c.dyi : 0.0;
            const double qyh = (j < g.ny - 1) ? -0.5 * (kc_c + kn) * (spf[buf][ty + 1][tx] - pf_c) * c.dyi : 0.0;
            const double qzl = (pz > 0) ? -0.5 * (kc_p + kc_c) * ((pf_c - pf_p) * c.dzi - c.rfg) : 0.0;
            const double qzh = (pz < g.nz - 1) ? -0.5 * (kc_c + kc_n) * ((pf_n - pf_c) * c.dzi - c.rfg) : 0.0;
            const double divq = (qxh - qxl) * c.dxi + (qyh - qyl) * c.dyi + (qzh - qzl) * c.dzi;

            const double pe = -pf_c;
            const double xseq = fmin(fmax(c.beta_x * pf_c + c.xs_half, 0.0), c.xs_max);
            const double bp = beta_p(c, phi_c);
            const double bphi = c.beta_d - c.beta_s / (1.0 - phi_c);
            const double dxsdt = (xseq - xs) * c.tau_inv;
            const double compaction = pe / (c.eta * (1.0 - phi_c));
            const double xs_n = xso + c.dt * dxsdt;
            const double pf_new = pf_c + dtau * dp - dtau * (pf_c - pfo) * c.dti;
            const double dphidt = (1.0 - phi_c) * (bphi * dp - compaction - c.onepdx / (1.0 - xs) * dxsdt);
            const double phi_new = fmin(fmax(phio + c.dt * dphidt, c.phi_min), c.phi_max);
            const double dp_new =
                (-divq + compaction + c.rho_term * (1.0 - phi_c) * c.onepdx / (1.0 - xs) * dxsdt) / bp;
            const int64_t o = (int64_t)pz * g.S + col;
            p.xs_o[o] = xs_n;
            p.pf_o[o] = pf_new;
            p.phi_o[o] = phi_new;
            p.dp_o[o] = dp_new;
            if (NORMS) {
                err = nanmax(err, fabs(phi_new - phi_c));
                err = nanmax(err, fabs(pf_new - pf_c) / 10.0);
                err = nanmax(err, fabs(xs_n - xs));
                // the next pseudo step's maximum, over this iteration's output
                kmax = nanmax(kmax, perm(c, phi_new) / beta_p(c, phi_new));
            }
        }
        pf_p = pf_c; kc_p = kc_c; phi_p = phi_c;
        pf_c = pf_n; kc_c = kc_n; phi_c = phi_n;
        pf_n = pf_nn; kc_n = kc_nn; phi_n = phi_nn;
        xs = xs2; dp = dp2; xso = xso2; pfo = pfo2; phio = phio2;
    }
    (void)phi_p;

    if constexpr (NORMS) {
        // wave64 butterfly in each of the H row waves (the halo wave holds
        // no tile cell), then across them through LDS
        __shared__ double red[2][WH];
        const int L = threadIdx.x, wave = L >> 6, lane = L & 63;
        if (wave < WH) {
            double v = err, u = kmax;
            for (int off = 32; off >= 1; off >>= 1) {
                v = nanmax(v, __shfl_xor(v, off, 64));
                u = nanmax(u, __shfl_xor(u, off, 64));
            }
            if (lane == 0) {
                red[0][wave] = v;
                red[1][wave] = u;
            }
        }
        __syncthreads();
        if (L < NNORM) {
            double r = 0.0;
            if (L < 2)
                for (int w = 0; w < WH; ++w) r = nanmax(r, red[L][w]);
            p.partials[(int64_t)blockIdx.x * NNORM + L] = r;
        }
    }
}

// Per-block maxima of k/beta_P over the cells (grid-stride), into partials.
__global__ __launch_bounds__(RB) void k_waves_kmax(Geom g, WavesCoef c, const double* __restrict__ phi,
                                                   double* __restrict__ partials) {
    __shared__ double red[RB / 64];
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    double m = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < ncell; t += (int64_t)gridDim.x * RB) {
        const int i = (int)(t % g.nx), j = (int)((t / g.nx) % g.ny), k = (int)(t / ((int64_t)g.nx * g.ny));
        const double f = phi[(int64_t)k * g.S + (int64_t)j * g.P + i];
        m = nanmax(m, perm(c, f) / beta_p(c, f));
    }
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < RB / 64; ++w) r = nanmax(r, red[w]);
        partials[blockIdx.x] = r;
    }
}

// dtau = h^2 / c_pf / max over the block maxima (one block).
__global__ __launch_bounds__(RB) void k_waves_dtau(const double* __restrict__ partials, int64_t nb, double h2_cpf,
                                                   double* __restrict__ dtau) {
    __shared__ double red[RB / 64];
    double m = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += RB) m = nanmax(m, partials[b]);
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < RB / 64; ++w) r = nanmax(r, red[w]);
        *dtau = h2_cpf / r;
    }
}

constexpr int64_t KMAX_BLOCKS = 2048;

}  // namespace
}  // namespace ptk

using namespace ptk;

struct pt_waves {
    Geom geom;
    pt_waves_params prm;
    WavesCoef coef;
    double* f[PT_W_NFIELDS][2];
    int cur[PT_W_NPING];
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    int64_t iter = 0;
    bool checked = false;
    bool kmax_fresh = false;   // the last sweep was a check: max k/beta_P of the present porosity is in hand
    std::string err;
};

namespace {

int64_t sweep_blocks(const Geom& g) { return iter_grid_blocks(g, WW, WH); }
// [sweep partials: blocks x 8][error: 8][dtau: 1][k/beta_P partials: KMAX_BLOCKS]
size_t waves_ws_needed(const pt_waves* w) {
    const int64_t n = sweep_blocks(w->geom) * NNORM + NNORM + 1 + KMAX_BLOCKS;
    return (size_t)((n + 31) / 32 * 32) * sizeof(double);
}
double* ws_partials(pt_waves* w) { return static_cast<double*>(w->ws); }
double* ws_error(pt_waves* w) { return ws_partials(w) + sweep_blocks(w->geom) * NNORM; }
double* ws_dtau(pt_waves* w) { return ws_error(w) + NNORM; }
double* ws_kmax(pt_waves* w) { return ws_dtau(w) + 1; }

pt_status wfail(pt_waves* w, pt_status s, const char* msg) {
    if (w) w->err = msg;
    return s;
}
pt_status whip(pt_waves* w, hipError_t e, const char* where) {
    if (w) w->err = std::string(where) + ": " + hipGetErrorString(e);
    return PT_EDEVICE;
}

bool waves_valid(const pt_waves_params* p) {
    if (!p || p->version != PT_WAVES_ABI_VERSION || p->nup < 1) return false;
    const double pos[] = {p->lx, p->ly, p->lz, p->phi0, p->k_muf0, p->eta, p->rho_f, p->tau, p->dt, p->c_pf};
    for (double v : pos)
        if (!(v > 0.0) || !std::isfinite(v)) return false;
    if (!(p->phi_min > 0.0 && p->phi_min <= p->phi_max && p->phi_max <= 1.0)) return false;
    if (!(p->xs_max > 0.0 && p->xs_max < 1.0) || !(p->delta_x > -1.0)) return false;
    return true;
}

void waves_coef(pt_waves* w) {
    const pt_waves_params& p = w->prm;
    WavesCoef& c = w->coef;
    const double dx = p.lx / w->geom.nx, dy = p.ly / w->geom.ny, dz = p.lz / w->geom.nz;
    const double h = std::fmin(dx, std::fmin(dy, dz));
    c.dxi = 1.0 / dx; c.dyi = 1.0 / dy; c.dzi = 1.0 / dz;
    c.rfg = p.rho_f * p.g;
    c.phi0_inv = 1.0 / p.phi0;
    c.k_muf0 = p.k_muf0;
    c.eta = p.eta;
    c.beta_d = p.beta_d; c.beta_s = p.beta_s; c.beta_f = p.beta_f;
    c.tau_inv = 1.0 / p.tau;
    c.beta_x = p.beta_x;
    c.xs_half = 0.5 * p.xs_max;
    c.xs_max = p.xs_max;
    c.dt = p.dt; c.dti = 1.0 / p.dt;
    c.phi_min = p.phi_min; c.phi_max = p.phi_max;
    c.onepdx = 1.0 + p.delta_x;
    c.rho_term = 1.0 - p.rho_s / (p.rho_f * (1.0 + p.delta_x));
    c.h2_cpf = h * h / p.c_pf;
}

pt_status waves_ready(pt_waves* w) {
    for (int f = 0; f < PT_W_NFIELDS; ++f) {
        if (!w->f[f][0]) return wfail(w, PT_EINVAL, "not every field is bound");
        if (f < PT_W_NPING && !w->f[f][1]) return wfail(w, PT_EINVAL, "both copies of the iterated fields must be bound");
    }
    if (!w->ws || w->ws_bytes < waves_ws_needed(w)) return wfail(w, PT_EINVAL, "workspace not bound or too small");
    return PT_OK;
}

double* wcur(pt_waves* w, int f) { return f < PT_W_NPING ? w->f[f][w->cur[f]] : w->f[f][0]; }
double* walt(pt_waves* w, int f) { return w->f[f][1 - w->cur[f]]; }

pt_status waves_iteration(pt_waves* w, bool refresh_dtau, bool norms) {
    hipError_t e = hipSuccess;
    if (refresh_dtau) {
        if (w->kmax_fresh) {
            // the check sweep just before took the maximum over its output
            hipLaunchKernelGGL(k_waves_dtau, dim3(1), dim3(RB), 0, w->stream, ws_error(w) + 1, (int64_t)1,
                               w->coef.h2_cpf, ws_dtau(w));
        } else {
            const int64_t ncell = (int64_t)w->geom.nx * w->geom.ny * w->geom.nz;
            const int64_t nb = std::min<int64_t>(KMAX_BLOCKS, (ncell + RB - 1) / RB);
            hipLaunchKernelGGL(k_waves_kmax, dim3((unsigned)nb), dim3(RB), 0, w->stream, w->geom, w->coef,
                               wcur(w, PT_W_PHI), ws_kmax(w));
            hipLaunchKernelGGL(k_waves_dtau, dim3(1), dim3(RB), 0, w->stream, ws_kmax(w), nb, w->coef.h2_cpf,
                               ws_dtau(w));
        }
        e = hipGetLastError();
        if (e != hipSuccess) return whip(w, e, "pseudo step");
    }
    WavesPtrs p{};
    p.xs = wcur(w, PT_W_XS); p.pf = wcur(w, PT_W_PF); p.phi = wcur(w, PT_W_PHI); p.dp = wcur(w, PT_W_DPFDT);
    p.xso = wcur(w, PT_W_XSO); p.pfo = wcur(w, PT_W_PFO); p.phio = wcur(w, PT_W_PHIO);
    p.xs_o = walt(w, PT_W_XS); p.pf_o = walt(w, PT_W_PF); p.phi_o = walt(w, PT_W_PHI); p.dp_o = walt(w, PT_W_DPFDT);
    p.dtau = ws_dtau(w);
    p.partials = ws_partials(w);
    const Geom v = sweep_geom(w->geom, WW, WH);
    const dim3 grid((unsigned)sweep_blocks(w->geom)), block(WW * WH);
    if (norms) hipLaunchKernelGGL(k_waves_sweep<true>, grid, block, 0, w->stream, v, w->coef, p);
    else hipLaunchKernelGGL(k_waves_sweep<false>, grid, block, 0, w->stream, v, w->coef, p);
    e = hipGetLastError();
    if (e != hipSuccess) return whip(w, e, "waves sweep");
    if (norms) {
        e = launch_reduce_max(ws_partials(w), sweep_blocks(w->geom), ws_error(w), w->stream);
        if (e != hipSuccess) return whip(w, e, "waves error");
        w->checked = true;
    }
    w->kmax_fresh = norms;
    for (int f = 0; f < PT_W_NPING; ++f) w->cur[f] ^= 1;
    w->iter += 1;
    return PT_OK;
}

pt_status waves_read_error(pt_waves* w, double* err) {
    double host = 0.0;
    hipError_t e = hipMemcpyAsync(&host, ws_error(w), sizeof(double), hipMemcpyDeviceToHost, w->stream);
    const hipError_t es = hipStreamSynchronize(w->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return whip(w, e, "error copy");
    *err = host;
    if (!std::isfinite(host)) return wfail(w, PT_EDIVERGED, "non-finite stopping quantity");
    return PT_OK;
}

}  // namespace

extern "C" {

pt_status pt_waves_create(int32_t nx, int32_t ny, int32_t nz, int64_t row_pitch, const pt_waves_params* params,
                          pt_waves** out) {
    if (!out) return PT_EINVAL;
    *out = nullptr;
    if (nx < 2 || ny < 2 || nz < 2 || row_pitch < (int64_t)nx + 1 || !waves_valid(params)) return PT_EINVAL;
    pt_waves* w = new (std::nothrow) pt_waves();
    if (!w) return PT_EINVAL;
    w->geom.nx = nx; w->geom.ny = ny; w->geom.nz = nz;
    w->geom.P = row_pitch;
    w->geom.S = row_pitch * (int64_t)(ny + 1);
    w->geom.kz = KZ_MAX;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        w->geom.cus = cus;
    (void)hipGetLastError();
    w->prm = *params;
    std::memset(w->f, 0, sizeof(w->f));
    std::memset(w->cur, 0, sizeof(w->cur));
    waves_coef(w);
    *out = w;
    return PT_OK;
}

pt_status pt_waves_destroy(pt_waves* w) {
    delete w;
    return PT_OK;
}

int64_t pt_waves_field_elems(const pt_waves* w) { return w ? w->geom.S * (int64_t)(w->geom.nz + 1) : 0; }

pt_status pt_waves_bind_field(pt_waves* w, int32_t field, int32_t copy, void* dev_ptr) {
    if (!w) return PT_EINVAL;
    if (field < 0 || field >= PT_W_NFIELDS) return wfail(w, PT_EINVAL, "bad field id");
    if (copy < 0 || copy > 1 || (copy == 1 && field >= PT_W_NPING)) return wfail(w, PT_EINVAL, "bad copy index");
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u)) return wfail(w, PT_EINVAL, "null or unaligned pointer");
    w->f[field][copy] = static_cast<double*>(dev_ptr);
    return PT_OK;
}

pt_status pt_waves_workspace_size(const pt_waves* w, size_t* bytes) {
    if (!w || !bytes) return PT_EINVAL;
    *bytes = waves_ws_needed(w);
    return PT_OK;
}

pt_status pt_waves_bind_workspace(pt_waves* w, void* dev_ptr, size_t bytes) {
    if (!w) return PT_EINVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) || bytes < waves_ws_needed(w))
        return wfail(w, PT_EINVAL, "workspace missing, unaligned or too small");
    w->ws = dev_ptr;
    w->ws_bytes = bytes;
    return PT_OK;
}

pt_status pt_waves_set_stream(pt_waves* w, void* hip_stream) {
    if (!w) return PT_EINVAL;
    w->stream = static_cast<hipStream_t>(hip_stream);
    return PT_OK;
}

pt_status pt_waves_current(const pt_waves* w, int32_t field, int32_t* copy) {
    if (!w || !copy || field < 0 || field >= PT_W_NFIELDS) return PT_EINVAL;
    *copy = field < PT_W_NPING ? w->cur[field] : 0;
    return PT_OK;
}

pt_status pt_waves_begin_step(pt_waves* w) {
    if (!w) return PT_EINVAL;
    pt_status st = waves_ready(w);
    if (st != PT_OK) return st;
    const int64_t n = w->geom.S * (int64_t)(w->geom.nz + 1);
    const int pairs[3][2] = {{PT_W_XS, PT_W_XSO}, {PT_W_PF, PT_W_PFO}, {PT_W_PHI, PT_W_PHIO}};
    for (auto& pr : pairs) {
        hipError_t e = launch_copy(wcur(w, pr[0]), w->f[pr[1]][0], n, w->stream);
        if (e != hipSuccess) return whip(w, e, "old values");
    }
    w->iter = 0;
    w->kmax_fresh = false;
    return PT_OK;
}

pt_status pt_waves_iterate(pt_waves* w, int64_t n) {
    if (!w || n < 0) return PT_EINVAL;
    pt_status st = waves_ready(w);
    if (st != PT_OK) return st;
    const int64_t nup = w->prm.nup;
    for (int64_t m = 0; m < n; ++m) {
        const int64_t it = w->iter + 1;
        st = waves_iteration(w, (it - 1) % nup == 0, it % nup == 0);
        if (st != PT_OK) return st;
    }
    return PT_OK;
}

pt_status pt_waves_last_error(pt_waves* w, double* err) {
    if (!w || !err) return PT_EINVAL;
    if (!w->checked) return wfail(w, PT_EINVAL, "no stopping quantity computed yet");
    return waves_read_error(w, err);
}

pt_status pt_waves_solve_step(pt_waves* w, double eps, int64_t iter_max, int64_t* iters, double* err) {
    if (!w || !(eps > 0.0) || iter_max < 1) return PT_EINVAL;
    pt_status st = waves_ready(w);
    if (st != PT_OK) return st;
    const int64_t nup = w->prm.nup;
    double e = INFINITY;
    while (w->iter < iter_max) {
        const int64_t chunk = std::min<int64_t>(nup - (w->iter % nup), iter_max - w->iter);
        st = pt_waves_iterate(w, chunk);
        if (st != PT_OK) return st;
        if (w->iter % nup == 0) {
            st = waves_read_error(w, &e);
            if (st != PT_OK) break;
            if (e < eps) break;
        }
    }
    if (iters) *iters = w->iter;
    if (err) *err = e;
    if (st != PT_OK) return st;
    return (e < eps) ? PT_OK : PT_ENOTCONV;
}

const char* pt_waves_last_message(const pt_waves* w) { return w ? w->err.c_str() : "null handle"; }

}  // extern "C"
