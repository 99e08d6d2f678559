// Adjoint of a run of Picard steps (steps x stages), reverse sweep kernels.
//
// Forward (per physical step; the stress history is updated from the run's
// second step on):  So = a So_prev + b E(V_prev) (eq (21), backward Euler);
// old values Pto, Pfo, Lo; then per stage the refresh K = k0 (phi/phi0)^3,
// eta = eta0 Mn (phi0/phi) R (eqs (23), (25)), s = 1 - phi; the linear stage
// F(x) = 0 of eqs (17)-(20); and the porosity step L = Lo - dt Phi (eq (22)).
//
// Reverse, per stage (gather form, one thread per point of the padded box):
//   k_adj_porosity  adjoint of the porosity step: adds -xbar to the
//                   transposed solve's right-hand side, accumulates the old
//                   values' adjoints, and leaves eta_bar, s_bar of Phi;
//   (transposed stage solve by the FP64 correction sweep: J_F is symmetric)
//   k_adj_coef      theta_bar = -lambda^T dF/dtheta for K, chi = 1/(eta s),
//                   s (buoyancy), Pto, Pfo and the history term, and the
//                   refresh chain to the incoming porosity and to ln k0;
// per step boundary:
//   k_adj_step      old values -> the previous step's final state; history
//                   term -> So_bar (a D^T, D the stress divergence);
//   k_adj_history   V_bar = E^T (b So_bar) into the right-hand side, then
//   k_adj_scale     So_bar <- a So_bar for the previous history.
// The switch R (Pf > Pt at refresh) is piecewise constant and has no
// derivative.  These kernels run a few times per stage: plain stencils that
// read neighbours through the caches.
#include "pt_internal.h"

namespace ptk {

namespace {

constexpr int AB = 256;

struct Idx {
    int i, j, k;
};

__device__ __forceinline__ bool box_index(const Geom& g, int64_t t, Idx& q) {
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

__device__ __forceinline__ double maxwell_a(double mu, double gdts_inv) {
    const double xi = mu * gdts_inv;
    return xi / (1.0 + xi);
}
__device__ __forceinline__ double maxwell_b(double mu, double gdts_inv) {
    const double xi = mu * gdts_inv;
    return 2.0 * mu / (1.0 + xi);
}

inline dim3 grid_of(const Geom& g) {
    const int64_t n = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    return dim3((unsigned)((n + AB - 1) / AB));
}

// ---- porosity step -----------------------------------------------------------
// Phi = beta_phi((Pf-Pfo) - (Pt-Pto))/dt + (Pf-Pt)/eta + adv, where an interior
// face between cells lo and hi adds 1/2 V (s_hi - s_lo)/h to the rate of both.
// With phib = -dt Lbar: xbar_Pf += phib (beta_phi/dt + 1/eta), xbar_Pt -= the
// same, Pfo_bar -= phib beta_phi/dt, Pto_bar += phib beta_phi/dt,
// Lo_bar += Lbar; a face adds w (s_hi - s_lo) to V_bar and +-w V to s_bar,
// w = 1/2 (phib_lo + phib_hi)/h.
__global__ __launch_bounds__(AB) void k_adj_porosity(Geom g, Coef c, AdjPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    const int64_t o = at(g, i, j, k);
    auto phib = [&](int ii, int jj, int kk) { return -c.dt * a.lbar[at(g, ii, jj, kk)]; };
    auto sf = [&](int ii, int jj, int kk) { return exp(a.lp[at(g, ii, jj, kk)]); };
    if (j < g.ny && k < g.nz && i >= 1 && i < g.nx) {
        const double w = 0.5 * (phib(i - 1, j, k) + phib(i, j, k)) * c.dxi;
        a.rvx[o] -= w * (sf(i, j, k) - sf(i - 1, j, k));
    }
    if (i < g.nx && k < g.nz && j >= 1 && j < g.ny) {
        const double w = 0.5 * (phib(i, j - 1, k) + phib(i, j, k)) * c.dyi;
        a.rvy[o] -= w * (sf(i, j, k) - sf(i, j - 1, k));
    }
    if (i < g.nx && j < g.ny && k >= 1 && k < g.nz) {
        const double w = 0.5 * (phib(i, j, k - 1) + phib(i, j, k)) * c.dzi;
        a.rvz[o] -= w * (sf(i, j, k) - sf(i, j, k - 1));
    }
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    const double pb = phib(i, j, k);
    const double eta = a.eta[o], pt = a.pt[o], pf = a.pf[o];
    const double c1 = c.beta_phi * c.dti + 1.0 / eta;
    a.rpf[o] -= pb * c1;
    a.rpt[o] += pb * c1;
    a.pfo_bar[o] -= pb * c.beta_phi * c.dti;
    a.pto_bar[o] += pb * c.beta_phi * c.dti;
    a.lo_bar[o] += a.lbar[o];
    a.eta_bar[o] = -pb * (pf - pt) / (eta * eta);
    double sb = 0.0;
    if (i >= 1) sb += 0.5 * (phib(i - 1, j, k) + pb) * c.dxi * a.vx[o];
    if (i + 1 < g.nx) sb -= 0.5 * (pb + phib(i + 1, j, k)) * c.dxi * a.vx[at(g, i + 1, j, k)];
    if (j >= 1) sb += 0.5 * (phib(i, j - 1, k) + pb) * c.dyi * a.vy[o];
    if (j + 1 < g.ny) sb -= 0.5 * (pb + phib(i, j + 1, k)) * c.dyi * a.vy[at(g, i, j + 1, k)];
    if (k >= 1) sb += 0.5 * (phib(i, j, k - 1) + pb) * c.dzi * a.vz[o];
    if (k + 1 < g.nz) sb -= 0.5 * (pb + phib(i, j, k + 1)) * c.dzi * a.vz[at(g, i, j, k + 1)];
    a.s_bar[o] = sb;
}

// ---- stage parameters and the refresh chain ------------------------------------
// K_bar   = sum over the cell's interior faces of 1/2 g_f (lam_lo - lam_hi)/h,
//           g_f = (Pf_hi - Pf_lo)/h + b (Darcy, b the buoyancy term on z-faces);
// chi_bar = -(lam_Pt - lam_Pf)(Pt - Pf);
// s_bar  += 1/2 (rhos g - rhof g) (lam_Vz below + lam_Vz above) (buoyancy);
// Pto_bar += beta_d/dt (lam_Pt - alpha lam_Pf); Pfo_bar += beta_d/dt
// ((alpha/B) lam_Pf - alpha lam_Pt); history-term adjoint -= lam_V.
// Refresh chain: eta_bar -= chi_bar/(eta^2 s), s_bar -= chi_bar/(eta s^2),
// L_bar = -3 K_bar K s/phi + eta_bar eta s/phi + s_bar s, grad += K_bar K.
// The right-hand side is cleared for the next stage.
__global__ __launch_bounds__(AB) void k_adj_coef(Geom g, Coef c, AdjPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    const int64_t o = at(g, i, j, k);
    if (j < g.ny && k < g.nz && i >= 1 && i < g.nx) a.fbx[o] -= a.lvx[o];
    if (i < g.nx && k < g.nz && j >= 1 && j < g.ny) a.fby[o] -= a.lvy[o];
    if (i < g.nx && j < g.ny && k >= 1 && k < g.nz) a.fbz[o] -= a.lvz[o];
    a.rvx[o] = 0.0;
    a.rvy[o] = 0.0;
    a.rvz[o] = 0.0;
    a.rpt[o] = 0.0;
    a.rpf[o] = 0.0;
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    double kb = 0.0;
    auto face = [&](int64_t lo, int64_t hi, double hinv, double b) {
        const double gf = (a.pf[hi] - a.pf[lo]) * hinv + b;
        kb += 0.5 * gf * (a.lpf[lo] - a.lpf[hi]) * hinv;
    };
    if (i > 0) face(at(g, i - 1, j, k), o, c.dxi, 0.0);
    if (i < g.nx - 1) face(o, at(g, i + 1, j, k), c.dxi, 0.0);
    if (j > 0) face(at(g, i, j - 1, k), o, c.dyi, 0.0);
    if (j < g.ny - 1) face(o, at(g, i, j + 1, k), c.dyi, 0.0);
    if (k > 0) face(at(g, i, j, k - 1), o, c.dzi, c.buoy);
    if (k < g.nz - 1) face(o, at(g, i, j, k + 1), c.dzi, c.buoy);
    const double lpt = a.lpt[o], lpf = a.lpf[o];
    const double chib = -(lpt - lpf) * (a.pt[o] - a.pf[o]);
    double sbuoy = 0.0;
    if (k >= 1) sbuoy += a.lvz[o];
    if (k + 1 < g.nz) sbuoy += a.lvz[at(g, i, j, k + 1)];
    sbuoy *= 0.5 * (c.rhosg - c.rhofg);
    a.pto_bar[o] += c.beta_d * c.dti * (lpt - c.alpha * lpf);
    a.pfo_bar[o] += c.beta_d * c.dti * (c.ab * lpf - c.alpha * lpt);
    const double s = exp(a.lp[o]);
    const double phi = 1.0 - s;
    const double K = a.kc[o], eta = a.eta[o];
    const double etab = a.eta_bar[o] - chib / (eta * eta * s);
    const double sbt = a.s_bar[o] + sbuoy - chib / (eta * s * s);
    a.lbar_out[o] = -3.0 * kb * K * s / phi + etab * eta * s / phi + sbt * s;
    a.grad[o] += kb * K;
}

// ---- step boundary -------------------------------------------------------------
// Lo, Pto, Pfo were the previous step's final ln(1-phi), Pt, Pf: their
// adjoints join L_bar and the right-hand side of the previous step's last
// stage.  The history term div(a So) gives So_bar += a D^T w (w its adjoint;
// D^T of the divergence of cell normal stresses and interior-edge shear
// stresses), with a at cells and (four-cell mean mu) at edges.
__global__ __launch_bounds__(AB) void k_adj_step(Geom g, Coef c, AdjPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    const int64_t o = at(g, i, j, k);
    auto mus = [&](int ii, int jj, int kk) { return a.mus[at(g, ii, jj, kk)]; };
    auto wx = [&](int ii, int jj, int kk) { return a.fbx[at(g, ii, jj, kk)]; };
    auto wy = [&](int ii, int jj, int kk) { return a.fby[at(g, ii, jj, kk)]; };
    auto wz = [&](int ii, int jj, int kk) { return a.fbz[at(g, ii, jj, kk)]; };
    if (i < g.nx && j < g.ny && k < g.nz) {
        a.lbar_out[o] = a.lbar[o] + a.lo_bar[o];
        a.rpt[o] = -a.pto_bar[o];
        a.rpf[o] = -a.pfo_bar[o];
        a.pto_bar[o] = 0.0;
        a.pfo_bar[o] = 0.0;
        a.lo_bar[o] = 0.0;
        const double ac = maxwell_a(mus(i, j, k), c.gdts_inv);
        a.sbxx[o] += ac * (wx(i, j, k) - wx(i + 1, j, k)) * c.dxi;
        a.sbyy[o] += ac * (wy(i, j, k) - wy(i, j + 1, k)) * c.dyi;
        a.sbzz[o] += ac * (wz(i, j, k) - wz(i, j, k + 1)) * c.dzi;
    }
    if (k < g.nz && i >= 1 && i < g.nx && j >= 1 && j < g.ny) {
        const double mue = 0.25 * (mus(i - 1, j - 1, k) + mus(i, j - 1, k) + mus(i - 1, j, k) + mus(i, j, k));
        a.sbxy[o] += maxwell_a(mue, c.gdts_inv) *
                     ((wx(i, j - 1, k) - wx(i, j, k)) * c.dyi + (wy(i - 1, j, k) - wy(i, j, k)) * c.dxi);
    }
    if (j < g.ny && i >= 1 && i < g.nx && k >= 1 && k < g.nz) {
        const double mue = 0.25 * (mus(i - 1, j, k - 1) + mus(i, j, k - 1) + mus(i - 1, j, k) + mus(i, j, k));
        a.sbxz[o] += maxwell_a(mue, c.gdts_inv) *
                     ((wx(i, j, k - 1) - wx(i, j, k)) * c.dzi + (wz(i - 1, j, k) - wz(i, j, k)) * c.dxi);
    }
    if (i < g.nx && j >= 1 && j < g.ny && k >= 1 && k < g.nz) {
        const double mue = 0.25 * (mus(i, j - 1, k - 1) + mus(i, j, k - 1) + mus(i, j - 1, k) + mus(i, j, k));
        a.sbyz[o] += maxwell_a(mue, c.gdts_inv) *
                     ((wy(i, j, k - 1) - wy(i, j, k)) * c.dzi + (wz(i, j - 1, k) - wz(i, j, k)) * c.dyi);
    }
}

// History update So = a So_prev + b E(V_prev): V_bar = E^T (b So_bar) on the
// interior faces, into the right-hand side (-xbar).  E: deviatoric normal
// strain rates at cells, 1/2 (dVx/dy + dVy/dx) etc. at interior edges.
__global__ __launch_bounds__(AB) void k_adj_history(Geom g, Coef c, AdjPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    const int64_t o = at(g, i, j, k);
    auto mus = [&](int ii, int jj, int kk) { return a.mus[at(g, ii, jj, kk)]; };
    // deviatoric part of b So_bar at a cell, component 0/1/2
    auto dev = [&](int ii, int jj, int kk, int comp) {
        const int64_t p = at(g, ii, jj, kk);
        const double b = maxwell_b(mus(ii, jj, kk), c.gdts_inv);
        const double tr = (a.sbxx[p] + a.sbyy[p] + a.sbzz[p]) * c.third;
        const double v = comp == 0 ? a.sbxx[p] : (comp == 1 ? a.sbyy[p] : a.sbzz[p]);
        return b * (v - tr);
    };
    auto txy = [&](int ii, int jj, int kk) {  // b_e So_bar on an interior xy-edge, else 0
        if (ii < 1 || ii >= g.nx || jj < 1 || jj >= g.ny) return 0.0;
        const double mue = 0.25 * (mus(ii - 1, jj - 1, kk) + mus(ii, jj - 1, kk) + mus(ii - 1, jj, kk) + mus(ii, jj, kk));
        return maxwell_b(mue, c.gdts_inv) * a.sbxy[at(g, ii, jj, kk)];
    };
    auto txz = [&](int ii, int jj, int kk) {
        if (ii < 1 || ii >= g.nx || kk < 1 || kk >= g.nz) return 0.0;
        const double mue = 0.25 * (mus(ii - 1, jj, kk - 1) + mus(ii, jj, kk - 1) + mus(ii - 1, jj, kk) + mus(ii, jj, kk));
        return maxwell_b(mue, c.gdts_inv) * a.sbxz[at(g, ii, jj, kk)];
    };
    auto tyz = [&](int ii, int jj, int kk) {
        if (jj < 1 || jj >= g.ny || kk < 1 || kk >= g.nz) return 0.0;
        const double mue = 0.25 * (mus(ii, jj - 1, kk - 1) + mus(ii, jj, kk - 1) + mus(ii, jj - 1, kk) + mus(ii, jj, kk));
        return maxwell_b(mue, c.gdts_inv) * a.sbyz[at(g, ii, jj, kk)];
    };
    if (j < g.ny && k < g.nz && i >= 1 && i < g.nx) {
        const double v = (dev(i - 1, j, k, 0) - dev(i, j, k, 0)) * c.dxi +
                         0.5 * (txy(i, j, k) - txy(i, j + 1, k)) * c.dyi +
                         0.5 * (txz(i, j, k) - txz(i, j, k + 1)) * c.dzi;
        a.rvx[o] -= v;
    }
    if (i < g.nx && k < g.nz && j >= 1 && j < g.ny) {
        const double v = (dev(i, j - 1, k, 1) - dev(i, j, k, 1)) * c.dyi +
                         0.5 * (txy(i, j, k) - txy(i + 1, j, k)) * c.dxi +
                         0.5 * (tyz(i, j, k) - tyz(i, j, k + 1)) * c.dzi;
        a.rvy[o] -= v;
    }
    if (i < g.nx && j < g.ny && k >= 1 && k < g.nz) {
        const double v = (dev(i, j, k - 1, 2) - dev(i, j, k, 2)) * c.dzi +
                         0.5 * (txz(i, j, k) - txz(i + 1, j, k)) * c.dxi +
                         0.5 * (tyz(i, j, k) - tyz(i, j + 1, k)) * c.dyi;
        a.rvz[o] -= v;
    }
}

// So_bar of the previous history = a So_bar (cells, interior edges; boundary
// edges carry no stress); the history-term adjoint restarts at zero.
__global__ __launch_bounds__(AB) void k_adj_scale(Geom g, Coef c, AdjPtrs a) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    const int i = q.i, j = q.j, k = q.k;
    const int64_t o = at(g, i, j, k);
    auto mus = [&](int ii, int jj, int kk) { return a.mus[at(g, ii, jj, kk)]; };
    a.fbx[o] = 0.0;
    a.fby[o] = 0.0;
    a.fbz[o] = 0.0;
    if (i < g.nx && j < g.ny && k < g.nz) {
        const double ac = maxwell_a(mus(i, j, k), c.gdts_inv);
        a.sbxx[o] *= ac;
        a.sbyy[o] *= ac;
        a.sbzz[o] *= ac;
    }
    if (k < g.nz) {
        double v = 0.0;
        if (i >= 1 && i < g.nx && j >= 1 && j < g.ny)
            v = maxwell_a(0.25 * (mus(i - 1, j - 1, k) + mus(i, j - 1, k) + mus(i - 1, j, k) + mus(i, j, k)),
                          c.gdts_inv) * a.sbxy[o];
        a.sbxy[o] = v;
    }
    if (j < g.ny) {
        double v = 0.0;
        if (i >= 1 && i < g.nx && k >= 1 && k < g.nz)
            v = maxwell_a(0.25 * (mus(i - 1, j, k - 1) + mus(i, j, k - 1) + mus(i - 1, j, k) + mus(i, j, k)),
                          c.gdts_inv) * a.sbxz[o];
        a.sbxz[o] = v;
    }
    if (i < g.nx) {
        double v = 0.0;
        if (j >= 1 && j < g.ny && k >= 1 && k < g.nz)
            v = maxwell_a(0.25 * (mus(i, j - 1, k - 1) + mus(i, j, k - 1) + mus(i, j - 1, k) + mus(i, j, k)),
                          c.gdts_inv) * a.sbyz[o];
        a.sbyz[o] = v;
    }
}

// Old pressures that make the stage residual at zero equal the transposed
// solve's right-hand side (rhs slots hold -xbar): with gravity off and the
// history term set to -xbar_V, F(0) = (-xbar_V, beta_d/dt (-Pto + alpha Pfo),
// beta_d/dt (alpha Pto - (alpha/B) Pfo)) = -xbar, so that F(lambda) =
// J_F lambda - xbar and a defect-correction solve of F = 0 is the transposed
// solve.
__global__ __launch_bounds__(AB) void k_adj_oldvalues(Geom g, Coef c, const double* __restrict__ rpt,
                                                      const double* __restrict__ rpf, double* __restrict__ pto,
                                                      double* __restrict__ pfo) {
    Idx q;
    if (!box_index(g, (int64_t)blockIdx.x * AB + threadIdx.x, q)) return;
    if (q.i >= g.nx || q.j >= g.ny || q.k >= g.nz) return;
    const int64_t o = at(g, q.i, q.j, q.k);
    const double xt = -rpt[o], xf = -rpf[o];
    const double f = (xf + c.alpha * xt) * c.dt / (c.beta_d * (c.ab - c.alpha * c.alpha));
    pfo[o] = f;
    pto[o] = c.alpha * f + xt * c.dt / c.beta_d;
}

// Largest |value| over five padded boxes (the transposed solve's right-hand
// side): per-block maxima into slot 0 of the norm partials, other slots 0.
struct Five {
    const double* f[5];
};
__global__ __launch_bounds__(AB) void k_absmax5(Geom g, Five fv, double* __restrict__ partials) {
    __shared__ double red[AB / 64];
    const int64_t n = (int64_t)g.S * (g.nz + 1);
    double m = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * AB + threadIdx.x; t < n; t += (int64_t)gridDim.x * AB) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const double v = fabs(fv.f[q][t]);
            m = (v > m || v != v) ? v : m;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double v = __shfl_xor(m, off, 64);
        m = (v > m || v != v) ? v : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x < NNORM) {
        double r = 0.0;
        if (threadIdx.x == 0)
            for (int w = 0; w < AB / 64; ++w) r = (red[w] > r || red[w] != red[w]) ? red[w] : r;
        partials[(int64_t)blockIdx.x * NNORM + threadIdx.x] = r;
    }
}

}  // namespace

hipError_t launch_adj_porosity(const Geom& g, const Coef& c, const AdjPtrs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_porosity, grid_of(g), dim3(AB), 0, s, g, c, a);
    return hipGetLastError();
}

hipError_t launch_adj_coef(const Geom& g, const Coef& c, const AdjPtrs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_coef, grid_of(g), dim3(AB), 0, s, g, c, a);
    return hipGetLastError();
}

hipError_t launch_adj_step(const Geom& g, const Coef& c, const AdjPtrs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_step, grid_of(g), dim3(AB), 0, s, g, c, a);
    return hipGetLastError();
}

hipError_t launch_adj_history(const Geom& g, const Coef& c, const AdjPtrs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_history, grid_of(g), dim3(AB), 0, s, g, c, a);
    hipLaunchKernelGGL(k_adj_scale, grid_of(g), dim3(AB), 0, s, g, c, a);
    return hipGetLastError();
}

hipError_t launch_adj_oldvalues(const Geom& g, const Coef& c, const double* rpt, const double* rpf, double* pto,
                                double* pfo, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_oldvalues, grid_of(g), dim3(AB), 0, s, g, c, rpt, rpf, pto, pfo);
    return hipGetLastError();
}

hipError_t launch_absmax5(const Geom& g, const double* const* f, double* partials, int64_t nblocks,
                          hipStream_t s) {
    Five fv;
    for (int q = 0; q < 5; ++q) fv.f[q] = f[q];
    hipLaunchKernelGGL(k_absmax5, dim3((unsigned)nblocks), dim3(AB), 0, s, g, fv, partials);
    return hipGetLastError();
}

}  // namespace ptk
