// Vector kernels of the Krylov-accelerated multigrid stage solve (the
// thesis's outlook names multigrid as the accelerator of the PT solvers; a
// Krylov subspace around the cycle keeps it convergent where strong
// coefficient contrasts make single cycles amplify some error components).
//
// A vector holds the five unknowns of the stage (Vx, Vy, Vz, Pt, Pf) or the
// five residuals (momentum x, y, z, r_Pt, r_Pf) of the fine grid in its
// padded boxes.  Only the entries that carry an equation take part: every
// cell for the pressures, the interior faces for the velocities (face i of
// x at index i, i >= 1; likewise j and k).  Wall faces, padding and the
// unused slots keep their values.  Inner products weight the momentum rows
// by wv and the pressure rows by wp (squared weights passed in), the scales
// of the stopping norm.
//
// Directions are kept in FP64: the operator amplifies the rounding error of
// a smooth direction by up to its condition number, so an FP32 direction
// would move the residual by far more than its stored image A p predicts.
// Their images A p are differences of residuals, which are FP32 already.
//
// Reductions run on a fixed grid with a fixed summation order, so results
// do not depend on timing.
#include "pt_internal.h"

namespace ptk {
namespace {

constexpr int KB = 256;

__device__ __forceinline__ bool active(int q, int i, int j, int k) {
    return q == 0 ? i >= 1 : q == 1 ? j >= 1 : q == 2 ? k >= 1 : true;
}

// Sum of NS per-thread values over the block into part[blockIdx.x * KRY_SLOTS + s].
template <int NS>
__device__ __forceinline__ void block_sums(double (&acc)[NS], double* __restrict__ part) {
    __shared__ double red[KB / 64][NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        double v = acc[s];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[s] = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) red[wave][s] = acc[s];
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double v = 0.0;
        for (int w = 0; w < KB / 64; ++w) v += red[w][threadIdx.x];
        part[(int64_t)blockIdx.x * KRY_SLOTS + threadIdx.x] = v;
    }
}

// Work items: VW consecutive columns i0 .. i0 + VW - 1 of one cell row (j, k),
// loaded and stored as whole 16- and 32-byte vectors for VW = 4: the row
// pitch is a multiple of 4 and every box starts on a 32-byte boundary
// (checked when the workspace is bound), and the last vector of a row ends
// within the pitch.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

struct Item {
    int64_t o;
    int i0, j, k;
};

template <int VW>
__device__ __forceinline__ Item item(const Geom& g, int64_t it, int groups) {
    const int64_t r = it / groups;
    Item t;
    t.i0 = VW * (int)(it - r * groups);
    t.j = (int)(r % g.ny);
    t.k = (int)(r / g.ny);
    t.o = (int64_t)t.k * g.S + (int64_t)t.j * g.P + t.i0;
    return t;
}

template <int VW>
__device__ __forceinline__ void ld(const double* p, double (&v)[VW]) {
    if constexpr (VW == 4) {
        const d2v a = *reinterpret_cast<const d2v*>(p), b = *reinterpret_cast<const d2v*>(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else {
        v[0] = *p;
    }
}
template <int VW>
__device__ __forceinline__ void ld(const float* p, double (&v)[VW]) {
    if constexpr (VW == 4) {
        const f4v a = *reinterpret_cast<const f4v*>(p);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else {
        v[0] = *p;
    }
}
template <int VW>
__device__ __forceinline__ void st(double* p, const double (&v)[VW]) {
    if constexpr (VW == 4) {
        d2v a, b;
        a.x = v[0]; a.y = v[1]; b.x = v[2]; b.y = v[3];
        *reinterpret_cast<d2v*>(p) = a;
        *reinterpret_cast<d2v*>(p + 2) = b;
    } else {
        *p = v[0];
    }
}
template <int VW>
__device__ __forceinline__ void st(float* p, const float (&v)[VW]) {
    if constexpr (VW == 4) {
        f4v a;
        a.x = v[0]; a.y = v[1]; a.z = v[2]; a.w = v[3];
        *reinterpret_cast<f4v*>(p) = a;
    } else {
        *p = v[0];
    }
}

// Which lanes of an item carry an equation of component q.
template <int VW>
__device__ __forceinline__ void lanes(const Geom& g, int q, const Item& t, bool (&m)[VW], bool& any) {
    any = false;
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        const int i = t.i0 + e;
        m[e] = i < g.nx && active(q, i, t.j, t.k);
        any = any || m[e];
    }
}

// Totals s < na: <r_k, A p_s>_W; KRY_MAX + s: <r_y, A p_s>_W.
template <int VW>
__global__ __launch_bounds__(KB) void k_kry_dots(Geom g, KryVecs v, double* __restrict__ part) {
    double acc[2 * KRY_MAX];
#pragma unroll
    for (int s = 0; s < 2 * KRY_MAX; ++s) acc[s] = 0.0;
    const int groups = (g.nx + VW - 1) / VW;
    const int64_t n = (int64_t)g.ny * g.nz * groups;
    for (int64_t it = (int64_t)blockIdx.x * KB + threadIdx.x; it < n; it += (int64_t)gridDim.x * KB) {
        const Item t = item<VW>(g, it, groups);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            bool m[VW], any;
            lanes<VW>(g, q, t, m, any);
            if (!any) continue;
            const double w2 = q < 3 ? v.wv2 : v.wp2;
            double rk[VW], ry[VW];
            ld<VW>(v.rk[q] + t.o, rk);
            ld<VW>(v.ry[q] + t.o, ry);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                rk[e] = m[e] ? w2 * rk[e] : 0.0;
                ry[e] = m[e] ? w2 * ry[e] : 0.0;
            }
#pragma unroll
            for (int s = 0; s < KRY_MAX; ++s)
                if (s < v.na) {
                    double a[VW];
                    ld<VW>(v.ap[s][q] + t.o, a);
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        acc[s] += rk[e] * a[e];
                        acc[KRY_MAX + s] += ry[e] * a[e];
                    }
                }
        }
    }
    block_sums<2 * KRY_MAX>(acc, part);
}

// One step: x' = y + sum gamma_s p_s into the saved copy and the fine
// fields; the new direction p = (y - x) - sum beta_s p_s (FP64) and its
// image A p = (r_k - r_y) - sum beta_s A p_s (FP32) into p_new, ap_new
// (which may be the slot of a stored direction: every stored value of an
// entry is read before it is written); total 0 = <A p, A p>_W of the
// stored image.  Lanes without an equation keep their values (the fine
// fields' walls and padding, zeros elsewhere).
template <int VW>
__global__ __launch_bounds__(KB) void k_kry_update(Geom g, KryVecs v, double* __restrict__ part) {
    double acc[1] = {0.0};
    const int groups = (g.nx + VW - 1) / VW;
    const int64_t n = (int64_t)g.ny * g.nz * groups;
    for (int64_t it = (int64_t)blockIdx.x * KB + threadIdx.x; it < n; it += (int64_t)gridDim.x * KB) {
        const Item t = item<VW>(g, it, groups);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            bool m[VW], any;
            lanes<VW>(g, q, t, m, any);
            if (!any) continue;
            double yv[VW], xv[VW], rk[VW], ry[VW];
            ld<VW>(v.y[q] + t.o, yv);
            ld<VW>(v.x[q] + t.o, xv);
            ld<VW>(v.rk[q] + t.o, rk);
            ld<VW>(v.ry[q] + t.o, ry);
            double xn[VW], z[VW], az[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                xn[e] = yv[e];
                z[e] = yv[e] - xv[e];
                az[e] = rk[e] - ry[e];
            }
#pragma unroll
            for (int s = 0; s < KRY_MAX; ++s)
                if (s < v.na) {
                    double ps[VW], as[VW];
                    ld<VW>(v.p[s][q] + t.o, ps);
                    ld<VW>(v.ap[s][q] + t.o, as);
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        xn[e] += v.gamma[s] * ps[e];
                        z[e] -= v.beta[s] * ps[e];
                        az[e] -= v.beta[s] * as[e];
                    }
                }
            const double w2 = q < 3 ? v.wv2 : v.wp2;
            double xo[VW], yo[VW], po[VW];
            float ao[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const float azf = (float)az[e];
                xo[e] = m[e] ? xn[e] : xv[e];
                yo[e] = m[e] ? xn[e] : yv[e];
                po[e] = m[e] ? z[e] : 0.0;
                ao[e] = m[e] ? azf : 0.0f;
                if (m[e]) acc[0] += w2 * (double)azf * (double)azf;
            }
            st<VW>(v.p_new[q] + t.o, po);
            st<VW>(v.ap_new[q] + t.o, ao);
            st<VW>(v.x[q] + t.o, xo);
            st<VW>(v.y[q] + t.o, yo);
        }
    }
    block_sums<1>(acc, part);
}

// The saved copy <- the fine fields.
template <int VW>
__global__ __launch_bounds__(KB) void k_kry_save(Geom g, KryVecs v) {
    const int groups = (g.nx + VW - 1) / VW;
    const int64_t n = (int64_t)g.ny * g.nz * groups;
    for (int64_t it = (int64_t)blockIdx.x * KB + threadIdx.x; it < n; it += (int64_t)gridDim.x * KB) {
        const Item t = item<VW>(g, it, groups);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            bool m[VW], any;
            lanes<VW>(g, q, t, m, any);
            if (!any) continue;
            double yv[VW], xv[VW];
            ld<VW>(v.y[q] + t.o, yv);
            ld<VW>(v.x[q] + t.o, xv);
#pragma unroll
            for (int e = 0; e < VW; ++e) xv[e] = m[e] ? yv[e] : xv[e];
            st<VW>(v.x[q] + t.o, xv);
        }
    }
}

// out[s] = sum over blocks of part[b * KRY_SLOTS + s] (one block, fixed order).
__global__ __launch_bounds__(KB) void k_kry_reduce(const double* __restrict__ part, int64_t nb,
                                                   double* __restrict__ out) {
    __shared__ double red[KB / 64][KRY_SLOTS];
    double acc[KRY_SLOTS];
#pragma unroll
    for (int s = 0; s < KRY_SLOTS; ++s) acc[s] = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += KB) {
#pragma unroll
        for (int s = 0; s < KRY_SLOTS; ++s) acc[s] += part[b * KRY_SLOTS + s];
    }
#pragma unroll
    for (int s = 0; s < KRY_SLOTS; ++s) {
        double x = acc[s];
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        acc[s] = x;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int s = 0; s < KRY_SLOTS; ++s) red[wave][s] = acc[s];
    }
    __syncthreads();
    if (threadIdx.x < KRY_SLOTS) {
        double x = 0.0;
        for (int w = 0; w < KB / 64; ++w) x += red[w][threadIdx.x];
        out[threadIdx.x] = x;
    }
}

int64_t kry_grid(const Geom& g) {
    const int64_t items = (int64_t)g.ny * g.nz * ((g.nx + KRY_VW - 1) / KRY_VW);
    return std::max<int64_t>(1, std::min<int64_t>((items + KB - 1) / KB, KRY_BLOCKS));
}

}  // namespace

hipError_t launch_kry_dots(const Geom& g, const KryVecs& v, double* part, hipStream_t s) {
    const int64_t nb = kry_grid(g);
    hipLaunchKernelGGL(k_kry_dots<KRY_VW>, dim3((unsigned)nb), dim3(KB), 0, s, g, v, part);
    hipLaunchKernelGGL(k_kry_reduce, dim3(1), dim3(KB), 0, s, part, nb, part + (int64_t)KRY_BLOCKS * KRY_SLOTS);
    return hipGetLastError();
}

hipError_t launch_kry_update(const Geom& g, const KryVecs& v, double* part, hipStream_t s) {
    const int64_t nb = kry_grid(g);
    hipLaunchKernelGGL(k_kry_update<KRY_VW>, dim3((unsigned)nb), dim3(KB), 0, s, g, v, part);
    hipLaunchKernelGGL(k_kry_reduce, dim3(1), dim3(KB), 0, s, part, nb, part + (int64_t)KRY_BLOCKS * KRY_SLOTS);
    return hipGetLastError();
}

hipError_t launch_kry_save(const Geom& g, const KryVecs& v, hipStream_t s) {
    hipLaunchKernelGGL(k_kry_save<KRY_VW>, dim3((unsigned)kry_grid(g)), dim3(KB), 0, s, g, v);
    return hipGetLastError();
}

}  // namespace ptk
