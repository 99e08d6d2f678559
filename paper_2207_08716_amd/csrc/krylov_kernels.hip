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

// Totals s < na: <r_k, A p_s>_W; KRY_MAX + s: <r_y, A p_s>_W.
__global__ __launch_bounds__(KB) void k_kry_dots(Geom g, KryVecs v, double* __restrict__ part) {
    double acc[2 * KRY_MAX];
#pragma unroll
    for (int s = 0; s < 2 * KRY_MAX; ++s) acc[s] = 0.0;
    const int64_t nrows = (int64_t)g.ny * g.nz;
    for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int j = (int)(r % g.ny), k = (int)(r / g.ny);
        const int64_t row = (int64_t)k * g.S + (int64_t)j * g.P;
        for (int i = threadIdx.x; i < g.nx; i += KB) {
            const int64_t o = row + i;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                if (!active(q, i, j, k)) continue;
                const double w2 = q < 3 ? v.wv2 : v.wp2;
                const double rk = w2 * (double)v.rk[q][o], ry = w2 * (double)v.ry[q][o];
#pragma unroll
                for (int s = 0; s < KRY_MAX; ++s)
                    if (s < v.na) {
                        const double a = (double)v.ap[s][q][o];
                        acc[s] += rk * a;
                        acc[KRY_MAX + s] += ry * a;
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
// stored image.
__global__ __launch_bounds__(KB) void k_kry_update(Geom g, KryVecs v, double* __restrict__ part) {
    double acc[1] = {0.0};
    const int64_t nrows = (int64_t)g.ny * g.nz;
    for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int j = (int)(r % g.ny), k = (int)(r / g.ny);
        const int64_t row = (int64_t)k * g.S + (int64_t)j * g.P;
        for (int i = threadIdx.x; i < g.nx; i += KB) {
            const int64_t o = row + i;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                if (!active(q, i, j, k)) continue;
                const double yv = v.y[q][o];
                double xn = yv;
                double z = yv - v.x[q][o];
                double az = (double)v.rk[q][o] - (double)v.ry[q][o];
#pragma unroll
                for (int s = 0; s < KRY_MAX; ++s)
                    if (s < v.na) {
                        const double ps = v.p[s][q][o];
                        xn += v.gamma[s] * ps;
                        z -= v.beta[s] * ps;
                        az -= v.beta[s] * (double)v.ap[s][q][o];
                    }
                const float azf = (float)az;
                v.p_new[q][o] = z;
                v.ap_new[q][o] = azf;
                v.x[q][o] = xn;
                v.y[q][o] = xn;
                acc[0] += (q < 3 ? v.wv2 : v.wp2) * (double)azf * (double)azf;
            }
        }
    }
    block_sums<1>(acc, part);
}

// The saved copy <- the fine fields.
__global__ __launch_bounds__(KB) void k_kry_save(Geom g, KryVecs v) {
    const int64_t nrows = (int64_t)g.ny * g.nz;
    for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int j = (int)(r % g.ny), k = (int)(r / g.ny);
        const int64_t row = (int64_t)k * g.S + (int64_t)j * g.P;
        for (int i = threadIdx.x; i < g.nx; i += KB) {
            const int64_t o = row + i;
#pragma unroll
            for (int q = 0; q < 5; ++q)
                if (active(q, i, j, k)) v.x[q][o] = v.y[q][o];
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

int64_t kry_grid(const Geom& g) { return std::min<int64_t>((int64_t)g.ny * g.nz, KRY_BLOCKS); }

}  // namespace

hipError_t launch_kry_dots(const Geom& g, const KryVecs& v, double* part, hipStream_t s) {
    const int64_t nb = kry_grid(g);
    hipLaunchKernelGGL(k_kry_dots, dim3((unsigned)nb), dim3(KB), 0, s, g, v, part);
    hipLaunchKernelGGL(k_kry_reduce, dim3(1), dim3(KB), 0, s, part, nb, part + (int64_t)KRY_BLOCKS * KRY_SLOTS);
    return hipGetLastError();
}

hipError_t launch_kry_update(const Geom& g, const KryVecs& v, double* part, hipStream_t s) {
    const int64_t nb = kry_grid(g);
    hipLaunchKernelGGL(k_kry_update, dim3((unsigned)nb), dim3(KB), 0, s, g, v, part);
    hipLaunchKernelGGL(k_kry_reduce, dim3(1), dim3(KB), 0, s, part, nb, part + (int64_t)KRY_BLOCKS * KRY_SLOTS);
    return hipGetLastError();
}

hipError_t launch_kry_save(const Geom& g, const KryVecs& v, hipStream_t s) {
    hipLaunchKernelGGL(k_kry_save, dim3((unsigned)kry_grid(g)), dim3(KB), 0, s, g, v);
    return hipGetLastError();
}

}  // namespace ptk
