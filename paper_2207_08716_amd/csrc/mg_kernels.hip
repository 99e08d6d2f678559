// Grid transfers of the geometric multigrid solver for the linear Picard
// stage (the thesis's outlook: geometric multigrid with weighted-Jacobi
// smoothing, which the PT iteration becomes without damping).
//
// A coarse grid has ceil(n/2) cells per axis on the same domain, so grids
// with odd counts (511 -> 256 -> 128 ...) are not nested.  Transfers are
// tensor products of one-dimensional linear interpolation between the two
// grids' point positions, per staggering: cell centres (i + 1/2) h, taken
// constant beyond the outermost coarse centres, and faces i h, which both
// grids have at the walls.  Prolongation P interpolates a coarse correction
// to the fine points; restriction is P's transpose with every row
// normalised to weight sum 1 (an average of the fine values around a coarse
// point).  Normal faces on the walls carry no equation: the restriction
// skips them and gives zero there, the prolongation leaves them alone.
#include "pt_internal.h"

namespace ptk {
namespace {

constexpr int TB = 256;

// Fine index i of an axis with nf fine and nc coarse cells, in coarse
// units: the coarse index j0 and the weight t of j0 + 1 (1 - t of j0).
__device__ __forceinline__ void pw(int i, int nf, int nc, bool face, int& j0, double& t) {
    if (face) {
        const double u = (double)i * nc / nf;
        j0 = min((int)floor(u), nc - 1);
        t = u - j0;
    } else {
        const double u = ((double)i + 0.5) * nc / nf - 0.5;
        if (u <= 0.0) {
            j0 = 0;
            t = 0.0;
        } else if (u >= (double)(nc - 1)) {
            j0 = nc - 1;
            t = 0.0;
        } else {
            j0 = (int)floor(u);
            t = u - j0;
        }
    }
}

// P's entry (fine i, coarse J) of one axis.
__device__ __forceinline__ double pweight(int i, int J, int nf, int nc, bool face) {
    int j0;
    double t;
    pw(i, nf, nc, face, j0, t);
    return J == j0 ? 1.0 - t : (J == j0 + 1 ? t : 0.0);
}

// Fine indices whose interpolation can involve coarse index J.
__device__ __forceinline__ void prange(int J, int nf, int nc, bool face, int& lo, int& hi) {
    const double r = (double)nf / nc;
    if (face) {
        lo = max(0, (int)floor((J - 1) * r));
        hi = min(nf, (int)ceil((J + 1) * r));
    } else {
        lo = max(0, (int)floor((J - 0.5) * r - 0.5));
        hi = min(nf - 1, (int)ceil((J + 1.5) * r - 0.5));
    }
}

// The x taps of a restriction, in registers: fine indices lo .. lo + 7 and
// P's entries for coarse index I (a coarse grid has ceil(n/2) cells, so the
// ratio is at most 2 and the candidate range spans at most 7 fine points).
constexpr int MAXT = 8;
static_assert(MG_TAB == 2 + MAXT, "a restriction row holds its first index, its count and MAXT weights");
struct Taps {
    int lo, n;
    double w[MAXT];
    double sum;
};
__device__ __forceinline__ void taps(int J, int nf, int nc, bool face, bool skip_walls, Taps& t) {
    int lo, hi;
    prange(J, nf, nc, face, lo, hi);
    if (skip_walls) {
        lo = max(lo, 1);
        hi = min(hi, nf - 1);
    }
    t.lo = lo;
    t.n = min(hi - lo + 1, MAXT);
    t.sum = 0.0;
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const double w = (q < t.n) ? pweight(lo + q, J, nf, nc, face) : 0.0;
        t.w[q] = w;
        t.sum += w;
    }
}

struct Ext {
    int nx, ny, nz;     // cells of the grid
    int64_t P, S;       // row and plane pitch
};
__host__ __device__ inline Ext ext(const Geom& g) { return Ext{g.nx, g.ny, g.nz, g.P, g.S}; }

// One axis of the separable restriction.  The restriction is a tensor
// product of one-dimensional rows, each normalised to weight sum 1, so it
// runs as three passes (x, then y, then z), each reading its input once in
// rows instead of gathering every coarse point's 3D neighbourhood.  dst
// holds the points (i, j, k) < (ex, ey, ez) whose coordinate along `axis`
// is coarse and whose other coordinates are src's; strides sP, sS (src) and
// dP, dS (dst).  tab: the axis's normalised rows (MG_TAB doubles per coarse
// index: first fine index, count, weights), built once per hierarchy.
// Launched on a 3D grid of GX x GY blocks (x: i, y: j, z: k), so that no
// thread divides its index.
constexpr int GX = 64, GY = 4;

// mean: 0 arithmetic; 1 harmonic, 2 geometric (the x pass averages 1/v or
// ln v, the z pass maps the average back), so that the passes stay linear.
template <typename TI>
__global__ __launch_bounds__(GX * GY) void k_mg_r1(const TI* __restrict__ src, int64_t sP, int64_t sS,
                                                  double* __restrict__ dst, int64_t dP, int64_t dS, int ex, int ey,
                                                  int axis, const double* __restrict__ tab, int mean) {
    const int i = blockIdx.x * GX + threadIdx.x, j = blockIdx.y * GY + threadIdx.y, k = blockIdx.z;
    if (i < ex && j < ey) {
        const int64_t step = axis == 0 ? 1 : (axis == 1 ? sP : sS);
        const int J = axis == 0 ? i : (axis == 1 ? j : k);
        const double* row = tab + (int64_t)J * MG_TAB;
        const int lo = (int)row[0], cnt = (int)row[1];
        const int64_t base = (axis == 0 ? (int64_t)k * sS + (int64_t)j * sP
                                        : (axis == 1 ? (int64_t)k * sS + i : (int64_t)j * sP + i)) +
                             (int64_t)lo * step;
        double r = 0.0;
#pragma unroll
        for (int q = 0; q < MAXT; ++q)
            if (q < cnt) {
                double v = (double)src[base + q * step];
                if (axis == 0 && mean) v = mean == 1 ? 1.0 / v : log(v);
                r += row[2 + q] * v;
            }
        if (axis == 2 && mean && cnt > 0) r = mean == 1 ? 1.0 / r : exp(r);
        dst[(int64_t)k * dS + (int64_t)j * dP + i] = r;
    }
}

dim3 grid3(int ex, int ey, int ez) { return dim3((unsigned)((ex + GX - 1) / GX), (unsigned)((ey + GY - 1) / GY), (unsigned)ez); }

// The normalised restriction rows of one axis (fine nf, coarse nc points;
// face: the field sits on faces normal to it, whose wall faces carry no
// equation: skipped as inputs, rows of weight 0 for the coarse walls).
__global__ __launch_bounds__(TB) void k_mg_taps(double* __restrict__ tab, int nf, int nc, bool face) {
    const int J = blockIdx.x * TB + threadIdx.x;
    if (J > nc - 1 + face) return;
    double* row = tab + (int64_t)J * MG_TAB;
    Taps tt;
    taps(J, nf, nc, face, face, tt);
    const bool none = (face && (J == 0 || J == nc)) || !(tt.sum > 0.0);
    row[0] = tt.lo;
    row[1] = none ? 0 : tt.n;
#pragma unroll
    for (int q = 0; q < MAXT; ++q) row[2 + q] = none ? 0.0 : tt.w[q] / tt.sum;
}

// Restricted pressure residuals (a, b) folded into old-pressure fields in
// place: pto = m00 a + m01 b, pfo = m10 a + m11 b, the values whose terms
// in r_Pt and r_Pf at the zero state are a and b.
__global__ __launch_bounds__(TB) void k_mg_fold(Ext c, double* __restrict__ pto, double* __restrict__ pfo,
                                                double m00, double m01, double m10, double m11) {
    const int64_t n = (int64_t)c.nx * c.ny * c.nz;
    for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TB) {
        const int I = (int)(t % c.nx), J = (int)((t / c.nx) % c.ny), K = (int)(t / ((int64_t)c.nx * c.ny));
        const int64_t o = (int64_t)K * c.S + (int64_t)J * c.P + I;
        const double a = pto[o], b = pfo[o];
        pto[o] = m00 * a + m01 * b;
        pfo[o] = m10 * a + m11 * b;
    }
}

// fine += P coarse for one field of staggering (fx, fy, fz); the walls'
// normal faces keep their values.
__global__ __launch_bounds__(GX * GY) void k_mg_prolong_add(Ext f, Ext c, bool fx, bool fy, bool fz,
                                                            const double* __restrict__ src,
                                                            double* __restrict__ dst) {
    const int ex = f.nx + fx, ey = f.ny + fy;
    const int i = blockIdx.x * GX + threadIdx.x, j = blockIdx.y * GY + threadIdx.y, k = blockIdx.z;
    if (i < ex && j < ey) {
        if ((fx && (i == 0 || i == f.nx)) || (fy && (j == 0 || j == f.ny)) || (fz && (k == 0 || k == f.nz))) return;
        int x0, y0, z0;
        double tx, ty, tz;
        pw(i, f.nx, c.nx, fx, x0, tx);
        pw(j, f.ny, c.ny, fy, y0, ty);
        pw(k, f.nz, c.nz, fz, z0, tz);
        // the second point of an axis: inside the coarse extent (its weight
        // is zero where the first point is the last one)
        const int x1 = min(x0 + 1, c.nx - 1 + fx), y1 = min(y0 + 1, c.ny - 1 + fy), z1 = min(z0 + 1, c.nz - 1 + fz);
        auto at = [&](int a, int b, int d) { return src[(int64_t)d * c.S + (int64_t)b * c.P + a]; };
        const double v0 = (1.0 - tx) * at(x0, y0, z0) + tx * at(x1, y0, z0);
        const double v1 = (1.0 - tx) * at(x0, y1, z0) + tx * at(x1, y1, z0);
        const double v2 = (1.0 - tx) * at(x0, y0, z1) + tx * at(x1, y0, z1);
        const double v3 = (1.0 - tx) * at(x0, y1, z1) + tx * at(x1, y1, z1);
        const double v = (1.0 - tz) * ((1.0 - ty) * v0 + ty * v1) + tz * ((1.0 - ty) * v2 + ty * v3);
        dst[(int64_t)k * f.S + (int64_t)j * f.P + i] += v;
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)std::min<int64_t>((n + TB - 1) / TB, 65536); }

}  // namespace

namespace {

// The three passes of a separable restriction of an FP32 fine field
// (scratch sa: (nz_f + 1) (ny_f + 1) P_c doubles, sb: (nz_f + 1) (ny_c + 1) P_c;
// tab: the rows of the x, y, z axes for this field's staggering).
template <typename TI>
hipError_t restrict_sep(const Geom& gf, const Geom& gc, int kind, const TI* src, double* dst, double* sa,
                        double* sb, const double* const tab[3], int mean, hipStream_t s) {
    const bool fx = kind == 1, fy = kind == 2, fz = kind == 3;
    const int64_t aS = gc.P * (int64_t)(gf.ny + 1), bS = gc.P * (int64_t)(gc.ny + 1);
    const dim3 blk(GX, GY);
    hipLaunchKernelGGL(k_mg_r1<TI>, grid3(gc.nx + fx, gf.ny + fy, gf.nz + fz), blk, 0, s, src, gf.P, gf.S, sa,
                       gc.P, aS, gc.nx + fx, gf.ny + fy, 0, tab[0], mean);
    hipLaunchKernelGGL(k_mg_r1<double>, grid3(gc.nx + fx, gc.ny + fy, gf.nz + fz), blk, 0, s, (const double*)sa,
                       gc.P, aS, sb, gc.P, bS, gc.nx + fx, gc.ny + fy, 1, tab[1], mean);
    hipLaunchKernelGGL(k_mg_r1<double>, grid3(gc.nx + fx, gc.ny + fy, gc.nz + fz), blk, 0, s, (const double*)sb,
                       gc.P, bS, dst, gc.P, gc.S, gc.nx + fx, gc.ny + fy, 2, tab[2], mean);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mg_taps(double* tab, int nf, int nc, int face, hipStream_t s) {
    hipLaunchKernelGGL(k_mg_taps, dim3((unsigned)((nc + 1 + TB - 1) / TB)), dim3(TB), 0, s, tab, nf, nc, face != 0);
    return hipGetLastError();
}

hipError_t launch_mg_restrict(const Geom& gf, const Geom& gc, const double* src, double* dst, int mean, double* sa,
                              double* sb, const double* const tab[3], hipStream_t s) {
    return restrict_sep(gf, gc, 0, src, dst, sa, sb, tab, mean, s);
}

hipError_t launch_mg_restrict32(const Geom& gf, const Geom& gc, int kind, const float* src, double* dst,
                                double* sa, double* sb, const double* const tab[3], hipStream_t s) {
    return restrict_sep(gf, gc, kind, src, dst, sa, sb, tab, 0, s);
}

hipError_t launch_mg_restrict_fold(const Geom& gf, const Geom& gc, const float* rpt, const float* rpf, double* pto,
                                   double* pfo, const double m[4], double* sa, double* sb, const double* const tab[3],
                                   hipStream_t s) {
    hipError_t e = restrict_sep(gf, gc, 0, rpt, pto, sa, sb, tab, 0, s);
    if (e == hipSuccess) e = restrict_sep(gf, gc, 0, rpf, pfo, sa, sb, tab, 0, s);
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)gc.nx * gc.ny * gc.nz;
    hipLaunchKernelGGL(k_mg_fold, dim3(blocks_for(n)), dim3(TB), 0, s, ext(gc), pto, pfo, m[0], m[1], m[2], m[3]);
    return hipGetLastError();
}

hipError_t launch_mg_prolong_add(const Geom& gf, const Geom& gc, int kind, const double* src, double* dst,
                                 hipStream_t s) {
    const bool fx = kind == 1, fy = kind == 2, fz = kind == 3;
    hipLaunchKernelGGL(k_mg_prolong_add, grid3(gf.nx + fx, gf.ny + fy, gf.nz + fz), dim3(GX, GY), 0, s, ext(gf),
                       ext(gc), fx, fy, fz, src, dst);
    return hipGetLastError();
}

}  // namespace ptk
