// The paper's mixed-precision gradient for SIE lenses on gfx950 (Sec. 3.2,
// Sec. 3.3, Appendix A.3): grad Psi in single precision at every pixel, in
// double precision inside blocks of pixels centred on the halos (pc x pc for
// the cluster-scale halos, pg x pg for the galaxy-scale ones), then in double
// precision again wherever the source-plane criteria of Sec. 3.3, evaluated on
// that field, ask for it.
//
// Launch sequence (one call, the caller's stream):
//   k_mix_prep     constants of every potential (one workgroup), SIE check,
//                  counters reset
//   k_mix_field32  FP32 field at every node (SIE form alpha = K m / R with
//                  R = sqrt(d . M d): one reciprocal square root per
//                  potential), written as double; mask cleared
//   k_mix_patches  one workgroup per halo marks its block in the mask
//   k_mix_scan<0>  appends the block pixels to the DP list
//   k_mix_dp       FP64 gradient of the listed pixels
//   k_mix_scan<1>  criteria on the field so far; appends flagged pixels
//   k_mix_dp       FP64 gradient of those pixels
//   k_mix_stats    counts and status to the caller's stats
#include "lens_path.hpp"

namespace lens {

// ---------------------------------------------------------------- constants

__global__ __launch_bounds__(256) void k_mix_prep(PotPtrs pot, GridDesc g, double* __restrict__ tab64,
                                                  float* __restrict__ tab32, double* __restrict__ bterm,
                                                  MixState* __restrict__ st)
{
    __shared__ int s_bad;
    if (threadIdx.x == 0) {
        s_bad = 0;
        st->n_list = 0;
        st->n_patch = 0;
    }
    __syncthreads();
    bool bad = false;
    for (int p = threadIdx.x; p < pot.n; p += 256) {
        double row[T64_STRIDE], terms[3];
        prep_one(pot, g, p, p, tab64, tab32, bterm, row, terms);
        // the criteria and blocks are derived for the SIE (Sec. 3.2): no core, no cut
        bad |= terms[2] != 0.0 || pot.r_core[p] != 0.0 || !isinf(pot.r_cut[p]) || pot.r_cut[p] < 0.0;
    }
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) st->status = s_bad ? kStatusInvalid : kStatusOk;
}

// ---------------------------------------------------------------- FP32 field

// FP32 SIE contribution of table row c for NPL nodes of a row: node-unit
// offsets from the exact centre split (as in the general FP32 field), m = M d,
// R^2 = d . m clamped below at 1e-30 (the centre, where m = 0, contributes 0),
// alpha += (K/h) m / R.
template <int NPL>
__device__ __forceinline__ void sie32_pot(const float* __restrict__ c, float4 rc, const float* fi, float* sx,
                                          float* sy)
{
    const float cxh = c[T32_CXH], cxl = c[T32_CXL];
    const float A = c[T32_A], B = c[T32_B], K = c[T32_K];
    const float nyv = rc.x, bny = rc.y, cny = rc.z;  // the row part (pots_wg)
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        const float nxv = (fi[k] - cxh) - cxl;
        const float m1 = fmaf(A, nxv, bny);
        const float m2 = fmaf(B, nxv, cny);
        const float R2 = fmaxf(fmaf(nxv, m1, nyv * m2), 1e-30f);
        const float kr = K * __builtin_amdgcn_rsqf(R2);
        sx[k] = fmaf(kr, m1, sx[k]);
        sy[k] = fmaf(kr, m2, sy[k]);
    }
}

// Workgroup = 256 * NPL consecutive nodes of row blockIdx.y; each thread NPL
// consecutive nodes.  Writes the FP32 field as double and clears the mask.
template <int NPL>
__global__ __launch_bounds__(256) void k_mix_field32(const float* __restrict__ tab32, int np, int nx,
                                                     double* __restrict__ ax, double* __restrict__ ay,
                                                     unsigned char* __restrict__ mask,
                                                     const MixState* __restrict__ st)
{
    const int j = blockIdx.y;
    const int i0 = (blockIdx.x * 256 + threadIdx.x) * NPL;
    if ((int)(blockIdx.x * 256 * NPL) >= nx) return;
    const float fj = (float)j;
    float fi[NPL], sx[NPL], sy[NPL];
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        fi[k] = (float)(i0 + k);
        sx[k] = 0.0f;
        sy[k] = 0.0f;
    }
    const bool bad = st->status != kStatusOk;
    if (!bad)  // uniform over the launch
        pots_wg<T32_STRIDE, T32_CYH, T32_CYL, T32_B, T32_C>(
            tab32, np, fj, [&](const float* c, float4 rc) { sie32_pot<NPL>(c, rc, fi, sx, sy); });
    const size_t row = (size_t)j * nx;
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        if (i0 + k < nx) {
            ax[row + i0 + k] = bad ? __builtin_nan("") : (double)sx[k];
            ay[row + i0 + k] = bad ? __builtin_nan("") : (double)sy[k];
            mask[row + i0 + k] = 0;
        }
    }
}

// ---------------------------------------------------------------- DP blocks and criteria

// Workgroup p marks the block of halo p: p x p pixels (pc for the first
// n_cluster halos, pg for the others) spanning node indices [k - size/2,
// k - size/2 + size) on each axis, k = (x_c - x0)/h rounded half away from
// zero, clipped to the grid.
__global__ __launch_bounds__(256) void k_mix_patches(PotPtrs pot, GridDesc g, int n_cluster, int pc, int pg,
                                                     unsigned char* __restrict__ mask,
                                                     const MixState* __restrict__ st)
{
    if (st->status != kStatusOk) return;
    const int p = blockIdx.x;
    const long long size = p < n_cluster ? pc : pg;
    const long long ki = llround((pot.x[p] - g.x0) / g.h), kj = llround((pot.y[p] - g.y0) / g.h);
    long long i0 = ki - size / 2, i1 = ki - size / 2 + size, j0 = kj - size / 2, j1 = kj - size / 2 + size;
    i0 = i0 < 0 ? 0 : i0;
    j0 = j0 < 0 ? 0 : j0;
    i1 = i1 > g.nx ? g.nx : i1;
    j1 = j1 > g.ny ? g.ny : j1;
    if (i0 >= i1 || j0 >= j1) return;
    const long long w = i1 - i0, n = w * (j1 - j0);
    for (long long q = threadIdx.x; q < n; q += 256) {
        const long long j = j0 + q / w, i = i0 + q % w;
        mask[j * g.nx + i] = 1;
    }
}

constexpr int kScanPer = 16;               // pixels per thread of the scan
constexpr int kScanChunk = 256 * kScanPer;  // pixels per workgroup

// Appends the pixels of chunk blockIdx.x (4096 consecutive pixels) that need
// double precision to list[]: MODE 0, the block pixels (mask 1); MODE 1, the
// pixels outside the blocks where the criteria of Sec. 3.3 hold on the field
// so far (marked 2):
//     d1 = ax(i,j) - ax(i-1,j), d2 = ay(i,j) - ay(i,j-1),
//     d3 = ax(i,j) - ax(i,j-1), d4 = ay(i,j) - ay(i-1,j),
//     |dx - d1| < t12, |dx - d2| < t12, |d3| > t34 or |d4| > t34,
// a difference whose neighbour is outside the image not being evaluated.  The
// workgroup compacts its pixels through a prefix sum in LDS: one list-counter
// atomic per chunk.
template <int MODE>
__global__ __launch_bounds__(256) void k_mix_scan(const double* __restrict__ ax, const double* __restrict__ ay,
                                                  int nx, long long n_nodes, double dx, double t12, double t34,
                                                  unsigned char* __restrict__ mask, unsigned* __restrict__ list,
                                                  MixState* __restrict__ st)
{
    __shared__ unsigned s_wave[4];
    __shared__ unsigned s_base;
    if (st->status != kStatusOk) return;
    const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
    const long long c0 = (long long)blockIdx.x * kScanChunk;
    unsigned bits = 0, cnt = 0;
#pragma unroll 4
    for (int k = 0; k < kScanPer; k++) {
        const long long n = c0 + k * 256 + t;
        if (n >= n_nodes) break;
        bool need = false;
        const unsigned char m = mask[n];
        if (MODE == 0) {
            need = m == 1;
        } else if (m == 0) {
            const long long j = n / nx, i = n - j * nx;
            const double x = ax[n], y = ay[n];
            if (i > 0) {
                const double d1 = x - ax[n - 1], d4 = y - ay[n - 1];
                need = fabs(dx - d1) < t12 || fabs(d4) > t34;
            }
            if (j > 0) {
                const double d2 = y - ay[n - nx], d3 = x - ax[n - nx];
                need = need || fabs(dx - d2) < t12 || fabs(d3) > t34;
            }
            if (need) mask[n] = 2;
        }
        bits |= (need ? 1u : 0u) << k;
        cnt += need ? 1u : 0u;
    }
    // exclusive prefix of the per-thread counts over the workgroup
    unsigned inc = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned v = __shfl_up(inc, d, 64);
        if (lane >= d) inc += v;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    if (t == 0) {
        const unsigned total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
        s_base = total ? atomicAdd(&st->n_list, total) : 0u;
    }
    __syncthreads();
    unsigned pos = s_base + inc - cnt;
    for (int w = 0; w < wave; w++) pos += s_wave[w];
    for (int k = 0; k < kScanPer; k++)
        if (bits & (1u << k)) list[pos++] = (unsigned)(c0 + k * 256 + t);
}

// 1/sqrt(x) in FP64 for a positive normal x: the hardware estimate (relative
// error below 2^-24 on gfx950, measured) refined by one Newton-Raphson step
// y <- y (3/2 - x y^2 / 2), which squares the error: ~2^-47 relative.
__device__ __forceinline__ double rsq64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return fma(y, fma(-0.5 * x * y, y, 0.5), y);
}

// FP64 SIE contribution of table row t at (t1, t2): alpha += K m / R, m = M d,
// R^2 = d . m, clamped below at 1e-300 (the centre, where m = 0, contributes 0).
__device__ __forceinline__ void sie64_add(const double* __restrict__ t, double t1, double t2, double& s1,
                                          double& s2)
{
    const double d1 = t1 - t[T64_XC], d2 = t2 - t[T64_YC];
    const double m1 = fma(t[T64_A], d1, t[T64_B] * d2);
    const double m2 = fma(t[T64_B], d1, t[T64_C] * d2);
    const double R2 = fmax(fma(d1, m1, d2 * m2), 1e-300);
    const double kr = t[T64_K] * rsq64(R2);
    s1 = fma(kr, m1, s1);
    s2 = fma(kr, m2, s2);
}

// FP64 gradient of list entries [lo, hi), lo = the block count (MODE 1) or 0
// (MODE 0), hi = the list length.
template <int MODE>
__global__ __launch_bounds__(256) void k_mix_dp(const double* __restrict__ tab64, int np, GridDesc g,
                                                const unsigned* __restrict__ list, double* __restrict__ ax,
                                                double* __restrict__ ay, MixState* __restrict__ st)
{
    if (st->status != kStatusOk) return;
    const unsigned hi = st->n_list;
    const unsigned lo = MODE == 0 ? 0u : st->n_patch;
    for (unsigned e = lo + blockIdx.x * 256 + threadIdx.x; e < hi; e += gridDim.x * 256) {
        const unsigned n = list[e];
        const int j = (int)(n / (unsigned)g.nx), i = (int)(n - (unsigned)j * (unsigned)g.nx);
        const double t1 = node_coord(g.x0, i, g.h), t2 = node_coord(g.y0, j, g.h);
        double s1 = 0.0, s2 = 0.0;
#pragma unroll 4
        for (int p = 0; p < np; p++) sie64_add(tab64 + (size_t)p * T64_STRIDE, t1, t2, s1, s2);
        ax[n] = s1;
        ay[n] = s2;
    }
}

// The block count is the list length after k_mix_scan<0> (read before the
// criteria scan appends).
__global__ void k_mix_mark(MixState* __restrict__ st)
{
    if (threadIdx.x == 0) st->n_patch = st->n_list;
}

__global__ void k_mix_stats(const MixState* __restrict__ st, long long* __restrict__ stats)
{
    if (threadIdx.x == 0) {
        const bool ok = st->status == kStatusOk;
        stats[0] = ok ? (long long)st->n_patch : 0;
        stats[1] = ok ? (long long)(st->n_list - st->n_patch) : 0;
        stats[2] = ok ? (long long)st->n_list : 0;
        stats[3] = st->status;
    }
}

// ---------------------------------------------------------------- launcher

hipError_t launch_mixed(const PotPtrs& pot, const GridDesc& g, const MixedLaunch& ml, hipStream_t s)
{
    const long long n_nodes = (long long)g.nx * g.ny;
    k_mix_prep<<<1, 256, 0, s>>>(pot, g, ml.tab64, ml.tab32, ml.bterm, ml.st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int npl = ml.npl;
    const dim3 fgrid((unsigned)((g.nx + 256 * npl - 1) / (256 * npl)), (unsigned)g.ny);
    switch (npl) {
    case 1: e = launch_ev(ml.ev, k_mix_field32<1>, fgrid, dim3(256), s, (const float*)ml.tab32, pot.n, g.nx, ml.ax,
                      ml.ay, ml.mask, (const MixState*)ml.st); break;
    case 2: e = launch_ev(ml.ev, k_mix_field32<2>, fgrid, dim3(256), s, (const float*)ml.tab32, pot.n, g.nx, ml.ax,
                      ml.ay, ml.mask, (const MixState*)ml.st); break;
    default: e = launch_ev(ml.ev, k_mix_field32<4>, fgrid, dim3(256), s, (const float*)ml.tab32, pot.n, g.nx, ml.ax,
                       ml.ay, ml.mask, (const MixState*)ml.st); break;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pot.n > 0) {
        k_mix_patches<<<(unsigned)pot.n, 256, 0, s>>>(pot, g, ml.n_cluster, ml.pc, ml.pg, ml.mask, ml.st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const long long sb = (n_nodes + kScanChunk - 1) / kScanChunk;
    const unsigned scan_blocks = (unsigned)(sb < 1 ? 1 : sb);
    k_mix_scan<0><<<scan_blocks, 256, 0, s>>>(ml.ax, ml.ay, g.nx, n_nodes, g.h, ml.t12, ml.t34, ml.mask, ml.list,
                                              ml.st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mix_mark<<<1, 64, 0, s>>>(ml.st);
    k_mix_dp<0><<<2048, 256, 0, s>>>(ml.tab64, pot.n, g, ml.list, ml.ax, ml.ay, ml.st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mix_scan<1><<<scan_blocks, 256, 0, s>>>(ml.ax, ml.ay, g.nx, n_nodes, g.h, ml.t12, ml.t34, ml.mask, ml.list,
                                              ml.st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mix_dp<1><<<2048, 256, 0, s>>>(ml.tab64, pot.n, g, ml.list, ml.ax, ml.ay, ml.st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_mix_stats<<<1, 64, 0, s>>>(ml.st, ml.stats);
    return hipGetLastError();
}

}  // namespace lens
