// Pseudo-elliptical NFW deflection on gfx950: the second profile family the
// paper names for its method (Sec. 5), in the frame construction of
// Algorithm 1 (Sec. 2.2.2).  With m = M d (M = Rot(Phi) diag(1-eps, 1+eps)
// Rot(-Phi), d = theta - centre), R^2 = d . m and x = R / r_s,
//     alpha = 4 kappa_s (g(x) / x^2) m,   g(x) = ln(x/2) + F(x),
//     F(x) = atanh(s)/s, s = sqrt(1 - x^2) (x < 1);  atan(r)/r, r = sqrt(x^2 - 1) (x > 1)
// (the textbook arccosh / arccos forms of F written through s and r).  Below
// x = 1/2 the two logarithms of g cancel; there g/x^2 is evaluated as
//     [ln(2/x)/(1 + s) + log1p(-x^2 / (2 (1 + s))) / x^2] / s,
// the same quantity with the cancellation done exactly.  The centre (R = 0)
// contributes 0.  FP32: node offsets from the exact split of the centre, as in
// the isothermal FP32 field; FP64: theta - centre in FP64.
#include "lens_path.hpp"

namespace lens {

enum : int { N64_XC = 0, N64_YC, N64_A, N64_B, N64_C, N64_IRS2, N64_K4, N64_STRIDE = 8 };
enum : int {
    N32_CXH = 0, N32_CXL, N32_CYH, N32_CYL, N32_A, N32_B, N32_C, N32_IRS2, N32_K, N32_STRIDE = 12
};

// Constants of every halo (one thread each) and the status: invalid for a
// non-finite or out-of-domain parameter (0 <= eps < 1, r_s > 0, kappa_s >= 0)
// or a centre beyond 2^22 nodes of the grid origin.
__global__ __launch_bounds__(256) void k_nfw_prep(NfwPtrs h, GridDesc g, double* __restrict__ t64,
                                                  float* __restrict__ t32, int* __restrict__ st,
                                                  int* __restrict__ status)
{
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    bool bad = false;
    for (int p = threadIdx.x; p < h.n; p += 256) {
        const double xc = h.x[p], yc = h.y[p], eps = h.eps[p], phi = h.phi[p], rs = h.r_s[p], ks = h.kappa_s[p];
        const bool ok = isfinite(xc) && isfinite(yc) && isfinite(phi) && eps >= 0.0 && eps < 1.0 && rs > 0.0 &&
                        isfinite(rs) && ks >= 0.0 && isfinite(ks);
        double s2, c2;
        sincos(2.0 * phi, &s2, &c2);
        const double A = 1.0 - eps * c2, B = -eps * s2, C = 1.0 + eps * c2;
        double* u = t64 + (size_t)p * N64_STRIDE;
        u[N64_XC] = xc;
        u[N64_YC] = yc;
        u[N64_A] = A;
        u[N64_B] = B;
        u[N64_C] = C;
        u[N64_IRS2] = 1.0 / (rs * rs);
        u[N64_K4] = 4.0 * ks;
        u[N64_STRIDE - 1] = 0.0;
        const double cxn = (xc - g.x0) / g.h, cyn = (yc - g.y0) / g.h;
        const bool near = fabs(cxn) < 4194304.0 && fabs(cyn) < 4194304.0;
        const double cxh = near ? rint(cxn) : 0.0, cyh = near ? rint(cyn) : 0.0;
        const double h2 = g.h * g.h;
        float* v = t32 + (size_t)p * N32_STRIDE;
        v[N32_CXH] = (float)cxh;
        v[N32_CXL] = (float)(cxn - cxh);
        v[N32_CYH] = (float)cyh;
        v[N32_CYL] = (float)(cyn - cyh);
        v[N32_A] = (float)(A * h2);
        v[N32_B] = (float)(B * h2);
        v[N32_C] = (float)(C * h2);
        v[N32_IRS2] = (float)(1.0 / (rs * rs));
        v[N32_K] = (float)(4.0 * ks / g.h);
        for (int k = N32_K + 1; k < N32_STRIDE; k++) v[k] = 0.0f;
        bad |= !(ok && near);
    }
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        *st = s_bad ? kStatusInvalid : kStatusOk;
        if (status) *status = *st;
    }
}

// g(x) / x^2 for x^2 > 0 (see the file comment).
__device__ __forceinline__ float nfw_gx2(float x2)
{
    const float x = sqrtf(x2);
    if (x < 0.5f) {
        const float s = sqrtf(1.0f - x2);
        return (logf(2.0f / x) / (1.0f + s) + log1pf(-x2 / (2.0f * (1.0f + s))) / x2) / s;
    }
    float F;
    if (x2 < 1.0f) {
        const float s = sqrtf(1.0f - x2);
        F = s > 0.0f ? atanhf(s) / s : 1.0f;
    } else {
        const float r = sqrtf(x2 - 1.0f);
        F = r > 0.0f ? atanf(r) / r : 1.0f;
    }
    return (logf(0.5f * x) + F) / x2;
}

__device__ __forceinline__ double nfw_gx2(double x2)
{
    const double x = sqrt(x2);
    if (x < 0.5) {
        const double s = sqrt(1.0 - x2);
        return (log(2.0 / x) / (1.0 + s) + log1p(-x2 / (2.0 * (1.0 + s))) / x2) / s;
    }
    double F;
    if (x2 < 1.0) {
        const double s = sqrt(1.0 - x2);
        F = s > 0.0 ? atanh(s) / s : 1.0;
    } else {
        const double r = sqrt(x2 - 1.0);
        F = r > 0.0 ? atan(r) / r : 1.0;
    }
    return (log(0.5 * x) + F) / x2;
}

// FP32 field: NPL consecutive nodes of row blockIdx.y per thread.
template <int NPL>
__global__ __launch_bounds__(256) void k_nfw32(const float* __restrict__ t32, int np, int nx,
                                               float* __restrict__ ax, float* __restrict__ ay,
                                               const int* __restrict__ st)
{
    const int j = blockIdx.y;
    const int i0 = (blockIdx.x * 256 + threadIdx.x) * NPL;
    if ((int)(blockIdx.x * 256 * NPL) >= nx) return;
    const bool bad = *st != kStatusOk;
    float sx[NPL], sy[NPL];
#pragma unroll
    for (int k = 0; k < NPL; k++) sx[k] = sy[k] = 0.0f;
    const float fj = (float)j;
    if (!bad)  // uniform over the launch
        pots_wg<N32_STRIDE, N32_CYH, N32_CYL, N32_B, N32_C>(t32, np, fj, [&](const float* c, float4 rc) {
            const float A = c[N32_A], B = c[N32_B], irs2 = c[N32_IRS2], K = c[N32_K];
            const float nyv = rc.x, bny = rc.y, cny = rc.z;  // the row part
#pragma unroll
            for (int k = 0; k < NPL; k++) {
                const float nxv = ((float)(i0 + k) - c[N32_CXH]) - c[N32_CXL];
                const float m1 = fmaf(A, nxv, bny), m2 = fmaf(B, nxv, cny);
                const float R2 = fmaf(nxv, m1, nyv * m2);
                if (R2 > 0.0f) {
                    const float kg = K * nfw_gx2(R2 * irs2);
                    sx[k] = fmaf(kg, m1, sx[k]);
                    sy[k] = fmaf(kg, m2, sy[k]);
                }
            }
        });
    const size_t row = (size_t)j * nx;
#pragma unroll
    for (int k = 0; k < NPL; k++)
        if (i0 + k < nx) {
            ax[row + i0 + k] = bad ? __builtin_nanf("") : sx[k];
            ay[row + i0 + k] = bad ? __builtin_nanf("") : sy[k];
        }
}

// FP64 field: one node per thread.
__global__ __launch_bounds__(256) void k_nfw64(const double* __restrict__ t64, int np, GridDesc g,
                                               double* __restrict__ ax, double* __restrict__ ay,
                                               const int* __restrict__ st)
{
    const int j = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= g.nx) return;
    const bool bad = *st != kStatusOk;
    const double t1 = node_coord(g.x0, i, g.h), t2 = node_coord(g.y0, j, g.h);
    double s1 = 0.0, s2 = 0.0;
    for (int p = 0; p < np && !bad; p++) {
        const double* c = t64 + (size_t)p * N64_STRIDE;
        const double d1 = t1 - c[N64_XC], d2 = t2 - c[N64_YC];
        const double m1 = c[N64_A] * d1 + c[N64_B] * d2, m2 = c[N64_B] * d1 + c[N64_C] * d2;
        const double R2 = d1 * m1 + d2 * m2;
        if (R2 > 0.0) {
            const double kg = c[N64_K4] * nfw_gx2(R2 * c[N64_IRS2]);
            s1 += kg * m1;
            s2 += kg * m2;
        }
    }
    const size_t n = (size_t)j * g.nx + i;
    ax[n] = bad ? __builtin_nan("") : s1;
    ay[n] = bad ? __builtin_nan("") : s2;
}

// ---------------------------------------------------------------- launcher

size_t nfw_scratch(int np) { return (size_t)(np > 0 ? np : 1) * (N64_STRIDE * 8 + N32_STRIDE * 4) + 256; }

hipError_t launch_nfw(const NfwPtrs& h, const GridDesc& g, bool fp32, void* ax, void* ay, int* status,
                      void* scratch, const KernelEvents* ev, hipStream_t s)
{
    const int np = h.n > 0 ? h.n : 1;
    double* t64 = (double*)scratch;
    float* t32 = (float*)(t64 + (size_t)np * N64_STRIDE);
    int* st = (int*)(t32 + (size_t)np * N32_STRIDE);
    k_nfw_prep<<<1, 256, 0, s>>>(h, g, t64, t32, st, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fp32) {
        const dim3 grid((unsigned)((g.nx + 511) / 512), (unsigned)g.ny);
        return launch_ev(ev, k_nfw32<2>, grid, dim3(256), s, (const float*)t32, h.n, g.nx, (float*)ax, (float*)ay,
                         (const int*)st);
    }
    const dim3 grid((unsigned)((g.nx + 255) / 256), (unsigned)g.ny);
    return launch_ev(ev, k_nfw64, grid, dim3(256), s, (const double*)t64, h.n, g, (double*)ax, (double*)ay,
                     (const int*)st);
}

}  // namespace lens
