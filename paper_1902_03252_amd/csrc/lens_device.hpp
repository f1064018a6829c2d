// Device-side building blocks of the gfx950 chi^2 path.
//
// Deflection of one pseudo-elliptical cored/cut isothermal potential
// (Algorithm 1 of Rexroth et al. 2019, radial profile generalised as the paper
// suggests in Sec. 5).  Algorithm 1 translates, rotates by -Phi, scales the
// two axes by (1 -/+ eps), forms R and rotates back by +Phi.  The two
// rotations and the axis scaling collapse into one symmetric matrix
//     M = Rot(Phi) diag(1-eps, 1+eps) Rot(-Phi) = [[A, B], [B, C]],
//     A = (1-eps) cos^2 + (1+eps) sin^2,  B = -2 eps cos sin,
//     C = (1-eps) sin^2 + (1+eps) cos^2,
// so that with d = theta - theta_c:
//     R^2 = d . M d,   grad Psi = K f(R) M d,
//     f(R) = 1/(sqrt(a^2+R^2) + a) - 1/(sqrt(s^2+R^2) + s),
// K = b0 s/(s - a), b0 = 4 pi (sigma_v/c)^2 (Sec. 2.2.2).  For a = 0 and
// s = inf, K f M d = b0 M d / R: the SIE gradient of Sec. 2.2.2.  The matrix
// form needs 4 multiply-adds for the quadratic form and the gradient
// direction instead of 8 for the two explicit rotations; per-potential
// constants are precomputed once (FP64) by the prep kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lens {

// ---------------------------------------------------------------- tables

// FP64 table, arcsec units, one 128-byte row per potential.
enum : int {
    T64_XC = 0, T64_YC, T64_A, T64_B, T64_C, T64_A2, T64_S2, T64_RA, T64_RS, T64_K, T64_SINF,
    T64_STRIDE = 16
};

// FP32 table, grid-node units, one 96-byte row per potential.  The centre is
// stored as (index of the nearest node) + (fraction): with node index i an
// exact float, (i - c_hi) is exact and (i - c_hi) - c_lo carries only a
// relative rounding error, so the FP32 offset from a potential's centre is
// accurate to a few ulps of the offset itself, wherever the potential sits.
// This removes the paper's error growth near potential centres far from the
// origin (the |theta_center| / |Delta theta| term of its Appendix A).
// The general field uses M scaled by 1/sqrt(A h^2) (AP, BP, CQ) so that
// R^2 = m1'^2 + DQ n_y^2 with m1' = AP n_x + BP n_y (see field32_pot); the SIE
// field of the paper's own benchmark uses M h^2 and K/h directly.
enum : int {
    T32_CXH = 0, T32_CXL, T32_CYH, T32_CYL,  // centre in node units (hi + lo)
    T32_A, T32_B, T32_C,                     // M h^2 (SIE field)
    T32_K,                                   // K / h (SIE field)
    T32_AP, T32_BP, T32_CQ,                  // sqrt(A h^2), B h^2 / sqrt(A h^2), C h^2 / sqrt(A h^2)
    T32_DQ,                                  // det(M h^2) / (A h^2) = (1 - eps^2) h^4 / (A h^2)
    T32_A2,                                  // a^2 (arcsec^2)
    T32_S2A2,                                // s^2 - a^2
    T32_RA,                                  // a (arcsec)
    T32_KP,                                  // K' = (K / h) sqrt(A h^2)
    T32_KINV, T32_RSK,                       // 1 / K', s / K' (the FP32 values)
    T32_STRIDE = 24
};

// Per-system row (FP64): barycentre, its node-unit split, D_LS/D_OS and the
// FP32 error bound of the source-plane vertex positions.
enum : int {
    SYS_BX = 0, SYS_BY, SYS_BXH, SYS_BXL, SYS_BYH, SYS_BYL, SYS_R, SYS_EB, SYS_STRIDE = 8
};

// Device-side state of one evaluation (counters zeroed by the prep kernel).
struct EvalState {
    unsigned long long n_hits;       // certain hits appended by the triangle stage
    unsigned long long n_flags;      // undecided FP32 tests sent to the fallback
    unsigned long long n_fb_hits;    // hits found by the fallback
    int status;                      // LENS_OK / LENS_ERR_INVALID / LENS_ERR_CAPACITY
    unsigned head_ticket;            // "last workgroup" ticket, zero between launches
    double e_alpha;                  // bound on |alpha_fp32 - alpha| per component
    double w_sum;                    // sum of per-potential deflection bounds
};

constexpr int kStatusOk = 0;
constexpr int kStatusInvalid = 1;
constexpr int kStatusCapacity = 3;

// ---------------------------------------------------------------- wave helpers

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ double wave_sum(double v)
{
    // butterfly: every lane ends with the same, order-fixed result
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ float wave_min(float v)
{
    for (int m = 32; m >= 1; m >>= 1) v = fminf(v, __shfl_xor(v, m, 64));
    return v;
}

// FP64 coordinate of grid node i on one axis, x0 + i h, with the product and
// the sum rounded separately (no fused multiply-add): every FP64 node
// position of the library is formed this way, so that FP64 offsets
// theta - theta_c are the same numbers wherever they are computed, also at a
// node that coincides (or nearly coincides) with a potential's centre.
__device__ __forceinline__ double node_coord(double x0, double i, double h)
{
#pragma clang fp contract(off)
    return x0 + i * h;
}

// FP64 source-plane coordinate theta - r alpha (the lens equation of
// Sec. 2.2.2), product and difference rounded separately like node_coord.
__device__ __forceinline__ double src_map(double t, double r, double a)
{
#pragma clang fp contract(off)
    return t - r * a;
}

// ---------------------------------------------------------------- FP64 deflection

// FP64 square root and reciprocal of positive normal arguments from the
// hardware estimates (relative error below 2^-24 on gfx950, measured).  The
// root: one Goldschmidt iteration (g ~ sqrt(x) within ~2^-47) and one Newton
// correction g + (x - g^2) h with the unrefined h ~ 1/(2 sqrt(x)), whose own
// 2^-24 error enters only multiplied by the 2^-47 residual (Markstein,
// "IA-64 and elementary functions", 2000).  The reciprocal: r (1 + e + e^2)
// with e = 1 - x r, the second-order Newton-Raphson step, error ~e^3 plus
// rounding.  Both within about 1 ulp, at half the instructions of the
// correctly rounded library sequences.  A zero argument gives NaN (callers
// keep it positive).
__device__ __forceinline__ double sqrt_est64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double g = x * y, h = 0.5 * y;
    const double g1 = fma(g, fma(-g, h, 0.5), g);
    return fma(fma(-g1, g1, x), h, g1);
}

__device__ __forceinline__ double rcp_est64(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
}

// The row part of a potential's FP64 deflection at ordinate t2: d2 = t2 - y_c
// and the products B d2, C d2, common to every point of that ordinate.
struct Row64 {
    double d2, bd2, cd2;
};

__device__ __forceinline__ Row64 alpha64_rowc(const double* __restrict__ t, double t2)
{
    const double d2 = t2 - t[T64_YC];
    return {d2, t[T64_B] * d2, t[T64_C] * d2};
}

// Adds the deflection of the potential in row `t` (FP64 table) at the point
// (t1, ordinate of rc) to (s1, s2), given the row part rc.  The first root
// takes max(|a^2 + R^2|, 1e-300): at the centre of a singular profile (a = 0,
// R^2 = 0, m = 0 exactly) f is then finite (~1e150) and the contribution f m
// exactly zero, the centre convention, without a test; |.| keeps a
// rounding-level negative R^2 (eps near 1) from a NaN.  Everywhere else the
// clamp is inactive (a^2 + R^2 >= 1e-300 unless the point lies within 1e-150"
// of a singular centre without coinciding with it).
__device__ __forceinline__ void add_alpha64(const double* __restrict__ t, double t1, const Row64& rc, double& s1,
                                            double& s2)
{
    const double d1 = t1 - t[T64_XC];
    const double m1 = fma(t[T64_A], d1, rc.bd2);
    const double m2 = fma(t[T64_B], d1, rc.cd2);
    const double R2 = fma(d1, m1, rc.d2 * m2);
    const double qa = sqrt_est64(fmax(fabs(t[T64_A2] + R2), 1e-300)) + t[T64_RA];
    double f;
    if (__double_as_longlong(t[T64_SINF]) != 0) {  // uncut (a scalar test of the stored 1.0 / +0.0)
        f = rcp_est64(qa);
    } else {
        const double qs = sqrt_est64(t[T64_S2] + R2) + t[T64_RS];
        f = (qs - qa) * rcp_est64(qa * qs);
    }
    const double kf = t[T64_K] * f;
    s1 += kf * m1;
    s2 += kf * m2;
}

// The same at the point (t1, t2).
__device__ __forceinline__ void add_alpha64(const double* __restrict__ t, double t1, double t2, double& s1,
                                            double& s2)
{
    add_alpha64(t, t1, alpha64_rowc(t, t2), s1, s2);
}

// Deflection at (t1[k], t2), k < N, of every potential of the FP64 table, for
// a workgroup of 256 threads whose points share the ordinate t2 (all threads
// call it): the row parts of up to 256 potentials at a time are computed once,
// one potential per thread, into LDS.  Same arithmetic as add_alpha64 at each
// point.
template <int N>
__device__ __forceinline__ void alpha64_all_wg(const double* __restrict__ tab, int np, const double* t1, double t2,
                                               double* s1, double* s2)
{
    __shared__ Row64 srow[256];
    for (int p0 = 0; p0 < np; p0 += 256) {
        const int pc = np - p0 < 256 ? np - p0 : 256;
        if (p0 > 0) __syncthreads();  // the previous chunk has been read
        if ((int)threadIdx.x < pc) srow[threadIdx.x] = alpha64_rowc(tab + (size_t)(p0 + threadIdx.x) * T64_STRIDE, t2);
        __syncthreads();
        for (int p = 0; p < pc; p++) {
            const Row64 rc = srow[p];
#pragma unroll
            for (int k = 0; k < N; k++) add_alpha64(tab + (size_t)(p0 + p) * T64_STRIDE, t1[k], rc, s1[k], s2[k]);
        }
    }
}

__device__ __forceinline__ void alpha64_all_wg(const double* __restrict__ tab, int np, double t1, double t2,
                                               double& s1, double& s2)
{
    alpha64_all_wg<1>(tab, np, &t1, t2, &s1, &s2);
}

// grad Psi at one point with the potentials split over the 64 lanes of a
// wave and a fixed butterfly reduction (deterministic).  All lanes return the
// same value.
__device__ __forceinline__ void alpha64_wave(const double* __restrict__ tab, int np, double t1, double t2,
                                             double& a1, double& a2)
{
    double s1 = 0.0, s2 = 0.0;
    for (int p = lane_id(); p < np; p += 64) add_alpha64(tab + (size_t)p * T64_STRIDE, t1, t2, s1, s2);
    a1 = wave_sum(s1);
    a2 = wave_sum(s2);
}

// ---------------------------------------------------------------- exact orientation

// Error-free transformations (Knuth's TwoSum; TwoProduct through the fused
// multiply-add).  Exact barring overflow/underflow.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e)
{
    p = a * b;
    e = fma(a, b, -p);
}

// Sign of the exact sum of n doubles by growing a non-overlapping expansion
// (Shewchuk 1997, "Adaptive precision floating-point arithmetic"): the sign of
// an expansion is the sign of its largest non-zero component.
__device__ __noinline__ int exact_sum_sign(const double* terms, int n)
{
    double h[16];
    int m = 0;
    for (int k = 0; k < n; k++) {
        double q = terms[k];
        for (int i = 0; i < m; i++) {
            double s, e;
            two_sum(q, h[i], s, e);
            h[i] = e;
            q = s;
        }
        h[m++] = q;
    }
    for (int i = m - 1; i >= 0; i--)
        if (h[i] != 0.0) return h[i] > 0.0 ? 1 : -1;
    return 0;
}

// Exact sign of (a - p) x (b - p) for FP64 inputs.  A forward error bound
// decides almost every case in plain FP64; otherwise the determinant is
// expanded exactly: each difference is a two-term sum (TwoSum), each product
// of two-term sums four TwoProducts, 16 terms in all.
__device__ __forceinline__ int orient_exact(double ax, double ay, double bx, double by, double px, double py)
{
    const double l = (ax - px) * (by - py);
    const double r = (ay - py) * (bx - px);
    const double det = l - r;
    // |fl(det) - det| <= (3u + O(u^2)) (|l| + |r|) + u |det|, u = 2^-53; use 8u
    const double bound = 8.881784197001252e-16 * (fabs(l) + fabs(r));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    double x1, x1e, y2, y2e, y1, y1e, x2, x2e;
    two_sum(ax, -px, x1, x1e);
    two_sum(by, -py, y2, y2e);
    two_sum(ay, -py, y1, y1e);
    two_sum(bx, -px, x2, x2e);
    double t[16];
    two_prod(x1, y2, t[0], t[1]);
    two_prod(x1, y2e, t[2], t[3]);
    two_prod(x1e, y2, t[4], t[5]);
    two_prod(x1e, y2e, t[6], t[7]);
    two_prod(-y1, x2, t[8], t[9]);
    two_prod(-y1, x2e, t[10], t[11]);
    two_prod(-y1e, x2, t[12], t[13]);
    two_prod(-y1e, x2e, t[14], t[15]);
    return exact_sum_sign(t, 16);
}

// Containment of p in the triangle (v0, v1, v2) decided exactly on the FP64
// vertex values: exact bounding-box rejection, then the three exact edge
// signs; strict inequalities (a point on an edge is a miss).
__device__ __forceinline__ bool contains_exact(const double* vx, const double* vy, double px, double py)
{
    const double xmin = fmin(vx[0], fmin(vx[1], vx[2])), xmax = fmax(vx[0], fmax(vx[1], vx[2]));
    const double ymin = fmin(vy[0], fmin(vy[1], vy[2])), ymax = fmax(vy[0], fmax(vy[1], vy[2]));
    if (px < xmin || px > xmax || py < ymin || py > ymax) return false;
    const int s0 = orient_exact(vx[0], vy[0], vx[1], vy[1], px, py);
    const int s1 = orient_exact(vx[1], vy[1], vx[2], vy[2], px, py);
    const int s2 = orient_exact(vx[2], vy[2], vx[0], vy[0], px, py);
    return (s0 > 0 && s1 > 0 && s2 > 0) || (s0 < 0 && s1 < 0 && s2 < 0);
}

// Grid-node indices of the three vertices of triangle `tid` (Fig. 1 split).
__device__ __forceinline__ void triangle_nodes(int nx, int tid, int* ni, int* nj)
{
    const int cell = tid >> 1, k = tid & 1;
    const int i = cell % (nx - 1), j = cell / (nx - 1);
    if (k == 0) {
        ni[0] = i; nj[0] = j; ni[1] = i + 1; nj[1] = j; ni[2] = i; nj[2] = j + 1;
    } else {
        ni[0] = i + 1; nj[0] = j + 1; ni[1] = i; nj[1] = j + 1; ni[2] = i + 1; nj[2] = j;
    }
}

}  // namespace lens
