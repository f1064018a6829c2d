// Device code shared by the single-evaluation and the batched chi^2 kernels:
// constants, per-potential tables, the FP32 field inner loop, the tile
// machinery of the triangle stage, FP64 vertices and image positions.
#pragma once

#include "lens_device.hpp"
#include "lens_internal.hpp"

#include <math.h>

namespace lens {

constexpr double kPi = 3.14159265358979323846;
constexpr double kCkms = 299792.458;                 // km/s
constexpr double kArcsecPerRad = 206264.80624709636;  // 180 * 3600 / pi
constexpr double kU32 = 5.9604644775390625e-08;       // 2^-24, unit roundoff of FP32
constexpr double kNodeSplitErr = 2.9802322387695312e-08;  // 2^-25 node units

// Ticket of the "last workgroup finishes the job" pattern: every workgroup
// publishes its global writes, then takes a ticket; the one that takes the
// last ticket sees every other workgroup's writes and resets the ticket for
// the next launch.
__device__ __forceinline__ bool last_of(unsigned* ticket, unsigned count, int* s_flag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *s_flag = atomicAdd(ticket, 1u) == count - 1;
    __syncthreads();
    if (!*s_flag) return false;
    __threadfence();
    if (threadIdx.x == 0) *ticket = 0;
    return true;
}

__device__ __forceinline__ bool last_workgroup(unsigned* ticket, int* s_flag)
{
    return last_of(ticket, gridDim.x, s_flag);
}

// ============================================================== prep

// FP64 table row of potential p (arcsec units), computed from the raw
// parameters; returns whether the parameters lie in the model's domain.
__device__ __forceinline__ bool row64(const PotPtrs& pot, int p, double* t, double& K, double& a1, double& a2)
{
    const double xc = pot.x[p], yc = pot.y[p], eps = pot.eps[p], phi = pot.phi[p];
    const double a = pot.r_core[p], s = pot.r_cut[p], sig = pot.sigma_v[p];
    const bool ok = isfinite(xc) && isfinite(yc) && isfinite(eps) && isfinite(phi) && isfinite(a) &&
                    isfinite(sig) && eps >= 0.0 && eps < 1.0 && a >= 0.0 && sig >= 0.0 && s > a;
    const bool sinf = isinf(s);
    double c, sn;
    sincos(phi, &sn, &c);
    a1 = 1.0 - eps;
    a2 = 1.0 + eps;
    const double ratio = sig / kCkms;
    const double b0 = 4.0 * kPi * ratio * ratio * kArcsecPerRad;
    K = sinf ? b0 : b0 * s / (s - a);
    t[T64_XC] = xc;
    t[T64_YC] = yc;
    t[T64_A] = a1 * c * c + a2 * sn * sn;
    t[T64_B] = -2.0 * eps * c * sn;
    t[T64_C] = a1 * sn * sn + a2 * c * c;
    t[T64_A2] = a * a;
    t[T64_S2] = sinf ? 0.0 : s * s;
    t[T64_RA] = a;
    t[T64_RS] = sinf ? 0.0 : s;
    t[T64_K] = K;
    t[T64_SINF] = sinf ? 1.0 : 0.0;
    for (int k = T64_SINF + 1; k < T64_STRIDE; k++) t[k] = 0.0;
    return ok;
}

// Constants of parameter column p written to table row q; the FP64 row is
// also copied to row_copy and the three bound terms returned in terms when
// these are not null.
inline __device__ void prep_one(const PotPtrs& pot, const GridDesc& g, int p, int q, double* __restrict__ tab64,
                                float* __restrict__ tab32, double* __restrict__ bterm,
                                double* row_copy = nullptr, double* terms = nullptr)
{
    double row[T64_STRIDE], K, a1, a2;
    bool ok = row64(pot, p, row, K, a1, a2);
    double* t = tab64 + (size_t)q * T64_STRIDE;
    for (int k = 0; k < T64_STRIDE; k++) t[k] = row[k];
    if (row_copy)
        for (int k = 0; k < T64_STRIDE; k++) row_copy[k] = row[k];
    const double xc = row[T64_XC], yc = row[T64_YC], A = row[T64_A], B = row[T64_B], C = row[T64_C];
    const double a = row[T64_RA], s = pot.r_cut[p];
    const bool sinf = row[T64_SINF] != 0.0;
    const double cxn = (xc - g.x0) / g.h, cyn = (yc - g.y0) / g.h;
    ok = ok && fabs(cxn) < 4194304.0 && fabs(cyn) < 4194304.0;  // |centre| < 2^22 nodes
    const double cxh = ok ? rint(cxn) : 0.0, cyh = ok ? rint(cyn) : 0.0;
    // The fraction is taken from the FP64 offset of the nearest node itself,
    // formed as every FP64 node offset is (node_coord, then the difference):
    // at that node the FP32 offset (i - c_hi) - c_lo = -c_lo is then that FP64
    // offset up to one FP32 rounding, a relative error even when the centre
    // lies on (or within rounding of) the node.
    const double cxl = -(node_coord(g.x0, cxh, g.h) - xc) / g.h;
    const double cyl = -(node_coord(g.y0, cyh, g.h) - yc) / g.h;
    const double h2 = g.h * g.h;
    float* u = tab32 + (size_t)q * T32_STRIDE;
    u[T32_CXH] = (float)cxh;
    u[T32_CXL] = (float)cxl;
    u[T32_CYH] = (float)cyh;
    u[T32_CYL] = (float)cyl;
    // SIE field (the paper's benchmark): M h^2 and K/h; a potential with K/h
    // below 1e-15 (sigma_v = 0, or a deflection below 1e-14") is stored with
    // M = 0 and K = 0
    const float k32 = (float)(K / g.h);
    const bool kz = !(k32 >= 1e-15f);
    u[T32_A] = kz ? 0.0f : (float)(A * h2);
    u[T32_B] = kz ? 0.0f : (float)(B * h2);
    u[T32_C] = kz ? 0.0f : (float)(C * h2);
    u[T32_K] = kz ? 0.0f : k32;
    // General field (field32_pot): M scaled by 1/sqrt(A h^2) and K' = (K/h)
    // sqrt(A h^2) = K sqrt(A).  A finite cut radius beyond 1e18" is stored as
    // uncut (its term 1/B_ < 5e-19 is below the rounding of 1/A_ for any
    // A_ < 1e9"), an uncut profile with s = 1e18 (s^2 - a^2 = 1e36), and a
    // singular one with a = 1e-20 in A_ only.  A potential with K' below 1e-12
    // is stored with zero coefficients and K' = 0 (its finite f multiplies
    // m = 0) and its whole deflection, at most w_p, is charged to the bound
    // below; 1/K' <= 1e12 keeps B_/K' <= 2e30.
    const bool sbig = sinf || s > 1e18;
    const double sA = sqrt(A * h2);
    const float kp = (float)(K * sqrt(A));
    const bool kzp = !(kp >= 1e-12f);
    u[T32_AP] = kzp ? 0.0f : (float)sA;
    u[T32_BP] = kzp ? 0.0f : (float)(B * h2 / sA);
    u[T32_CQ] = kzp ? 0.0f : (float)(C * h2 / sA);
    u[T32_DQ] = (float)(a1 * a2 * h2 / A);
    u[T32_A2] = (float)(a * a);
    u[T32_S2A2] = sbig ? 1e36f : (float)(s * s - a * a);
    u[T32_RA] = a > 0.0 ? (float)a : 1e-20f;
    u[T32_KP] = kzp ? 0.0f : kp;
    const float kinv = kzp ? 1.0f : (float)(1.0 / (double)kp);
    u[T32_KINV] = kinv;
    u[T32_RSK] = (float)((double)(sbig ? 1e18f : (float)s) * (double)kinv);
    for (int k = T32_RSK + 1; k < T32_STRIDE; k++) u[k] = 0.0f;

    // Offset error term j_p.  Every node other than the nearest one lies at
    // least half a node from the centre on one axis, so R >= sqrt(1 - eps) h
    // max(rn, 1/2) there (R^2 >= (1 - eps) |d|^2), and its offset differs from
    // the FP64 node offset by at most derr (FP32 rounding of the fraction, the
    // FP64 reference's own rounding of the node positions and of theta -
    // theta_c); J bounds the Jacobian of grad Psi_p at that radius.  At the
    // nearest node the difference is relative (one FP32 rounding of c_lo,
    // above): |Jacobian| |Delta d| <= (2 K (1 + eps) / ((1 - eps) R)) u |d| <=
    // 2 u K (1 + eps) / (1 - eps)^1.5, whatever the distance.
    const double w = K * a2 / sqrt(a1);
    const double rn = sqrt(cxl * cxl + cyl * cyl);
    const double rho = sqrt(a1) * g.h * fmax(rn, 0.5);
    const double J = 2.0 * K * a2 / (a1 * (sqrt(a * a + rho * rho) + a));
    const double span = fabs(g.x0) + fabs(g.y0) + (double)(g.nx + g.ny) * g.h + fabs(xc) + fabs(yc);
    // (two nodes' roundings of x0 + i h and theta - theta_c, each <= 2^-53 (2 |x0| + 3 n h + |x_c|)
    // per axis, below 1e-15 span)
    const double derr = g.h * kNodeSplitErr + 1e-15 * span;
    // That relative argument needs the FP32 evaluation at the nearest node to
    // be accurate itself: for a (nearly) singular profile whose centre lies
    // within 1e-10" of a node without coinciding with it, the 1e-20" stand-in
    // core and the FP32 range of R^2 are not negligible there, and the term
    // 2 w_p (any deflection direction) is taken instead: the bound then admits
    // little, and the mixed path defers to the FP64 fallback or reports
    // capacity.  A centre exactly on a node is exact in both precisions (zero
    // offsets, zero contribution).
    const bool near_singular = rn > 0.0 && g.h * rn < 1e-10 && a < 1e-10;
    // The FP32 products stay finite while qa B_/K' <= (sqrt(a^2 + R^2) + a)
    // (2 s + R) / K' does (R <= sqrt(1 + eps) |d|, |d| <= span); beyond, the
    // same 2 w_p is taken.
    const double rmax = sqrt(a2) * span, se = sbig ? 1e18 : s;
    const bool range = !kzp && (sqrt(a * a + rmax * rmax) + a) * (2.0 * se + rmax) * (double)kinv > 1e37;
    const double jt = J * derr + 2.0 * kU32 * K * a2 / (a1 * sqrt(a1)) +
                      ((near_singular || range) ? 2.0 * w : 0.0) + (kzp ? w : 0.0);
    bterm[3 * q + 0] = ok ? w : 0.0;
    bterm[3 * q + 1] = ok ? jt : 0.0;
    bterm[3 * q + 2] = ok ? 0.0 : 1.0;
    if (terms) {
        terms[0] = ok ? w : 0.0;
        terms[1] = ok ? jt : 0.0;
        terms[2] = ok ? 0.0 : 1.0;
    }
}

// Index of the system that owns observed image j: sys_off is non-decreasing
// for valid input; the search is clamped so that invalid input stays in range
// (it is then reported as invalid).
__device__ __forceinline__ int system_of(const int* __restrict__ sys_off, int nsys, int j)
{
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys_off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- field

// FP32 contribution of one potential row `c` for NPL nodes of a row, one
// branch-free formula for all four radial-profile kinds:
//     f = (B_ - A_) / (A_ B_),  A_ = sqrt(a^2 + R^2) + a,  B_ = sqrt(s^2 + R^2) + s.
// With M h^2 = [[A, B], [B, C]] and n the node-unit offset, the table holds
// M scaled by 1/sqrt(A): m' = (sqrt(A) n_x + B/sqrt(A) n_y, B/sqrt(A) n_x +
// C/sqrt(A) n_y) = M h^2 n / sqrt(A), and R^2 = n . M h^2 n =
// m'_1^2 + (det(M h^2)/A) n_y^2 (completing the square in n_x): a sum of two
// non-negative terms, so a^2 + R^2 is one fused multiply-add of m'_1 onto a
// row constant E = (det/A) n_y^2 + a^2, never negative.  The deflection
// K f M d = (K' f) m' with K' = (K/h) sqrt(A), and K' f = K' (B_ - A_) /
// (A_ B_) is evaluated as (K' b - A_) / (A_ b) with b = B_ / K' =
// sqrt(s^2 + R^2) / K' + s / K' (one fused multiply-add; 1/K' and s/K' are
// stored).  An uncut profile is stored with s = 1e18 (s^2 - a^2 = 1e36):
// B_ = 2e18 in FP32, B_ - A_ rounds to B_, and f = 1/A_ to a few ulps.  A
// singular profile (a = 0) is stored with a = 1e-20 arcsec in A_ only (a^2
// stays 0), so that A_ B_ > 0 everywhere: at the centre the offsets are
// exactly zero and the contribution is exactly zero (the centre convention);
// elsewhere the change of f, below 1e-20/R relative, lies inside the FP32
// error bound (its Jacobian term).  Offsets from the centre use the exact
// hi/lo split (see the FP32 table); hardware sqrt/rcp (1 ulp) are accounted
// for in the error bound (a float32 emulation with 1-ulp root and reciprocal
// errors over random profiles, eps up to 0.95, and radii from 1e-3 to 1e4
// nodes stays under 9 u w_p, inside the bound's 64 u w_p per potential).
// This is the node part for NPL consecutive nodes in each of NR consecutive
// rows (sx, sy: [NR][NPL]), given the row parts rc[r] = (B/sqrt(A) n_y,
// C/sqrt(A) n_y, E, s/K') of the same potential for those rows (see
// field32_all_wg): the column offset n_x = (i - c_hi) - c_lo, two
// instructions, is formed once per column and shared by the NR rows; per
// node and potential, 11 vector instructions and 3 transcendentals (2 roots,
// 1 reciprocal).  Every node's arithmetic is the same whatever NPL and NR.
template <int NPL, int NR = 1>
__device__ __forceinline__ void field32_pot(const float* __restrict__ c, const float4* rc, const float* fi,
                                            float* sx, float* sy)
{
    const float cxh = c[T32_CXH], cxl = c[T32_CXL];
    const float ap = c[T32_AP], bp = c[T32_BP];
    const float s2a2 = c[T32_S2A2], ra = c[T32_RA], kp = c[T32_KP], kinv = c[T32_KINV];
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        const float nxv = (fi[k] - cxh) - cxl;
#pragma unroll
        for (int r = 0; r < NR; r++) {
            const float m1 = fmaf(ap, nxv, rc[r].x);
            const float m2 = fmaf(bp, nxv, rc[r].y);
            const float qa2 = fmaf(m1, m1, rc[r].z);  // a^2 + R^2 >= 0
            const float qa = __builtin_amdgcn_sqrtf(qa2) + ra;
            const float qsk = fmaf(__builtin_amdgcn_sqrtf(qa2 + s2a2), kinv, rc[r].w);  // B_ / K'
            const float kf = fmaf(qsk, kp, -qa) * __builtin_amdgcn_rcpf(qa * qsk);
            sx[r * NPL + k] = fmaf(kf, m1, sx[r * NPL + k]);
            sy[r * NPL + k] = fmaf(kf, m2, sy[r * NPL + k]);
        }
    }
}

// Runs f(c, rc) for every row c of an FP32 table of np rows (STRIDE floats
// each), in order, with rc[r] = rowf(c, n_y), n_y = (j - c[IYH]) - c[IYL],
// for the NR grid rows j = fj, fj + 1, ...: the row part of a potential,
// common to every node of grid row j.  For a workgroup of 256 threads on
// those rows (all threads call it, with the same fj): the row parts of up to
// 256 potentials at a time are computed once, one potential per thread, into
// LDS, so that the per-potential work of every wave is the node part only
// (the row part is uniform over the workgroup but, with no scalar FP32 ALU,
// costs a full vector instruction per wave).
// srow: LDS of NR * 256 float4 (row r of potential p at r * 256 + p).
template <int STRIDE, int IYH, int IYL, int NR, class RF, class F>
__device__ __forceinline__ void pots_wg_rows(const float* __restrict__ tab, int np, float fj, float4* __restrict__ srow,
                                             RF&& rowf, F&& f)
{
    for (int p0 = 0; p0 < np; p0 += 256) {
        const int pc = np - p0 < 256 ? np - p0 : 256;
        if (p0 > 0) __syncthreads();  // the previous chunk has been read
        if ((int)threadIdx.x < pc) {
            const float* c = tab + (size_t)(p0 + threadIdx.x) * STRIDE;
#pragma unroll
            for (int r = 0; r < NR; r++) srow[r * 256 + threadIdx.x] = rowf(c, ((fj + (float)r) - c[IYH]) - c[IYL]);
        }
        __syncthreads();
        for (int p = 0; p < pc; p++) {
            float4 rc[NR];
#pragma unroll
            for (int r = 0; r < NR; r++) rc[r] = srow[r * 256 + p];
            f(tab + (size_t)(p0 + p) * STRIDE, rc);
        }
    }
}

// One grid row (pots_wg_rows with NR = 1) and the row part (n_y, B n_y, C n_y)
// of a table holding M h^2 at IB, IC: f(c, rc) with the row part itself.
template <int STRIDE, int IYH, int IYL, int IB, int IC, class F>
__device__ __forceinline__ void pots_wg(const float* __restrict__ tab, int np, float fj, F&& f)
{
    __shared__ float4 srow[256];
    pots_wg_rows<STRIDE, IYH, IYL, 1>(
        tab, np, fj, srow, [](const float* c, float nyv) { return make_float4(nyv, c[IB] * nyv, c[IC] * nyv, 0.0f); },
        [&](const float* c, const float4* rc) { f(c, rc[0]); });
}

// Deflection of NPL nodes in each of NR rows (fj, fj + 1, ...) by every
// potential of the FP32 table, for a workgroup of 256 threads on those rows
// (pots_wg_rows with the row part of field32_pot; s / K' rides along with it,
// as field32_pot's fused multiply-add can take only one scalar operand).
// sx, sy: [NR][NPL]; srow: LDS of NR * 256 float4.
template <int NPL, int NR = 1>
__device__ __forceinline__ void field32_all_wg(const float* __restrict__ tab, int np, float fj, const float* fi,
                                               float* sx, float* sy, float4* __restrict__ srow)
{
    pots_wg_rows<T32_STRIDE, T32_CYH, T32_CYL, NR>(
        tab, np, fj, srow,
        [](const float* c, float nyv) {
            return make_float4(c[T32_BP] * nyv, c[T32_CQ] * nyv, fmaf(c[T32_DQ] * nyv, nyv, c[T32_A2]), c[T32_RSK]);
        },
        [&](const float* c, const float4* rc) { field32_pot<NPL, NR>(c, rc, fi, sx, sy); });
}

// Range partials of the triangle stage, written by the field kernel: for grid
// row j and column group c (nodes [c*TX, c*TX + TX) of the row), the min/max
// of each deflection component over the group and the deflection at its first
// node, which is the halo column of tile column c - 1.  rr is
// [rows][tiles_x + 1][kRR] (min ax, max ax, min ay, max ay, ax, ay at the
// first node, 2 unused); groups c <= tiles_x carry the first node, groups
// c < tiles_x the ranges.  The lanes of a group are an aligned group of
// TX/NPL lanes of one wave; all 64 lanes must call this together.  Nodes at
// i >= nx do not count.  (kRR is declared with the launch interface.)

template <typename V, int NPL>
__device__ __forceinline__ void tile_partials(const V* sx, const V* sy, int i0, int j, int nx, int tx_shift,
                                              int tiles_x, V* __restrict__ rr)
{
    V mnx = V(INFINITY), mxx = V(-INFINITY), mny = V(INFINITY), mxy = V(-INFINITY);
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        if (i0 + k < nx) {
            mnx = fmin(mnx, sx[k]);
            mxx = fmax(mxx, sx[k]);
            mny = fmin(mny, sy[k]);
            mxy = fmax(mxy, sy[k]);
        }
    }
    const int seg = (1 << tx_shift) / NPL;  // lanes per tile column, a power of two <= 64
    for (int m = 1; m < seg; m <<= 1) {
        mnx = fmin(mnx, __shfl_xor(mnx, m, 64));
        mxx = fmax(mxx, __shfl_xor(mxx, m, 64));
        mny = fmin(mny, __shfl_xor(mny, m, 64));
        mxy = fmax(mxy, __shfl_xor(mxy, m, 64));
    }
    const int col = i0 >> tx_shift;
    if ((i0 & ((1 << tx_shift) - 1)) == 0 && i0 < nx && col <= tiles_x) {
        V* q = rr + ((size_t)j * (tiles_x + 1) + col) * kRR;
        if (col < tiles_x) {
            q[0] = mnx;
            q[1] = mxx;
            q[2] = mny;
            q[3] = mxy;
        }
        q[4] = sx[0];
        q[5] = sy[0];
    }
}

// ---------------------------------------------------------------- triangles


enum : int { kMiss = 0, kHit = 1, kFlag = 2 };

// Appends `key` for every lane with `pred` set: one atomic per wave, slots
// from the ballot prefix count.  Must be called by all 64 lanes together.
__device__ __forceinline__ void wave_append(bool pred, unsigned long long key, unsigned long long* counter,
                                            unsigned long long* list, long long cap)
{
    const unsigned long long m = __ballot(pred);
    if (m == 0) return;
    const int leader = __ffsll((long long)m) - 1;
    const int cnt = __popcll(m);
    long long base = 0;
    if (lane_id() == leader) base = (long long)atomicAdd(counter, (unsigned long long)cnt);
    base = __shfl(base, leader, 64);
    const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    if (pred && base + off < cap) list[base + off] = key;
}

// Value of lane l (wave-uniform l) in every lane.
__device__ __forceinline__ double bcast(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ unsigned long long hit_key(int s, int tid)
{
    return ((unsigned long long)(unsigned)s << 32) | (unsigned)tid;
}

// FP32 containment decision with a certified sign (mixed path).  d* are the
// vertex offsets B_k - barycentre; each component is within E of the exact
// FP64 value.  Returns kMiss / kHit when certain, kFlag otherwise.
__device__ __forceinline__ int decide32(const float* dx, const float* dy, float E, int mode, float tau,
                                        unsigned& nbbox)
{
    const float xmin = fminf(dx[0], fminf(dx[1], dx[2])), xmax = fmaxf(dx[0], fmaxf(dx[1], dx[2]));
    const float ymin = fminf(dy[0], fminf(dy[1], dy[2])), ymax = fmaxf(dy[0], fmaxf(dy[1], dy[2]));
    if (mode == 1) {  // literal threshold
        if (xmin > 0.0f || xmax < 0.0f || ymin > 0.0f || ymax < 0.0f) return kMiss;
        nbbox++;
        int pos = 0, neg = 0;
        bool small = false;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int k1 = k == 2 ? 0 : k + 1;
            const float c = fmaf(dx[k], dy[k1], -(dy[k] * dx[k1]));
            small = small || fabsf(c) < tau;
            pos += c > 0.0f;
            neg += c < 0.0f;
        }
        if (small) return kFlag;
        return (pos == 3 || neg == 3) ? kHit : kMiss;
    }
    if (xmin > E || xmax < -E || ymin > E || ymax < -E) return kMiss;
    nbbox++;
    int pos = 0, neg = 0;
    const float e2 = 2.0f * E * E;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int k1 = k == 2 ? 0 : k + 1;
        const float p = dy[k] * dx[k1];
        const float q = dx[k] * dy[k1];
        const float c = fmaf(dx[k], dy[k1], -p);
        const float s1 = fabsf(dx[k]) + fabsf(dy[k]) + fabsf(dx[k1]) + fabsf(dy[k1]);
        // |c_exact - c| <= E s1 + 2E^2 + 2u (|q| + |p|), evaluated with margin
        const float T = (E * s1 + e2 + 1.2e-7f * (fabsf(q) + fabsf(p))) * 1.001f;
        pos += c > T;
        neg += c < -T;
    }
    if (pos > 0 && neg > 0) return kMiss;
    if (pos == 3 || neg == 3) return kHit;
    return kFlag;
}

// ---------------------------------------------------------------- tiles

// A tile of TX x TY cells with its one-node halo of (TX+1) x (TY+1) nodes.
template <int TX_, int TY_>
struct TileShape {
    static constexpr int TX = TX_, TY = TY_;
    static constexpr int TNX = TX + 1, TNY = TY + 1;
    static_assert(TX * TY % 256 == 0, "a tile is a whole number of cells per wave step");
};

// Tile geometry from a linear tile index.
struct Tile {
    int ci0, cj0, ncx, ncy;
};

template <class S>
__device__ __forceinline__ Tile tile_of(const GridDesc& g, int tiles_x, int tile)
{
    Tile T;
    T.ci0 = (tile % tiles_x) * S::TX;
    T.cj0 = (tile / tiles_x) * S::TY;
    T.ncx = min(S::TX, g.nx - 1 - T.ci0);
    T.ncy = min(S::TY, g.ny - 1 - T.cj0);
    return T;
}

// Deflection range of tile T (with its halo) for every lane of a wave, from
// the field kernel's row partials: lanes over the tile's node rows, then a
// butterfly min/max.
template <class S, typename V>
__device__ __forceinline__ void tile_range_wave(const V* __restrict__ rr, int tiles_x, const Tile& T, double* rng)
{
    const int lane = lane_id();
    const int col = T.ci0 / S::TX;
    V mnx = V(INFINITY), mxx = V(-INFINITY), mny = V(INFINITY), mxy = V(-INFINITY);
    if (lane <= T.ncy) {
        const int j = T.cj0 + lane;
        const V* q = rr + ((size_t)j * (tiles_x + 1) + col) * kRR;
        mnx = q[0];
        mxx = q[1];
        mny = q[2];
        mxy = q[3];
        if (T.ncx == S::TX) {  // halo column: first node of the next column group
            const V vx = q[kRR + 4], vy = q[kRR + 5];
            mnx = fmin(mnx, vx);
            mxx = fmax(mxx, vx);
            mny = fmin(mny, vy);
            mxy = fmax(mxy, vy);
        }
    }
    for (int m = 32; m >= 1; m >>= 1) {
        mnx = fmin(mnx, __shfl_xor(mnx, m, 64));
        mxx = fmax(mxx, __shfl_xor(mxx, m, 64));
        mny = fmin(mny, __shfl_xor(mny, m, 64));
        mxy = fmax(mxy, __shfl_xor(mxy, m, 64));
    }
    rng[0] = mnx;
    rng[1] = mxx;
    rng[2] = mny;
    rng[3] = mxy;
}

// Deflection range of one tile per lane (the lane's own tile T) from the
// field kernel's row partials: the same minimum and maximum over the tile's node
// rows and halo column as tile_range_wave.
template <class S, typename V>
__device__ __forceinline__ void tile_range_lane(const V* __restrict__ rr, int tiles_x, const Tile& T, double* rng)
{
    const int col = T.ci0 / S::TX;
    const bool halo = T.ncx == S::TX;  // halo column: first node of the next column group
    V mnx = V(INFINITY), mxx = V(-INFINITY), mny = V(INFINITY), mxy = V(-INFINITY);
    // every row's loads issued at once, without branches: a fixed trip count
    // with rows past the tile's last node row clamped to it (a repeated row
    // leaves the minimum and maximum unchanged), and the halo record always
    // loaded (it lies inside the partials, past the grid's last column group
    // unwritten) and selected only for a full-width tile
#pragma unroll
    for (int r = 0; r <= S::TY; r++) {
        const V* q = rr + ((size_t)(T.cj0 + min(r, T.ncy)) * (tiles_x + 1) + col) * kRR;
        const V a0 = q[0], a1 = q[1], a2 = q[2], a3 = q[3], hx = q[kRR + 4], hy = q[kRR + 5];
        mnx = fmin(mnx, halo ? fmin(a0, hx) : a0);
        mxx = fmax(mxx, halo ? fmax(a1, hx) : a1);
        mny = fmin(mny, halo ? fmin(a2, hy) : a2);
        mxy = fmax(mxy, halo ? fmax(a3, hy) : a3);
    }
    rng[0] = mnx;
    rng[1] = mxx;
    rng[2] = mny;
    rng[3] = mxy;
}

// Loads tile T's nodes (with the halo) into a wave-private LDS tile.
template <class S, typename V>
__device__ __forceinline__ void stage_tile_wave(const V* __restrict__ ax, const V* __restrict__ ay, const GridDesc& g,
                                                const Tile& T, V (*sx)[S::TNX], V (*sy)[S::TNX])
{
    const int lane = lane_id();
    constexpr int N = S::TNX * S::TNY;
#pragma unroll
    for (int k = 0; k < (N + 63) / 64; k++) {
        const int q = lane + 64 * k;
        const int li = q % S::TNX, lj = q / S::TNX;
        if (q < N && li <= T.ncx && lj <= T.ncy) {
            const size_t n = (size_t)(T.cj0 + lj) * g.nx + (T.ci0 + li);
            sx[lj][li] = ax[n];
            sy[lj][li] = ay[n];
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A tile's nodes (with the halo) held in registers, lane-strided as
// stage_tile_wave places them: fetched while the wave still works on the
// previous tile, then written to the wave's LDS tile.
template <class S, typename V>
struct TileRegs {
    static constexpr int N = S::TNX * S::TNY, K = (N + 63) / 64;
    V x[K], y[K];
};

template <class S, typename V>
__device__ __forceinline__ void fetch_tile_regs(const V* __restrict__ ax, const V* __restrict__ ay,
                                                const GridDesc& g, const Tile& T, TileRegs<S, V>& t)
{
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < TileRegs<S, V>::K; k++) {
        const int q = lane + 64 * k;
        const int li = q % S::TNX, lj = q / S::TNX;
        const bool in = q < TileRegs<S, V>::N && li <= T.ncx && lj <= T.ncy;
        const size_t n = in ? (size_t)(T.cj0 + lj) * g.nx + (T.ci0 + li) : 0;
        t.x[k] = ax[n];
        t.y[k] = ay[n];
    }
}

template <class S, typename V>
__device__ __forceinline__ void store_tile_regs(const TileRegs<S, V>& t, const Tile& T, V (*sx)[S::TNX],
                                                V (*sy)[S::TNX])
{
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < TileRegs<S, V>::K; k++) {
        const int q = lane + 64 * k;
        const int li = q % S::TNX, lj = q / S::TNX;
        if (q < TileRegs<S, V>::N && li <= T.ncx && lj <= T.ncy) {
            sx[lj][li] = t.x[k];
            sy[lj][li] = t.y[k];
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sums a wave-uniform count a and a per-lane count b over the workgroup and
// writes them to the workgroup's statistics slot.  All threads must call it.
__device__ __forceinline__ void write_part_sum(unsigned* part, size_t slot, unsigned a, unsigned b,
                                               unsigned (*s)[2])
{
    for (int m = 32; m >= 1; m >>= 1) b += __shfl_xor(b, m, 64);
    if (lane_id() == 0) {
        s[threadIdx.x >> 6][0] = a;
        s[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned sa = 0, sb = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) {
            sa += s[w][0];
            sb += s[w][1];
        }
        part[2 * slot + 0] = sa;
        part[2 * slot + 1] = sb;
    }
}

// Whether the tile's source-plane box [theta_min - r alpha_max, theta_max -
// r alpha_min] (per axis, widened by eb) contains the barycentre (bx, by);
// the box contains every source-plane vertex of the tile.
__device__ __forceinline__ bool tile_box_contains(const GridDesc& g, const Tile& T, const double* rng, double r,
                                                  double eb, double bx, double by)
{
    const double tx0 = node_coord(g.x0, T.ci0, g.h), tx1 = node_coord(g.x0, T.ci0 + T.ncx, g.h);
    const double ty0 = node_coord(g.y0, T.cj0, g.h), ty1 = node_coord(g.y0, T.cj0 + T.ncy, g.h);
    return bx >= tx0 - r * rng[1] - eb && bx <= tx1 - r * rng[0] + eb && by >= ty0 - r * rng[3] - eb &&
           by <= ty1 - r * rng[2] + eb;
}

// All triangles of a staged FP32 tile against one system (mixed path): the
// certified FP32 decision for each, hits and undecided tests appended with
// one atomic per wave.  fr = {r, E_B, bx_hi, bx_lo, by_hi, by_lo} as float;
// an appended key is (hit_base | triangle id) or (flag_base | triangle id).
// NT threads share the tile, a multiple of its width, so a thread keeps its
// column in every pass; the passes' results are kept as bits and the appends
// run only when some thread of the wave has a hit or an undecided test.
template <class S, int NT = 256>
__device__ __forceinline__ void tri32_system(const GridDesc& g, const Tile& T, const float (*sx)[S::TNX],
                                             const float (*sy)[S::TNX], const float* fr,
                                             unsigned long long hit_base, unsigned long long flag_base, int mode,
                                             float tau, unsigned long long* hit_counter,
                                             unsigned long long* hit_keys, long long hit_cap,
                                             unsigned long long* flag_counter, unsigned long long* flag_keys,
                                             long long flag_cap, unsigned& nbbox, int tix = threadIdx.x)
{
    constexpr int IT = S::TX * S::TY / NT;  // cells per thread
    static_assert(NT % S::TX == 0 && IT * 4 <= 64, "column per thread; 4 result bits per cell");
    const float r = fr[0], E = fr[1], bxh = fr[2], bxl = fr[3], byh = fr[4], byl = fr[5];
    const float h32 = (float)g.h;
    const int li = tix % S::TX, lj0 = tix / S::TX;
    const int gi = T.ci0 + li;
    // offsets theta - barycentre in node units (exact hi part), then arcsec
    const float ex0 = (((float)gi - bxh) - bxl) * h32;
    const float ex1 = (((float)(gi + 1) - bxh) - bxl) * h32;
    unsigned long long bits = 0;
#pragma unroll 1
    for (int it = 0; it < IT; it++) {
        const int lj = lj0 + (NT / S::TX) * it;
        const int gj = T.cj0 + lj;
        const float ey0 = (((float)gj - byh) - byl) * h32;
        const float ey1 = (((float)(gj + 1) - byh) - byl) * h32;
        const float d00x = fmaf(-r, sx[lj][li], ex0), d00y = fmaf(-r, sy[lj][li], ey0);
        const float d10x = fmaf(-r, sx[lj][li + 1], ex1), d10y = fmaf(-r, sy[lj][li + 1], ey0);
        const float d01x = fmaf(-r, sx[lj + 1][li], ex0), d01y = fmaf(-r, sy[lj + 1][li], ey1);
        const float d11x = fmaf(-r, sx[lj + 1][li + 1], ex1), d11y = fmaf(-r, sy[lj + 1][li + 1], ey1);
        if (li < T.ncx && lj < T.ncy) {
            const float tx[3] = {d00x, d10x, d01x}, ty[3] = {d00y, d10y, d01y};
            const float ux[3] = {d11x, d01x, d10x}, uy[3] = {d11y, d01y, d10y};
            const int res0 = decide32(tx, ty, E, mode, tau, nbbox);
            const int res1 = decide32(ux, uy, E, mode, tau, nbbox);
            bits |= (unsigned long long)(res0 | (res1 << 2)) << (4 * it);
        }
    }
    if (__ballot(bits != 0) == 0) return;  // the common case: no hit, nothing undecided
#pragma unroll 1
    for (int it = 0; it < IT; it++) {
        const unsigned rb = (unsigned)(bits >> (4 * it)) & 15u;
        const int gj = T.cj0 + lj0 + (NT / S::TX) * it;
        const unsigned tid0 = (unsigned)(2 * (gj * (g.nx - 1) + gi));
        wave_append((rb & 3u) == kHit, hit_base | tid0, hit_counter, hit_keys, hit_cap);
        wave_append((rb >> 2) == kHit, hit_base | (tid0 + 1), hit_counter, hit_keys, hit_cap);
        wave_append((rb & 3u) == kFlag, flag_base | tid0, flag_counter, flag_keys, flag_cap);
        wave_append((rb >> 2) == kFlag, flag_base | (tid0 + 1), flag_counter, flag_keys, flag_cap);
    }
}

// All triangles of a staged FP64 tile against one system (FP64 path): exact
// bounding box, then exact orientation signs; hits kept as bits and appended
// only when some thread of the wave has one (as tri32_system).
template <class S, int NT = 256>
__device__ __forceinline__ void tri64_system(const GridDesc& g, const Tile& T, const double (*sx)[S::TNX],
                                             const double (*sy)[S::TNX], double r, double bx, double by,
                                             unsigned long long hit_base, unsigned long long* hit_counter,
                                             unsigned long long* hit_keys, long long hit_cap, unsigned& nbbox,
                                             int tix = threadIdx.x)
{
    constexpr int IT = S::TX * S::TY / NT;
    static_assert(NT % S::TX == 0 && IT * 2 <= 64, "column per thread; 2 result bits per cell");
    const int li = tix % S::TX, lj0 = tix / S::TX;
    const int gi = T.ci0 + li;
    const double t0x = node_coord(g.x0, gi, g.h), t1x = node_coord(g.x0, gi + 1, g.h);
    unsigned long long bits = 0;
#pragma unroll 1
    for (int it = 0; it < IT; it++) {
        const int lj = lj0 + (NT / S::TX) * it;
        const int gj = T.cj0 + lj;
        if (li < T.ncx && lj < T.ncy) {
            const double t0y = node_coord(g.y0, gj, g.h), t1y = node_coord(g.y0, gj + 1, g.h);
            const double b00x = src_map(t0x, r, sx[lj][li]), b00y = src_map(t0y, r, sy[lj][li]);
            const double b10x = src_map(t1x, r, sx[lj][li + 1]), b10y = src_map(t0y, r, sy[lj][li + 1]);
            const double b01x = src_map(t0x, r, sx[lj + 1][li]), b01y = src_map(t1y, r, sy[lj + 1][li]);
            const double b11x = src_map(t1x, r, sx[lj + 1][li + 1]), b11y = src_map(t1y, r, sy[lj + 1][li + 1]);
            const double vx0[3] = {b00x, b10x, b01x}, vy0[3] = {b00y, b10y, b01y};
            const double vx1[3] = {b11x, b01x, b10x}, vy1[3] = {b11y, b01y, b10y};
            const double lo0 = fmin(vx0[0], fmin(vx0[1], vx0[2])), hi0 = fmax(vx0[0], fmax(vx0[1], vx0[2]));
            const double lo1 = fmin(vy0[0], fmin(vy0[1], vy0[2])), hi1 = fmax(vy0[0], fmax(vy0[1], vy0[2]));
            if (!(bx < lo0 || bx > hi0 || by < lo1 || by > hi1)) {
                nbbox++;
                if (contains_exact(vx0, vy0, bx, by)) bits |= 1ull << (2 * it);
            }
            const double lo2 = fmin(vx1[0], fmin(vx1[1], vx1[2])), hi2 = fmax(vx1[0], fmax(vx1[1], vx1[2]));
            const double lo3 = fmin(vy1[0], fmin(vy1[1], vy1[2])), hi3 = fmax(vy1[0], fmax(vy1[1], vy1[2]));
            if (!(bx < lo2 || bx > hi2 || by < lo3 || by > hi3)) {
                nbbox++;
                if (contains_exact(vx1, vy1, bx, by)) bits |= 2ull << (2 * it);
            }
        }
    }
    if (__ballot(bits != 0) == 0) return;
#pragma unroll 1
    for (int it = 0; it < IT; it++) {
        const int gj = T.cj0 + lj0 + (NT / S::TX) * it;
        const unsigned tid0 = (unsigned)(2 * (gj * (g.nx - 1) + gi));
        wave_append(((bits >> (2 * it)) & 1ull) != 0, hit_base | tid0, hit_counter, hit_keys, hit_cap);
        wave_append(((bits >> (2 * it)) & 2ull) != 0, hit_base | (tid0 + 1), hit_counter, hit_keys, hit_cap);
    }
}

// ---------------------------------------------------------------- FP64 vertices and positions

// FP64 source-plane vertices B_k of triangle `tid` for a system with distance
// ratio r: grad Psi at the three vertices with the potentials spread over the
// wave (fixed butterfly reduction); tx, ty are the image-plane vertices.
__device__ __forceinline__ void vertices64(const double* __restrict__ tab64, int np, GridDesc g, int tid,
                                           double r, double* vx, double* vy, double* tx, double* ty)
{
    int ni[3], nj[3];
    triangle_nodes(g.nx, tid, ni, nj);
    double s[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 3; v++) {
        tx[v] = node_coord(g.x0, ni[v], g.h);
        ty[v] = node_coord(g.y0, nj[v], g.h);
    }
    for (int p = lane_id(); p < np; p += 64) {
        const double* t = tab64 + (size_t)p * T64_STRIDE;
#pragma unroll
        for (int v = 0; v < 3; v++) add_alpha64(t, tx[v], ty[v], s[2 * v], s[2 * v + 1]);
    }
#pragma unroll
    for (int v = 0; v < 3; v++) {
        vx[v] = src_map(tx[v], r, wave_sum(s[2 * v]));
        vy[v] = src_map(ty[v], r, wave_sum(s[2 * v + 1]));
    }
}

// Predicted image position (Sec. 2.2.2, READING: barycentric interpolation):
// image-plane vertices weighted by lambda_k = c_{k+1} / (c_0 + c_1 + c_2),
// c_k = (B_k - p) x (B_{k+1} - p) from the FP64 source-plane triangle.
__device__ __forceinline__ void image_position(const double* vx, const double* vy, const double* tx,
                                               const double* ty, double px, double py, double& ox, double& oy)
{
    double c[3];
#pragma unroll
    for (int v = 0; v < 3; v++) {
        const int w = v == 2 ? 0 : v + 1;
        c[v] = (vx[v] - px) * (vy[w] - py) - (vy[v] - py) * (vx[w] - px);
    }
    const double sum = c[0] + c[1] + c[2];
    const double l0 = c[1] / sum, l1 = c[2] / sum, l2 = c[0] / sum;
    ox = l0 * tx[0] + l1 * tx[1] + l2 * tx[2];
    oy = l0 * ty[0] + l1 * ty[1] + l2 * ty[2];
}

// ---------------------------------------------------------------- hit lists

constexpr int kSortCap = (int)kHitScratch;  // 8192 = 2^13
constexpr int kIdxBits = 13;
constexpr int kTailStage = 1024;            // hits, images and systems staged in LDS

__device__ __forceinline__ int lower_bound_key(const unsigned long long* k, int n, unsigned long long v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (k[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}


}  // namespace lens
