// HIP kernels of the image-plane chi^2 path for gfx950 (MI355X).
//
// One chi^2 evaluation (Rexroth et al. 2019, Sec. 2.2.1-2.2.2, Fig. 1):
//   k_head   per-potential constants (FP64 and FP32 tables), domain checks,
//            observed images -> source plane in FP64; the last workgroup
//            forms the barycentres, the FP32 error bound and one row per
//            system, and resets the counters
//   k_field  deflection at every grid node (FP32 or FP64)          <- the time
//   k_tri    persistent workgroups over tiles of cells: cull (tile, system)
//            pairs, triangle containment, ballot/prefix-sum compaction of hits
//            and of undecided FP32 tests
//   k_fbpos  one wave per item: FP64 re-test of each undecided test (mixed
//            path) and the FP64 image position of every hit
//   k_tail   one workgroup: sort of the hits, matching of observed to
//            predicted images, FP64 chi^2 in a fixed order
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
__device__ __forceinline__ bool last_workgroup(unsigned* ticket, int* s_flag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *s_flag = atomicAdd(ticket, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!*s_flag) return false;
    __threadfence();
    if (threadIdx.x == 0) *ticket = 0;
    return true;
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
    const double c = cos(phi), sn = sin(phi);
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

__device__ void prep_one(const PotPtrs& pot, const GridDesc& g, int p, double* __restrict__ tab64,
                         float* __restrict__ tab32, double* __restrict__ bterm)
{
    double row[T64_STRIDE], K, a1, a2;
    bool ok = row64(pot, p, row, K, a1, a2);
    double* t = tab64 + (size_t)p * T64_STRIDE;
    for (int k = 0; k < T64_STRIDE; k++) t[k] = row[k];
    const double xc = row[T64_XC], yc = row[T64_YC], A = row[T64_A], B = row[T64_B], C = row[T64_C];
    const double a = row[T64_RA], s = pot.r_cut[p];
    const bool sinf = row[T64_SINF] != 0.0;
    const double cxn = (xc - g.x0) / g.h, cyn = (yc - g.y0) / g.h;
    ok = ok && fabs(cxn) < 4194304.0 && fabs(cyn) < 4194304.0;  // |centre| < 2^22 nodes
    const double cxh = rint(cxn), cyh = rint(cyn);
    const double cxl = cxn - cxh, cyl = cyn - cyh;
    const double h2 = g.h * g.h;
    float* u = tab32 + (size_t)p * T32_STRIDE;
    u[T32_CXH] = (float)cxh;
    u[T32_CXL] = (float)cxl;
    u[T32_CYH] = (float)cyh;
    u[T32_CYL] = (float)cyl;
    u[T32_A] = (float)(A * h2);
    u[T32_B] = (float)(B * h2);
    u[T32_C] = (float)(C * h2);
    u[T32_A2] = (float)(a * a);
    u[T32_S2A2] = sinf ? 0.0f : (float)(s * s - a * a);
    u[T32_RA] = (float)a;
    u[T32_RS] = sinf ? 0.0f : (float)s;
    u[T32_K] = (float)(K / g.h);
    u[T32_KIND] = (float)((a == 0.0 ? 2 : 0) + (sinf ? 1 : 0));
    for (int k = T32_KIND + 1; k < T32_STRIDE; k++) u[k] = 0.0f;

    const double w = K * a2 / sqrt(a1);
    const double rho = sqrt(a1) * g.h * sqrt(cxl * cxl + cyl * cyl);
    const double den = a1 * (sqrt(a * a + rho * rho) + a);
    const double J = den > 0.0 ? 2.0 * K * a2 / den : INFINITY;
    // absolute offset error: FP32 rounding of the centre fraction, plus the FP64
    // reference's own rounding of theta - theta_c
    const double span = fabs(g.x0) + fabs(g.y0) + (double)(g.nx + g.ny) * g.h + fabs(xc) + fabs(yc);
    const double derr = g.h * kNodeSplitErr + 4.5e-16 * span;
    bterm[3 * p + 0] = ok ? w : 0.0;
    bterm[3 * p + 1] = ok ? J * derr : 0.0;
    bterm[3 * p + 2] = ok ? 0.0 : 1.0;
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

// Head of every evaluation, one wave per observed image (at least enough
// workgroups of 4 waves for one thread per potential), in two phases:
//  1. every thread with a potential index writes that potential's constants
//     (prep_one); every wave with an observed image j computes its source
//     position beta_ij = theta_ij - r_i grad Psi(theta_ij) in FP64 (Sec. 2.2.2),
//     grad Psi evaluated at the observed position itself from the raw
//     parameters (the same row64 arithmetic as the table), potentials over the
//     lanes;
//  2. the last workgroup to finish reduces the bound terms in a fixed order,
//       E_alpha = u (64 + P) sum_p w_p + sum_p j_p + 1e-9,   u = 2^-24,
//     (64 u w_p bounds the rounding of one potential's FP32 evaluation --
//     about 30 u w_p by operation count, doubled -- (P-1) u W the sequential
//     FP32 sum over potentials, sum_p j_p the Jacobian-amplified absolute
//     offset error), and writes one row per system: barycentre (unweighted
//     mean of its beta_ij), its node-unit split, D_LS/D_OS and the FP32 error
//     bound of source-plane offsets
//       E_B = r E_alpha + 4u Theta + 2u r (W + E_alpha) + 2^-25 h + 1e-9,
//     W = sum_p w_p, Theta = max |theta - barycentre| over the grid; it sets
//     the status from every domain check and zeroes the counters.
__global__ __launch_bounds__(256) void k_head(PotPtrs pot, GridDesc g, ObsPtrs obs, double* __restrict__ tab64,
                                              float* __restrict__ tab32, double* __restrict__ bterm,
                                              double* __restrict__ beta_x, double* __restrict__ beta_y,
                                              double* __restrict__ sysrow, EvalState* __restrict__ st)
{
    __shared__ double sw[256], sj[256], sb[256];
    __shared__ int last, sys_bad;
    const int t = threadIdx.x;
    const int np = pot.n;
    for (int p = blockIdx.x * 256 + t; p < np; p += gridDim.x * 256) prep_one(pot, g, p, tab64, tab32, bterm);
    const int nwaves = gridDim.x * 4;
    for (int j = blockIdx.x * 4 + (t >> 6); j < obs.n_img; j += nwaves) {
        const double t1 = obs.x[j], t2 = obs.y[j];
        double s1 = 0.0, s2 = 0.0;
        for (int p = lane_id(); p < np; p += 64) {
            double row[T64_STRIDE], K, a1, a2;
            row64(pot, p, row, K, a1, a2);
            add_alpha64(row, t1, t2, s1, s2);
        }
        const double a1 = wave_sum(s1), a2 = wave_sum(s2);
        const int s = system_of(obs.sys_off, obs.n_sys, j);
        const double r = obs.dls[s];
        if (lane_id() == 0) {
            beta_x[j] = t1 - r * a1;
            beta_y[j] = t2 - r * a2;
        }
    }
    if (!last_workgroup(&st->head_ticket, &last)) return;

    double w = 0.0, jt = 0.0, bad = 0.0;
    for (int p = t; p < np; p += 256) {
        w += bterm[3 * p + 0];
        jt += bterm[3 * p + 1];
        bad += bterm[3 * p + 2];
    }
    sw[t] = w;
    sj[t] = jt;
    sb[t] = bad;
    if (t == 0) sys_bad = obs.n_sys > 0 && (obs.sys_off[0] != 0 || obs.sys_off[obs.n_sys] != obs.n_img);
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if (t < m) {
            sw[t] += sw[t + m];
            sj[t] += sj[t + m];
            sb[t] += sb[t + m];
        }
        __syncthreads();
    }
    const double W = sw[0];
    const double e_alpha = kU32 * (64.0 + np) * W + sj[0] + 1e-9;
    const double xlo = g.x0, xhi = g.x0 + (g.nx - 1) * g.h, ylo = g.y0, yhi = g.y0 + (g.ny - 1) * g.h;
    for (int s = t; s < obs.n_sys; s += 256) {
        const int j0 = obs.sys_off[s], j1 = obs.sys_off[s + 1];
        bool ok = j0 <= j1 && j0 >= 0 && j1 <= obs.n_img;
        double bx = 0.0, by = 0.0;
        if (ok) {
            for (int j = j0; j < j1; j++) {
                bx += beta_x[j];
                by += beta_y[j];
                ok = ok && obs.sigma[j] > 0.0 && isfinite(obs.sigma[j]) && isfinite(obs.x[j]) && isfinite(obs.y[j]);
            }
            if (j1 > j0) {
                bx /= (j1 - j0);
                by /= (j1 - j0);
            }
        }
        const double r = obs.dls[s];
        ok = ok && isfinite(r) && r >= 0.0;
        const double bxn = (bx - g.x0) / g.h, byn = (by - g.y0) / g.h;
        ok = ok && fabs(bxn) < 4194304.0 && fabs(byn) < 4194304.0;
        const double theta = fmax(fmax(fabs(xlo - bx), fabs(xhi - bx)), fmax(fabs(ylo - by), fabs(yhi - by)));
        const double eb = r * e_alpha + 4.0 * kU32 * theta + 2.0 * kU32 * r * (W + e_alpha) +
                          g.h * kNodeSplitErr + 1e-9;
        double* row = sysrow + (size_t)s * SYS_STRIDE;
        row[SYS_BX] = bx;
        row[SYS_BY] = by;
        row[SYS_BXH] = rint(bxn);
        row[SYS_BXL] = bxn - rint(bxn);
        row[SYS_BYH] = rint(byn);
        row[SYS_BYL] = byn - rint(byn);
        row[SYS_R] = r;
        row[SYS_EB] = eb * (1.0 + 1e-6);
        if (!ok) atomicOr(&sys_bad, 1);
    }
    __syncthreads();
    if (t == 0) {
        st->n_hits = 0;
        st->n_flags = 0;
        st->n_fb_hits = 0;
        st->w_sum = W;
        st->e_alpha = e_alpha;
        st->status = (sb[0] != 0.0 || sys_bad) ? kStatusInvalid : kStatusOk;
    }
}

// ============================================================== deflection field

// FP32 contribution of one potential row `c` (node units) for NPL nodes of a
// row.  KIND selects the radial profile at compile time: bit 0 = no cut
// radius, bit 1 = no core.  f = (B_ - A_) / (A_ B_) with A_ = sqrt(a^2+R^2)+a,
// B_ = sqrt(s^2+R^2)+s; without a cut f = 1/A_; for the singular uncut case
// f = 1/R = rsq(R^2).  Offsets from the centre use the exact hi/lo split
// (see the FP32 table); hardware sqrt/rcp/rsq (1 ulp) are accounted for in
// the error bound.
template <int KIND, int NPL>
__device__ __forceinline__ void field32_pot(const float* __restrict__ c, float fj, const float* fi, float* sx,
                                            float* sy)
{
    const float cxh = c[T32_CXH], cxl = c[T32_CXL], cyh = c[T32_CYH], cyl = c[T32_CYL];
    const float A = c[T32_A], B = c[T32_B], C = c[T32_C];
    const float a2 = c[T32_A2], s2a2 = c[T32_S2A2], ra = c[T32_RA], rs = c[T32_RS], K = c[T32_K];
    const float nyv = (fj - cyh) - cyl;
    const float bny = B * nyv, cny = C * nyv;
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        const float nxv = (fi[k] - cxh) - cxl;
        const float m1 = fmaf(A, nxv, bny);
        const float m2 = fmaf(B, nxv, cny);
        const float qa2 = fmaf(nxv, m1, fmaf(nyv, m2, a2));  // a^2 + R^2 (node units^2 * h^2)
        float f;
        if constexpr (KIND == 0) {          // cored, cut
            const float qa = __builtin_amdgcn_sqrtf(qa2) + ra;
            const float qs = __builtin_amdgcn_sqrtf(qa2 + s2a2) + rs;
            f = (qs - qa) * __builtin_amdgcn_rcpf(qa * qs);
        } else if constexpr (KIND == 1) {   // cored, uncut
            f = __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(qa2) + ra);
        } else if constexpr (KIND == 2) {   // singular, cut
            const float R2 = fmaxf(qa2, 0.0f);
            const float qa = __builtin_amdgcn_sqrtf(R2);
            const float qs = __builtin_amdgcn_sqrtf(R2 + s2a2) + rs;
            f = R2 > 0.0f ? (qs - qa) * __builtin_amdgcn_rcpf(qa * qs) : 0.0f;
        } else {                            // singular isothermal ellipsoid
            const float R2 = fmaxf(qa2, 0.0f);
            f = R2 > 0.0f ? __builtin_amdgcn_rsqf(R2) : 0.0f;
        }
        const float kf = K * f;
        sx[k] = fmaf(kf, m1, sx[k]);
        sy[k] = fmaf(kf, m2, sy[k]);
    }
}

// Each thread owns NPL consecutive nodes of one grid row; a workgroup of 256
// threads covers 256*NPL nodes of that row, so the row offset is uniform and
// every per-potential constant is a wave-uniform (scalar) operand.
template <int NPL>
__global__ __launch_bounds__(256) void k_field32(const float* __restrict__ tab32, int np, int nx, int ny,
                                                 float* __restrict__ ax, float* __restrict__ ay,
                                                 const EvalState* __restrict__ st)
{
    const int j = blockIdx.y;
    const int i0 = (blockIdx.x * 256 + threadIdx.x) * NPL;
    if (i0 >= nx) return;
    const float fj = (float)j;
    float fi[NPL], sx[NPL], sy[NPL];
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        fi[k] = (float)(i0 + k);
        sx[k] = 0.0f;
        sy[k] = 0.0f;
    }
    for (int p = 0; p < np; p++) {
        const float* c = tab32 + (size_t)p * T32_STRIDE;
        const int kind = (int)c[T32_KIND];
        if (kind == 0) field32_pot<0, NPL>(c, fj, fi, sx, sy);
        else if (kind == 1) field32_pot<1, NPL>(c, fj, fi, sx, sy);
        else if (kind == 2) field32_pot<2, NPL>(c, fj, fi, sx, sy);
        else field32_pot<3, NPL>(c, fj, fi, sx, sy);
    }
    const bool bad = st != nullptr && st->status != kStatusOk;
    const size_t row = (size_t)j * nx;
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        if (i0 + k < nx) {
            ax[row + i0 + k] = bad ? __builtin_nanf("") : sx[k];
            ay[row + i0 + k] = bad ? __builtin_nanf("") : sy[k];
        }
    }
}

// FP64 field: one node per thread, the same matrix form in arcsec.
__global__ __launch_bounds__(256) void k_field64(const double* __restrict__ tab64, int np, GridDesc g,
                                                 double* __restrict__ ax, double* __restrict__ ay,
                                                 const EvalState* __restrict__ st)
{
    const int j = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= g.nx) return;
    const double t1 = g.x0 + i * g.h, t2 = g.y0 + j * g.h;
    double s1 = 0.0, s2 = 0.0;
    for (int p = 0; p < np; p++) add_alpha64(tab64 + (size_t)p * T64_STRIDE, t1, t2, s1, s2);
    const bool bad = st != nullptr && st->status != kStatusOk;
    const size_t n = (size_t)j * g.nx + i;
    ax[n] = bad ? __builtin_nan("") : s1;
    ay[n] = bad ? __builtin_nan("") : s2;
}

// ============================================================== triangle stage

constexpr int TX = kTileX, TY = kTileY;    // cells per tile
constexpr int TNX = TX + 1, TNY = TY + 1;   // nodes per tile (one-node halo)
constexpr int TLOADS = (TNX * TNY + 255) / 256;
constexpr int kCellIters = (TX * TY + 255) / 256;  // cells per thread
static_assert(TX * TY % 256 == 0, "a tile is a whole number of cells per thread");
constexpr int SYS_CHUNK = 128;              // systems staged in LDS at a time

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

// Per-system data of one chunk of systems, staged in LDS by the tile kernels.
struct SysChunk {
    double bx[SYS_CHUNK], by[SYS_CHUNK], r[SYS_CHUNK], eb[SYS_CHUNK];
    float f[SYS_CHUNK][6];  // r, E_B, bx_hi, bx_lo, by_hi, by_lo as float
};

__device__ __forceinline__ void load_chunk(SysChunk& c, const double* __restrict__ sysrow, int nsys, int base)
{
    const int t = threadIdx.x;
    const int s = base + t;
    if (t < SYS_CHUNK && s < nsys) {
        const double* row = sysrow + (size_t)s * SYS_STRIDE;
        const double bx = row[SYS_BX], by = row[SYS_BY], r = row[SYS_R], eb = row[SYS_EB];
        c.bx[t] = bx;
        c.by[t] = by;
        c.r[t] = r;
        c.eb[t] = eb;
        c.f[t][0] = (float)r;
        c.f[t][1] = (float)eb;
        c.f[t][2] = (float)row[SYS_BXH];
        c.f[t][3] = (float)row[SYS_BXL];
        c.f[t][4] = (float)row[SYS_BYH];
        c.f[t][5] = (float)row[SYS_BYL];
    }
}

// Tile geometry from a linear tile index.
struct Tile {
    int ci0, cj0, ncx, ncy;
};

__device__ __forceinline__ Tile tile_of(const GridDesc& g, int tiles_x, int tile)
{
    Tile T;
    T.ci0 = (tile % tiles_x) * TX;
    T.cj0 = (tile / tiles_x) * TY;
    T.ncx = min(TX, g.nx - 1 - T.ci0);
    T.ncy = min(TY, g.ny - 1 - T.cj0);
    return T;
}

// Issues every load of a tile's node values (with the one-node halo) into
// registers; nothing waits for them here.
template <typename V>
__device__ __forceinline__ void load_tile(const V* __restrict__ ax, const V* __restrict__ ay, const GridDesc& g,
                                          const Tile& T, V* vx, V* vy)
{
#pragma unroll
    for (int k = 0; k < TLOADS; k++) {
        const int q = threadIdx.x + 256 * k;
        const int li = q % TNX, lj = q / TNX;
        const bool in = q < TNX * TNY && li <= T.ncx && lj <= T.ncy;
        const size_t n = in ? (size_t)(T.cj0 + lj) * g.nx + (T.ci0 + li) : 0;
        vx[k] = in ? ax[n] : V(0);
        vy[k] = in ? ay[n] : V(0);
    }
}

// Stores the registers of a tile to LDS and leaves the tile's deflection range
// (min/max of each component over its nodes) in rng[0..3] for every thread.
// Contains the workgroup barrier that publishes the LDS tile.
template <typename V>
__device__ __forceinline__ void stage_tile(const Tile& T, const V* vx, const V* vy, V (*sx)[TNX], V (*sy)[TNX],
                                           V (*wred)[4], V* rng)
{
    V xmn = V(INFINITY), xmx = V(-INFINITY), ymn = V(INFINITY), ymx = V(-INFINITY);
#pragma unroll
    for (int k = 0; k < TLOADS; k++) {
        const int q = threadIdx.x + 256 * k;
        const int li = q % TNX, lj = q / TNX;
        if (q < TNX * TNY) {
            sx[lj][li] = vx[k];
            sy[lj][li] = vy[k];
            if (li <= T.ncx && lj <= T.ncy) {
                xmn = vx[k] < xmn ? vx[k] : xmn;
                xmx = vx[k] > xmx ? vx[k] : xmx;
                ymn = vy[k] < ymn ? vy[k] : ymn;
                ymx = vy[k] > ymx ? vy[k] : ymx;
            }
        }
    }
    for (int m = 32; m >= 1; m >>= 1) {
        const V a = __shfl_xor(xmn, m, 64), b = __shfl_xor(xmx, m, 64);
        const V c = __shfl_xor(ymn, m, 64), d = __shfl_xor(ymx, m, 64);
        xmn = a < xmn ? a : xmn;
        xmx = b > xmx ? b : xmx;
        ymn = c < ymn ? c : ymn;
        ymx = d > ymx ? d : ymx;
    }
    if (lane_id() == 0) {
        const int w = threadIdx.x >> 6;
        wred[w][0] = xmn;
        wred[w][1] = xmx;
        wred[w][2] = ymn;
        wred[w][3] = ymx;
    }
    __syncthreads();
    rng[0] = wred[0][0];
    rng[1] = wred[0][1];
    rng[2] = wred[0][2];
    rng[3] = wred[0][3];
    for (int w = 1; w < 4; w++) {
        rng[0] = wred[w][0] < rng[0] ? wred[w][0] : rng[0];
        rng[1] = wred[w][1] > rng[1] ? wred[w][1] : rng[1];
        rng[2] = wred[w][2] < rng[2] ? wred[w][2] : rng[2];
        rng[3] = wred[w][3] > rng[3] ? wred[w][3] : rng[3];
    }
}

// Writes the workgroup's statistics to its own slot (no contended atomic).
__device__ __forceinline__ void write_part(unsigned* part, unsigned ntile, unsigned nbbox, unsigned* sbb)
{
    for (int m = 32; m >= 1; m >>= 1) nbbox += __shfl_xor(nbbox, m, 64);
    if (lane_id() == 0) sbb[threadIdx.x >> 6] = nbbox;
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 0] = ntile;
        part[2 * blockIdx.x + 1] = sbb[0] + sbb[1] + sbb[2] + sbb[3];
    }
}

// Mixed path.  Persistent workgroups (4 waves) walk the tiles of TX x TY
// cells; the loads of the next tile are in flight while the current one is
// processed.  A tile's FP32 deflections (with a one-node halo) are staged in
// LDS.  The box [theta_min - r alpha_max, theta_max - r alpha_min] (per axis,
// widened by E_B) contains every source-plane vertex of the tile, so a system
// whose barycentre lies outside it is skipped for the whole tile.  Systems
// are tested 64 at a time, one per lane, and the survivors enumerated from
// the ballot mask.
__global__ __launch_bounds__(256) void k_tri32(const float* __restrict__ ax, const float* __restrict__ ay,
                                               GridDesc g, int tiles_x, int n_tiles, int nsys,
                                               const double* __restrict__ sysrow, EvalState* __restrict__ st,
                                               int mode, float tau, unsigned long long* __restrict__ hit_keys,
                                               long long hit_cap, unsigned long long* __restrict__ flag_keys,
                                               long long flag_cap, unsigned* __restrict__ part)
{
    __shared__ float sx[TNY][TNX], sy[TNY][TNX];
    __shared__ float wred[4][4];
    __shared__ SysChunk chunk;
    __shared__ unsigned sbb[4];
    const bool one_chunk = nsys <= SYS_CHUNK;
    if (one_chunk) load_chunk(chunk, sysrow, nsys, 0);
    const float h32 = (float)g.h;
    const int lane = lane_id();
    unsigned nbbox = 0, ntile = 0;
    float vx[TLOADS], vy[TLOADS];
    int tile = blockIdx.x;
    Tile T = tile_of(g, tiles_x, tile);
    if (tile < n_tiles) load_tile(ax, ay, g, T, vx, vy);
    for (; tile < n_tiles; tile += gridDim.x) {
        float rng[4];
        stage_tile(T, vx, vy, sx, sy, wred, rng);
        const Tile cur = T;
        const int next = tile + gridDim.x;
        if (next < n_tiles) {
            T = tile_of(g, tiles_x, next);
            load_tile(ax, ay, g, T, vx, vy);
        }
        const double tx0 = g.x0 + cur.ci0 * g.h, tx1 = g.x0 + (cur.ci0 + cur.ncx) * g.h;
        const double ty0 = g.y0 + cur.cj0 * g.h, ty1 = g.y0 + (cur.cj0 + cur.ncy) * g.h;
        const double xmn = rng[0], xmx = rng[1], ymn = rng[2], ymx = rng[3];
        for (int cbase = 0; cbase < nsys; cbase += SYS_CHUNK) {
            if (!one_chunk) {
                __syncthreads();
                load_chunk(chunk, sysrow, nsys, cbase);
                __syncthreads();
            }
            const int nc = min(SYS_CHUNK, nsys - cbase);
            for (int sbase = 0; sbase < nc; sbase += 64) {
                const int sl = sbase + lane;
                bool pass = false;
                if (sl < nc) {
                    const double r = chunk.r[sl], eb = chunk.eb[sl], bx = chunk.bx[sl], by = chunk.by[sl];
                    pass = bx >= tx0 - r * xmx - eb && bx <= tx1 - r * xmn + eb && by >= ty0 - r * ymx - eb &&
                           by <= ty1 - r * ymn + eb;
                }
                unsigned long long m = __ballot(pass);
                ntile += __popcll(m);
                while (m) {
                    const int sb = __ffsll((long long)m) - 1;
                    m &= m - 1;
                    const int s = sbase + sb;
                    const int sys = cbase + s;
                    const float r = chunk.f[s][0], E = chunk.f[s][1];
                    const float bxh = chunk.f[s][2], bxl = chunk.f[s][3], byh = chunk.f[s][4], byl = chunk.f[s][5];
#pragma unroll
                    for (int it = 0; it < kCellIters; it++) {
                        const int cidx = threadIdx.x + 256 * it;
                        const int li = cidx % TX, lj = cidx / TX;
                        const bool valid = li < cur.ncx && lj < cur.ncy;
                        const int gi = cur.ci0 + li, gj = cur.cj0 + lj;
                        // offsets theta - barycentre in node units (exact hi part), then arcsec
                        const float ex0 = (((float)gi - bxh) - bxl) * h32;
                        const float ex1 = (((float)(gi + 1) - bxh) - bxl) * h32;
                        const float ey0 = (((float)gj - byh) - byl) * h32;
                        const float ey1 = (((float)(gj + 1) - byh) - byl) * h32;
                        const float d00x = fmaf(-r, sx[lj][li], ex0), d00y = fmaf(-r, sy[lj][li], ey0);
                        const float d10x = fmaf(-r, sx[lj][li + 1], ex1), d10y = fmaf(-r, sy[lj][li + 1], ey0);
                        const float d01x = fmaf(-r, sx[lj + 1][li], ex0), d01y = fmaf(-r, sy[lj + 1][li], ey1);
                        const float d11x = fmaf(-r, sx[lj + 1][li + 1], ex1);
                        const float d11y = fmaf(-r, sy[lj + 1][li + 1], ey1);
                        int res0 = kMiss, res1 = kMiss;
                        if (valid) {
                            const float tx[3] = {d00x, d10x, d01x}, ty[3] = {d00y, d10y, d01y};
                            const float ux[3] = {d11x, d01x, d10x}, uy[3] = {d11y, d01y, d10y};
                            res0 = decide32(tx, ty, E, mode, tau, nbbox);
                            res1 = decide32(ux, uy, E, mode, tau, nbbox);
                        }
                        const int tid0 = 2 * (gj * (g.nx - 1) + gi);
                        wave_append(res0 == kHit, hit_key(sys, tid0), &st->n_hits, hit_keys, hit_cap);
                        wave_append(res1 == kHit, hit_key(sys, tid0 + 1), &st->n_hits, hit_keys, hit_cap);
                        wave_append(res0 == kFlag, hit_key(sys, tid0), &st->n_flags, flag_keys, flag_cap);
                        wave_append(res1 == kFlag, hit_key(sys, tid0 + 1), &st->n_flags, flag_keys, flag_cap);
                    }
                }
            }
        }
        __syncthreads();  // the LDS tile is overwritten by the next iteration
    }
    write_part(part, ntile, nbbox, sbb);
}

// FP64 path: same walk, FP64 deflections in LDS, every surviving triangle
// decided exactly (exact bounding box, then exact orientation signs).
__global__ __launch_bounds__(256) void k_tri64(const double* __restrict__ ax, const double* __restrict__ ay,
                                               GridDesc g, int tiles_x, int n_tiles, int nsys,
                                               const double* __restrict__ sysrow, EvalState* __restrict__ st,
                                               unsigned long long* __restrict__ hit_keys, long long hit_cap,
                                               unsigned* __restrict__ part)
{
    __shared__ double sx[TNY][TNX], sy[TNY][TNX];
    __shared__ double wred[4][4];
    __shared__ SysChunk chunk;
    __shared__ unsigned sbb[4];
    const bool one_chunk = nsys <= SYS_CHUNK;
    if (one_chunk) load_chunk(chunk, sysrow, nsys, 0);
    const int lane = lane_id();
    unsigned nbbox = 0, ntile = 0;
    double vx[TLOADS], vy[TLOADS];
    int tile = blockIdx.x;
    Tile T = tile_of(g, tiles_x, tile);
    if (tile < n_tiles) load_tile(ax, ay, g, T, vx, vy);
    for (; tile < n_tiles; tile += gridDim.x) {
        double rng[4];
        stage_tile(T, vx, vy, sx, sy, wred, rng);
        const Tile cur = T;
        const int next = tile + gridDim.x;
        if (next < n_tiles) {
            T = tile_of(g, tiles_x, next);
            load_tile(ax, ay, g, T, vx, vy);
        }
        const double tx0 = g.x0 + cur.ci0 * g.h, tx1 = g.x0 + (cur.ci0 + cur.ncx) * g.h;
        const double ty0 = g.y0 + cur.cj0 * g.h, ty1 = g.y0 + (cur.cj0 + cur.ncy) * g.h;
        for (int cbase = 0; cbase < nsys; cbase += SYS_CHUNK) {
            if (!one_chunk) {
                __syncthreads();
                load_chunk(chunk, sysrow, nsys, cbase);
                __syncthreads();
            }
            const int nc = min(SYS_CHUNK, nsys - cbase);
            for (int sbase = 0; sbase < nc; sbase += 64) {
                const int sl = sbase + lane;
                bool pass = false;
                if (sl < nc) {
                    const double r = chunk.r[sl], bx = chunk.bx[sl], by = chunk.by[sl];
                    const double eb = 1e-9;  // FP64 rounding of the box, far below this margin
                    pass = bx >= tx0 - r * rng[1] - eb && bx <= tx1 - r * rng[0] + eb &&
                           by >= ty0 - r * rng[3] - eb && by <= ty1 - r * rng[2] + eb;
                }
                unsigned long long m = __ballot(pass);
                ntile += __popcll(m);
                while (m) {
                    const int sb = __ffsll((long long)m) - 1;
                    m &= m - 1;
                    const int s = sbase + sb;
                    const int sys = cbase + s;
                    const double r = chunk.r[s], bx = chunk.bx[s], by = chunk.by[s];
#pragma unroll 1
                    for (int it = 0; it < kCellIters; it++) {
                        const int cidx = threadIdx.x + 256 * it;
                        const int li = cidx % TX, lj = cidx / TX;
                        const bool valid = li < cur.ncx && lj < cur.ncy;
                        const int gi = cur.ci0 + li, gj = cur.cj0 + lj;
                        bool h0 = false, h1 = false;
                        if (valid) {
                            const double t0x = g.x0 + gi * g.h, t1x = g.x0 + (gi + 1) * g.h;
                            const double t0y = g.y0 + gj * g.h, t1y = g.y0 + (gj + 1) * g.h;
                            const double b00x = t0x - r * sx[lj][li], b00y = t0y - r * sy[lj][li];
                            const double b10x = t1x - r * sx[lj][li + 1], b10y = t0y - r * sy[lj][li + 1];
                            const double b01x = t0x - r * sx[lj + 1][li], b01y = t1y - r * sy[lj + 1][li];
                            const double b11x = t1x - r * sx[lj + 1][li + 1], b11y = t1y - r * sy[lj + 1][li + 1];
                            const double vx0[3] = {b00x, b10x, b01x}, vy0[3] = {b00y, b10y, b01y};
                            const double vx1[3] = {b11x, b01x, b10x}, vy1[3] = {b11y, b01y, b10y};
                            const double lo0 = fmin(vx0[0], fmin(vx0[1], vx0[2]));
                            const double hi0 = fmax(vx0[0], fmax(vx0[1], vx0[2]));
                            const double lo1 = fmin(vy0[0], fmin(vy0[1], vy0[2]));
                            const double hi1 = fmax(vy0[0], fmax(vy0[1], vy0[2]));
                            if (!(bx < lo0 || bx > hi0 || by < lo1 || by > hi1)) {
                                nbbox++;
                                h0 = contains_exact(vx0, vy0, bx, by);
                            }
                            const double lo2 = fmin(vx1[0], fmin(vx1[1], vx1[2]));
                            const double hi2 = fmax(vx1[0], fmax(vx1[1], vx1[2]));
                            const double lo3 = fmin(vy1[0], fmin(vy1[1], vy1[2]));
                            const double hi3 = fmax(vy1[0], fmax(vy1[1], vy1[2]));
                            if (!(bx < lo2 || bx > hi2 || by < lo3 || by > hi3)) {
                                nbbox++;
                                h1 = contains_exact(vx1, vy1, bx, by);
                            }
                        }
                        const int tid0 = 2 * (gj * (g.nx - 1) + gi);
                        wave_append(h0, hit_key(sys, tid0), &st->n_hits, hit_keys, hit_cap);
                        wave_append(h1, hit_key(sys, tid0 + 1), &st->n_hits, hit_keys, hit_cap);
                    }
                }
            }
        }
        __syncthreads();
    }
    write_part(part, ntile, nbbox, sbb);
}

// ============================================================== FP64 fallback and positions

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
        tx[v] = g.x0 + ni[v] * g.h;
        ty[v] = g.y0 + nj[v] * g.h;
    }
    for (int p = lane_id(); p < np; p += 64) {
        const double* t = tab64 + (size_t)p * T64_STRIDE;
#pragma unroll
        for (int v = 0; v < 3; v++) add_alpha64(t, tx[v], ty[v], s[2 * v], s[2 * v + 1]);
    }
#pragma unroll
    for (int v = 0; v < 3; v++) {
        vx[v] = tx[v] - r * wave_sum(s[2 * v]);
        vy[v] = ty[v] - r * wave_sum(s[2 * v + 1]);
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

// ---------------------------------------------------------------- fallback and positions

constexpr int kSortCap = (int)kHitScratch;  // 8192 = 2^13
constexpr int kIdxBits = 13;
constexpr int kTailStage = 1024;            // hits, images and systems staged in LDS

// Persistent waves over the items [certain hits..., undecided tests...]:
// the position of every certain hit goes to pos[item]; each undecided test is
// decided exactly on its FP64 vertices and, if it is a hit, appended with its
// position to the fallback list.
__global__ __launch_bounds__(256) void k_fbpos(const double* __restrict__ tab64, int np, GridDesc g,
                                               const double* __restrict__ sysrow, EvalState* __restrict__ st,
                                               const unsigned long long* __restrict__ hit_keys, long long hit_cap,
                                               const unsigned long long* __restrict__ flag_keys, long long flag_cap,
                                               unsigned long long* __restrict__ fb_keys, long long fb_cap,
                                               double* __restrict__ pos, double* __restrict__ fb_pos)
{
    if (st->status != kStatusOk) return;
    const long long nwaves = (long long)gridDim.x * (blockDim.x >> 6);
    const long long w0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nc = (long long)min((unsigned long long)hit_cap, st->n_hits);
    const long long nf = (long long)min((unsigned long long)flag_cap, st->n_flags);
    for (long long item = w0; item < nc + nf; item += nwaves) {
        const bool flagged = item >= nc;
        const unsigned long long key = flagged ? flag_keys[item - nc] : hit_keys[item];
        const int sys = (int)(key >> 32), tid = (int)(key & 0xffffffffu);
        const double* row = sysrow + (size_t)sys * SYS_STRIDE;
        double vx[3], vy[3], tx[3], ty[3];
        vertices64(tab64, np, g, tid, row[SYS_R], vx, vy, tx, ty);
        if (lane_id() == 0) {
            const double px = row[SYS_BX], py = row[SYS_BY];
            if (!flagged) {
                image_position(vx, vy, tx, ty, px, py, pos[2 * item], pos[2 * item + 1]);
            } else if (contains_exact(vx, vy, px, py)) {
                const unsigned long long slot = atomicAdd(&st->n_fb_hits, 1ull);
                if ((long long)slot < fb_cap) {
                    fb_keys[slot] = key;
                    image_position(vx, vy, tx, ty, px, py, fb_pos[2 * slot], fb_pos[2 * slot + 1]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------- tail

__device__ __forceinline__ int lower_bound_key(const unsigned long long* k, int n, unsigned long long v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (k[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}


// One workgroup of 1024 threads after every hit is known.  Merges the certain
// and the fallback hits, sorts them by (system, triangle id) -- rank sort of
// packed keys (system << 44 | triangle id << 13 | source index) for up to 1024
// hits, bitonic sort beyond -- and writes the sorted (system, id) pairs with
// their positions.  Each observed image is paired with the nearest predicted
// image of its system (ties to the lower triangle id), chi2_i = sum_j
// |x_obs - x|^2 / sigma^2 in image order, +inf without any predicted image,
// and chi^2 = sum_i chi2_i in a fixed order (Sec. 2.2.1).  Two rounds of
// independent global loads (the counters, then every key, position and
// observation at once); everything after that works in LDS.  Reports capacity
// overflow of any list.
__global__ __launch_bounds__(1024) void k_tail(ObsPtrs obs, EvalState* __restrict__ st, long long hit_cap,
                                               long long flag_cap, long long fb_cap, int hit_capacity,
                                               const unsigned long long* __restrict__ hit_keys,
                                               const unsigned long long* __restrict__ fb_keys,
                                               const double* __restrict__ pos, const double* __restrict__ fb_pos,
                                               int* __restrict__ out_hits, double* __restrict__ img_xy,
                                               int* __restrict__ n_pred, double* __restrict__ contrib,
                                               double* __restrict__ chi2, double* __restrict__ chi2_sys,
                                               int* __restrict__ match, long long* __restrict__ stats,
                                               long long n_tests, const unsigned* __restrict__ part, int n_parts)
{
    __shared__ unsigned long long key[kSortCap];
    __shared__ double upx[kTailStage], upy[kTailStage];  // positions in unsorted order
    __shared__ double sox[kTailStage], soy[kTailStage], ssg[kTailStage], scon[kTailStage];
    __shared__ int soff[kTailStage + 1];
    __shared__ int sfirst[kTailStage], send[kTailStage];
    __shared__ double scs[kTailStage];
    __shared__ unsigned long long s_tile, s_bbox;
    const int t = threadIdx.x;
    const int nimg = obs.n_img, nsys = obs.n_sys;
    const bool staged = nimg <= kTailStage && nsys <= kTailStage;
    // round 1: counters, statistics partials, observations (all independent)
    const unsigned long long nc = st->n_hits, nf = st->n_flags, nfb = st->n_fb_hits;
    const int status0 = st->status;
    unsigned long long pt = 0, pb = 0;
    for (int q = t; q < n_parts; q += 1024) {
        pt += part[2 * q];
        pb += part[2 * q + 1];
    }
    if (staged) {
        if (t < nimg) {
            sox[t] = obs.x[t];
            soy[t] = obs.y[t];
            ssg[t] = obs.sigma[t];
        }
        if (t <= nsys) soff[t] = obs.sys_off[t];
        if (t < nsys) {
            sfirst[t] = 0;
            send[t] = 0;
        }
    }
    if (t == 0) {
        s_tile = 0;
        s_bbox = 0;
    }
    __syncthreads();
    if (pt) atomicAdd(&s_tile, pt);
    if (pb) atomicAdd(&s_bbox, pb);
    const unsigned long long total = nc + nfb;
    const bool over = nc > (unsigned long long)hit_cap || nf > (unsigned long long)flag_cap ||
                      nfb > (unsigned long long)fb_cap || total > (unsigned long long)hit_capacity ||
                      total > (unsigned long long)kSortCap;
    const int status = (status0 == kStatusOk && over) ? kStatusCapacity : status0;
    const int n = status == kStatusOk ? (int)total : 0, ncert = (int)nc;
    const bool fast = staged && n <= kTailStage;
    // round 2: keys and positions
    int npad = 1;
    while (npad < n) npad <<= 1;
    for (int q = t; q < npad; q += 1024) {
        unsigned long long k = ~0ull;
        if (q < n) {
            const unsigned long long h = q < ncert ? hit_keys[q] : fb_keys[q - ncert];
            k = ((h >> 32) << 44) | ((h & 0x7fffffffull) << kIdxBits) | (unsigned long long)q;
            if (fast) {
                const double* src = q < ncert ? pos + 2 * q : fb_pos + 2 * (q - ncert);
                upx[q] = src[0];
                upy[q] = src[1];
            }
        }
        key[q] = k;
    }
    __syncthreads();
    if (t == 0) {
        st->status = status;
        stats[0] = (long long)total;
        stats[1] = (long long)nf;
        stats[2] = (long long)s_tile;
        stats[3] = (long long)s_bbox;
        stats[4] = status;
        stats[5] = (long long)nfb;
        stats[6] = n_tests;
        stats[7] = 0;
    }
    if (status != kStatusOk) {
        for (int s = t; s < nsys; s += 1024) {
            chi2_sys[s] = __builtin_nan("");
            n_pred[s] = 0;
        }
        for (int j = t; j < nimg; j += 1024)
            if (match) match[j] = -1;
        if (t == 0) chi2[0] = __builtin_nan("");
        return;
    }
    if (n <= 1024) {
        // rank sort (keys are unique): one barrier instead of log^2 of them
        unsigned long long mine = 0;
        int rank = 0;
        if (t < n) {
            mine = key[t];
            int q = 0;
            for (; q + 8 <= n; q += 8) {
#pragma unroll
                for (int u = 0; u < 8; u++) rank += key[q + u] < mine;
            }
            for (; q < n; q++) rank += key[q] < mine;
        }
        __syncthreads();
        if (t < n) key[rank] = mine;
        __syncthreads();
    } else {
        for (int size = 2; size <= npad; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int q = t; q < npad / 2; q += 1024) {
                    const int lo = 2 * q - (q & (stride - 1));
                    const int hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const unsigned long long a = key[lo], b = key[hi];
                    if ((a > b) == up) {
                        key[lo] = b;
                        key[hi] = a;
                    }
                }
                __syncthreads();
            }
        }
    }
    if (fast) {
        // sorted output, and the [first, end) range of every system from the
        // boundaries of the sorted list
        if (t < n) {
            const unsigned long long k = key[t];
            const int idx = (int)(k & ((1ull << kIdxBits) - 1));
            const int s = (int)(k >> 44);
            out_hits[2 * t + 0] = s;
            out_hits[2 * t + 1] = (int)((k >> kIdxBits) & 0x7fffffffull);
            img_xy[2 * t + 0] = upx[idx];
            img_xy[2 * t + 1] = upy[idx];
            if (t == 0 || (int)(key[t - 1] >> 44) != s) sfirst[s] = t;
            if (t == n - 1 || (int)(key[t + 1] >> 44) != s) send[s] = t + 1;
        }
        __syncthreads();
        if (t < nimg) {
            int lo = 0, hi = nsys - 1;  // system of image t
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (soff[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int q0 = sfirst[lo], q1 = send[lo];
            int best = -1;
            double bd = 0.0;
            for (int q = q0; q < q1; q++) {
                const int idx = (int)(key[q] & ((1ull << kIdxBits) - 1));
                const double dx = sox[t] - upx[idx], dy = soy[t] - upy[idx];
                const double d2 = dx * dx + dy * dy;
                if (best < 0 || d2 < bd) {
                    best = q;
                    bd = d2;
                }
            }
            if (match) match[t] = best;
            scon[t] = best >= 0 ? bd / (ssg[t] * ssg[t]) : 0.0;
        }
        __syncthreads();
        if (t < nsys) {
            const int q0 = sfirst[t], q1 = send[t];
            double cs = 0.0;
            for (int j = soff[t]; j < soff[t + 1]; j++) cs += scon[j];
            cs = q1 > q0 ? cs : INFINITY;
            chi2_sys[t] = cs;
            n_pred[t] = q1 - q0;
            scs[t] = cs;
        }
        __syncthreads();
        if (t < 64) {  // one wave: fixed-order sum over the systems
            double v = 0.0;
            for (int s = t; s < nsys; s += 64) v += scs[s];
            v = wave_sum(v);
            if (t == 0) chi2[0] = v;
        }
        return;
    }
    // general path (more than 1024 hits, images or systems): global operands
    for (int q = t; q < n; q += 1024) {
        const unsigned long long k = key[q];
        const int idx = (int)(k & ((1ull << kIdxBits) - 1));
        out_hits[2 * q + 0] = (int)(k >> 44);
        out_hits[2 * q + 1] = (int)((k >> kIdxBits) & 0x7fffffffull);
        const double* src = idx < ncert ? pos + 2 * idx : fb_pos + 2 * (idx - ncert);
        img_xy[2 * q + 0] = src[0];
        img_xy[2 * q + 1] = src[1];
    }
    __syncthreads();
    for (int j = t; j < nimg; j += 1024) {
        const int s = system_of(obs.sys_off, nsys, j);
        const int q0 = lower_bound_key(key, n, (unsigned long long)s << 44);
        const int q1 = lower_bound_key(key, n, (unsigned long long)(s + 1) << 44);
        int best = -1;
        double bd = 0.0;
        for (int q = q0; q < q1; q++) {
            const double dx = obs.x[j] - img_xy[2 * q], dy = obs.y[j] - img_xy[2 * q + 1];
            const double d2 = dx * dx + dy * dy;
            if (best < 0 || d2 < bd) {
                best = q;
                bd = d2;
            }
        }
        if (match) match[j] = best;
        contrib[j] = best >= 0 ? bd / (obs.sigma[j] * obs.sigma[j]) : 0.0;
    }
    __syncthreads();
    for (int s = t; s < nsys; s += 1024) {
        const int q0 = lower_bound_key(key, n, (unsigned long long)s << 44);
        const int q1 = lower_bound_key(key, n, (unsigned long long)(s + 1) << 44);
        double cs = 0.0;
        for (int j = obs.sys_off[s]; j < obs.sys_off[s + 1]; j++) cs += contrib[j];
        chi2_sys[s] = q1 > q0 ? cs : INFINITY;
        n_pred[s] = q1 - q0;
    }
    __syncthreads();
    if (t < 64) {
        double v = 0.0;
        for (int s = t; s < nsys; s += 64) v += chi2_sys[s];
        v = wave_sum(v);
        if (t == 0) chi2[0] = v;
    }
}

// ============================================================== cosmology

// D_LS / D_OS in a flat universe, one workgroup per source: composite Simpson
// quadrature of 1/E(z) for the comoving distances to the lens and the source,
// (chi_s - chi_l) / chi_s; fixed-order reduction.
__device__ double comoving_block(double z, double om, double ol, double* red)
{
    const int n = 1 << 18;  // even number of panels
    const double h = z / n;
    double s = 0.0;
    for (int k = threadIdx.x; k <= n; k += blockDim.x) {
        const double a = 1.0 + k * h;
        const double f = 1.0 / sqrt(om * a * a * a + ol);
        const double wgt = (k == 0 || k == n) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
        s += wgt * f;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int m = blockDim.x >> 1; m >= 1; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    const double out = red[0] * h / 3.0;
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(256) void k_dls(double zl, const double* __restrict__ zs, int n, double om, double ol,
                                             double* __restrict__ out)
{
    __shared__ double red[256];
    const int s = blockIdx.x;
    if (s >= n) return;
    const double z = zs[s];
    const double cl = comoving_block(zl, om, ol, red);
    const double cs = comoving_block(z, om, ol, red);
    if (threadIdx.x == 0) out[s] = z > zl ? (cs - cl) / cs : 0.0;
}

// ============================================================== exports

__global__ void k_export(const double* __restrict__ sysrow, int nsys, const EvalState* __restrict__ st,
                         double* __restrict__ bar_x, double* __restrict__ bar_y, int* __restrict__ status)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0 && status) *status = st->status;
    if (s < nsys && bar_x) {
        bar_x[s] = sysrow[(size_t)s * SYS_STRIDE + SYS_BX];
        bar_y[s] = sysrow[(size_t)s * SYS_STRIDE + SYS_BY];
    }
}

// ============================================================== launchers

static inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

static inline unsigned clampu(long long v, long long lo, long long hi) { return (unsigned)(v < lo ? lo : v > hi ? hi : v); }

hipError_t launch_head(const PotPtrs& pot, const GridDesc& g, const ObsPtrs& obs, double* tab64, float* tab32,
                       double* bterm, double* bx, double* by, double* sysrow, EvalState* st, hipStream_t s)
{
    long long nb = cdiv(obs.n_img, 4);
    if (nb < cdiv(pot.n, 256)) nb = cdiv(pot.n, 256);
    k_head<<<clampu(nb, 1, 1024), 256, 0, s>>>(pot, g, obs, tab64, tab32, bterm, bx, by, sysrow, st);
    return hipGetLastError();
}

hipError_t launch_field32(const float* tab32, int np, const GridDesc& g, float* ax, float* ay,
                          const EvalState* st, int npl, hipStream_t s)
{
    switch (npl) {
    case 1: k_field32<1><<<dim3(cdiv(g.nx, 256), g.ny), 256, 0, s>>>(tab32, np, g.nx, g.ny, ax, ay, st); break;
    case 2: k_field32<2><<<dim3(cdiv(g.nx, 512), g.ny), 256, 0, s>>>(tab32, np, g.nx, g.ny, ax, ay, st); break;
    case 4: k_field32<4><<<dim3(cdiv(g.nx, 1024), g.ny), 256, 0, s>>>(tab32, np, g.nx, g.ny, ax, ay, st); break;
    default: k_field32<8><<<dim3(cdiv(g.nx, 2048), g.ny), 256, 0, s>>>(tab32, np, g.nx, g.ny, ax, ay, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_field64(const double* tab64, int np, const GridDesc& g, double* ax, double* ay,
                          const EvalState* st, hipStream_t s)
{
    k_field64<<<dim3(cdiv(g.nx, 256), g.ny), 256, 0, s>>>(tab64, np, g, ax, ay, st);
    return hipGetLastError();
}

int tri_blocks(const GridDesc& g)
{
    const long long n_tiles = (long long)cdiv(g.nx - 1, TX) * cdiv(g.ny - 1, TY);
    return (int)(n_tiles < kTriBlocks ? n_tiles : kTriBlocks);
}

hipError_t launch_tri32(const float* ax, const float* ay, const GridDesc& g, int nsys, const double* sysrow,
                        EvalState* st, int mode, float tau, unsigned long long* hit_keys, long long hit_cap,
                        unsigned long long* flag_keys, long long flag_cap, unsigned* part, hipStream_t s)
{
    const int tiles_x = (int)cdiv(g.nx - 1, TX);
    const int n_tiles = tiles_x * (int)cdiv(g.ny - 1, TY);
    k_tri32<<<tri_blocks(g), 256, 0, s>>>(ax, ay, g, tiles_x, n_tiles, nsys, sysrow, st, mode, tau, hit_keys,
                                          hit_cap, flag_keys, flag_cap, part);
    return hipGetLastError();
}

hipError_t launch_tri64(const double* ax, const double* ay, const GridDesc& g, int nsys, const double* sysrow,
                        EvalState* st, unsigned long long* hit_keys, long long hit_cap, unsigned* part,
                        hipStream_t s)
{
    const int tiles_x = (int)cdiv(g.nx - 1, TX);
    const int n_tiles = tiles_x * (int)cdiv(g.ny - 1, TY);
    k_tri64<<<tri_blocks(g), 256, 0, s>>>(ax, ay, g, tiles_x, n_tiles, nsys, sysrow, st, hit_keys, hit_cap, part);
    return hipGetLastError();
}

hipError_t launch_fbpos(const double* tab64, int np, const GridDesc& g, const double* sysrow, EvalState* st,
                        const unsigned long long* hit_keys, long long hit_cap, const unsigned long long* flag_keys,
                        long long flag_cap, unsigned long long* fb_keys, long long fb_cap, double* pos,
                        double* fb_pos, hipStream_t s)
{
    k_fbpos<<<256, 256, 0, s>>>(tab64, np, g, sysrow, st, hit_keys, hit_cap, flag_keys, flag_cap, fb_keys, fb_cap,
                                pos, fb_pos);
    return hipGetLastError();
}

hipError_t launch_tail(const TailLaunch& tl, EvalState* st, const unsigned long long* fb_keys, const double* pos,
                       const double* fb_pos, hipStream_t s)
{
    k_tail<<<1, 1024, 0, s>>>(tl.obs, st, tl.hit_cap, tl.flag_cap, tl.fb_cap, tl.hit_capacity, tl.hit_keys, fb_keys,
                              pos, fb_pos, tl.out_hits, tl.img_xy, tl.n_pred, tl.contrib, tl.chi2, tl.chi2_sys,
                              tl.match, tl.stats, tl.n_tests, tl.part, tl.n_parts);
    return hipGetLastError();
}

hipError_t launch_dls(double zl, const double* zs, int n, double om, double ol, double* out, hipStream_t s)
{
    if (n > 0) k_dls<<<n, 256, 0, s>>>(zl, zs, n, om, ol, out);
    return hipGetLastError();
}

hipError_t launch_export(const double* sysrow, int nsys, const EvalState* st, double* bar_x, double* bar_y,
                         int* status, hipStream_t s)
{
    k_export<<<cdiv(nsys > 0 ? nsys : 1, 256), 256, 0, s>>>(sysrow, nsys, st, bar_x, bar_y, status);
    return hipGetLastError();
}

}  // namespace lens
