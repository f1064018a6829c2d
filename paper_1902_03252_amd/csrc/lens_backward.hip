// Backward form of the deflection model on gfx950: vector-Jacobian products of
// the deflection gradient with respect to the seven parameters of every
// potential, and the source-plane chi^2 with its gradient.
//
// The paper (Rexroth et al. 2019) has no derivatives; these are the analytic
// derivatives of the deflection of Algorithm 1 generalised to the cored/cut
// profile (Sec. 2.2.2 and Sec. 5), in the matrix form used by the forward
// kernels:
//     d = theta - c,  m = M d,  R^2 = d . m,  alpha = K f(R) m,
//     M = [[A, B], [B, C]] = Rot(Phi) diag(1-eps, 1+eps) Rot(-Phi),
//     f = 1/(qa + a) - 1/(qs + s),  qa = sqrt(a^2 + R^2),  qs = sqrt(s^2 + R^2),
//     K = b0 s/(s - a),  b0 = 4 pi (sigma_v/c)^2.
// With F' = df/d(R^2) = -1/(2 qa (qa+a)^2) + 1/(2 qs (qs+s)^2) and a cotangent
// g, the product g . d alpha/dq is
//     (dK/dq f + K df/dq|_R + K F' dR^2/dq) (g . m) + K f (g . dm/dq)
// where, per parameter:
//     x_c:  dR^2 = -2 m_1,      dm = -(A, B)
//     y_c:  dR^2 = -2 m_2,      dm = -(B, C)
//     eps:  dM = [[-cos 2Phi, -sin 2Phi], [-sin 2Phi, cos 2Phi]],   dR^2 = d.dM d, dm = dM d
//     Phi:  dM = 2 eps [[sin 2Phi, -cos 2Phi], [-cos 2Phi, -sin 2Phi]]
//     a:    dK = K/(s-a),        df = -1/(qa (qa+a))
//     s:    dK = -K a/(s (s-a)), df = 1/(qs (qs+s))          (0 for s = inf)
//     sigma_v: dK = 2 K/sigma_v (computed without the division)
// The centre of a singular profile contributes nothing, as in the forward path.
//
// Summed over nodes, the seven products factor into per-potential constants
// times seven node sums (Fg = F' (g . m), U = d1^2 - d2^2, V = 2 d1 d2,
// X = g1 d1 - g2 d2, Y = g1 d2 + g2 d1):
//     T1 = sum 2 Fg d1 + f g1      x_c:  -K (A T1 + B T2)
//     T2 = sum 2 Fg d2 + f g2      y_c:  -K (B T1 + C T2)
//     W1 = sum Fg U + f X          eps:  K (-cos 2Phi W1 - sin 2Phi W2)
//     W2 = sum Fg V + f Y          Phi:  2 eps K (sin 2Phi W1 - cos 2Phi W2)
//     F = sum f (g . m)            a:    K/(s-a) F + K Da
//     Da = sum -(g . m)/(qa A_)    s:    -K a/(s (s-a)) F + K Ds
//     Ds = sum (g . m)/(qs B_)     sigma_v: 2 K/sigma_v F
// so the kernels accumulate the node sums and apply the constants once.
#include "lens_path.hpp"

namespace lens {

// Derivative constants of one potential, arcsec units.
enum : int {
    D_XC = 0, D_YC, D_A, D_B, D_C, D_AE, D_BE, D_AP, D_BP, D_RA, D_A2, D_RS, D_S2, D_S2A2, D_SMA, D_K, D_KA, D_KS,
    D_KSIG, D_SINF, D_OK, D_CXH, D_CXL, D_CYH, D_CYL, D_STRIDE = 28
};

__device__ __forceinline__ void dconst(const PotPtrs& pot, int p, double* d)
{
    double row[T64_STRIDE], K, a1, a2;
    const bool ok = row64(pot, p, row, K, a1, a2);
    const double eps = pot.eps[p], phi = pot.phi[p], a = pot.r_core[p], s = pot.r_cut[p];
    const double sig = pot.sigma_v[p];
    const bool sinf = isinf(s);
    const double c2 = cos(2.0 * phi), s2 = sin(2.0 * phi);
    d[D_XC] = row[T64_XC];
    d[D_YC] = row[T64_YC];
    d[D_A] = row[T64_A];
    d[D_B] = row[T64_B];
    d[D_C] = row[T64_C];
    d[D_AE] = -c2;
    d[D_BE] = -s2;
    d[D_AP] = 2.0 * eps * s2;
    d[D_BP] = -2.0 * eps * c2;
    d[D_RA] = a;
    d[D_A2] = a * a;
    d[D_RS] = sinf ? 0.0 : s;
    d[D_S2] = sinf ? 0.0 : s * s;
    d[D_S2A2] = sinf ? 0.0 : (s - a) * (s + a);
    d[D_SMA] = sinf ? 0.0 : s - a;
    d[D_K] = K;
    d[D_KA] = sinf ? 0.0 : K / (s - a);
    d[D_KS] = sinf ? 0.0 : -K * a / (s * (s - a));
    // dK/dsigma = 2 K / sigma = 2 * 4 pi sigma / c^2 * (s/(s-a))
    const double k1 = 8.0 * kPi * sig / (kCkms * kCkms) * kArcsecPerRad;
    d[D_KSIG] = sinf ? k1 : k1 * s / (s - a);
    d[D_SINF] = sinf ? 1.0 : 0.0;
    d[D_OK] = ok ? 1.0 : 0.0;
}

// Square root and reciprocal square root of a positive argument.  FP64: the
// hardware estimate y of 1/sqrt(x) (relative error below 2^-24 on gfx950,
// measured) refined by one Newton step, y (1 + (1 - x y^2) / 2), whose
// relative error is 1.5 times the square of the estimate's (below 2^-47), and
// the root as x times it: both within ~2^-47 relative, far inside the
// products' 1e-11 bar.  FP32: the hardware instructions (1 ulp).
__device__ __forceinline__ void sqrt_rsq(double x, double& s, double& is)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    is = fma(0.5 * y, e, y);
    s = x * is;
}
__device__ __forceinline__ void sqrt_rsq(float x, float& s, float& is)
{
    s = __builtin_amdgcn_sqrtf(x);
    is = __builtin_amdgcn_rsqf(x);
}
// Reciprocal of a positive normal argument: the hardware estimate (2^-24)
// refined by one Newton-Raphson step (~2^-48) in FP64; the hardware
// instruction (FP32, 1 ulp).
__device__ __forceinline__ double brcp(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float brcp(float v) { return __builtin_amdgcn_rcpf(v); }

template <typename T>
struct DConst {
    T A, B, C, Ae, Be, Ap, Bp, a, a2, s, s2, s2a2, sma, K, Ka, Ks, Ksig;
    bool sinf;
};

template <typename T>
__device__ __forceinline__ DConst<T> load_dconst(const double* d)
{
    DConst<T> k;
    k.A = (T)d[D_A];
    k.B = (T)d[D_B];
    k.C = (T)d[D_C];
    k.Ae = (T)d[D_AE];
    k.Be = (T)d[D_BE];
    k.Ap = (T)d[D_AP];
    k.Bp = (T)d[D_BP];
    k.a = (T)d[D_RA];
    k.a2 = (T)d[D_A2];
    k.s = (T)d[D_RS];
    k.s2 = (T)d[D_S2];
    k.s2a2 = (T)d[D_S2A2];
    k.sma = (T)d[D_SMA];
    k.K = (T)d[D_K];
    k.Ka = (T)d[D_KA];
    k.Ks = (T)d[D_KS];
    k.Ksig = (T)d[D_KSIG];
    k.sinf = d[D_SINF] != 0.0;
    return k;
}

// sum[0..6] += the node sums (T1, T2, W1, W2, F, Da, Ds) of one node at offset
// d with cotangent g, for a cut (CUT) or uncut profile.  Straight-line code so
// that calls in one basic block interleave; for a singular profile (SING) the
// centre runs with g = 0 and R^2 = 1, so that its products are exact zeros.
template <typename T, bool CUT, bool SING>
__device__ __forceinline__ void vjp_sums(const DConst<T>& k, T d1, T d2, T g1, T g2, T* sum)
{
    const T m1 = k.A * d1 + k.B * d2, m2 = k.B * d1 + k.C * d2;
    T R2 = d1 * m1 + d2 * m2;
    if constexpr (SING) {
        const bool c = R2 == (T)0;
        R2 = c ? (T)1 : R2;
        g1 = c ? (T)0 : g1;
        g2 = c ? (T)0 : g2;
    }
    // f and F' without cancellation: with A_ = qa + a, B_ = qs + s,
    //   qs - qa = (s^2 - a^2)/(qs + qa),  B_ - A_ = (qs - qa) + (s - a),
    //   f = (B_ - A_)/(A_ B_),
    //   F' = -[(qs - qa) B_^2 + qa (B_ - A_)(B_ + A_)] / (2 qa qs A_^2 B_^2).
    // The reciprocals 1/(A_ B_), 1/A_, 1/B_ and 1/(qs + qa) come from the one
    // reciprocal of A_ B_ (qs + qa).
    T qa, iqa;
    sqrt_rsq(k.a2 + R2, qa, iqa);
    const T A_ = qa + k.a;
    const T gm = g1 * m1 + g2 * m2;
    T f, Fp, dfa;
    if constexpr (!CUT) {
        const T iA = brcp(A_);
        f = iA;
        Fp = (T)(-0.5) * iA * iA * iqa;
        dfa = -iA * iqa;
    } else {
        T qs, iqs;
        sqrt_rsq(k.s2 + R2, qs, iqs);
        const T B_ = qs + k.s, S = qs + qa, AB = A_ * B_;
        const T inv = brcp(AB * S), iAB = S * inv;
        const T dq = k.s2a2 * (AB * inv);
        const T dB = dq + k.sma;
        f = dB * iAB;
        Fp = (T)(-0.5) * (dq * B_ * B_ + qa * dB * (B_ + A_)) * (iqa * iqs) * (iAB * iAB);
        dfa = -(B_ * iAB) * iqa;
        sum[6] += ((A_ * iAB) * iqs) * gm;
    }
    const T Fg = Fp * gm, Fg2 = Fg + Fg;
    sum[0] += Fg2 * d1 + f * g1;
    sum[1] += Fg2 * d2 + f * g2;
    sum[2] += Fg * (d1 * d1 - d2 * d2) + f * (g1 * d1 - g2 * d2);
    sum[3] += Fg2 * (d1 * d2) + f * (g1 * d2 + g2 * d1);
    sum[4] += f * gm;
    sum[5] += dfa * gm;
}

// sum[0..6] += the node sums of two nodes (one basic block).
template <typename T, bool CUT, bool SING>
__device__ __forceinline__ void vjp_sums2(const DConst<T>& k, T d1a, T d2a, T g1a, T g2a, T d1b, T d2b, T g1b,
                                          T g2b, T* sum)
{
    vjp_sums<T, CUT, SING>(k, d1a, d2a, g1a, g2a, sum);
    vjp_sums<T, CUT, SING>(k, d1b, d2b, g1b, g2b, sum);
}

// Dispatch on the profile kind (uniform over the wave).
template <typename T>
__device__ __forceinline__ void vjp_pair(const DConst<T>& k, T d1a, T d2a, T g1a, T g2a, T d1b, T d2b, T g1b,
                                         T g2b, T* sum)
{
    if (k.sinf) {
        if (k.a == (T)0)
            vjp_sums2<T, false, true>(k, d1a, d2a, g1a, g2a, d1b, d2b, g1b, g2b, sum);
        else
            vjp_sums2<T, false, false>(k, d1a, d2a, g1a, g2a, d1b, d2b, g1b, g2b, sum);
    } else {
        if (k.a == (T)0)
            vjp_sums2<T, true, true>(k, d1a, d2a, g1a, g2a, d1b, d2b, g1b, g2b, sum);
        else
            vjp_sums2<T, true, false>(k, d1a, d2a, g1a, g2a, d1b, d2b, g1b, g2b, sum);
    }
}

// Product c of (x_c, y_c, eps, Phi, a, s, sigma_v) from the FP64 node sums.
__device__ __forceinline__ double vjp_combine(const double* d, const double* sum, int c)
{
    const double K = d[D_K];
    switch (c) {
    case 0: return -K * (d[D_A] * sum[0] + d[D_B] * sum[1]);
    case 1: return -K * (d[D_B] * sum[0] + d[D_C] * sum[1]);
    case 2: return K * (d[D_AE] * sum[2] + d[D_BE] * sum[3]);
    case 3: return K * (d[D_AP] * sum[2] + d[D_BP] * sum[3]);
    case 4: return d[D_KA] * sum[4] + K * sum[5];
    case 5: return d[D_SINF] != 0.0 ? 0.0 : d[D_KS] * sum[4] + K * sum[6];
    default: return d[D_KSIG] * sum[4];
    }
}

// ============================================================== field VJP

// Rows per wave (nodes per thread, their cotangents held in registers) and
// potentials per workgroup of the field VJP: FP32 products 16 rows and 4
// potentials, FP64 products 8 rows and 2 potentials (twice the registers per
// value and three times the work per term).
#ifndef LENS_VJP32_ROWS
#define LENS_VJP32_ROWS 8
#endif
#ifndef LENS_VJP32_GROUP
#define LENS_VJP32_GROUP 4
#endif
#ifndef LENS_VJP64_ROWS
#define LENS_VJP64_ROWS 4
#endif
#ifndef LENS_VJP64_GROUP
#define LENS_VJP64_GROUP 2
#endif
template <typename T>
struct VjpCfg {
    static constexpr int rows = LENS_VJP32_ROWS, group = LENS_VJP32_GROUP;
};
template <>
struct VjpCfg<double> {
    static constexpr int rows = LENS_VJP64_ROWS, group = LENS_VJP64_GROUP;
};
// the smaller tile height (more tiles) sizes the scratch
constexpr int kVjpMinRows = VjpCfg<double>::rows < VjpCfg<float>::rows ? VjpCfg<double>::rows : VjpCfg<float>::rows;

// Derivative constants of every potential, plus (FP32 path) the node-unit
// split of its centre as in the FP32 field: slot D_CX.. of row p.
__global__ __launch_bounds__(64) void k_vjp_prep(PotPtrs pot, GridDesc g, double* __restrict__ dtab,
                                                 int* __restrict__ status)
{
    const int p = blockIdx.x * 64 + threadIdx.x;
    if (p == 0 && status) *status = kStatusOk;
    if (p >= pot.n) return;
    double* d = dtab + (size_t)p * D_STRIDE;
    dconst(pot, p, d);
    const double cxn = (d[D_XC] - g.x0) / g.h, cyn = (d[D_YC] - g.y0) / g.h;
    d[D_CXH] = (float)rint(cxn);
    d[D_CXL] = (float)(cxn - rint(cxn));
    d[D_CYH] = (float)rint(cyn);
    d[D_CYL] = (float)(cyn - rint(cyn));
}

// The seven node sums of one potential over a thread's R rows (cotangents
// g1, g2 in registers, rows past the grid at g = 0), for one profile kind.
template <typename T, int R, bool CUT, bool SING>
__device__ __forceinline__ void vjp_rows(const DConst<T>& k, T d1, const T* d2, const T* g1, const T* g2, T* acc)
{
#pragma unroll
    for (int r = 0; r < R; r += 2)
        vjp_sums2<T, CUT, SING>(k, d1, d2[r], g1[r], g2[r], d1, d2[r + 1], g1[r + 1], g2[r + 1], acc);
}

// Workgroup (tile, group): a 64-column tile of 4 R rows, lane = column and
// wave = a band of R rows, times the potentials [group*G, +G), whose
// constants every lane reads from the same address.  Each thread loads its
// R nodes' cotangents once (one round of independent loads), then for every
// potential of the group accumulates the seven node sums in T over those
// nodes and leaves them in LDS.  The workgroup then reduces the 256 partial
// sums of each (potential, sum) in FP64 in a fixed order (runs of 256/S
// consecutive threads, then the S runs), applies the potential's constants
// and writes the seven products to part[(k*P + p)*n_tiles + tile].
// Held to at most 96 VGPRs (five waves per SIMD): the FP64 form then keeps
// one register in scratch and runs 3-4 % faster than at 100 VGPRs and four
// waves; the FP32 form needs 85 anyway.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_vjp(
    const double* __restrict__ dtab, int np, GridDesc g, const double* __restrict__ gx,
    const double* __restrict__ gy, int tiles_x, int n_tiles, double* __restrict__ part)
{
    constexpr int R = VjpCfg<T>::rows, G = VjpCfg<T>::group;
    constexpr int S = G * 7 * 16 <= 256 ? 16 : G * 7 * 8 <= 256 ? 8 : 4;  // runs per (potential, sum)
    static_assert(G * 7 * S <= 256 && 256 % S == 0, "one thread per run");
    __shared__ T red[G * 7][256];
    __shared__ double run[G * 7][S];
    __shared__ double tot[G * 7];
    const int tile = blockIdx.x % n_tiles, grp = blockIdx.x / n_tiles;
    const int p0 = grp * G, npg = min(G, np - p0);
    const int t = threadIdx.x, lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int i = (tile % tiles_x) * 64 + lane;
    const int jb = (tile / tiles_x) * (4 * R) + wave * R;
    const bool col = i < g.nx;
    const int ic = col ? i : 0;
    T g1[R], g2[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const bool in = col && jb + r < g.ny;
        const size_t n = in ? (size_t)(jb + r) * g.nx + ic : 0;
        g1[r] = in ? (T)gx[n] : (T)0;
        g2[r] = in ? (T)gy[n] : (T)0;
    }
    const float ihf = (float)g.h;
    for (int q = 0; q < npg; q++) {
        const double* d = dtab + (size_t)(p0 + q) * D_STRIDE;
        const DConst<T> k = load_dconst<T>(d);
        T d1, d2[R];
        if constexpr (sizeof(T) == 8) {
            d1 = node_coord(g.x0, i, g.h) - d[D_XC];
#pragma unroll
            for (int r = 0; r < R; r++) d2[r] = node_coord(g.y0, jb + r, g.h) - d[D_YC];
        } else {
            // offsets from the node-unit split of the centre, as in the FP32 field
            d1 = (((float)i - (float)d[D_CXH]) - (float)d[D_CXL]) * ihf;
#pragma unroll
            for (int r = 0; r < R; r++) d2[r] = (((float)(jb + r) - (float)d[D_CYH]) - (float)d[D_CYL]) * ihf;
        }
        T acc[7];
#pragma unroll
        for (int c = 0; c < 7; c++) acc[c] = (T)0;
        if (k.sinf) {
            if (k.a == (T)0)
                vjp_rows<T, R, false, true>(k, d1, d2, g1, g2, acc);
            else
                vjp_rows<T, R, false, false>(k, d1, d2, g1, g2, acc);
        } else {
            if (k.a == (T)0)
                vjp_rows<T, R, true, true>(k, d1, d2, g1, g2, acc);
            else
                vjp_rows<T, R, true, false>(k, d1, d2, g1, g2, acc);
        }
#pragma unroll
        for (int c = 0; c < 7; c++) red[q * 7 + c][t] = acc[c];
    }
    __syncthreads();
    if (t < npg * 7 * S) {
        const int qc = t / S, r0 = (t - qc * S) * (256 / S);
        double v = 0.0;
        for (int k = 0; k < 256 / S; k++) v += (double)red[qc][r0 + k];
        run[qc][t - qc * S] = v;
    }
    __syncthreads();
    if (t < npg * 7) {
        double v = 0.0;
        for (int k = 0; k < S; k++) v += run[t][k];
        tot[t] = v;
    }
    __syncthreads();
    if (t < 7 * npg) {
        const int q = t / 7, c = t - 7 * q;
        part[((size_t)c * np + p0 + q) * n_tiles + tile] =
            vjp_combine(dtab + (size_t)(p0 + q) * D_STRIDE, tot + 7 * q, c);
    }
}

// One wave per output (k, p): fixed-order sum over the chunks; NaN and
// LENS_ERR_INVALID for parameters outside the model's domain.
__global__ __launch_bounds__(256) void k_vjp_final(PotPtrs pot, const double* __restrict__ part, int n_chunks,
                                                   double* __restrict__ grad, int* __restrict__ status)
{
    const int o = (int)((blockIdx.x * 256 + threadIdx.x) >> 6);
    if (o >= 7 * pot.n) return;
    const int p = o % pot.n;
    double v = 0.0;
    for (int c = lane_id(); c < n_chunks; c += 64) v += part[(size_t)o * n_chunks + c];
    v = wave_sum(v);
    if (lane_id() == 0) {
        double row[T64_STRIDE], K, a1, a2;
        const bool ok = row64(pot, p, row, K, a1, a2);
        grad[o] = ok ? v : __builtin_nan("");
        if (!ok && status) *status = kStatusInvalid;
    }
}

// ============================================================== source-plane chi^2

// beta_j = theta_j - r alpha(theta_j) (one wave per image, FP64), then the
// last workgroup forms, per system, the barycentre, chi2_i = sum_j
// |beta_j - bar|^2 / sigma_j^2 and the cotangent of alpha at theta_j,
//     G_j = -r_i (2 w_j - (2/n_i) sum_k w_k),  w_j = (beta_j - bar)/sigma_j^2,
// so that d chi^2/d q = sum_j G_j . d alpha(theta_j)/d q.  Writes chi2 (if
// not null), the cotangents and the status.
__global__ __launch_bounds__(256) void k_src_fwd(PotPtrs pot, ObsPtrs obs, double* __restrict__ beta,
                                                 double* __restrict__ cot, double* __restrict__ csys,
                                                 SrcState* __restrict__ st, double* __restrict__ chi2,
                                                 int* __restrict__ status)
{
    __shared__ int s_last, s_bad;
    const int t = threadIdx.x, lane = lane_id();
    if (t == 0) s_bad = 0;
    __syncthreads();
    for (int j = blockIdx.x * 4 + (t >> 6); j < obs.n_img; j += gridDim.x * 4) {
        const double t1 = obs.x[j], t2 = obs.y[j];
        double s1 = 0.0, s2 = 0.0;
        bool bad = false;
        for (int p = lane; p < pot.n; p += 64) {
            double row[T64_STRIDE], K, a1, a2;
            bad |= !row64(pot, p, row, K, a1, a2);
            add_alpha64(row, t1, t2, s1, s2);
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        const int i = system_of(obs.sys_off, obs.n_sys, j);
        const double r = obs.dls[i];
        if (__ballot(bad) != 0 && lane == 0) s_bad = 1;
        if (lane == 0) {
            beta[2 * j] = src_map(t1, r, s1);
            beta[2 * j + 1] = src_map(t2, r, s2);
        }
    }
    __syncthreads();
    if (t == 0 && s_bad) atomicOr(&st->bad, 1);
    if (!last_workgroup(&st->ticket, &s_last)) return;
    bool ok = atomicOr(&st->bad, 0) == 0 && obs.sys_off[0] == 0 && obs.sys_off[obs.n_sys] == obs.n_img;
    for (int i = t; i < obs.n_sys; i += 256) {
        const int j0 = obs.sys_off[i], j1 = obs.sys_off[i + 1];
        const double r = obs.dls[i];
        bool oki = j0 <= j1 && j0 >= 0 && j1 <= obs.n_img && isfinite(r) && r >= 0.0;
        double bx = 0.0, by = 0.0, c = 0.0, wx = 0.0, wy = 0.0;
        if (oki) {
            for (int j = j0; j < j1; j++) {
                bx += beta[2 * j];
                by += beta[2 * j + 1];
                oki = oki && obs.sigma[j] > 0.0 && isfinite(obs.sigma[j]);
            }
            const int n = j1 - j0;
            if (n > 0) {
                bx /= n;
                by /= n;
            }
            for (int j = j0; j < j1; j++) {
                const double dx = beta[2 * j] - bx, dy = beta[2 * j + 1] - by, is2 = 1.0 / (obs.sigma[j] * obs.sigma[j]);
                c += (dx * dx + dy * dy) * is2;
                wx += dx * is2;
                wy += dy * is2;
            }
            for (int j = j0; j < j1; j++) {
                const double is2 = 1.0 / (obs.sigma[j] * obs.sigma[j]);
                const double gxj = 2.0 * (beta[2 * j] - bx) * is2 - 2.0 * wx / n;
                const double gyj = 2.0 * (beta[2 * j + 1] - by) * is2 - 2.0 * wy / n;
                cot[2 * j] = -r * gxj;
                cot[2 * j + 1] = -r * gyj;
            }
        }
        csys[i] = c;
        ok = ok && oki;
    }
    ok = __syncthreads_and(ok);
    if (t < 64) {
        double v = 0.0;
        for (int i = t; i < obs.n_sys; i += 64) v += csys[i];
        v = wave_sum(v);
        if (t == 0) {
            if (chi2) *chi2 = ok ? v : __builtin_nan("");
            if (status) *status = ok ? kStatusOk : kStatusInvalid;
            st->status = ok ? kStatusOk : kStatusInvalid;
            st->bad = 0;
        }
    }
}

// One wave per potential: d chi^2/d q = scale * sum_j G_j . d alpha_p(theta_j)/d q.
// With has_upd, the HMC kick (and drift) of the entries it writes follow.
__global__ __launch_bounds__(256) void k_src_bwd(PotPtrs pot, ObsPtrs obs, const double* __restrict__ cot,
                                                 const SrcState* __restrict__ st, const double* __restrict__ g_chi2,
                                                 double* __restrict__ grad, HmcUpdate upd, int has_upd)
{
    __shared__ double sc[4][D_STRIDE];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int p = blockIdx.x * 4 + wave;
    if (p < pot.n && lane == 0) dconst(pot, p, sc[wave]);
    __syncthreads();
    if (p >= pot.n) return;
    const double* d = sc[wave];
    const DConst<double> k = load_dconst<double>(d);
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int j = lane; j < obs.n_img; j += 64)
        vjp_pair<double>(k, obs.x[j] - d[D_XC], obs.y[j] - d[D_YC], cot[2 * j], cot[2 * j + 1], 0.0, 0.0, 0.0, 0.0,
                         acc);
#pragma unroll
    for (int c = 0; c < 7; c++) acc[c] = wave_sum(acc[c]);
    const double scale = g_chi2 ? *g_chi2 : 1.0;
    const bool ok = st->status == kStatusOk;
    if (lane >= 7) return;
    const size_t k7 = (size_t)lane * pot.n + p;
    const double gv = ok ? scale * vjp_combine(d, acc, lane) : __builtin_nan("");
    grad[k7] = gv;
    if (has_upd && upd.step[k7] != 0.0) {
        upd.p[k7] -= upd.kick * upd.step[k7] * (0.5 * gv);
        if (upd.drift) upd.q[k7] += upd.step[k7] * upd.p[k7];
    }
}

__global__ void k_status(int* status, int v)
{
    if (threadIdx.x == 0) *status = v;
}

// ============================================================== launchers

static int vjp_tiles_x(const GridDesc& g) { return (g.nx + 63) / 64; }

// Tiles of 64 columns x 4 rows-per-wave rows.
static int vjp_chunks(const GridDesc& g, int rows) { return vjp_tiles_x(g) * ((g.ny + 4 * rows - 1) / (4 * rows)); }

size_t vjp_scratch(int np, const GridDesc& g)
{
    return ((size_t)7 * vjp_chunks(g, kVjpMinRows) + D_STRIDE) * (size_t)np * 8;
}

hipError_t launch_vjp(const PotPtrs& pot, const GridDesc& g, bool fp32, const double* gx, const double* gy,
                      double* scratch, double* grad, int* status, const KernelEvents* ev, hipStream_t s)
{
    if (pot.n == 0) {
        if (status) k_status<<<1, 64, 0, s>>>(status, kStatusOk);
        return hipGetLastError();
    }
    const int rows = fp32 ? VjpCfg<float>::rows : VjpCfg<double>::rows;
    const int group = fp32 ? VjpCfg<float>::group : VjpCfg<double>::group;
    const int nc = vjp_chunks(g, rows), tx = vjp_tiles_x(g);
    double* dtab = scratch;
    double* part = scratch + (size_t)D_STRIDE * pot.n;
    k_vjp_prep<<<(unsigned)((pot.n + 63) / 64), 64, 0, s>>>(pot, g, dtab, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nb = (long long)nc * ((pot.n + group - 1) / group);
    e = fp32 ? launch_ev(ev, k_vjp<float>, dim3((unsigned)nb), dim3(256), s, (const double*)dtab, pot.n, g, gx, gy,
                         tx, nc, part)
             : launch_ev(ev, k_vjp<double>, dim3((unsigned)nb), dim3(256), s, (const double*)dtab, pot.n, g, gx, gy,
                         tx, nc, part);
    if (e != hipSuccess) return e;
    k_vjp_final<<<(unsigned)((7ll * pot.n + 3) / 4), 256, 0, s>>>(pot, part, nc, grad, status);
    return hipGetLastError();
}

hipError_t launch_src(const PotPtrs& pot, const ObsPtrs& obs, double* beta, double* cot, double* csys,
                      SrcState* st, double* chi2, int* status, const double* g_chi2, double* grad,
                      const HmcUpdate* upd, hipStream_t s)
{
    long long nb = (obs.n_img + 3) / 4;
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    k_src_fwd<<<(unsigned)nb, 256, 0, s>>>(pot, obs, beta, cot, csys, st, chi2, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !grad || pot.n == 0) return e;
    const HmcUpdate none = {nullptr, nullptr, nullptr, 0.0, 0};
    k_src_bwd<<<(unsigned)((pot.n + 3) / 4), 256, 0, s>>>(pot, obs, cot, st, g_chi2, grad, upd ? *upd : none,
                                                          upd ? 1 : 0);
    return hipGetLastError();
}

}  // namespace lens
