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
#include "lens_path.hpp"

namespace lens {

// Derivative constants of one potential, arcsec units.
enum : int {
    D_XC = 0, D_YC, D_A, D_B, D_C, D_AE, D_BE, D_AP, D_BP, D_RA, D_A2, D_RS, D_S2, D_S2A2, D_SMA, D_K, D_KA, D_KS,
    D_KSIG, D_SINF, D_OK, D_STRIDE = 24
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

__device__ __forceinline__ double bsqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float bsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double brcp(double v) { return 1.0 / v; }
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

// acc[0..6] += g . d alpha / d (x_c, y_c, eps, Phi, a, s, sigma_v) at offset d.
template <typename T>
__device__ __forceinline__ void vjp_term(const DConst<T>& k, T d1, T d2, T g1, T g2, T* acc)
{
    const T m1 = k.A * d1 + k.B * d2, m2 = k.B * d1 + k.C * d2;
    const T R2 = d1 * m1 + d2 * m2;
    if (k.a == (T)0 && R2 == (T)0) return;
    // f and F' without cancellation: with A_ = qa + a, B_ = qs + s,
    //   qs - qa = (s^2 - a^2)/(qs + qa),  B_ - A_ = (qs - qa) + (s - a),
    //   f = (B_ - A_)/(A_ B_),
    //   F' = -[(qs - qa) B_^2 + qa (B_ - A_)(B_ + A_)] / (2 qa qs A_^2 B_^2).
    const T qa = bsqrt(k.a2 + R2);
    const T A_ = qa + k.a, iA = brcp(A_), iqa = brcp(qa);
    T f, Fp, dfa = -iA * iqa, dfs = (T)0;
    if (k.sinf) {
        f = iA;
        Fp = (T)(-0.5) * iA * iA * iqa;
    } else {
        const T qs = bsqrt(k.s2 + R2);
        const T B_ = qs + k.s, iB = brcp(B_), iqs = brcp(qs);
        const T dq = k.s2a2 * brcp(qs + qa);
        const T dB = dq + k.sma;
        f = dB * iA * iB;
        Fp = (T)(-0.5) * (dq * B_ * B_ + qa * dB * (B_ + A_)) * (iqa * iqs) * (iA * iA) * (iB * iB);
        dfs = iB * iqs;
    }
    const T gm = g1 * m1 + g2 * m2;
    const T Kf = k.K * f, KFp = k.K * Fp;
    acc[0] -= (T)2 * KFp * m1 * gm + Kf * (g1 * k.A + g2 * k.B);
    acc[1] -= (T)2 * KFp * m2 * gm + Kf * (g1 * k.B + g2 * k.C);
    const T e1 = k.Ae * d1 + k.Be * d2, e2 = k.Be * d1 - k.Ae * d2;
    acc[2] += KFp * (d1 * e1 + d2 * e2) * gm + Kf * (g1 * e1 + g2 * e2);
    const T p1 = k.Ap * d1 + k.Bp * d2, p2 = k.Bp * d1 - k.Ap * d2;
    acc[3] += KFp * (d1 * p1 + d2 * p2) * gm + Kf * (g1 * p1 + g2 * p2);
    acc[4] += (k.Ka * f + k.K * dfa) * gm;
    acc[5] += (k.Ks * f + k.K * dfs) * gm;
    acc[6] += k.Ksig * f * gm;
}

// ============================================================== field VJP

constexpr int kVjpNpt = 16;   // nodes per thread
constexpr int kVjpGroup = 2;  // potentials per workgroup
constexpr int kVjpChunk = 256 * kVjpNpt;

// Workgroup (chunk, group): nodes [chunk*4096, +4096) of the row-major grid,
// strided over the threads; potentials [group*2, +2).  Per potential every
// thread sums its nodes' seven products in T, the workgroup reduces them in
// FP64 in a fixed order and writes part[(k*P + p)*n_chunks + chunk].
template <typename T>
__global__ __launch_bounds__(256) void k_vjp(PotPtrs pot, GridDesc g, const double* __restrict__ gx,
                                             const double* __restrict__ gy, int n_chunks,
                                             double* __restrict__ part, int* __restrict__ status)
{
    __shared__ double sc[kVjpGroup][D_STRIDE];
    __shared__ double red[4][8];
    const int chunk = blockIdx.x % n_chunks, grp = blockIdx.x / n_chunks;
    const int p0 = grp * kVjpGroup, npg = min(kVjpGroup, pot.n - p0);
    const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
    if (blockIdx.x == 0 && t == 0 && status) *status = kStatusOk;
    if (t < npg) dconst(pot, p0 + t, sc[t]);
    const long long n_nodes = (long long)g.nx * g.ny;
    T g1[kVjpNpt], g2[kVjpNpt];
    int ni[kVjpNpt], nj[kVjpNpt];
#pragma unroll
    for (int u = 0; u < kVjpNpt; u++) {
        const long long n = (long long)chunk * kVjpChunk + u * 256 + t;
        const bool in = n < n_nodes;
        const long long nn = in ? n : 0;
        nj[u] = (int)(nn / g.nx);
        ni[u] = (int)(nn - (long long)nj[u] * g.nx);
        g1[u] = in ? (T)gx[nn] : (T)0;
        g2[u] = in ? (T)gy[nn] : (T)0;
    }
    __syncthreads();
    for (int q = 0; q < npg; q++) {
        const double* d = sc[q];
        const DConst<T> k = load_dconst<T>(d);
        T acc[7] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
        if constexpr (sizeof(T) == 8) {
            const double xc = d[D_XC], yc = d[D_YC];
#pragma unroll
            for (int u = 0; u < kVjpNpt; u++) {
                if (g1[u] == (T)0 && g2[u] == (T)0) continue;  // nothing to add (and no 0 * inf)
                const double d1 = (g.x0 + ni[u] * g.h) - xc, d2 = (g.y0 + nj[u] * g.h) - yc;
                vjp_term<T>(k, d1, d2, g1[u], g2[u], acc);
            }
        } else {
            // offsets from the node-unit split of the centre, as in the FP32 field
            const double cxn = (d[D_XC] - g.x0) / g.h, cyn = (d[D_YC] - g.y0) / g.h;
            const float cxh = (float)rint(cxn), cyh = (float)rint(cyn);
            const float cxl = (float)(cxn - rint(cxn)), cyl = (float)(cyn - rint(cyn));
            const float h = (float)g.h;
#pragma unroll
            for (int u = 0; u < kVjpNpt; u++) {
                if (g1[u] == (T)0 && g2[u] == (T)0) continue;
                const float d1 = (((float)ni[u] - cxh) - cxl) * h, d2 = (((float)nj[u] - cyh) - cyl) * h;
                vjp_term<T>(k, d1, d2, g1[u], g2[u], acc);
            }
        }
#pragma unroll
        for (int c = 0; c < 7; c++) {
            const double v = wave_sum((double)acc[c]);
            if (lane == 0) red[wave][c] = v;
        }
        __syncthreads();
        if (t < 7) {
            const double v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
            part[((size_t)t * pot.n + p0 + q) * n_chunks + chunk] = v;
        }
        __syncthreads();
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
            beta[2 * j] = t1 - r * s1;
            beta[2 * j + 1] = t2 - r * s2;
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
__global__ __launch_bounds__(256) void k_src_bwd(PotPtrs pot, ObsPtrs obs, const double* __restrict__ cot,
                                                 const SrcState* __restrict__ st, const double* __restrict__ g_chi2,
                                                 double* __restrict__ grad)
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
        vjp_term<double>(k, obs.x[j] - d[D_XC], obs.y[j] - d[D_YC], cot[2 * j], cot[2 * j + 1], acc);
    const double scale = g_chi2 ? *g_chi2 : 1.0;
    const bool ok = st->status == kStatusOk;
#pragma unroll
    for (int c = 0; c < 7; c++) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) grad[(size_t)c * pot.n + p] = ok ? scale * v : __builtin_nan("");
    }
}

__global__ void k_status(int* status, int v)
{
    if (threadIdx.x == 0) *status = v;
}

// ============================================================== launchers

int vjp_chunks(const GridDesc& g) { return (int)(((long long)g.nx * g.ny + kVjpChunk - 1) / kVjpChunk); }

hipError_t launch_vjp(const PotPtrs& pot, const GridDesc& g, bool fp32, const double* gx, const double* gy,
                      double* part, double* grad, int* status, const KernelEvents* ev, hipStream_t s)
{
    if (pot.n == 0) {
        if (status) k_status<<<1, 64, 0, s>>>(status, kStatusOk);
        return hipGetLastError();
    }
    const int nc = vjp_chunks(g);
    const long long nb = (long long)nc * ((pot.n + kVjpGroup - 1) / kVjpGroup);
    hipError_t e = fp32 ? launch_ev(ev, k_vjp<float>, dim3((unsigned)nb), dim3(256), s, pot, g, gx, gy, nc, part, status)
                        : launch_ev(ev, k_vjp<double>, dim3((unsigned)nb), dim3(256), s, pot, g, gx, gy, nc, part,
                                    status);
    if (e != hipSuccess) return e;
    k_vjp_final<<<(unsigned)((7ll * pot.n + 3) / 4), 256, 0, s>>>(pot, part, nc, grad, status);
    return hipGetLastError();
}

hipError_t launch_src(const PotPtrs& pot, const ObsPtrs& obs, double* beta, double* cot, double* csys,
                      SrcState* st, double* chi2, int* status, const double* g_chi2, double* grad, hipStream_t s)
{
    long long nb = (obs.n_img + 3) / 4;
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    k_src_fwd<<<(unsigned)nb, 256, 0, s>>>(pot, obs, beta, cot, csys, st, chi2, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !grad || pot.n == 0) return e;
    k_src_bwd<<<(unsigned)((pot.n + 3) / 4), 256, 0, s>>>(pot, obs, cot, st, g_chi2, grad);
    return hipGetLastError();
}

}  // namespace lens
