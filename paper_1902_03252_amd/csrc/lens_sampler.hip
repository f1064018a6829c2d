// Sampler steps over the lens model's parameters on gfx950: the role of the
// paper's sampler (Sec. 2.2.1, whose chi^2 it evaluates) taken by
//   - Hamiltonian Monte Carlo on the source-plane chi^2 (potential energy
//     U = chi^2 / 2, unit masses in the coordinates z = q / step, leapfrog
//     integration, Metropolis acceptance on the energy error): the momentum
//     kicks and position drifts are applied by the source-plane gradient
//     kernel to the entries it writes, so a leapfrog step is two kernels;
//   - independent random-walk Metropolis chains on the image-plane chi^2
//     (log-likelihood -chi^2 / 2), all chains' proposals evaluated by one
//     batched chi^2 call.
// The random numbers (momenta, proposal noise, acceptance uniforms) are the
// caller's inputs, so that a step is a deterministic function of them.
// Parameters are a device table [7][n] (rows x, y, eps, phi, r_core, r_cut,
// sigma_v); a parameter with step 0 is held fixed.
#include "lens_path.hpp"

namespace lens {

// q = state; p = momentum (0 where the step is 0).
__global__ __launch_bounds__(256) void k_hmc_begin(const double* __restrict__ state,
                                                   const double* __restrict__ momentum,
                                                   const double* __restrict__ step, int n7, double* __restrict__ q,
                                                   double* __restrict__ p)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n7) return;
    q[k] = state[k];
    p[k] = step[k] != 0.0 ? momentum[k] : 0.0;
}

// H = chi^2 / 2 + |p|^2 / 2 before (momentum input) and after (p) the
// trajectory, fixed-order sums; accept when both chi^2 are valid and
// u < exp(H0 - H1).  On acceptance the state becomes q.  chi2 receives the
// chi^2 of the resulting state.
__global__ __launch_bounds__(256) void k_hmc_accept(double* __restrict__ state, const double* __restrict__ q,
                                                    const double* __restrict__ momentum,
                                                    const double* __restrict__ p, const double* __restrict__ step,
                                                    int n7, const double* __restrict__ chi2_pair,
                                                    const int* __restrict__ status_pair, const double* __restrict__ u,
                                                    double* __restrict__ chi2, int* __restrict__ accepted)
{
    __shared__ double s0[4], s1[4];
    __shared__ int s_acc;
    const int t = threadIdx.x, lane = lane_id(), wave = t >> 6;
    double k0 = 0.0, k1 = 0.0;
    for (int k = t; k < n7; k += 256) {
        if (step[k] == 0.0) continue;
        k0 += momentum[k] * momentum[k];
        k1 += p[k] * p[k];
    }
    k0 = wave_sum(k0);
    k1 = wave_sum(k1);
    if (lane == 0) {
        s0[wave] = k0;
        s1[wave] = k1;
    }
    __syncthreads();
    if (t == 0) {
        const double c0 = chi2_pair[0], c1 = chi2_pair[1];
        const double h0 = 0.5 * c0 + 0.5 * ((s0[0] + s0[1]) + (s0[2] + s0[3]));
        const double h1 = 0.5 * c1 + 0.5 * ((s1[0] + s1[1]) + (s1[2] + s1[3]));
        const bool valid = status_pair[0] == kStatusOk && status_pair[1] == kStatusOk && isfinite(c1) &&
                           isfinite(h1);
        const bool acc = valid && log(u[0]) < h0 - h1;
        s_acc = acc;
        *chi2 = acc ? c1 : c0;
        *accepted = acc ? 1 : 0;
    }
    __syncthreads();
    if (s_acc)
        for (int k = t; k < n7; k += 256) state[k] = q[k];
}

// Random-walk proposals of every chain: proposal = state + step * noise, with
// the step of parameter (row, potential) shared by all chains (n potentials per
// chain, B chains, tables [7][B*n]).  Multiply and add are rounded separately.
__global__ __launch_bounds__(256) void k_mh_propose(const double* __restrict__ state,
                                                    const double* __restrict__ step,
                                                    const double* __restrict__ noise, int n, long long bn,
                                                    double* __restrict__ prop)
{
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= 7 * bn) return;
    const int row = (int)(k / bn);
    const int pidx = (int)((k - (long long)row * bn) % n);
    const double s = step[(size_t)row * n + pidx];
    prop[k] = s != 0.0 ? __dadd_rn(state[k], __dmul_rn(s, noise[k])) : state[k];
}

// Chain b accepts its proposal when the proposal's evaluation is valid and
// log u_b < -(chi2_new - chi2_cur) / 2; accepted chains copy the proposal into
// their state and chi^2.  One workgroup per chain.
__global__ __launch_bounds__(256) void k_mh_accept(double* __restrict__ state, const double* __restrict__ prop,
                                                   int n, long long bn, const double* __restrict__ chi2_new,
                                                   const int* __restrict__ status_new, const double* __restrict__ u,
                                                   double* __restrict__ chi2, int* __restrict__ accepted)
{
    __shared__ int s_acc;
    const int b = blockIdx.x;
    if (threadIdx.x == 0) {
        const double cn = chi2_new[b], cc = chi2[b];
        const bool valid = status_new[b] == kStatusOk && isfinite(cn);
        const bool acc = valid && (!isfinite(cc) || log(u[b]) < -0.5 * (cn - cc));
        s_acc = acc;
        accepted[b] = acc ? 1 : 0;
        if (acc) chi2[b] = cn;
    }
    __syncthreads();
    if (!s_acc) return;
    for (int k = threadIdx.x; k < 7 * n; k += 256) {
        const int row = k / n, pidx = k - row * n;
        const size_t idx = (size_t)row * bn + (size_t)b * n + pidx;
        state[idx] = prop[idx];
    }
}

// ---------------------------------------------------------------- launchers

static unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

hipError_t launch_hmc_begin(const double* state, const double* momentum, const double* step, int n7, double* q,
                            double* p, hipStream_t s)
{
    k_hmc_begin<<<blocks_for(n7), 256, 0, s>>>(state, momentum, step, n7, q, p);
    return hipGetLastError();
}

hipError_t launch_hmc_accept(double* state, const double* q, const double* momentum, const double* p,
                             const double* step, int n7, const double* chi2_pair, const int* status_pair,
                             const double* u, double* chi2, int* accepted, hipStream_t s)
{
    k_hmc_accept<<<1, 256, 0, s>>>(state, q, momentum, p, step, n7, chi2_pair, status_pair, u, chi2, accepted);
    return hipGetLastError();
}

hipError_t launch_mh_propose(const double* state, const double* step, const double* noise, int n, int b,
                             double* prop, hipStream_t s)
{
    const long long bn = (long long)b * n;
    k_mh_propose<<<blocks_for(7 * bn), 256, 0, s>>>(state, step, noise, n, bn, prop);
    return hipGetLastError();
}

hipError_t launch_mh_accept(double* state, const double* prop, int n, int b, const double* chi2_new,
                            const int* status_new, const double* u, double* chi2, int* accepted, hipStream_t s)
{
    k_mh_accept<<<(unsigned)b, 256, 0, s>>>(state, prop, n, (long long)b * n, chi2_new, status_new, u, chi2,
                                            accepted);
    return hipGetLastError();
}

}  // namespace lens
