// HIP kernels of the image-plane chi^2 path for gfx950 (MI355X).
//
// One chi^2 evaluation (Rexroth et al. 2019, Sec. 2.2.1-2.2.2, Fig. 1):
//   k_prep    per-potential constants (FP64 and FP32 tables), domain terms
//   k_field*h deflection at every grid node (FP32 or FP64) and the per-tile
//             deflection ranges; its first rows of workgroups run the head:
//             observed images -> source plane in FP64, then (last of them)
//             the barycentres, the FP32 error bound, one row per system and
//             the counters                                       <- the time
//   k_cull    one wave per tile of cells: the tile's deflection range bounds
//             its source-plane vertices; every system whose barycentre the
//             bound admits gives a (tile, system) pair
//   k_pairs   persistent waves over the pairs: triangle containment (FP32
//             certified signs or FP64 exact); hits and undecided tests
//             appended
//   k_fbpos   FP64 re-test of the undecided tests, FP64 position of every hit
//   k_tail    one workgroup: sort of the hits, matching of observed to
//             predicted images, FP64 chi^2 in a fixed order
// k_head (prep and head in one kernel) serves lens_deflect and
// lens_source_positions, and the chi^2 path when the fused grid would exceed
// 65535 rows of workgroups.
#include "lens_path.hpp"

#include <algorithm>
#include <type_traits>

namespace lens {

// Head of every evaluation, one wave per observed image (at least enough
// workgroups of 4 waves for one thread per potential), in two phases:
//  1. every thread with a potential index writes that potential's constants
//     (prep_one); every wave with an observed image j computes grad Psi at the
//     observed position itself in FP64 from the raw parameters (the same
//     row64 arithmetic as the table), potentials over the lanes;
//  2. the last workgroup to finish forms the source positions
//     beta_ij = theta_ij - r_i grad Psi(theta_ij) (Sec. 2.2.2), one system per
//     thread, reduces the bound terms in a fixed order,
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
// Source-plane part of the head: grad Psi (FP64) at observed images j =
// wave, wave + n_waves, ... (one wave per image, the potentials over the lanes
// and a fixed butterfly sum), stored in beta_x/beta_y for head_finish.  TABLE:
// the prepared table rows are read; otherwise each lane recomputes its rows
// from the parameters.
template <bool TABLE>
__device__ __forceinline__ void head_images(const PotPtrs& pot, const double* __restrict__ tab64,
                                            const ObsPtrs& obs, double* __restrict__ beta_x,
                                            double* __restrict__ beta_y, int wave, int n_waves)
{
    const int np = pot.n;
    for (int j = wave; j < obs.n_img; j += n_waves) {
        const double t1 = obs.x[j], t2 = obs.y[j];
        double a1, a2;
        if constexpr (TABLE) {
            alpha64_wave(tab64, np, t1, t2, a1, a2);
        } else {
            double s1 = 0.0, s2 = 0.0;
            for (int p = lane_id(); p < np; p += 64) {
                double row[T64_STRIDE], K, b1, b2;
                row64(pot, p, row, K, b1, b2);
                add_alpha64(row, t1, t2, s1, s2);
            }
            a1 = wave_sum(s1);
            a2 = wave_sum(s2);
        }
        if (lane_id() == 0) {  // grad Psi for now; head_finish turns it into beta
            beta_x[j] = a1;
            beta_y[j] = a2;
        }
    }
}

// The last workgroup's part of the head (256 threads): the FP32 error bound
// E_alpha from the per-potential terms, beta_ij = theta_ij - r_i grad Psi,
// barycentres and one row per system with its FP32 bound E_B, counters reset
// and the status.  Up to kHeadStage images the images are spread over the
// threads (one round of independent loads) and staged in LDS for the
// per-system sums; beyond, each system's thread walks its images.  Both forms
// sum a system's images in image order.
constexpr int kHeadStage = 512;

// LDS of head_finish, laid out in a caller's buffer so that the fused field
// kernels can overlay it on the field loop's row parts.
struct HeadLds {
    double sw[4], sj[4], sb[4];
    double sbx[kHeadStage], sby[kHeadStage];
    int soff[kHeadStage + 1];
    int sys_bad;
};

__device__ __forceinline__ void head_finish(HeadLds& L, int np, const GridDesc& g, const ObsPtrs& obs,
                                            const double* __restrict__ bterm, double* __restrict__ beta_x,
                                            double* __restrict__ beta_y, double* __restrict__ sysrow,
                                            EvalState* __restrict__ st)
{
    double* sw = L.sw;
    double* sj = L.sj;
    double* sb = L.sb;
    int& sys_bad = L.sys_bad;
    double* sbx = L.sbx;
    double* sby = L.sby;
    int* soff = L.soff;
    const int t = threadIdx.x;
    const int nsys = obs.n_sys, nimg = obs.n_img;
    const bool staged = nsys > 0 && nimg <= kHeadStage && nsys < kHeadStage;
    double w = 0.0, jt = 0.0, bad = 0.0;
    for (int p = t; p < np; p += 256) {
        w += bterm[3 * p + 0];
        jt += bterm[3 * p + 1];
        bad += bterm[3 * p + 2];
    }
    if (staged)
        for (int q = t; q <= nsys; q += 256) soff[q] = obs.sys_off[q];
    w = wave_sum(w);
    jt = wave_sum(jt);
    bad = wave_sum(bad);
    if (lane_id() == 0) {
        sw[t >> 6] = w;
        sj[t >> 6] = jt;
        sb[t >> 6] = bad;
    }
    if (t == 0) sys_bad = nsys > 0 && (obs.sys_off[0] != 0 || obs.sys_off[nsys] != nimg);
    __syncthreads();
    if (staged) {
        // beta of every image, one thread each; an image whose system is out of
        // order (invalid offsets) is left to the per-system check below
        bool img_bad = false;
        for (int j = t; j < nimg; j += 256) {
            int lo = 0, hi = nsys - 1;  // the system owning image j
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (soff[mid] <= j) lo = mid; else hi = mid - 1;
            }
            const double r = obs.dls[lo];
            const double b1 = src_map(obs.x[j], r, beta_x[j]), b2 = src_map(obs.y[j], r, beta_y[j]);
            sbx[j] = b1;
            sby[j] = b2;
            const double sg = obs.sigma[j];
            img_bad = img_bad || !(sg > 0.0 && isfinite(sg) && isfinite(obs.x[j]) && isfinite(obs.y[j]));
        }
        if (img_bad) atomicOr(&sys_bad, 1);
        __syncthreads();
        for (int j = t; j < nimg; j += 256) {
            beta_x[j] = sbx[j];
            beta_y[j] = sby[j];
        }
    }
    const double W = (sw[0] + sw[1]) + (sw[2] + sw[3]);
    const double Jsum = (sj[0] + sj[1]) + (sj[2] + sj[3]);
    const double Bsum = (sb[0] + sb[1]) + (sb[2] + sb[3]);
    const double e_alpha = kU32 * (64.0 + np) * W + Jsum + 1e-9;
    const double xlo = g.x0, xhi = g.x0 + (g.nx - 1) * g.h, ylo = g.y0, yhi = g.y0 + (g.ny - 1) * g.h;
    for (int s = t; s < nsys; s += 256) {
        const int j0 = staged ? soff[s] : obs.sys_off[s], j1 = staged ? soff[s + 1] : obs.sys_off[s + 1];
        bool ok = j0 <= j1 && j0 >= 0 && j1 <= nimg;
        double bx = 0.0, by = 0.0;
        const double r = obs.dls[s];
        if (ok) {
            for (int j = j0; j < j1; j++) {
                double b1, b2;
                if (staged) {
                    b1 = sbx[j];
                    b2 = sby[j];
                } else {
                    b1 = src_map(obs.x[j], r, beta_x[j]);
                    b2 = src_map(obs.y[j], r, beta_y[j]);
                    beta_x[j] = b1;
                    beta_y[j] = b2;
                    ok = ok && obs.sigma[j] > 0.0 && isfinite(obs.sigma[j]) && isfinite(obs.x[j]) &&
                         isfinite(obs.y[j]);
                }
                bx += b1;
                by += b2;
            }
            if (j1 > j0) {
                bx /= (j1 - j0);
                by /= (j1 - j0);
            }
        }
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
        st->status = (Bsum != 0.0 || sys_bad) ? kStatusInvalid : kStatusOk;
    }
}

__global__ __launch_bounds__(256) void k_head(PotPtrs pot, GridDesc g, ObsPtrs obs, double* __restrict__ tab64,
                                              float* __restrict__ tab32, double* __restrict__ bterm,
                                              double* __restrict__ beta_x, double* __restrict__ beta_y,
                                              double* __restrict__ sysrow, EvalState* __restrict__ st)
{
    __shared__ int last;
    __shared__ HeadLds hl;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < pot.n; p += gridDim.x * 256)
        prep_one(pot, g, p, p, tab64, tab32, bterm);
    head_images<false>(pot, nullptr, obs, beta_x, beta_y, blockIdx.x * 4 + (threadIdx.x >> 6), gridDim.x * 4);
    if (!last_workgroup(&st->head_ticket, &last)) return;
    head_finish(hl, pot.n, g, obs, bterm, beta_x, beta_y, sysrow, st);
}

// Constants of every potential only (the fused field kernels do the rest of
// the head); also clears the head's ticket for the field launch that follows
// (it is left at zero by every completed launch, and cleared here whatever
// the scratch held before).
__global__ __launch_bounds__(256) void k_prep(PotPtrs pot, GridDesc g, double* __restrict__ tab64,
                                              float* __restrict__ tab32, double* __restrict__ bterm,
                                              EvalState* __restrict__ st)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) st->head_ticket = 0;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < pot.n; p += gridDim.x * 256)
        prep_one(pot, g, p, p, tab64, tab32, bterm);
}

// ============================================================== deflection field

// Each thread owns NPL consecutive nodes in each of NR consecutive grid rows
// (rows j0 .. j0 + NR - 1); a workgroup of 256 threads covers 256*NPL columns
// of those rows, so the row offsets are uniform and every per-potential
// constant is a wave-uniform (scalar) operand.  With rr set, the kernel also
// writes the triangle stage's per-(row, tile column) deflection ranges (tile
// width 1 << tx_shift cells).
template <int NPL, int NR>
__device__ __forceinline__ void field32_block(const float* __restrict__ tab32, int np, int nx, int ny, int j0, int bx,
                                              float* __restrict__ ax, float* __restrict__ ay,
                                              const EvalState* __restrict__ st, float* __restrict__ rr,
                                              int tx_shift, int tiles_x, float4* __restrict__ srow)
{
    const int i0 = (bx * 256 + threadIdx.x) * NPL;
    if (bx * 256 * NPL >= nx) return;  // whole workgroup beyond the row
    float fi[NPL], sx[NR * NPL], sy[NR * NPL];
#pragma unroll
    for (int k = 0; k < NPL; k++) fi[k] = (float)(i0 + k);
#pragma unroll
    for (int q = 0; q < NR * NPL; q++) {
        sx[q] = 0.0f;
        sy[q] = 0.0f;
    }
    field32_all_wg<NPL, NR>(tab32, np, (float)j0, fi, sx, sy, srow);
    const bool bad = st != nullptr && st->status != kStatusOk;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int j = j0 + r;
        if (j >= ny) break;  // uniform over the workgroup
        if (rr) tile_partials<float, NPL>(sx + r * NPL, sy + r * NPL, i0, j, nx, tx_shift, tiles_x, rr);
        const size_t row = (size_t)j * nx;
#pragma unroll
        for (int k = 0; k < NPL; k++) {
            if (i0 + k < nx) {
                ax[row + i0 + k] = bad ? __builtin_nanf("") : sx[r * NPL + k];
                ay[row + i0 + k] = bad ? __builtin_nanf("") : sy[r * NPL + k];
            }
        }
    }
}

template <int NPL, int NR>
__global__ __launch_bounds__(256) void k_field32(const float* __restrict__ tab32, int np, int nx, int ny,
                                                 float* __restrict__ ax, float* __restrict__ ay,
                                                 const EvalState* __restrict__ st, float* __restrict__ rr,
                                                 int tx_shift, int tiles_x)
{
    __shared__ float4 srow[NR * 256];
    field32_block<NPL, NR>(tab32, np, nx, ny, blockIdx.y * NR, blockIdx.x, ax, ay, st, rr, tx_shift, tiles_x, srow);
}

constexpr int kNpl64 = 2;  // FP64 field nodes per thread

// FP64 field: kNpl64 consecutive nodes of one row per thread (a workgroup
// covers 256 * kNpl64 nodes), the same matrix form in arcsec; with rr set,
// also the triangle stage's row partials (as k_field32).
__device__ __forceinline__ void field64_row(const double* __restrict__ tab64, int np, const GridDesc& g, int j,
                                            int bx, double* __restrict__ ax, double* __restrict__ ay,
                                            const EvalState* __restrict__ st, double* __restrict__ rr, int tx_shift,
                                            int tiles_x)
{
    const int i0 = (bx * 256 + (int)threadIdx.x) * kNpl64;
    if (bx * 256 * kNpl64 >= g.nx) return;  // whole workgroup beyond the row
    const double t2 = node_coord(g.y0, j, g.h);
    double t1[kNpl64], s1[kNpl64], s2[kNpl64];
#pragma unroll
    for (int k = 0; k < kNpl64; k++) {
        t1[k] = node_coord(g.x0, i0 + k, g.h);
        s1[k] = 0.0;
        s2[k] = 0.0;
    }
    alpha64_all_wg<kNpl64>(tab64, np, t1, t2, s1, s2);
    if (rr) tile_partials<double, kNpl64>(s1, s2, i0, j, g.nx, tx_shift, tiles_x, rr);
    const bool bad = st != nullptr && st->status != kStatusOk;
    const size_t row = (size_t)j * g.nx;
#pragma unroll
    for (int k = 0; k < kNpl64; k++) {
        if (i0 + k < g.nx) {
            ax[row + i0 + k] = bad ? __builtin_nan("") : s1[k];
            ay[row + i0 + k] = bad ? __builtin_nan("") : s2[k];
        }
    }
}

__global__ __launch_bounds__(256) void k_field64(const double* __restrict__ tab64, int np, GridDesc g,
                                                 double* __restrict__ ax, double* __restrict__ ay,
                                                 const EvalState* __restrict__ st, double* __restrict__ rr,
                                                 int tx_shift, int tiles_x)
{
    field64_row(tab64, np, g, blockIdx.y, blockIdx.x, ax, ay, st, rr, tx_shift, tiles_x);
}

// ---------------------------------------------------------------- head fused into the field launch

// The head's source-plane part (after k_prep) run by the first `head_rows`
// rows of workgroups of a field launch, which the hardware dispatches first:
// one wave per observed image reads the prepared FP64 table; the last of these
// workgroups runs head_finish.  The field workgroups do not depend on it (they
// read only the FP32 / FP64 tables); the triangle stage after the launch does.
__device__ __forceinline__ void fused_head(HeadLds& L, const HeadArgs& h, int head_rows)
{
    __shared__ int last;
    const int nblk = head_rows * gridDim.x;
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    head_images<true>(h.pot, h.tab64, h.obs, h.bx, h.by, b * 4 + (threadIdx.x >> 6), nblk * 4);
    if (!last_of(&h.st->head_ticket, (unsigned)nblk, &last)) return;
    head_finish(L, h.pot.n, h.g, h.obs, h.bterm, h.bx, h.by, h.sysrow, h.st);
}

// One LDS buffer for both parts of a fused field launch (a workgroup runs
// either the head or the field): the head's arrays and the field loop's row
// parts overlay, so the launch needs the larger of the two, not their sum.
template <int BYTES>
struct alignas(16) FusedLds {
    unsigned char raw[BYTES];
};
constexpr int fused_lds_bytes(int field_bytes)
{
    return field_bytes > (int)sizeof(HeadLds) ? field_bytes : (int)sizeof(HeadLds);
}

template <int NPL, int NR>
__global__ __launch_bounds__(256) void k_field32h(const float* __restrict__ tab32, int np, int nx, int ny,
                                                  float* __restrict__ ax, float* __restrict__ ay,
                                                  float* __restrict__ rr, int tx_shift, int tiles_x, HeadArgs h,
                                                  int head_rows)
{
    __shared__ FusedLds<fused_lds_bytes(NR * 256 * (int)sizeof(float4))> lds;
    if ((int)blockIdx.y < head_rows) {
        fused_head(*reinterpret_cast<HeadLds*>(lds.raw), h, head_rows);
        return;
    }
    field32_block<NPL, NR>(tab32, np, nx, ny, (blockIdx.y - head_rows) * NR, blockIdx.x, ax, ay, nullptr, rr,
                           tx_shift, tiles_x, reinterpret_cast<float4*>(lds.raw));
}

__global__ __launch_bounds__(256) void k_field64h(const double* __restrict__ tab64, int np, GridDesc g,
                                                  double* __restrict__ ax, double* __restrict__ ay,
                                                  double* __restrict__ rr, int tx_shift, int tiles_x, HeadArgs h,
                                                  int head_rows)
{
    __shared__ HeadLds hl;
    if ((int)blockIdx.y < head_rows) {
        fused_head(hl, h, head_rows);
        return;
    }
    field64_row(tab64, np, g, blockIdx.y - head_rows, blockIdx.x, ax, ay, nullptr, rr, tx_shift, tiles_x);
}

// ============================================================== triangle stage

// Culling, one wave per (block of 64 consecutive tiles of S::TX x S::TY
// cells, chunk of `sc` systems) with `tpw` blocks per wave, lane = tile: each
// lane bounds its tile's source-plane vertices by the box [theta_min -
// r alpha_max, theta_max - r alpha_min] from the field kernel's row partials
// plus the halo column (consecutive tiles read consecutive partials), widened
// by the FP32 bound E_B (mixed path) or 1e-9" (FP64 path), and tests the
// barycentre of every system of its chunk (the chunk's rows loaded at once,
// lane = system, then broadcast); every passing (tile, system) pair is
// appended to the wave's own region (ballot and lane prefix) and the wave's
// count written to counts[wave]: no atomic, no barrier.  Small grids split the
// systems over more waves, large grids give a wave several blocks.
template <class S, typename V>
__global__ __launch_bounds__(256) void k_cull(const V* __restrict__ rr, GridDesc g, int tiles_x, int n_tiles,
                                              int tpw, int sc, int n_chunks, int n_cull, int nsys,
                                              const double* __restrict__ sysrow, unsigned long long* __restrict__ pairs,
                                              long long region, unsigned* __restrict__ counts,
                                              unsigned* __restrict__ part)
{
    const int lane = lane_id();
    const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (w >= n_cull) return;  // the whole wave
    const int blk = w / n_chunks, s0 = (w - blk * n_chunks) * sc;
    const int ns = min(sc, nsys - s0);  // <= 64
    // the chunk's system rows, lane = system
    double r = 0.0, eb = 0.0, bx = 0.0, by = 0.0;
    if (lane < ns) {
        const double* row = sysrow + (size_t)(s0 + lane) * SYS_STRIDE;
        r = row[SYS_R];
        eb = sizeof(V) == 4 ? row[SYS_EB] : 1e-9;
        bx = row[SYS_BX];
        by = row[SYS_BY];
    }
    unsigned long long* out = pairs + (size_t)w * region;
    unsigned cnt = 0;  // pairs of the wave so far (uniform)
    for (int k = 0; k < tpw; k++) {
        const int tile = (blk * tpw + k) * 64 + lane;
        const bool act = tile < n_tiles;
        Tile T = {0, 0, 0, 0};
        double rng[4] = {0.0, 0.0, 0.0, 0.0};
        if (act) {
            T = tile_of<S>(g, tiles_x, tile);
            tile_range_lane<S, V>(rr, tiles_x, T, rng);
        }
        for (int c = 0; c < ns; c++) {
            const bool pass =
                act && tile_box_contains(g, T, rng, bcast(r, c), bcast(eb, c), bcast(bx, c), bcast(by, c));
            const unsigned long long m = __ballot(pass);
            const int off =
                __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            if (pass) out[cnt + off] = ((unsigned long long)(unsigned)tile << 32) | (unsigned)(s0 + c);
            cnt += (unsigned)__popcll(m);
        }
    }
    if (lane == 0) {
        counts[w] = cnt;
        part[2 * w + 0] = cnt;
        part[2 * w + 1] = 0;
    }
}

// Containment of one (tile, system) pair by one wave: the tile's cells are
// strided over the lanes, up to four cells per lane per step, with every vertex
// load of a step issued before any decision.  Mixed path: FP32 vertex offsets
// and the certified sign test; FP64 path: exact containment on the FP64
// field's vertices.  Certain hits and undecided tests are appended (system <<
// 32 | triangle id) with one atomic per wave.  All 64 lanes call it together.
template <class S, typename V>
__device__ __forceinline__ void pair_test(const V* __restrict__ ax, const V* __restrict__ ay, const GridDesc& g,
                                          const Tile& T, int sys, const double* __restrict__ sysrow,
                                          EvalState* __restrict__ st, int mode, float tau,
                                          unsigned long long* __restrict__ hit_keys, long long hit_cap,
                                          unsigned long long* __restrict__ flag_keys, long long flag_cap,
                                          unsigned& nbbox)
{
    constexpr int Q = S::TX * S::TY / 64;  // cells per lane for one pair
    constexpr int QB = Q < 4 ? Q : 4;      // cells per lane per step
    const int lane = lane_id();
    // the system's row, read once per pair (sys is wave-uniform: scalar loads)
    const double* row = sysrow + (size_t)sys * SYS_STRIDE;
    const double rr64 = row[SYS_R], rbx = row[SYS_BX], rby = row[SYS_BY];
    const float r32 = (float)rr64, e32 = (float)row[SYS_EB];
    const float bxh = (float)row[SYS_BXH], bxl = (float)row[SYS_BXL];
    const float byh = (float)row[SYS_BYH], byl = (float)row[SYS_BYL];
    for (int q0 = 0; q0 < Q; q0 += QB) {
        V va[QB][8];
#pragma unroll
        for (int b = 0; b < QB; b++) {
            const int c = lane + 64 * (q0 + b), li = c % S::TX, lj = c / S::TX;
            const bool valid = li < T.ncx && lj < T.ncy;
            const size_t n00 = valid ? (size_t)(T.cj0 + lj) * g.nx + (T.ci0 + li) : 0;
            const size_t n01 = n00 + g.nx;
            va[b][0] = ax[n00];
            va[b][1] = ax[n00 + 1];
            va[b][2] = ax[n01];
            va[b][3] = ax[n01 + 1];
            va[b][4] = ay[n00];
            va[b][5] = ay[n00 + 1];
            va[b][6] = ay[n01];
            va[b][7] = ay[n01 + 1];
        }
        unsigned bits = 0;  // 4 bits per cell: result of triangle 0, then triangle 1
#pragma unroll
        for (int b = 0; b < QB; b++) {
            const int c = lane + 64 * (q0 + b), li = c % S::TX, lj = c / S::TX;
            if (!(li < T.ncx && lj < T.ncy)) continue;
            const int gi = T.ci0 + li, gj = T.cj0 + lj;
            int res0 = kMiss, res1 = kMiss;
            if constexpr (sizeof(V) == 4) {
                const float r = r32, E = e32;
                const float h32 = (float)g.h;
                const float ex0 = (((float)gi - bxh) - bxl) * h32;
                const float ex1 = (((float)(gi + 1) - bxh) - bxl) * h32;
                const float ey0 = (((float)gj - byh) - byl) * h32;
                const float ey1 = (((float)(gj + 1) - byh) - byl) * h32;
                const float d00x = fmaf(-r, va[b][0], ex0), d00y = fmaf(-r, va[b][4], ey0);
                const float d10x = fmaf(-r, va[b][1], ex1), d10y = fmaf(-r, va[b][5], ey0);
                const float d01x = fmaf(-r, va[b][2], ex0), d01y = fmaf(-r, va[b][6], ey1);
                const float d11x = fmaf(-r, va[b][3], ex1), d11y = fmaf(-r, va[b][7], ey1);
                const float tx[3] = {d00x, d10x, d01x}, ty[3] = {d00y, d10y, d01y};
                const float ux[3] = {d11x, d01x, d10x}, uy[3] = {d11y, d01y, d10y};
                res0 = decide32(tx, ty, E, mode, tau, nbbox);
                res1 = decide32(ux, uy, E, mode, tau, nbbox);
            } else {
                const double r = rr64, bx = rbx, by = rby;
                const double t0x = node_coord(g.x0, gi, g.h), t1x = node_coord(g.x0, gi + 1, g.h);
                const double t0y = node_coord(g.y0, gj, g.h), t1y = node_coord(g.y0, gj + 1, g.h);
                const double b00x = src_map(t0x, r, va[b][0]), b00y = src_map(t0y, r, va[b][4]);
                const double b10x = src_map(t1x, r, va[b][1]), b10y = src_map(t0y, r, va[b][5]);
                const double b01x = src_map(t0x, r, va[b][2]), b01y = src_map(t1y, r, va[b][6]);
                const double b11x = src_map(t1x, r, va[b][3]), b11y = src_map(t1y, r, va[b][7]);
                const double vx0[3] = {b00x, b10x, b01x}, vy0[3] = {b00y, b10y, b01y};
                const double vx1[3] = {b11x, b01x, b10x}, vy1[3] = {b11y, b01y, b10y};
                if (!(bx < fmin(vx0[0], fmin(vx0[1], vx0[2])) || bx > fmax(vx0[0], fmax(vx0[1], vx0[2])) ||
                      by < fmin(vy0[0], fmin(vy0[1], vy0[2])) || by > fmax(vy0[0], fmax(vy0[1], vy0[2])))) {
                    nbbox++;
                    res0 = contains_exact(vx0, vy0, bx, by) ? kHit : kMiss;
                }
                if (!(bx < fmin(vx1[0], fmin(vx1[1], vx1[2])) || bx > fmax(vx1[0], fmax(vx1[1], vx1[2])) ||
                      by < fmin(vy1[0], fmin(vy1[1], vy1[2])) || by > fmax(vy1[0], fmax(vy1[1], vy1[2])))) {
                    nbbox++;
                    res1 = contains_exact(vx1, vy1, bx, by) ? kHit : kMiss;
                }
            }
            bits |= (unsigned)(res0 | (res1 << 2)) << (4 * b);
        }
        if (__ballot(bits != 0) == 0) continue;  // the common case: no hit, nothing undecided
        const unsigned long long base = (unsigned long long)(unsigned)sys << 32;
#pragma unroll 1
        for (int b = 0; b < QB; b++) {
            const unsigned rb = (bits >> (4 * b)) & 15u;
            const int c = lane + 64 * (q0 + b), li = c % S::TX, lj = c / S::TX;
            const unsigned tid0 = (unsigned)(2 * ((T.cj0 + lj) * (g.nx - 1) + (T.ci0 + li)));
            wave_append((rb & 3u) == kHit, base | tid0, &st->n_hits, hit_keys, hit_cap);
            wave_append((rb >> 2) == kHit, base | (tid0 + 1), &st->n_hits, hit_keys, hit_cap);
            wave_append((rb & 3u) == kFlag, base | tid0, &st->n_flags, flag_keys, flag_cap);
            wave_append((rb >> 2) == kFlag, base | (tid0 + 1), &st->n_flags, flag_keys, flag_cap);
        }
    }
}

// Containment of the (tile, system) pairs, persistent waves, one pair at a
// time (pair_test).
template <class S, typename V>
__global__ __launch_bounds__(256) void k_pairs(const V* __restrict__ ax, const V* __restrict__ ay, GridDesc g,
                                               int tiles_x, const double* __restrict__ sysrow,
                                               EvalState* __restrict__ st, int mode, float tau,
                                               const unsigned long long* __restrict__ pairs, long long region,
                                               const unsigned* __restrict__ counts, int n_cull,
                                               unsigned long long* __restrict__ hit_keys, long long hit_cap,
                                               unsigned long long* __restrict__ flag_keys, long long flag_cap,
                                               unsigned* __restrict__ part, int part_base)
{
    __shared__ unsigned sp[4][2];
    const int lane = lane_id(), t = threadIdx.x;
    // exclusive prefix of the culling counts in LDS: thread t owns counts
    // [CT t, CT t + CT) (n_cull <= kMaxCull), wave scans, then the wave totals
    constexpr int CT = kMaxCull / 256;
    __shared__ unsigned spre[kMaxCull + 1];
    __shared__ unsigned swt[4];
    const int wave = t >> 6;
    unsigned cl[CT], lsum = 0;
#pragma unroll
    for (int j = 0; j < CT; j++) {
        const int c = CT * t + j;
        cl[j] = c < n_cull ? counts[c] : 0u;
        lsum += cl[j];
    }
    unsigned incl = lsum;
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned v = __shfl_up(incl, d, 64);
        if (lane >= d) incl += v;
    }
    if (lane == 63) swt[wave] = incl;
    __syncthreads();
    unsigned run = incl - lsum;
    for (int w = 0; w < wave; w++) run += swt[w];
#pragma unroll
    for (int j = 0; j < CT; j++) {
        const int c = CT * t + j;
        if (c < n_cull) spre[c] = run;
        run += cl[j];
    }
    const unsigned total = swt[0] + swt[1] + swt[2] + swt[3];
    __syncthreads();
    const long long nw = (long long)gridDim.x * 4;
    const long long w0 = (long long)blockIdx.x * 4 + wave;
    const long long n_pairs = st->status == kStatusOk ? (long long)total : 0;
    unsigned nbbox = 0;
    // key of pair u: the last culling wave whose prefix is <= u, then its region
    auto pair_key = [&](long long u) -> unsigned long long {
        const unsigned pidx = (unsigned)u;
        int lo = 0, hi = n_cull - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (spre[mid] <= pidx) lo = mid; else hi = mid - 1;
        }
        return pairs[(size_t)lo * region + (pidx - spre[lo])];
    };
    // the next pair's key is looked up and loaded before the current pair's tests
    unsigned long long nk = w0 < n_pairs ? pair_key(w0) : 0ull;
    for (long long u = w0; u < n_pairs; u += nw) {
        const unsigned long long pk = nk;
        if (u + nw < n_pairs) nk = pair_key(u + nw);
        // the key is the wave's own (every lane loaded the same one)
        const int tile = __builtin_amdgcn_readfirstlane((int)(pk >> 32));
        const int sys = __builtin_amdgcn_readfirstlane((int)(pk & 0xffffffffu));
        pair_test<S, V>(ax, ay, g, tile_of<S>(g, tiles_x, tile), sys, sysrow, st, mode, tau, hit_keys, hit_cap,
                        flag_keys, flag_cap, nbbox);
    }
    write_part_sum(part, (size_t)part_base + blockIdx.x, 0u, nbbox, sp);
}


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
        for (int q = t; q <= nsys; q += 1024) soff[q] = obs.sys_off[q];  // nsys + 1 <= 1025 entries
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
                      nfb > (unsigned long long)fb_cap ||
                      total > (unsigned long long)hit_capacity ||
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
    if (n > 256 && n <= 1024 && nsys <= kTailStage) {
        // counting by system, then rank by (triangle id, index) inside each
        // system's bucket: keys are unique, so the ranks give the sorted order
        // in O(n + sum of squared bucket sizes) instead of O(n^2) (below 257
        // keys the plain rank sort, with fewer barriers, is faster).  The
        // upper half of the key array holds the buckets, then the bucket
        // starts and fill counts.
        static_assert(kSortCap >= 4096, "room for 1024 keys and the bucket arrays");
        unsigned long long* tmp = key + kSortCap / 2;
        int* sbeg = reinterpret_cast<int*>(tmp + 1024);
        int* sfill = sbeg + kTailStage;
        int* swsum = sfill + kTailStage;
        if (t < nsys) sfill[t] = 0;
        __syncthreads();
        unsigned long long mine = 0;
        int sy = 0;
        if (t < n) {
            mine = key[t];
            sy = (int)(mine >> 44);
            atomicAdd(&sfill[sy], 1);
        }
        __syncthreads();
        const int cnt = t < nsys ? sfill[t] : 0;  // thread t: system t
        int incl = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d, 64);
            if ((t & 63) >= d) incl += v;
        }
        if ((t & 63) == 63) swsum[t >> 6] = incl;
        __syncthreads();
        int b0 = incl - cnt;
        for (int w = 0; w < (t >> 6); w++) b0 += swsum[w];
        if (t < nsys) {
            sbeg[t] = b0;
            sfill[t] = 0;
        }
        __syncthreads();
        if (t < n) tmp[sbeg[sy] + atomicAdd(&sfill[sy], 1)] = mine;
        __syncthreads();
        if (t < n) {
            const int q0 = sbeg[sy], q1 = q0 + sfill[sy];
            int rank = 0;
            for (int q = q0; q < q1; q++) rank += tmp[q] < mine;
            key[q0 + rank] = mine;
        }
        __syncthreads();
    } else if (n <= 1024) {
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

// Calls f(integral_constant<NPL>, integral_constant<NR>) for an FP32 field
// layout code (field_cols / field_rows); unknown codes take 2 x 1.
template <class F>
static hipError_t with_field_shape(int code, F f)
{
    using std::integral_constant;
    switch (code) {
    case 0x01: return f(integral_constant<int, 1>(), integral_constant<int, 1>());
    case 0x04: return f(integral_constant<int, 4>(), integral_constant<int, 1>());
    case 0x08: return f(integral_constant<int, 8>(), integral_constant<int, 1>());
    case 0x21: return f(integral_constant<int, 1>(), integral_constant<int, 2>());
    case 0x22: return f(integral_constant<int, 2>(), integral_constant<int, 2>());
    case 0x24: return f(integral_constant<int, 4>(), integral_constant<int, 2>());
    case 0x41: return f(integral_constant<int, 1>(), integral_constant<int, 4>());
    case 0x42: return f(integral_constant<int, 2>(), integral_constant<int, 4>());
    default: return f(integral_constant<int, 2>(), integral_constant<int, 1>());
    }
}

hipError_t launch_field32(const float* tab32, int np, const GridDesc& g, float* ax, float* ay,
                          const EvalState* st, int npl, float* rr, int tx_shift, int tiles_x,
                          const KernelEvents* ev, hipStream_t s)
{
    return with_field_shape(npl, [&](auto c, auto r) {
        constexpr int C = decltype(c)::value, R = decltype(r)::value;
        const dim3 grid(cdiv(g.nx, 256 * C), cdiv(g.ny, R));
        return launch_ev(ev, k_field32<C, R>, grid, dim3(256), s, tab32, np, g.nx, g.ny, ax, ay, st, rr, tx_shift,
                         tiles_x);
    });
}

hipError_t launch_prep(const PotPtrs& pot, const GridDesc& g, double* tab64, float* tab32, double* bterm,
                       EvalState* st, hipStream_t s)
{
    k_prep<<<clampu(cdiv(pot.n, 256), 1, 1024), 256, 0, s>>>(pot, g, tab64, tab32, bterm, st);
    return hipGetLastError();
}

// Zeroes n words (a fill kernel rather than a memset, so that a captured
// graph holds no memset node).
__global__ __launch_bounds__(64) void k_zero_u32(unsigned* __restrict__ p, int n)
{
    for (int k = threadIdx.x; k < n; k += 64) p[k] = 0u;
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s)
{
    k_zero_u32<<<1, 64, 0, s>>>(p, n);
    return hipGetLastError();
}

// Rows of head workgroups for a field launch `bx` workgroups wide: one wave
// per observed image, at least one workgroup (head_finish always runs).
static int head_rows_for(const ObsPtrs& obs, int bx)
{
    const long long blocks = obs.n_img > 0 ? cdiv(obs.n_img, 4) : 1;
    return (int)((blocks + bx - 1) / bx);
}

int fused_head_fits(const GridDesc& g, const ObsPtrs& obs, int npl, bool fp32)
{
    const int bx = (int)cdiv(g.nx, fp32 ? 256 * field_cols(npl) : 256 * kNpl64);
    const long long rows = fp32 ? cdiv(g.ny, field_rows(npl)) : g.ny;
    return rows + head_rows_for(obs, bx) <= 65535;
}

hipError_t launch_field32h(const float* tab32, int np, const GridDesc& g, float* ax, float* ay, int npl, float* rr,
                           int tx_shift, int tiles_x, const HeadArgs& h, const KernelEvents* ev, hipStream_t s)
{
    return with_field_shape(npl, [&](auto c, auto r) {
        constexpr int C = decltype(c)::value, R = decltype(r)::value;
        const int bx = (int)cdiv(g.nx, 256 * C);
        const int hr = head_rows_for(h.obs, bx);
        const dim3 grid((unsigned)bx, (unsigned)(cdiv(g.ny, R) + hr));
        return launch_ev(ev, k_field32h<C, R>, grid, dim3(256), s, tab32, np, g.nx, g.ny, ax, ay, rr, tx_shift,
                         tiles_x, h, hr);
    });
}

hipError_t launch_field64h(const double* tab64, int np, const GridDesc& g, double* ax, double* ay, double* rr,
                           int tx_shift, int tiles_x, const HeadArgs& h, const KernelEvents* ev, hipStream_t s)
{
    const int bx = (int)cdiv(g.nx, 256 * kNpl64);
    const int hr = head_rows_for(h.obs, bx);
    return launch_ev(ev, k_field64h, dim3((unsigned)bx, (unsigned)(g.ny + hr)), dim3(256), s, tab64, np, g, ax, ay,
                     rr, tx_shift, tiles_x, h, hr);
}

hipError_t launch_field64(const double* tab64, int np, const GridDesc& g, double* ax, double* ay,
                          const EvalState* st, double* rr, int tx_shift, int tiles_x, const KernelEvents* ev,
                          hipStream_t s)
{
    return launch_ev(ev, k_field64, dim3(cdiv(g.nx, 256 * kNpl64), g.ny), dim3(256), s, tab64, np, g, ax, ay, st, rr,
                     tx_shift, tiles_x);
}

// Tile shapes selectable per call (lens_chi2_opts.tile): 1 = 32x8 (default),
// 2 = 64x16, 3 = 64x8, 4 = 32x16.
template <class F>
static hipError_t with_shape(int shape, F f)
{
    switch (shape) {
    case 2: return f(TileShape<64, 16>());
    case 3: return f(TileShape<64, 8>());
    case 4: return f(TileShape<32, 16>());
    default: return f(TileShape<32, 8>());
    }
}

void tile_dims(int shape, int& tx, int& ty)
{
    switch (shape) {
    case 2: tx = 64; ty = 16; break;
    case 3: tx = 64; ty = 8; break;
    case 4: tx = 32; ty = 16; break;
    default: tx = 32; ty = 8; break;
    }
}

// Tiles of a grid for a tile-shape code; workgroups of the culling kernel.
long long tri_tiles(const GridDesc& g, int shape, int* tiles_x)
{
    int tx, ty;
    tile_dims(shape, tx, ty);
    *tiles_x = (int)cdiv(g.nx - 1, tx);
    return (long long)*tiles_x * cdiv(g.ny - 1, ty);
}

// Culling waves for a grid and nsys systems, at most kMaxCull: blocks of 64
// tiles times chunks of at most 64 systems.  Large grids give a wave several
// blocks (tpw) until blocks x the necessary chunks fit; small grids split the
// systems over more waves while that keeps at least 4 systems per wave.  Each
// wave's pair region holds 64 * tpw * sc pairs.
void cull_shape(const GridDesc& g, int shape, int nsys, int* n_cull, int* tpw, int* sc, int* n_chunks)
{
    int tiles_x;
    const long long n_tiles = tri_tiles(g, shape, &tiles_x);
    const long long ns = nsys > 0 ? nsys : 1;
    const long long chmin = (ns + 63) / 64;
    const long long budget = std::max(1ll, (long long)kMaxCull / chmin);
    long long nb = cdiv(n_tiles, 64);
    int k = 1;
    while (nb > budget) {
        k *= 2;
        nb = cdiv(n_tiles, 64ll * k);
    }
    long long ch = std::max(chmin, std::min((long long)kMaxCull / nb, std::max(chmin, ns / 4)));
    const long long per = (ns + ch - 1) / ch;  // <= 64
    ch = (ns + per - 1) / per;
    *tpw = k;
    *sc = (int)per;
    *n_chunks = (int)ch;
    *n_cull = (int)(nb * ch);
}

// Persistent workgroups of the positions / fallback kernel: enough waves that
// a large grid's hits and undecided tests (thousands) take a few items per
// wave, at least the count that serves small grids best.
int fbpos_blocks(long long n_tiles) { return (int)std::min(1024ll, std::max(256ll, n_tiles / 64)); }

hipError_t launch_cull(bool fp32, const void* rr, const GridDesc& g, int nsys,
                       const double* sysrow, unsigned long long* pairs, long long region, unsigned* counts,
                       unsigned* part, int shape, hipStream_t s)
{
    return with_shape(shape, [&](auto sh) {
        using S = decltype(sh);
        int tiles_x, nw, tpw, sc, nch;
        const int n_tiles = (int)tri_tiles(g, shape, &tiles_x);
        cull_shape(g, shape, nsys, &nw, &tpw, &sc, &nch);
        const unsigned nb = (unsigned)cdiv(nw, 4);
        if (fp32)
            k_cull<S, float><<<nb, 256, 0, s>>>((const float*)rr, g, tiles_x, n_tiles, tpw, sc, nch, nw, nsys, sysrow,
                                                pairs, region, counts, part);
        else
            k_cull<S, double><<<nb, 256, 0, s>>>((const double*)rr, g, tiles_x, n_tiles, tpw, sc, nch, nw, nsys,
                                                 sysrow, pairs, region, counts, part);
        return hipGetLastError();
    });
}

hipError_t launch_pairs(bool fp32, const void* ax, const void* ay, const GridDesc& g, const double* sysrow,
                        EvalState* st, int mode, float tau, const unsigned long long* pairs, long long region,
                        const unsigned* counts, int n_cull, unsigned long long* hit_keys, long long hit_cap,
                        unsigned long long* flag_keys, long long flag_cap, unsigned* part, int part_base, int shape,
                        hipStream_t s)
{
    return with_shape(shape, [&](auto sh) {
        using S = decltype(sh);
        int tiles_x;
        tri_tiles(g, shape, &tiles_x);
        if (fp32)
            k_pairs<S, float><<<kPairBlocks, 256, 0, s>>>((const float*)ax, (const float*)ay, g, tiles_x, sysrow, st,
                                                          mode, tau, pairs, region, counts, n_cull, hit_keys, hit_cap,
                                                          flag_keys, flag_cap, part, part_base);
        else
            k_pairs<S, double><<<kPairBlocks, 256, 0, s>>>((const double*)ax, (const double*)ay, g, tiles_x,
                                                           sysrow, st, mode, tau, pairs, region, counts, n_cull,
                                                           hit_keys, hit_cap, flag_keys, flag_cap, part, part_base);
        return hipGetLastError();
    });
}

hipError_t launch_fbpos(const double* tab64, int np, const GridDesc& g, const double* sysrow, EvalState* st,
                        const unsigned long long* hit_keys, long long hit_cap, const unsigned long long* flag_keys,
                        long long flag_cap, unsigned long long* fb_keys, long long fb_cap, double* pos,
                        double* fb_pos, int blocks, hipStream_t s)
{
    k_fbpos<<<blocks, 256, 0, s>>>(tab64, np, g, sysrow, st, hit_keys, hit_cap, flag_keys, flag_cap, fb_keys, fb_cap,
                                pos, fb_pos);
    return hipGetLastError();
}

hipError_t launch_tail(const TailLaunch& tl, EvalState* st, const unsigned long long* fb_keys, const double* pos,
                       const double* fb_pos, hipStream_t s)
{
    k_tail<<<1, 1024, 0, s>>>(tl.obs, st, tl.hit_cap, tl.flag_cap, tl.fb_cap, tl.hit_capacity,
                              tl.hit_keys, fb_keys,
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
