// Batched image-plane chi^2 on gfx950: n lens models (a sampler's proposals)
// with their own potentials and grids, sharing one set of observed systems,
// evaluated by a fixed number of batch-wide launches:
//   k_bhead   constants of every potential, source positions of every
//             (sample, observed image), FP64
//   k_bsys    one wave per sample: error bound, barycentres, system rows,
//             counters
//   k_bmap    work-item -> sample maps of the field and triangle stages
//   k_bfield  FP32 or FP64 deflection, one workgroup per (sample, row segment),
//             heaviest samples first
//   k_btri    one workgroup per (sample, tile), heaviest samples first
//   k_bfbpos  FP64 image positions of every hit (a workgroup per sample) and
//             the FP64 re-test of every undecided FP32 test
//   k_btail   one workgroup per sample: sort, matching, chi^2
// The per-sample work follows exactly the single-evaluation path (same device
// functions, Rexroth et al. 2019, Sec. 2.2.1-2.2.2 and Algorithm 1).
#include "lens_path.hpp"

namespace lens {

static_assert(kBatchMax == kTailStage, "the batch tail stages one sample's hits in LDS");

// Upper bound of the index k with off[k] <= v among off[0..n] (off[0] = 0).
__device__ __forceinline__ int find_segment(const long long* __restrict__ off, int n, long long v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ============================================================== head

__global__ __launch_bounds__(256) void k_bhead(BatchPlan bp, PotPtrs pot, ObsPtrs obs, double* __restrict__ tab64,
                                               float* __restrict__ tab32, double* __restrict__ bterm,
                                               double* __restrict__ beta_x, double* __restrict__ beta_y)
{
    const int t = threadIdx.x;
    const int p0 = bp.pot_off[0], np_all = bp.pot_off[bp.n] - p0;
    // constants: potential p (chunk-local index q) uses its sample's grid
    for (int q = blockIdx.x * 256 + t; q < np_all; q += gridDim.x * 256) {
        int lo = 0, hi = bp.n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (bp.pot_off[mid] - p0 <= q) lo = mid; else hi = mid - 1;
        }
        prep_one(pot, bp.grid[lo], p0 + q, q, tab64, tab32, bterm);
    }
    // source positions: one wave per (sample, observed image)
    const long long nwaves = (long long)gridDim.x * 4;
    const long long nitems = (long long)bp.n * obs.n_img;
    for (long long it = (long long)blockIdx.x * 4 + (t >> 6); it < nitems; it += nwaves) {
        const int s = (int)(it / obs.n_img), j = (int)(it % obs.n_img);
        const double t1 = obs.x[j], t2 = obs.y[j];
        double s1 = 0.0, s2 = 0.0;
        for (int p = bp.pot_off[s] + lane_id(); p < bp.pot_off[s + 1]; p += 64) {
            double row[T64_STRIDE], K, a1, a2;
            row64(pot, p, row, K, a1, a2);
            add_alpha64(row, t1, t2, s1, s2);
        }
        const double a1 = wave_sum(s1), a2 = wave_sum(s2);
        const double r = obs.dls[system_of(obs.sys_off, obs.n_sys, j)];
        if (lane_id() == 0) {
            beta_x[it] = src_map(t1, r, a1);
            beta_y[it] = src_map(t2, r, a2);
        }
    }
}

// One wave per sample: fixed-order bound reductions over its potentials, then
// its system rows (as the single-evaluation head), counters and status.
__global__ __launch_bounds__(256) void k_bsys(BatchPlan bp, ObsPtrs obs, const double* __restrict__ bterm,
                                              const double* __restrict__ beta_x, const double* __restrict__ beta_y,
                                              double* __restrict__ sysrow, BatchState bs)
{
    const int s = (int)((blockIdx.x * 256 + threadIdx.x) >> 6);
    if (s >= bp.n) return;
    const int lane = lane_id();
    const int p0 = bp.pot_off[0];
    const int pa = bp.pot_off[s] - p0, pb = bp.pot_off[s + 1] - p0;
    double w = 0.0, jt = 0.0, bad = 0.0;
    for (int q = pa + lane; q < pb; q += 64) {
        w += bterm[3 * q + 0];
        jt += bterm[3 * q + 1];
        bad += bterm[3 * q + 2];
    }
    const double W = wave_sum(w), J = wave_sum(jt), B = wave_sum(bad);
    const double e_alpha = kU32 * (64.0 + (pb - pa)) * W + J + 1e-9;
    const GridDesc g = bp.grid[s];
    const double xlo = g.x0, xhi = g.x0 + (g.nx - 1) * g.h, ylo = g.y0, yhi = g.y0 + (g.ny - 1) * g.h;
    bool ok = B == 0.0 && obs.sys_off[0] == 0 && obs.sys_off[obs.n_sys] == obs.n_img;
    for (int i = lane; i < obs.n_sys; i += 64) {
        const int j0 = obs.sys_off[i], j1 = obs.sys_off[i + 1];
        bool oki = j0 <= j1 && j0 >= 0 && j1 <= obs.n_img;
        double bx = 0.0, by = 0.0;
        if (oki) {
            for (int j = j0; j < j1; j++) {
                bx += beta_x[(size_t)s * obs.n_img + j];
                by += beta_y[(size_t)s * obs.n_img + j];
                oki = oki && obs.sigma[j] > 0.0 && isfinite(obs.sigma[j]) && isfinite(obs.x[j]) &&
                      isfinite(obs.y[j]);
            }
            if (j1 > j0) {
                bx /= (j1 - j0);
                by /= (j1 - j0);
            }
        }
        const double r = obs.dls[i];
        oki = oki && isfinite(r) && r >= 0.0;
        const double bxn = (bx - g.x0) / g.h, byn = (by - g.y0) / g.h;
        oki = oki && fabs(bxn) < 4194304.0 && fabs(byn) < 4194304.0;
        const double theta = fmax(fmax(fabs(xlo - bx), fabs(xhi - bx)), fmax(fabs(ylo - by), fabs(yhi - by)));
        const double eb = r * e_alpha + 4.0 * kU32 * theta + 2.0 * kU32 * r * (W + e_alpha) +
                          g.h * kNodeSplitErr + 1e-9;
        double* row = sysrow + ((size_t)s * obs.n_sys + i) * SYS_STRIDE;
        row[SYS_BX] = bx;
        row[SYS_BY] = by;
        row[SYS_BXH] = rint(bxn);
        row[SYS_BXL] = bxn - rint(bxn);
        row[SYS_BYH] = rint(byn);
        row[SYS_BYL] = byn - rint(byn);
        row[SYS_R] = r;
        row[SYS_EB] = eb * (1.0 + 1e-6);
        ok = ok && oki;
    }
    ok = __ballot(!ok) == 0;
    if (lane == 0) {
        bs.status[s] = ok ? kStatusOk : kStatusInvalid;
        bs.n_hits[s] = 0;
        bs.n_fb[s] = 0;
        if (s == 0) *bs.n_flags = 0;
    }
}

// Work-item -> position-in-plan maps (one workgroup per sample).
__global__ __launch_bounds__(256) void k_bmap(BatchPlan bp, int* __restrict__ fmap, int* __restrict__ tmap)
{
    const int k = blockIdx.x;
    for (long long i = bp.fitem_off[k] + threadIdx.x; i < bp.fitem_off[k + 1]; i += 256) fmap[i] = k;
    for (long long i = bp.titem_off[k] + threadIdx.x; i < bp.titem_off[k + 1]; i += 256) tmap[i] = k;
}

// ============================================================== field

// One workgroup per (sample, block of NR rows, row segment of 256*NPL nodes);
// the map gives the sample (heaviest samples first).  Same inner loop as the
// single-evaluation FP32 field (NPL nodes in each of NR rows per thread), and
// the same tile range partials (per sample).
template <int NPL, int NR>
__global__ __launch_bounds__(256) void k_bfield32(BatchPlan bp, const int* __restrict__ fmap,
                                                  const float* __restrict__ tab32, float* __restrict__ fx,
                                                  float* __restrict__ fy, float* __restrict__ rr)
{
    __shared__ float4 srow[NR * 256];
    const long long item = blockIdx.x;
    const int k = fmap[item];
    const int s = bp.perm[k];
    const GridDesc g = bp.grid[s];
    const int segs = (g.nx + 256 * NPL - 1) / (256 * NPL);
    const long long local = item - bp.fitem_off[k];
    const int j0 = (int)(local / segs) * NR, seg = (int)(local % segs);
    const int i0 = (seg * 256 + threadIdx.x) * NPL;
    const int p0 = bp.pot_off[0];
    const float* tab = tab32 + (size_t)(bp.pot_off[s] - p0) * T32_STRIDE;
    const int np = bp.pot_off[s + 1] - bp.pot_off[s];
    float fi[NPL], sx[NR * NPL], sy[NR * NPL];
#pragma unroll
    for (int q = 0; q < NPL; q++) fi[q] = (float)(i0 + q);
#pragma unroll
    for (int q = 0; q < NR * NPL; q++) {
        sx[q] = 0.0f;
        sy[q] = 0.0f;
    }
    field32_all_wg<NPL, NR>(tab, np, (float)j0, fi, sx, sy, srow);
    const int tiles_x = (g.nx - 2) / (1 << bp.tx_shift) + 1;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int j = j0 + r;
        if (j >= g.ny) break;  // uniform over the workgroup
        tile_partials<float, NPL>(sx + r * NPL, sy + r * NPL, i0, j, g.nx, bp.tx_shift, tiles_x, rr + bp.rr_off[s]);
        const size_t row = (size_t)bp.node_off[s] + (size_t)j * g.nx;
#pragma unroll
        for (int q = 0; q < NPL; q++) {
            if (i0 + q < g.nx) {
                fx[row + i0 + q] = sx[r * NPL + q];
                fy[row + i0 + q] = sy[r * NPL + q];
            }
        }
    }
}

// FP64 field: one workgroup per (sample, row segment of 256 nodes).
__global__ __launch_bounds__(256) void k_bfield64(BatchPlan bp, const int* __restrict__ fmap,
                                                  const double* __restrict__ tab64, double* __restrict__ fx,
                                                  double* __restrict__ fy, double* __restrict__ rr)
{
    const long long item = blockIdx.x;
    const int k = fmap[item];
    const int s = bp.perm[k];
    const GridDesc g = bp.grid[s];
    const int segs = (g.nx + 255) / 256;
    const long long local = item - bp.fitem_off[k];
    const int j = (int)(local / segs), i = (int)(local % segs) * 256 + threadIdx.x;
    const int p0 = bp.pot_off[0];
    const double* tab = tab64 + (size_t)(bp.pot_off[s] - p0) * T64_STRIDE;
    const int np = bp.pot_off[s + 1] - bp.pot_off[s];
    const double t1 = node_coord(g.x0, i, g.h), t2 = node_coord(g.y0, j, g.h);
    double s1 = 0.0, s2 = 0.0;
    alpha64_all_wg(tab, np, t1, t2, s1, s2);
    const int tiles_x = (g.nx - 2) / (1 << bp.tx_shift) + 1;
    tile_partials<double, 1>(&s1, &s2, i, j, g.nx, bp.tx_shift, tiles_x, rr + bp.rr_off[s]);
    if (i >= g.nx) return;
    const size_t n = (size_t)bp.node_off[s] + (size_t)j * g.nx + i;
    fx[n] = s1;
    fy[n] = s2;
}

// ============================================================== triangles

// One wave per (sample, tile row, block of 64 tile columns) work item,
// heaviest samples first; lane = tile column.  Each lane bounds its own
// tile's source-plane vertices from the range partials (loads of consecutive
// tiles are consecutive) and tests every system's barycentre against that
// box (system rows are wave-uniform), keeping a mask of the passing systems.
// The wave then stages each tile with a passing system in its own LDS tile
// (lane order) and tests its cells for those systems, all lanes over the
// cells.  Hits go to the sample's own list (system << 32 | triangle id),
// undecided tests to the batch list (sample << 44 | system << 31 | triangle
// id).
template <class S, typename V>
__global__ __launch_bounds__(256) void k_btri(BatchPlan bp, const int* __restrict__ tmap, long long n_items,
                                              int nsys, const double* __restrict__ sysrow, const V* __restrict__ fx,
                                              const V* __restrict__ fy, const V* __restrict__ rr, BatchState bs,
                                              int mode, double tau, int hcap, unsigned long long* __restrict__ hits,
                                              unsigned long long* __restrict__ flags, long long flag_cap,
                                              unsigned* __restrict__ part)
{
    __shared__ V sx[4][S::TNY][S::TNX], sy[4][S::TNY][S::TNX];
    __shared__ unsigned sp[4][2];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const long long item = (long long)blockIdx.x * 4 + wave;
    unsigned npair = 0, nbbox = 0;  // per lane: passing (tile, system) pairs of its tile; bbox passes
    if (item < n_items) {
        const int k = tmap[item];
        const int s = bp.perm[k];
        const GridDesc g = bp.grid[s];
        const int tiles_x = (g.nx - 2) / S::TX + 1;
        const int blocks_x = (tiles_x + 63) / 64;
        const int local = (int)(item - bp.titem_off[k]);
        const int band = local / blocks_x, cb = local - band * blocks_x;
        const int col = cb * 64 + lane;
        const bool act = col < tiles_x;
        const Tile T = tile_of<S>(g, tiles_x, band * tiles_x + (act ? col : 0));
        double rng[4] = {0.0, 0.0, 0.0, 0.0};
        if (act) tile_range_lane<S, V>(rr + bp.rr_off[s], tiles_x, T, rng);
        const double* rows = sysrow + (size_t)s * nsys * SYS_STRIDE;
        const V* sfx = fx + bp.node_off[s];
        const V* sfy = fy + bp.node_off[s];
        for (int sb = 0; sb < nsys; sb += 64) {
            const int ns = min(64, nsys - sb);
            // the chunk's system rows in one round of loads (lane = system), then broadcast
            double lr = 0.0, leb = 0.0, lbx = 0.0, lby = 0.0;
            if (lane < ns) {
                const double* row = rows + (size_t)(sb + lane) * SYS_STRIDE;
                lr = row[SYS_R];
                leb = sizeof(V) == 4 ? row[SYS_EB] : 1e-9;
                lbx = row[SYS_BX];
                lby = row[SYS_BY];
            }
            unsigned long long mask = 0;
            for (int c = 0; c < ns; c++) {
                if (act && tile_box_contains(g, T, rng, bcast(lr, c), bcast(leb, c), bcast(lbx, c), bcast(lby, c)))
                    mask |= 1ull << c;
            }
            npair += (unsigned)__popcll(mask);
            unsigned long long tiles = __ballot(mask != 0);
            // the passing tiles in lane order; for tiles of up to 40 bytes of
            // nodes per lane the next tile's nodes are loaded into registers
            // while the current one is tested
            constexpr bool kPre = TileRegs<S, V>::K * (int)sizeof(V) <= 40;
            int l = tiles ? __ffsll((long long)tiles) - 1 : 0;
            TileRegs<S, V> nxt;
            if (kPre && tiles)
                fetch_tile_regs<S, V>(sfx, sfy, g, tile_of<S>(g, tiles_x, band * tiles_x + cb * 64 + l), nxt);
            while (tiles) {
                tiles &= tiles - 1;
                unsigned long long m = __shfl(mask, l, 64);
                const Tile Tl = tile_of<S>(g, tiles_x, band * tiles_x + cb * 64 + l);
                if constexpr (kPre) {
                    store_tile_regs<S, V>(nxt, Tl, sx[wave], sy[wave]);
                    if (tiles) {
                        l = __ffsll((long long)tiles) - 1;
                        fetch_tile_regs<S, V>(sfx, sfy, g, tile_of<S>(g, tiles_x, band * tiles_x + cb * 64 + l), nxt);
                    }
                } else {
                    stage_tile_wave<S, V>(sfx, sfy, g, Tl, sx[wave], sy[wave]);
                    if (tiles) l = __ffsll((long long)tiles) - 1;
                }
                while (m) {
                    const int c = __ffsll((long long)m) - 1;
                    m &= m - 1;
                    const unsigned sys = (unsigned)(sb + c);
                    const double* row = rows + (size_t)sys * SYS_STRIDE;  // wave-uniform
                    if constexpr (sizeof(V) == 4) {
                        const float fr[6] = {(float)row[SYS_R],   (float)row[SYS_EB],  (float)row[SYS_BXH],
                                             (float)row[SYS_BXL], (float)row[SYS_BYH], (float)row[SYS_BYL]};
                        tri32_system<S, 64>(g, Tl, sx[wave], sy[wave], fr, ((unsigned long long)sys << 32),
                                            ((unsigned long long)s << 44) | ((unsigned long long)sys << 31), mode,
                                            (float)(tau * g.h * g.h), &bs.n_hits[s], hits + (size_t)s * hcap, hcap,
                                            bs.n_flags, flags, flag_cap, nbbox, lane);
                    } else {
                        tri64_system<S, 64>(g, Tl, sx[wave], sy[wave], row[SYS_R], row[SYS_BX], row[SYS_BY],
                                            ((unsigned long long)sys << 32), &bs.n_hits[s], hits + (size_t)s * hcap,
                                            hcap, nbbox, lane);
                    }
                }
            }
        }
    }
    // the pairs as a wave-uniform count, as write_part_sum takes them
    for (int m = 32; m >= 1; m >>= 1) npair += __shfl_xor(npair, m, 64);
    write_part_sum(part, blockIdx.x, npair, nbbox, sp);
}

// ============================================================== positions and fallback

// Workgroups [0, kBfbSub n): the FP64 position of every certain hit, one wave
// per hit, kBfbSub workgroups per sample.  The kBfbFlagBlocks workgroups
// beyond: persistent waves over the batch's undecided tests, each decided
// exactly on FP64 vertices and, if a hit, appended with its position to its
// sample's fallback list.  Each item is a chain of dependent steps (the three
// vertices over the potentials, the wave reductions, the position), so the
// launch spreads the items over many waves.
constexpr int kBfbSub = 4;
constexpr int kBfbFlagBlocks = 2048;
__global__ __launch_bounds__(256) void k_bfbpos(BatchPlan bp, int nsys, const double* __restrict__ tab64,
                                                const double* __restrict__ sysrow, BatchState bs, int hcap,
                                                const unsigned long long* __restrict__ hits,
                                                const unsigned long long* __restrict__ flags, long long flag_cap,
                                                unsigned long long* __restrict__ fb, double* __restrict__ pos,
                                                double* __restrict__ fb_pos)
{
    const int p0 = bp.pot_off[0];
    const int wave = threadIdx.x >> 6;
    if ((int)blockIdx.x < bp.n * kBfbSub) {
        const int s = blockIdx.x / kBfbSub, sub = blockIdx.x - s * kBfbSub;
        if (bs.status[s] != kStatusOk) return;
        const int nh = (int)min((unsigned long long)hcap, bs.n_hits[s]);
        const GridDesc g = bp.grid[s];
        const double* tab = tab64 + (size_t)(bp.pot_off[s] - p0) * T64_STRIDE;
        const int np = bp.pot_off[s + 1] - bp.pot_off[s];
        for (int q = sub * 4 + wave; q < nh; q += 4 * kBfbSub) {
            const unsigned long long key = hits[(size_t)s * hcap + q];
            const int sys = (int)(key >> 32), tid = (int)(key & 0xffffffffu);
            const double* row = sysrow + ((size_t)s * nsys + sys) * SYS_STRIDE;
            double vx[3], vy[3], tx[3], ty[3];
            vertices64(tab, np, g, tid, row[SYS_R], vx, vy, tx, ty);
            if (lane_id() == 0)
                image_position(vx, vy, tx, ty, row[SYS_BX], row[SYS_BY], pos[2 * ((size_t)s * hcap + q)],
                               pos[2 * ((size_t)s * hcap + q) + 1]);
        }
        return;
    }
    const long long nwaves = (long long)(gridDim.x - bp.n * kBfbSub) * 4;
    const long long w0 = (long long)(blockIdx.x - bp.n * kBfbSub) * 4 + wave;
    const long long nf = (long long)min((unsigned long long)flag_cap, *bs.n_flags);
    for (long long it = w0; it < nf; it += nwaves) {
        const unsigned long long key = flags[it];
        const int s = (int)(key >> 44), sys = (int)((key >> 31) & 0x1fff), tid = (int)(key & 0x7fffffffu);
        if (bs.status[s] != kStatusOk) continue;
        const GridDesc g = bp.grid[s];
        const double* tab = tab64 + (size_t)(bp.pot_off[s] - p0) * T64_STRIDE;
        const int np = bp.pot_off[s + 1] - bp.pot_off[s];
        const double* row = sysrow + ((size_t)s * nsys + sys) * SYS_STRIDE;
        double vx[3], vy[3], tx[3], ty[3];
        vertices64(tab, np, g, tid, row[SYS_R], vx, vy, tx, ty);
        if (lane_id() == 0 && contains_exact(vx, vy, row[SYS_BX], row[SYS_BY])) {
            const unsigned long long slot = atomicAdd(&bs.n_fb[s], 1ull);
            if ((long long)slot < hcap) {
                const size_t o = (size_t)s * hcap + slot;
                fb[o] = ((unsigned long long)sys << 32) | (unsigned)tid;
                image_position(vx, vy, tx, ty, row[SYS_BX], row[SYS_BY], fb_pos[2 * o], fb_pos[2 * o + 1]);
            }
        }
    }
}

// ============================================================== tail

// One workgroup of 256 threads per sample: merge the sample's certain and
// fallback hits, rank-sort them by (system, triangle id), pair each observed
// image with the nearest predicted image of its system (ties to the lower
// triangle id), chi2_i in image order (+inf without a predicted image) and
// chi^2 in a fixed order (Sec. 2.2.1).  Needs hcap <= 1024 and at most 1024
// images and systems (checked on the host).
__global__ __launch_bounds__(256) void k_btail(ObsPtrs obs, BatchState bs, int hcap,
                                               long long flag_cap, const unsigned long long* __restrict__ hits,
                                               const unsigned long long* __restrict__ fb,
                                               const double* __restrict__ pos, const double* __restrict__ fb_pos,
                                               double* __restrict__ chi2, double* __restrict__ chi2_sys,
                                               int* __restrict__ n_pred, int* __restrict__ status,
                                               unsigned long long* __restrict__ agg,
                                               const unsigned* __restrict__ part, long long n_parts,
                                               int* __restrict__ out_nh, int* __restrict__ out_hits,
                                               double* __restrict__ out_xy)
{
    constexpr int NT = 256, CAP = 2 * kTailStage;
    {  // chunk statistics (tile passes, bbox passes), one slice of the tiles per workgroup
        const long long per = (n_parts + gridDim.x - 1) / gridDim.x;
        const long long q0 = (long long)blockIdx.x * per, q1 = min(n_parts, q0 + per);
        unsigned long long a = 0, b = 0;
        for (long long q = q0 + threadIdx.x; q < q1; q += NT) {
            a += part[2 * q];
            b += part[2 * q + 1];
        }
        for (int m = 32; m >= 1; m >>= 1) {
            a += __shfl_xor(a, m, 64);
            b += __shfl_xor(b, m, 64);
        }
        if (lane_id() == 0 && (a | b) != 0) {
            atomicAdd(&agg[4], a);
            atomicAdd(&agg[5], b);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&agg[3], *bs.n_flags);  // undecided tests
    }
    __shared__ unsigned long long key[CAP];
    __shared__ double upx[CAP], upy[CAP];
    __shared__ double scon[kTailStage];
    __shared__ int sfirst[kTailStage], send[kTailStage];
    const int t = threadIdx.x, s = blockIdx.x;
    const int nimg = obs.n_img, nsys = obs.n_sys;
    const unsigned long long nc = bs.n_hits[s], nfb = bs.n_fb[s];
    int st = bs.status[s];
    const bool over = nc > (unsigned long long)hcap || nfb > (unsigned long long)hcap ||
                      *bs.n_flags > (unsigned long long)flag_cap;
    if (st == kStatusOk && over) st = kStatusCapacity;
    double* cs_out = chi2_sys + (size_t)s * nsys;
    int* np_out = n_pred + (size_t)s * nsys;
    if (t == 0) {
        status[s] = st;
        atomicAdd(&agg[0], nc + nfb);
        atomicAdd(&agg[1], nfb);
        if (st != kStatusOk) atomicAdd(&agg[2], 1ull);
    }
    if (st != kStatusOk) {
        for (int i = t; i < nsys; i += NT) {
            cs_out[i] = __builtin_nan("");
            np_out[i] = 0;
        }
        if (t == 0) {
            chi2[s] = __builtin_nan("");
            if (out_nh) out_nh[s] = 0;
        }
        return;
    }
    const int n = (int)(nc + nfb), ncert = (int)nc;
    for (int q = t; q < n; q += NT) {
        const bool c = q < ncert;
        const size_t o = (size_t)s * hcap + (c ? q : q - ncert);
        const unsigned long long h = c ? hits[o] : fb[o];
        key[q] = ((h >> 32) << 44) | ((h & 0x7fffffffull) << 12) | (unsigned long long)q;
        upx[q] = c ? pos[2 * o] : fb_pos[2 * o];
        upy[q] = c ? pos[2 * o + 1] : fb_pos[2 * o + 1];
    }
    for (int i = t; i < nsys; i += NT) {
        sfirst[i] = 0;
        send[i] = 0;
    }
    __syncthreads();
    {
        constexpr int PER = CAP / NT;
        unsigned long long mine[PER];
        int rank[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int q = t + NT * u;
            rank[u] = 0;
            mine[u] = q < n ? key[q] : 0;
            if (q < n)
                for (int r = 0; r < n; r++) rank[u] += key[r] < mine[u];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; u++)
            if (t + NT * u < n) key[rank[u]] = mine[u];
        __syncthreads();
    }
    for (int q = t; q < n; q += NT) {
        const int sy = (int)(key[q] >> 44);
        if (q == 0 || (int)(key[q - 1] >> 44) != sy) sfirst[sy] = q;
        if (q == n - 1 || (int)(key[q + 1] >> 44) != sy) send[sy] = q + 1;
        if (out_hits) {  // the sorted hits and their positions, as the single evaluation writes them
            const size_t o = (size_t)s * hcap + q;
            const int idx = (int)(key[q] & 0xfff);
            out_hits[2 * o] = sy;
            out_hits[2 * o + 1] = (int)((key[q] >> 12) & 0x7fffffffull);
            out_xy[2 * o] = upx[idx];
            out_xy[2 * o + 1] = upy[idx];
        }
    }
    if (out_nh && t == 0) out_nh[s] = n;
    __syncthreads();
    for (int j = t; j < nimg; j += NT) {
        const int i = system_of(obs.sys_off, nsys, j);
        int best = -1;
        double bd = 0.0;
        const double ox = obs.x[j], oy = obs.y[j];
        for (int q = sfirst[i]; q < send[i]; q++) {
            const int idx = (int)(key[q] & 0xfff);
            const double dx = ox - upx[idx], dy = oy - upy[idx];
            const double d2 = dx * dx + dy * dy;
            if (best < 0 || d2 < bd) {
                best = q;
                bd = d2;
            }
        }
        const double sg = obs.sigma[j];
        scon[j] = best >= 0 ? bd / (sg * sg) : 0.0;
    }
    __syncthreads();
    for (int i = t; i < nsys; i += NT) {
        double c = 0.0;
        for (int j = obs.sys_off[i]; j < obs.sys_off[i + 1]; j++) c += scon[j];
        c = send[i] > sfirst[i] ? c : INFINITY;
        cs_out[i] = c;
        np_out[i] = send[i] - sfirst[i];
        upx[i] = c;
    }
    __syncthreads();
    if (t < 64) {
        double v = 0.0;
        for (int i = t; i < nsys; i += 64) v += upx[i];
        v = wave_sum(v);
        if (t == 0) chi2[s] = v;
    }
}

// ============================================================== launchers

static inline unsigned bcdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_bhead(const BatchPlan& bp, const PotPtrs& pot, const ObsPtrs& obs, double* tab64, float* tab32,
                        double* bterm, double* bx, double* by, int np_chunk, hipStream_t s)
{
    long long nb = bcdiv((long long)bp.n * obs.n_img, 4);
    const long long nb2 = bcdiv(np_chunk, 256);
    if (nb < nb2) nb = nb2;
    if (nb < 1) nb = 1;
    if (nb > 4096) nb = 4096;
    k_bhead<<<(unsigned)nb, 256, 0, s>>>(bp, pot, obs, tab64, tab32, bterm, bx, by);
    return hipGetLastError();
}

hipError_t launch_bsys(const BatchPlan& bp, const ObsPtrs& obs, const double* bterm, const double* bx,
                       const double* by, double* sysrow, const BatchState& bs, hipStream_t s)
{
    k_bsys<<<bcdiv(bp.n, 4), 256, 0, s>>>(bp, obs, bterm, bx, by, sysrow, bs);
    return hipGetLastError();
}

hipError_t launch_bmap(const BatchPlan& bp, int* fmap, int* tmap, hipStream_t s)
{
    k_bmap<<<bp.n, 256, 0, s>>>(bp, fmap, tmap);
    return hipGetLastError();
}

hipError_t launch_bfield32(const BatchPlan& bp, const int* fmap, long long n_items, const float* tab32, float* fx,
                           float* fy, float* rr, int npl, const KernelEvents* ev, hipStream_t s)
{
    const dim3 grid((unsigned)n_items), block(256);
    switch (npl) {
    case 0x01: return launch_ev(ev, k_bfield32<1, 1>, grid, block, s, bp, fmap, tab32, fx, fy, rr);
    case 0x04: return launch_ev(ev, k_bfield32<4, 1>, grid, block, s, bp, fmap, tab32, fx, fy, rr);
    case 0x21: return launch_ev(ev, k_bfield32<1, 2>, grid, block, s, bp, fmap, tab32, fx, fy, rr);
    case 0x22: return launch_ev(ev, k_bfield32<2, 2>, grid, block, s, bp, fmap, tab32, fx, fy, rr);
    case 0x41: return launch_ev(ev, k_bfield32<1, 4>, grid, block, s, bp, fmap, tab32, fx, fy, rr);
    default: return launch_ev(ev, k_bfield32<2, 1>, grid, block, s, bp, fmap, tab32, fx, fy, rr);
    }
}

hipError_t launch_bfield64(const BatchPlan& bp, const int* fmap, long long n_items, const double* tab64, double* fx,
                           double* fy, double* rr, const KernelEvents* ev, hipStream_t s)
{
    return launch_ev(ev, k_bfield64, dim3((unsigned)n_items), dim3(256), s, bp, fmap, tab64, fx, fy, rr);
}

template <class F>
static hipError_t with_bshape(int shape, F f)
{
    switch (shape) {
    case 2: return f(TileShape<64, 16>());
    case 3: return f(TileShape<64, 8>());
    case 4: return f(TileShape<32, 16>());
    default: return f(TileShape<32, 8>());
    }
}

hipError_t launch_btri(const BatchPlan& bp, const int* tmap, long long n_items, int nsys, const double* sysrow,
                       const void* fx, const void* fy, const void* rr, bool fp32, const BatchState& bs, int mode,
                       double tau, int hcap, unsigned long long* hits, unsigned long long* flags, long long flag_cap,
                       unsigned* part, int shape, hipStream_t s)
{
    const unsigned nb = (unsigned)((n_items + 3) / 4);
    return with_bshape(shape, [&](auto sh) {
        using S = decltype(sh);
        if (fp32)
            k_btri<S, float><<<nb, 256, 0, s>>>(bp, tmap, n_items, nsys, sysrow, (const float*)fx, (const float*)fy,
                                                (const float*)rr, bs, mode, tau, hcap, hits, flags, flag_cap, part);
        else
            k_btri<S, double><<<nb, 256, 0, s>>>(bp, tmap, n_items, nsys, sysrow, (const double*)fx,
                                                 (const double*)fy, (const double*)rr, bs, mode, tau, hcap, hits,
                                                 flags, flag_cap, part);
        return hipGetLastError();
    });
}

hipError_t launch_bfbpos(const BatchPlan& bp, int nsys, const double* tab64, const double* sysrow,
                         const BatchState& bs, int hcap, const unsigned long long* hits,
                         const unsigned long long* flags, long long flag_cap, unsigned long long* fb, double* pos,
                         double* fb_pos, hipStream_t s)
{
    k_bfbpos<<<bp.n * kBfbSub + kBfbFlagBlocks, 256, 0, s>>>(bp, nsys, tab64, sysrow, bs, hcap, hits, flags,
                                                             flag_cap, fb, pos, fb_pos);
    return hipGetLastError();
}

hipError_t launch_btail(const BatchPlan& bp, const ObsPtrs& obs, const BatchState& bs, int hcap, long long flag_cap,
                        const unsigned long long* hits, const unsigned long long* fb, const double* pos,
                        const double* fb_pos, double* chi2, double* chi2_sys, int* n_pred, int* status,
                        unsigned long long* agg, const unsigned* part, long long n_parts, int* out_nh,
                        int* out_hits, double* out_xy, hipStream_t s)
{
    k_btail<<<bp.n, 256, 0, s>>>(obs, bs, hcap, flag_cap, hits, fb, pos, fb_pos, chi2, chi2_sys, n_pred, status,
                                 agg, part, n_parts, out_nh, out_hits, out_xy);
    return hipGetLastError();
}

__global__ void k_zero_u64(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_bstats(const unsigned long long* agg, long long n_tests, long long* stats)
{
    if (threadIdx.x == 0) {
        stats[0] = (long long)agg[0];  // hits
        stats[1] = (long long)agg[3];  // undecided FP32 tests
        stats[2] = (long long)agg[4];  // (tile, system) pairs
        stats[3] = (long long)agg[5];  // bounding-box passes
        stats[4] = agg[2] ? 1 : 0;     // any sample not OK
        stats[5] = (long long)agg[1];  // fallback hits
        stats[6] = n_tests;
        stats[7] = (long long)agg[2];  // samples not OK
    }
}

hipError_t launch_bstats(const unsigned long long* agg, long long n_tests, long long* stats, hipStream_t s)
{
    k_bstats<<<1, 64, 0, s>>>(agg, n_tests, stats);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s)
{
    k_zero_u64<<<bcdiv(n, 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace lens
