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
#include "lens_path.hpp"

namespace lens {

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
    for (int p = blockIdx.x * 256 + t; p < np; p += gridDim.x * 256) prep_one(pot, g, p, p, tab64, tab32, bterm);
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

// Each thread owns NPL consecutive nodes of one grid row; a workgroup of 256
// threads covers 256*NPL nodes of that row, so the row offset is uniform and
// every per-potential constant is a wave-uniform (scalar) operand.  With rr
// set, the kernel also writes the triangle stage's per-(row, tile column)
// deflection ranges (tile width 1 << tx_shift cells).
template <int NPL>
__global__ __launch_bounds__(256) void k_field32(const float* __restrict__ tab32, int np, int nx, int ny,
                                                 float* __restrict__ ax, float* __restrict__ ay,
                                                 const EvalState* __restrict__ st, float* __restrict__ rr,
                                                 int tx_shift, int tiles_x)
{
    const int j = blockIdx.y;
    const int i0 = (blockIdx.x * 256 + threadIdx.x) * NPL;
    if ((int)(blockIdx.x * 256 * NPL) >= nx) return;  // whole workgroup beyond the row
    const float fj = (float)j;
    float fi[NPL], sx[NPL], sy[NPL];
#pragma unroll
    for (int k = 0; k < NPL; k++) {
        fi[k] = (float)(i0 + k);
        sx[k] = 0.0f;
        sy[k] = 0.0f;
    }
    field32_all<NPL>(tab32, np, fj, fi, sx, sy);
    if (rr) tile_partials<NPL>(sx, sy, i0, j, nx, tx_shift, tiles_x, rr);
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

// Mixed path.  Persistent workgroups (4 waves) walk the tiles of S::TX x S::TY
// cells; the loads of the next tile are in flight while the current one is
// processed.  A tile's FP32 deflections (with a one-node halo) are staged in
// LDS; a system whose barycentre lies outside the tile's source-plane box is
// skipped for the whole tile.  Systems are tested 64 at a time, one per lane,
// and the survivors enumerated from the ballot mask.
template <class S>
__global__ __launch_bounds__(256) void k_tri32(const float* __restrict__ ax, const float* __restrict__ ay,
                                               GridDesc g, int tiles_x, int n_tiles, int nsys,
                                               const double* __restrict__ sysrow, EvalState* __restrict__ st,
                                               int mode, float tau, unsigned long long* __restrict__ hit_keys,
                                               long long hit_cap, unsigned long long* __restrict__ flag_keys,
                                               long long flag_cap, unsigned* __restrict__ part)
{
    __shared__ float sx[S::TNY][S::TNX], sy[S::TNY][S::TNX];
    __shared__ float wred[4][4];
    __shared__ SysChunk chunk;
    __shared__ unsigned sbb[4];
    const bool one_chunk = nsys <= SYS_CHUNK;
    if (one_chunk) load_chunk(chunk, sysrow, nsys, 0);
    const int lane = lane_id();
    unsigned nbbox = 0, ntile = 0;
    float vx[S::LOADS], vy[S::LOADS];
    int tile = blockIdx.x;
    Tile T = tile_of<S>(g, tiles_x, tile);
    if (tile < n_tiles) load_tile<S>(ax, ay, g, T, vx, vy);
    for (; tile < n_tiles; tile += gridDim.x) {
        float rngf[4];
        stage_tile<S>(T, vx, vy, sx, sy, wred, rngf);
        const Tile cur = T;
        const int next = tile + gridDim.x;
        if (next < n_tiles) {
            T = tile_of<S>(g, tiles_x, next);
            load_tile<S>(ax, ay, g, T, vx, vy);
        }
        const double rng[4] = {rngf[0], rngf[1], rngf[2], rngf[3]};
        for (int cbase = 0; cbase < nsys; cbase += SYS_CHUNK) {
            if (!one_chunk) {
                __syncthreads();
                load_chunk(chunk, sysrow, nsys, cbase);
                __syncthreads();
            }
            const int nc = min(SYS_CHUNK, nsys - cbase);
            for (int sbase = 0; sbase < nc; sbase += 64) {
                const int sl = sbase + lane;
                const bool pass = sl < nc && tile_box_contains(g, cur, rng, chunk.r[sl], chunk.eb[sl],
                                                               chunk.bx[sl], chunk.by[sl]);
                unsigned long long m = __ballot(pass);
                ntile += __popcll(m);
                while (m) {
                    const int s = sbase + __ffsll((long long)m) - 1;
                    m &= m - 1;
                    const unsigned long long base = (unsigned long long)(cbase + s) << 32;
                    tri32_system<S>(g, cur, sx, sy, chunk.f[s], base, base, mode, tau, &st->n_hits, hit_keys,
                                    hit_cap, &st->n_flags, flag_keys, flag_cap, nbbox);
                }
            }
        }
        __syncthreads();  // the LDS tile is overwritten by the next iteration
    }
    write_part(part, blockIdx.x, ntile, nbbox, sbb);
}

// Mixed path, one wave per tile: the tile's deflection range comes from the
// field kernel's row partials (plus the halo column), so a tile that no
// system's barycentre can reach costs a few small loads; only tiles with a
// surviving system are staged (in a wave-private LDS tile) and tested.
template <class S>
__global__ __launch_bounds__(256) void k_tri32w(const float* __restrict__ ax, const float* __restrict__ ay,
                                                const float* __restrict__ rr, GridDesc g, int tiles_x, int n_tiles,
                                                int nsys, const double* __restrict__ sysrow,
                                                EvalState* __restrict__ st, int mode, float tau,
                                                unsigned long long* __restrict__ hit_keys, long long hit_cap,
                                                unsigned long long* __restrict__ flag_keys, long long flag_cap,
                                                unsigned* __restrict__ part)
{
    __shared__ float sx[4][S::TNY][S::TNX], sy[4][S::TNY][S::TNX];
    __shared__ SysChunk chunk;
    __shared__ unsigned sbb[4];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int tile = blockIdx.x * 4 + wave;
    const bool one_chunk = nsys <= SYS_CHUNK;
    if (one_chunk) {
        load_chunk(chunk, sysrow, nsys, 0);
        __syncthreads();
    }
    unsigned nbbox = 0, ntile = 0;
    const bool active = tile < n_tiles;
    Tile T = {0, 0, 0, 0};
    double rng[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        T = tile_of<S>(g, tiles_x, tile);
        float r4[4];
        tile_range_wave<S>(ax, ay, rr, g, tiles_x, T, r4);
        rng[0] = r4[0];
        rng[1] = r4[1];
        rng[2] = r4[2];
        rng[3] = r4[3];
    }
    bool staged = false;
    for (int cbase = 0; cbase < nsys; cbase += SYS_CHUNK) {
        if (!one_chunk) {
            __syncthreads();
            load_chunk(chunk, sysrow, nsys, cbase);
            __syncthreads();
        }
        if (!active) continue;
        const int nc = min(SYS_CHUNK, nsys - cbase);
        for (int sbase = 0; sbase < nc; sbase += 64) {
            const int sl = sbase + lane;
            const bool pass = sl < nc && tile_box_contains(g, T, rng, chunk.r[sl], chunk.eb[sl], chunk.bx[sl],
                                                           chunk.by[sl]);
            unsigned long long m = __ballot(pass);
            ntile += __popcll(m);
            if (m != 0 && !staged) {
                stage_tile_wave<S>(ax, ay, g, T, sx[wave], sy[wave]);
                staged = true;
            }
            while (m) {
                const int s = sbase + __ffsll((long long)m) - 1;
                m &= m - 1;
                const unsigned long long base = (unsigned long long)(cbase + s) << 32;
                tri32_wave_system<S>(g, T, sx[wave], sy[wave], chunk.f[s], base, base, mode, tau, &st->n_hits,
                                     hit_keys, hit_cap, &st->n_flags, flag_keys, flag_cap, nbbox);
            }
        }
    }
    write_part(part, blockIdx.x, ntile, nbbox, sbb);
}

// FP64 path: same walk, FP64 deflections in LDS, every surviving triangle
// decided exactly.
template <class S>
__global__ __launch_bounds__(256) void k_tri64(const double* __restrict__ ax, const double* __restrict__ ay,
                                               GridDesc g, int tiles_x, int n_tiles, int nsys,
                                               const double* __restrict__ sysrow, EvalState* __restrict__ st,
                                               unsigned long long* __restrict__ hit_keys, long long hit_cap,
                                               unsigned* __restrict__ part)
{
    __shared__ double sx[S::TNY][S::TNX], sy[S::TNY][S::TNX];
    __shared__ double wred[4][4];
    __shared__ SysChunk chunk;
    __shared__ unsigned sbb[4];
    const bool one_chunk = nsys <= SYS_CHUNK;
    if (one_chunk) load_chunk(chunk, sysrow, nsys, 0);
    const int lane = lane_id();
    unsigned nbbox = 0, ntile = 0;
    double vx[S::LOADS], vy[S::LOADS];
    int tile = blockIdx.x;
    Tile T = tile_of<S>(g, tiles_x, tile);
    if (tile < n_tiles) load_tile<S>(ax, ay, g, T, vx, vy);
    for (; tile < n_tiles; tile += gridDim.x) {
        double rng[4];
        stage_tile<S>(T, vx, vy, sx, sy, wred, rng);
        const Tile cur = T;
        const int next = tile + gridDim.x;
        if (next < n_tiles) {
            T = tile_of<S>(g, tiles_x, next);
            load_tile<S>(ax, ay, g, T, vx, vy);
        }
        for (int cbase = 0; cbase < nsys; cbase += SYS_CHUNK) {
            if (!one_chunk) {
                __syncthreads();
                load_chunk(chunk, sysrow, nsys, cbase);
                __syncthreads();
            }
            const int nc = min(SYS_CHUNK, nsys - cbase);
            for (int sbase = 0; sbase < nc; sbase += 64) {
                const int sl = sbase + lane;
                // 1e-9 arcsec covers the FP64 rounding of the box
                const bool pass = sl < nc && tile_box_contains(g, cur, rng, chunk.r[sl], 1e-9, chunk.bx[sl],
                                                               chunk.by[sl]);
                unsigned long long m = __ballot(pass);
                ntile += __popcll(m);
                while (m) {
                    const int s = sbase + __ffsll((long long)m) - 1;
                    m &= m - 1;
                    tri64_system<S>(g, cur, sx, sy, chunk.r[s], chunk.bx[s], chunk.by[s],
                                    (unsigned long long)(cbase + s) << 32, &st->n_hits, hit_keys, hit_cap, nbbox);
                }
            }
        }
        __syncthreads();
    }
    write_part(part, blockIdx.x, ntile, nbbox, sbb);
}

// ============================================================== FP64 fallback, positions, tail

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
                          const EvalState* st, int npl, float* rr, int tx_shift, int tiles_x,
                          const KernelEvents* ev, hipStream_t s)
{
    switch (npl) {
    case 1: return launch_ev(ev, k_field32<1>, dim3(cdiv(g.nx, 256), g.ny), dim3(256), s, tab32, np, g.nx, g.ny, ax, ay, st, rr, tx_shift, tiles_x);
    case 2: return launch_ev(ev, k_field32<2>, dim3(cdiv(g.nx, 512), g.ny), dim3(256), s, tab32, np, g.nx, g.ny, ax, ay, st, rr, tx_shift, tiles_x);
    case 4: return launch_ev(ev, k_field32<4>, dim3(cdiv(g.nx, 1024), g.ny), dim3(256), s, tab32, np, g.nx, g.ny, ax, ay, st, rr, tx_shift, tiles_x);
    default: return launch_ev(ev, k_field32<8>, dim3(cdiv(g.nx, 2048), g.ny), dim3(256), s, tab32, np, g.nx, g.ny, ax, ay, st, rr, tx_shift, tiles_x);
    }
}

hipError_t launch_field64(const double* tab64, int np, const GridDesc& g, double* ax, double* ay,
                          const EvalState* st, const KernelEvents* ev, hipStream_t s)
{
    return launch_ev(ev, k_field64, dim3(cdiv(g.nx, 256), g.ny), dim3(256), s, tab64, np, g, ax, ay, st);
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

// Workgroups of the triangle stage: FP32, one wave per tile; FP64, persistent.
int tri_blocks(const GridDesc& g, int shape, bool fp32)
{
    int tx, ty;
    tile_dims(shape, tx, ty);
    const long long n_tiles = (long long)cdiv(g.nx - 1, tx) * cdiv(g.ny - 1, ty);
    if (fp32) return (int)cdiv(n_tiles, 4);
    return (int)(n_tiles < kTriBlocks ? n_tiles : kTriBlocks);
}

hipError_t launch_tri32(const float* ax, const float* ay, const float* rr, const GridDesc& g, int nsys,
                        const double* sysrow, EvalState* st, int mode, float tau, unsigned long long* hit_keys,
                        long long hit_cap, unsigned long long* flag_keys, long long flag_cap, unsigned* part,
                        int shape, hipStream_t s)
{
    return with_shape(shape, [&](auto sh) {
        using S = decltype(sh);
        const int tiles_x = (int)cdiv(g.nx - 1, S::TX);
        const int n_tiles = tiles_x * (int)cdiv(g.ny - 1, S::TY);
        k_tri32w<S><<<tri_blocks(g, shape, true), 256, 0, s>>>(ax, ay, rr, g, tiles_x, n_tiles, nsys, sysrow, st,
                                                               mode, tau, hit_keys, hit_cap, flag_keys, flag_cap,
                                                               part);
        return hipGetLastError();
    });
}

hipError_t launch_tri64(const double* ax, const double* ay, const GridDesc& g, int nsys, const double* sysrow,
                        EvalState* st, unsigned long long* hit_keys, long long hit_cap, unsigned* part, int shape,
                        hipStream_t s)
{
    return with_shape(shape, [&](auto sh) {
        using S = decltype(sh);
        const int tiles_x = (int)cdiv(g.nx - 1, S::TX);
        const int n_tiles = tiles_x * (int)cdiv(g.ny - 1, S::TY);
        k_tri64<S><<<tri_blocks(g, shape, false), 256, 0, s>>>(ax, ay, g, tiles_x, n_tiles, nsys, sysrow, st, hit_keys,
                                                        hit_cap, part);
        return hipGetLastError();
    });
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
