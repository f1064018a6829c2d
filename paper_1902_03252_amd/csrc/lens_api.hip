// C ABI of the gfx950 chi^2 library (declared in include/lens.h): argument
// checks on the host, context scratch, and the launch sequence of each entry
// point.  No C++ exception crosses this file's extern "C" functions.
#include "lens.h"
#include "lens_device.hpp"
#include "lens_internal.hpp"
#include "lens_tune.hpp"

#include <algorithm>
#include <climits>
#include <mutex>
#include <cmath>
#include <stdlib.h>
#include <string.h>
#include <vector>

using namespace lens;

namespace {

enum Buf { B_TAB64, B_TAB32, B_BTERM, B_FIELD, B_BX, B_BY, B_SYS, B_STATE, B_HITS, B_FLAGS, B_POS, B_CONTRIB,
           B_PART, B_BCOUNT, B_VJP, B_SRC, B_SRCST, B_RR, B_PAIRS, B_MIX, B_MLIST, B_MMASK, B_HMC, B_MHP, B_NFW, B_NBUF };

// Device work plan of one chunk of a batch (see lens_image_chi2_batched).
struct PlanChunk {
    int s0, n, np;            // first sample, samples, parameter columns
    long long n_fitems, n_tiles, n_nodes, n_tests, n_rr;
    void* host_stage;         // pinned source of the plan upload, freed with the plan
    void* dev_plan;
    int* fmap;
    int* tmap;
    BatchPlan bp;
};

struct PlanEntry {
    std::vector<int32_t> pot_off;
    std::vector<double> grids;  // x0, y0, h, nx, ny per sample
    int npl, shape, fp32;
    std::vector<PlanChunk> chunks;
};

constexpr int kMaxPlans = 16;  // cached batch plans per context

void release_plan(PlanEntry* e)
{
    for (PlanChunk& ch : e->chunks) {
        (void)hipHostFree(ch.host_stage);
        (void)hipFree(ch.dev_plan);
        (void)hipFree(ch.fmap);
        (void)hipFree(ch.tmap);
    }
    delete e;
}

}  // namespace

constexpr int kMaxPending = 1024;  // event pairs awaiting lens_field_timing

struct lens_ctx {
    int device;
    void* buf[B_NBUF];
    size_t cap[B_NBUF];
    // field-kernel timing
    int timing;
    int n_pending;
    hipEvent_t ev_start[kMaxPending], ev_stop[kMaxPending];
    int n_events;  // events created so far (pairs)
    double total_ms;
    long long launches;
    std::vector<PlanEntry*>* plans;  // batch plans, one per distinct shape class
    TuneTable* tune;                 // autotuned tile shape / nodes per thread per bucket
};

namespace {
void* noalloc_scratch(int dev);  // the fixed scratch of lens_image_chi2_noalloc (below)
}  // namespace

TuneTable* lens_ctx_tune(lens_ctx* ctx) { return ctx ? ctx->tune : nullptr; }
int lens_ctx_device(lens_ctx* ctx) { return ctx->device; }
int lens_ctx_timing(lens_ctx* ctx) { return ctx->timing; }

namespace {

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Grows scratch buffer `which` to at least `bytes`.  Growing frees the old
// block after a device synchronisation, so earlier asynchronous calls that
// still read it have finished.
int ensure(lens_ctx* c, int which, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (c->cap[which] >= bytes) return LENS_OK;
    size_t nb = c->cap[which] + c->cap[which] / 2;
    if (nb < bytes) nb = bytes;
    nb = (nb + 255) & ~(size_t)255;
    if (c->buf[which]) {
        if (hipDeviceSynchronize() != hipSuccess) return LENS_ERR_DEVICE;
        (void)hipFree(c->buf[which]);
        c->buf[which] = nullptr;
        c->cap[which] = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, nb) != hipSuccess) return LENS_ERR_DEVICE;
    if ((which == B_STATE || which == B_SRCST) && hipMemset(p, 0, nb) != hipSuccess)
        return LENS_ERR_DEVICE;  // tickets start at 0
    c->buf[which] = p;
    c->cap[which] = nb;
    return LENS_OK;
}

bool is_fin(double v) { return std::isfinite(v); }

int check_pot(const lens_potentials* pot)
{
    if (!pot || pot->n < 0) return LENS_ERR_INVALID;
    if (pot->n > 0 && (!pot->x || !pot->y || !pot->eps || !pot->phi || !pot->r_core || !pot->r_cut || !pot->sigma_v))
        return LENS_ERR_INVALID;
    return LENS_OK;
}

int check_grid(const lens_grid* g)
{
    if (!g || g->nx < 2 || g->ny < 2 || g->ny > 65535 || !(g->h > 0.0) || !is_fin(g->h) || !is_fin(g->x0) ||
        !is_fin(g->y0))
        return LENS_ERR_INVALID;
    if ((long long)(g->nx - 1) * (long long)(g->ny - 1) >= (1ll << 30)) return LENS_ERR_INVALID;  // int32 ids
    return LENS_OK;
}

int check_obs(const lens_obs* o)
{
    if (!o || o->n_sys < 1 || o->n_sys >= kMaxSystems || o->n_img < 0 || !o->sys_off || !o->dls_dos)
        return LENS_ERR_INVALID;
    if (o->n_img > 0 && (!o->x || !o->y || !o->sigma)) return LENS_ERR_INVALID;
    return LENS_OK;
}

PotPtrs pot_ptrs(const lens_potentials* p)
{
    PotPtrs q;
    q.n = p->n;
    q.x = p->x;
    q.y = p->y;
    q.eps = p->eps;
    q.phi = p->phi;
    q.r_core = p->r_core;
    q.r_cut = p->r_cut;
    q.sigma_v = p->sigma_v;
    return q;
}

GridDesc grid_desc(const lens_grid* g)
{
    GridDesc d;
    d.x0 = g->x0;
    d.y0 = g->y0;
    d.h = g->h;
    d.nx = g->nx;
    d.ny = g->ny;
    return d;
}

ObsPtrs obs_ptrs(const lens_obs* o)
{
    ObsPtrs q;
    q.n_sys = o->n_sys;
    q.n_img = o->n_img;
    q.sys_off = o->sys_off;
    q.x = o->x;
    q.y = o->y;
    q.sigma = o->sigma;
    q.dls = o->dls_dos;
    return q;
}

// Nodes per thread of the FP32 field kernel: enough waves to fill 256 CUs,
// as many nodes per thread as that allows (amortises the per-row work and
// overlaps the transcendental latency); from 8M nodes on, one column of four
// rows (the column offset shared by the rows; measured fastest at 4096^2).
// LENS_FIELD_NPL overrides.
int field_npl(const GridDesc& g)
{
    const char* env = getenv("LENS_FIELD_NPL");
    if (env) {
        const int v = (int)strtol(env, nullptr, 0);
        if (field_code_ok(v)) return v;
    }
    const long long nodes = (long long)g.nx * g.ny;
    if (nodes >= (8ll << 20)) return 0x41;
    if (nodes >= (1ll << 20)) return 2;
    return 1;
}

// Fills a zero tile shape / nodes per thread from the autotuned table entry of
// the call's bucket, when there is one.
void resolve_tuned(lens_ctx* ctx, int prec, int batched, long long side, long long np, int& shape, int& npl)
{
    if (shape && npl) return;
    int t = 0, n = 0;
    if (!tune_lookup(ctx ? ctx->tune : nullptr, prec, batched, tune_log2(side), tune_log2(np), &t, &n)) return;
    if (!shape) shape = t;
    if (!npl) npl = n;
}

// Folds every recorded (start, stop) pair into the totals.
int fold_timing(lens_ctx* c)
{
    for (int k = 0; k < c->n_pending; k++) {
        float ms = 0.0f;
        if (hipEventSynchronize(c->ev_stop[k]) != hipSuccess) return LENS_ERR_DEVICE;
        if (hipEventElapsedTime(&ms, c->ev_start[k], c->ev_stop[k]) != hipSuccess) return LENS_ERR_DEVICE;
        c->total_ms += ms;
        c->launches++;
    }
    c->n_pending = 0;
    return LENS_OK;
}

// Event pair for the next timed kernel: *ev is null when timing is off, else
// it points to the pair, which the kernel's dispatch records around itself.
int timing_begin(lens_ctx* c, KernelEvents* store, const KernelEvents** ev, int* slot)
{
    *slot = -1;
    *ev = nullptr;
    if (!c->timing) return LENS_OK;
    if (c->n_pending == kMaxPending) {
        int rc = fold_timing(c);
        if (rc) return rc;
    }
    const int k = c->n_pending;
    if (k >= c->n_events) {
        if (hipEventCreate(&c->ev_start[k]) != hipSuccess || hipEventCreate(&c->ev_stop[k]) != hipSuccess)
            return LENS_ERR_DEVICE;
        c->n_events = k + 1;
    }
    store->start = c->ev_start[k];
    store->stop = c->ev_stop[k];
    *ev = store;
    *slot = k;
    return LENS_OK;
}

// Marks the pair of a launched timed kernel as pending.
void timing_end(lens_ctx* c, int slot)
{
    if (slot >= 0) c->n_pending = slot + 1;
}

// Constants, source positions, barycentres and error bound: the head of every
// entry point (obs may have no systems and no images).
int head_buffers(lens_ctx* c, int np, const ObsPtrs& obs)
{
    int rc;
    if ((rc = ensure(c, B_TAB64, (size_t)np * T64_STRIDE * 8)) ||
        (rc = ensure(c, B_TAB32, (size_t)np * T32_STRIDE * 4)) || (rc = ensure(c, B_BTERM, (size_t)np * 3 * 8)) ||
        (rc = ensure(c, B_SYS, (size_t)(obs.n_sys > 0 ? obs.n_sys : 1) * SYS_STRIDE * 8)) ||
        (rc = ensure(c, B_STATE, sizeof(EvalState))))
        return rc;
    return LENS_OK;
}

int head(lens_ctx* c, const lens_potentials* pot, const GridDesc& g, const ObsPtrs& obs, double* bx, double* by,
         hipStream_t s)
{
    int rc;
    if ((rc = head_buffers(c, pot->n, obs))) return rc;
    if (launch_head(pot_ptrs(pot), g, obs, (double*)c->buf[B_TAB64], (float*)c->buf[B_TAB32],
                    (double*)c->buf[B_BTERM], bx, by, (double*)c->buf[B_SYS], (EvalState*)c->buf[B_STATE],
                    s) != hipSuccess)
        return LENS_ERR_DEVICE;
    return LENS_OK;
}

ObsPtrs no_obs()
{
    ObsPtrs q;
    memset(&q, 0, sizeof q);
    return q;
}

}  // namespace

int lens_default_field_npl(int nx, int ny)
{
    GridDesc g{};
    g.nx = nx;
    g.ny = ny;
    return field_npl(g);
}

extern "C" {

int lens_create(lens_ctx** ctx, int device)
{
    if (!ctx) return LENS_ERR_INVALID;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return LENS_ERR_DEVICE;
    if (device < 0 || device >= n) return LENS_ERR_INVALID;
    lens_ctx* c = (lens_ctx*)calloc(1, sizeof(lens_ctx));
    if (!c) return LENS_ERR_DEVICE;
    c->device = device;
    c->plans = new (std::nothrow) std::vector<PlanEntry*>();
    c->tune = tune_new();
    if (!c->plans || !c->tune) {
        delete c->plans;
        tune_delete(c->tune);
        free(c);
        return LENS_ERR_DEVICE;
    }
    // a missing or malformed cache file leaves the table empty
    const char* cache = getenv("LENS_AUTOTUNE_CACHE");
    hipDeviceProp_t prop;
    if (cache && *cache && hipGetDeviceProperties(&prop, device) == hipSuccess)
        (void)tune_load(c->tune, cache, prop.gcnArchName);
    {
        // set-up of the no-allocation entry point's fixed scratch on this
        // device (a failure is reported by that entry point)
        DeviceGuard dg(device);
        if (dg.ok) (void)noalloc_scratch(device);
    }
    *ctx = c;
    return LENS_OK;
}

void lens_destroy(lens_ctx* ctx)
{
    if (!ctx) return;
    {
        DeviceGuard dg(ctx->device);
        (void)hipDeviceSynchronize();
        for (int k = 0; k < B_NBUF; k++)
            if (ctx->buf[k]) (void)hipFree(ctx->buf[k]);
        for (int k = 0; k < ctx->n_events; k++) {
            (void)hipEventDestroy(ctx->ev_start[k]);
            (void)hipEventDestroy(ctx->ev_stop[k]);
        }
        if (ctx->plans) {
            for (PlanEntry* e : *ctx->plans) release_plan(e);
            delete ctx->plans;
        }
    }
    tune_delete(ctx->tune);
    free(ctx);
}

int lens_set_timing(lens_ctx* ctx, int enable)
{
    if (!ctx) return LENS_ERR_INVALID;
    ctx->timing = enable != 0;
    return LENS_OK;
}

int lens_field_timing(lens_ctx* ctx, double* total_ms, int64_t* launches, int reset)
{
    if (!ctx || !total_ms || !launches) return LENS_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    const int rc = fold_timing(ctx);
    *total_ms = ctx->total_ms;
    *launches = ctx->launches;
    if (reset) {
        ctx->total_ms = 0.0;
        ctx->launches = 0;
    }
    return rc;
}

const char* lens_strerror(int code)
{
    switch (code) {
    case LENS_OK: return "ok";
    case LENS_ERR_INVALID: return "invalid argument or parameter domain";
    case LENS_ERR_DEVICE: return "HIP device error";
    case LENS_ERR_CAPACITY: return "hit capacity exceeded";
    case LENS_ERR_SCRATCH: return "input needs more scratch than the fixed no-allocation buffer holds";
    default: return "unknown error";
    }
}

int lens_dls_dos(lens_ctx* ctx, double zl, const double* zs, int32_t n, double omega_m, double omega_l, double* out,
                 hipStream_t stream)
{
    if (!ctx || n < 0 || (n > 0 && (!zs || !out)) || !is_fin(zl) || zl < 0.0 || !is_fin(omega_m) ||
        !is_fin(omega_l) || fabs(omega_m + omega_l - 1.0) > 1e-12 || omega_m < 0.0)
        return LENS_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    return launch_dls(zl, zs, n, omega_m, omega_l, out, stream) == hipSuccess ? LENS_OK : LENS_ERR_DEVICE;
}

int lens_deflect(lens_ctx* ctx, const lens_potentials* pot, const lens_grid* grid, lens_precision prec, void* ax,
                 void* ay, int32_t* status, hipStream_t stream)
{
    if (!ctx || check_pot(pot) || check_grid(grid) || !ax || !ay) return LENS_ERR_INVALID;
    if (prec != LENS_FP64 && prec != LENS_FP32 && prec != LENS_MIXED) return LENS_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    const GridDesc g = grid_desc(grid);
    int rc = head(ctx, pot, g, no_obs(), nullptr, nullptr, stream);
    if (rc) return rc;
    const EvalState* st = (const EvalState*)ctx->buf[B_STATE];
    int slot;
    KernelEvents kev;
    const KernelEvents* ev;
    if ((rc = timing_begin(ctx, &kev, &ev, &slot))) return rc;
    hipError_t e;
    if (prec == LENS_FP64)
        e = launch_field64((const double*)ctx->buf[B_TAB64], pot->n, g, (double*)ax, (double*)ay, st, nullptr, 5, 1,
                           ev, stream);
    else
        e = launch_field32((const float*)ctx->buf[B_TAB32], pot->n, g, (float*)ax, (float*)ay, st, field_npl(g),
                           nullptr, 5, 1, ev, stream);
    if (e != hipSuccess) return LENS_ERR_DEVICE;
    timing_end(ctx, slot);
    if (status && launch_export(nullptr, 0, st, nullptr, nullptr, status, stream) != hipSuccess)
        return LENS_ERR_DEVICE;
    return LENS_OK;
}

int lens_deflect_mixed(lens_ctx* ctx, const lens_potentials* pot, const lens_grid* grid, const lens_mixed_opts* opts,
                       double* ax, double* ay, uint8_t* mask, int64_t* stats, hipStream_t stream)
{
    if (!ctx || check_pot(pot) || check_grid(grid) || !opts || !ax || !ay || !stats) return LENS_ERR_INVALID;
    if (opts->n_cluster < 0 || opts->n_cluster > pot->n || opts->patch_cluster < 0 || opts->patch_galaxy < 0 ||
        opts->patch_cluster > (1 << 20) || opts->patch_galaxy > (1 << 20) || !(opts->t12 >= 0.0) ||
        !is_fin(opts->t12) || !(opts->t34 >= 0.0) || !is_fin(opts->t34))
        return LENS_ERR_INVALID;
    const long long nn = (long long)grid->nx * grid->ny;
    if (nn >= (1ll << 32)) return LENS_ERR_INVALID;  // DP list entries are 32-bit pixel indices
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    const GridDesc g = grid_desc(grid);
    const size_t np = pot->n > 0 ? pot->n : 1;
    int rc;
    if ((rc = ensure(ctx, B_TAB64, np * T64_STRIDE * 8)) || (rc = ensure(ctx, B_TAB32, np * T32_STRIDE * 4)) ||
        (rc = ensure(ctx, B_BTERM, np * 3 * 8)) || (rc = ensure(ctx, B_MIX, sizeof(MixState))) ||
        (rc = ensure(ctx, B_MLIST, (size_t)nn * 4)) || (!mask && (rc = ensure(ctx, B_MMASK, (size_t)nn))))
        return rc;
    MixedLaunch ml;
    ml.tab64 = (double*)ctx->buf[B_TAB64];
    ml.tab32 = (float*)ctx->buf[B_TAB32];
    ml.bterm = (double*)ctx->buf[B_BTERM];
    ml.st = (MixState*)ctx->buf[B_MIX];
    ml.ax = ax;
    ml.ay = ay;
    ml.mask = mask ? mask : (unsigned char*)ctx->buf[B_MMASK];
    ml.list = (unsigned*)ctx->buf[B_MLIST];
    ml.stats = (long long*)stats;
    ml.n_cluster = opts->n_cluster;
    ml.pc = opts->patch_cluster;
    ml.pg = opts->patch_galaxy;
    ml.npl = std::min(field_cols(field_npl(g)) * field_rows(field_npl(g)), 4);
    ml.t12 = opts->t12;
    ml.t34 = opts->t34;
    int slot;
    KernelEvents kev;
    if ((rc = timing_begin(ctx, &kev, &ml.ev, &slot))) return rc;
    if (launch_mixed(pot_ptrs(pot), g, ml, stream) != hipSuccess) return LENS_ERR_DEVICE;
    timing_end(ctx, slot);
    return LENS_OK;
}

int lens_deflect_nfw(lens_ctx* ctx, const lens_nfw* halos, const lens_grid* grid, lens_precision prec, void* ax,
                     void* ay, int32_t* status, hipStream_t stream)
{
    if (!ctx || !halos || halos->n < 0 || check_grid(grid) || !ax || !ay) return LENS_ERR_INVALID;
    if (halos->n > 0 && (!halos->x || !halos->y || !halos->eps || !halos->phi || !halos->r_s || !halos->kappa_s))
        return LENS_ERR_INVALID;
    if (prec != LENS_FP64 && prec != LENS_FP32) return LENS_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    int rc;
    if ((rc = ensure(ctx, B_NFW, nfw_scratch(halos->n)))) return rc;
    NfwPtrs h;
    h.n = halos->n;
    h.x = halos->x;
    h.y = halos->y;
    h.eps = halos->eps;
    h.phi = halos->phi;
    h.r_s = halos->r_s;
    h.kappa_s = halos->kappa_s;
    int slot;
    KernelEvents kev;
    const KernelEvents* ev;
    if ((rc = timing_begin(ctx, &kev, &ev, &slot))) return rc;
    if (launch_nfw(h, grid_desc(grid), prec == LENS_FP32, ax, ay, status, ctx->buf[B_NFW], ev, stream) != hipSuccess)
        return LENS_ERR_DEVICE;
    timing_end(ctx, slot);
    return LENS_OK;
}

int lens_source_positions(lens_ctx* ctx, const lens_potentials* pot, const lens_obs* obs, double* beta_x,
                          double* beta_y, double* bar_x, double* bar_y, int32_t* status, hipStream_t stream)
{
    if (!ctx || check_pot(pot) || check_obs(obs) || !bar_x || !bar_y) return LENS_ERR_INVALID;
    if (obs->n_img > 0 && (!beta_x || !beta_y)) return LENS_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    GridDesc g;  // the split of the barycentres needs some grid; a unit grid at the origin
    g.x0 = 0.0;
    g.y0 = 0.0;
    g.h = 1.0;
    g.nx = 2;
    g.ny = 2;
    int rc = head(ctx, pot, g, obs_ptrs(obs), beta_x, beta_y, stream);
    if (rc) return rc;
    if (launch_export((const double*)ctx->buf[B_SYS], obs->n_sys, (const EvalState*)ctx->buf[B_STATE], bar_x,
                      bar_y, status, stream) != hipSuccess)
        return LENS_ERR_DEVICE;
    return LENS_OK;
}

}  // extern "C"

namespace {

// Launch shape and scratch layout of one chi^2 evaluation (lens_image_chi2 and
// lens_image_chi2_noalloc share them).
enum { CB_STATE, CB_TAB64, CB_TAB32, CB_BTERM, CB_SYS, CB_BX, CB_BY, CB_FIELD, CB_CONTRIB, CB_HITS, CB_POS, CB_FLAGS,
       CB_PART, CB_RR, CB_PAIRS, CB_N };

struct Chi2Plan {
    GridDesc g;
    ObsPtrs o;
    int np;
    bool mixed, fused;
    int shape, npl, tiles_x, tx_shift, n_cull, tpw, n_parts, fb_blocks;
    long long region, flag_cap;
    size_t nn, vbytes;
    size_t bytes[CB_N];
};

struct Chi2Bufs {
    void* p[CB_N];
};

int chi2_check(const lens_potentials* pot, const lens_grid* grid, const lens_obs* obs, const lens_chi2_opts* opts,
               const lens_chi2_out* out)
{
    if (check_pot(pot) || check_grid(grid) || check_obs(obs) || !opts || !out) return LENS_ERR_INVALID;
    if (opts->prec != LENS_FP64 && opts->prec != LENS_MIXED) return LENS_ERR_INVALID;
    if (opts->hit_capacity < 1 || opts->hit_capacity > kHitScratch) return LENS_ERR_INVALID;
    if (opts->prec == LENS_MIXED && (opts->fb_mode < 0 || opts->fb_mode > 1)) return LENS_ERR_INVALID;
    if (opts->prec == LENS_MIXED && opts->fb_mode == 1 && !(opts->fb_tau >= 0.0 && is_fin(opts->fb_tau)))
        return LENS_ERR_INVALID;
    if (!(opts->field_npl == 0 || field_code_ok(opts->field_npl)) || opts->tile < 0 || opts->tile > 4)
        return LENS_ERR_INVALID;
    if (!out->chi2 || !out->chi2_sys || !out->n_pred || !out->hits || !out->img_xy || !out->stats)
        return LENS_ERR_INVALID;
    return LENS_OK;
}

// Shape of the launches and bytes of every scratch buffer; flag_cap is the
// capacity of the undecided-test list (mixed path).
int chi2_plan(lens_ctx* ctx, const lens_potentials* pot, const lens_grid* grid, const lens_obs* obs,
              const lens_chi2_opts* opts, long long flag_cap, Chi2Plan& pl)
{
    pl.g = grid_desc(grid);
    pl.o = obs_ptrs(obs);
    pl.np = pot->n;
    pl.mixed = opts->prec == LENS_MIXED;
    pl.nn = (size_t)pl.g.nx * pl.g.ny;
    pl.shape = opts->tile;
    pl.npl = opts->field_npl;
    resolve_tuned(ctx, opts->prec, 0, std::max(pl.g.nx, pl.g.ny), pl.np, pl.shape, pl.npl);
    if (!pl.shape) pl.shape = 1;
    if (!pl.npl) pl.npl = field_npl(pl.g);
    int tile_x, tile_y;
    tile_dims(pl.shape, tile_x, tile_y);
    pl.tx_shift = tile_x == 64 ? 6 : 5;
    const long long n_tiles = tri_tiles(pl.g, pl.shape, &pl.tiles_x);
    int sc, nch;
    cull_shape(pl.g, pl.shape, pl.o.n_sys, &pl.n_cull, &pl.tpw, &sc, &nch);
    pl.fb_blocks = fbpos_blocks(n_tiles);
    pl.n_parts = pl.n_cull + kPairBlocks;
    // each culling wave owns room for every pair of its tiles and systems
    pl.region = 64ll * pl.tpw * sc;
    if (pl.region * pl.n_cull > (1ll << 28)) return LENS_ERR_CAPACITY;  // 2 GiB of pair keys
    pl.vbytes = pl.mixed ? 4 : 8;
    pl.flag_cap = pl.mixed ? flag_cap : 0;
    // the head's source-plane part runs inside the field launch when the grid allows
    pl.fused = fused_head_fits(pl.g, pl.o, pl.npl, pl.mixed) != 0;
    size_t* b = pl.bytes;
    b[CB_STATE] = sizeof(EvalState);
    b[CB_TAB64] = (size_t)pl.np * T64_STRIDE * 8;
    b[CB_TAB32] = (size_t)pl.np * T32_STRIDE * 4;
    b[CB_BTERM] = (size_t)pl.np * 3 * 8;
    b[CB_SYS] = (size_t)(pl.o.n_sys > 0 ? pl.o.n_sys : 1) * SYS_STRIDE * 8;
    b[CB_BX] = (size_t)pl.o.n_img * 8;
    b[CB_BY] = (size_t)pl.o.n_img * 8;
    b[CB_FIELD] = pl.nn * 2 * pl.vbytes;
    b[CB_CONTRIB] = (size_t)pl.o.n_img * 8;
    b[CB_HITS] = (size_t)kHitScratch * 2 * 8;
    b[CB_POS] = (size_t)kHitScratch * 4 * 8;
    b[CB_FLAGS] = (size_t)(pl.mixed ? pl.flag_cap : 1) * 8;
    b[CB_PART] = (size_t)pl.n_parts * 2 * 4;
    b[CB_RR] = (size_t)pl.g.ny * (pl.tiles_x + 1) * kRR * pl.vbytes;
    b[CB_PAIRS] = (size_t)pl.region * pl.n_cull * 8 + (size_t)pl.n_cull * 4;
    return LENS_OK;
}

// The launch sequence of one evaluation on the given scratch; ctx (may be
// null) only for the field kernel's timing.
int chi2_run(lens_ctx* ctx, const Chi2Plan& pl, const Chi2Bufs& b, const lens_potentials* pot,
             const lens_chi2_opts* opts, lens_chi2_out* out, hipStream_t stream)
{
    const GridDesc& g = pl.g;
    const ObsPtrs& o = pl.o;
    const int np = pl.np;
    const bool mixed = pl.mixed;
    const size_t nn = pl.nn;
    double* tab64 = (double*)b.p[CB_TAB64];
    float* tab32 = (float*)b.p[CB_TAB32];
    double* bterm = (double*)b.p[CB_BTERM];
    double* sysrow = (double*)b.p[CB_SYS];
    EvalState* st = (EvalState*)b.p[CB_STATE];
    double* bx = (double*)b.p[CB_BX];
    double* by = (double*)b.p[CB_BY];
    void* rr = b.p[CB_RR];
    unsigned* part = (unsigned*)b.p[CB_PART];
    unsigned long long* pairs = (unsigned long long*)b.p[CB_PAIRS];
    unsigned* counts = (unsigned*)(pairs + (size_t)pl.region * pl.n_cull);
    unsigned long long* hits = (unsigned long long*)b.p[CB_HITS];
    unsigned long long* fb_hits = hits + kHitScratch;
    double* pos = (double*)b.p[CB_POS];
    double* fb_pos = pos + 2 * kHitScratch;
    unsigned long long* flags = (unsigned long long*)b.p[CB_FLAGS];
    if (pl.fused) {
        if (launch_prep(pot_ptrs(pot), g, tab64, tab32, bterm, st, stream) != hipSuccess) return LENS_ERR_DEVICE;
    } else if (launch_head(pot_ptrs(pot), g, o, tab64, tab32, bterm, bx, by, sysrow, st, stream) != hipSuccess) {
        return LENS_ERR_DEVICE;
    }
    int rc, slot = -1;
    KernelEvents kev;
    const KernelEvents* ev = nullptr;
    if (ctx && (rc = timing_begin(ctx, &kev, &ev, &slot))) return rc;
    hipError_t e;
    void* field = b.p[CB_FIELD];
    const void* fx = field;
    const void* fy = (const char*)field + nn * pl.vbytes;
    HeadArgs ha;
    ha.pot = pot_ptrs(pot);
    ha.g = g;
    ha.obs = o;
    ha.tab64 = tab64;
    ha.bterm = bterm;
    ha.bx = bx;
    ha.by = by;
    ha.sysrow = sysrow;
    ha.st = st;
    if (mixed && pl.fused)
        e = launch_field32h(tab32, np, g, (float*)field, (float*)field + nn, pl.npl, (float*)rr, pl.tx_shift,
                            pl.tiles_x, ha, ev, stream);
    else if (mixed)
        e = launch_field32(tab32, np, g, (float*)field, (float*)field + nn, nullptr, pl.npl, (float*)rr, pl.tx_shift,
                           pl.tiles_x, ev, stream);
    else if (pl.fused)
        e = launch_field64h(tab64, np, g, (double*)field, (double*)field + nn, (double*)rr, pl.tx_shift, pl.tiles_x,
                            ha, ev, stream);
    else
        e = launch_field64(tab64, np, g, (double*)field, (double*)field + nn, nullptr, (double*)rr, pl.tx_shift,
                           pl.tiles_x, ev, stream);
    if (e != hipSuccess) return LENS_ERR_DEVICE;
    if (ctx) timing_end(ctx, slot);

    const float tau = (float)(opts->fb_tau * g.h * g.h);
    e = launch_cull(mixed, rr, g, o.n_sys, sysrow, pairs, pl.region, counts, part, pl.shape, stream);
    if (e == hipSuccess)
        e = launch_pairs(mixed, fx, fy, g, sysrow, st, opts->fb_mode, tau, pairs, pl.region, counts, pl.n_cull, hits,
                         kHitScratch, flags, pl.flag_cap, part, pl.n_cull, pl.shape, stream);
    if (e == hipSuccess)
        e = launch_fbpos(tab64, np, g, sysrow, st, hits, kHitScratch, flags, pl.flag_cap, fb_hits, kHitScratch, pos,
                         fb_pos, pl.fb_blocks, stream);
    if (e != hipSuccess) return LENS_ERR_DEVICE;
    TailLaunch tl;
    tl.obs = o;
    tl.hit_cap = kHitScratch;
    tl.flag_cap = pl.flag_cap;
    tl.fb_cap = kHitScratch;
    tl.hit_capacity = opts->hit_capacity;
    tl.hit_keys = hits;
    tl.out_hits = out->hits;
    tl.img_xy = out->img_xy;
    tl.n_pred = out->n_pred;
    tl.contrib = (double*)b.p[CB_CONTRIB];
    tl.chi2 = out->chi2;
    tl.chi2_sys = out->chi2_sys;
    tl.match = out->match;
    tl.stats = (long long*)out->stats;
    tl.n_tests = 2ll * (g.nx - 1) * (g.ny - 1) * o.n_sys;
    tl.part = part;
    tl.n_parts = pl.n_parts;
    e = launch_tail(tl, st, fb_hits, pos, fb_pos, stream);
    return e == hipSuccess ? LENS_OK : LENS_ERR_DEVICE;
}

const int kCtxBuf[CB_N] = {B_STATE, B_TAB64, B_TAB32, B_BTERM, B_SYS, B_BX, B_BY, B_FIELD, B_CONTRIB, B_HITS,
                           B_POS, B_FLAGS, B_PART, B_RR, B_PAIRS};

}  // namespace

extern "C" {

int lens_image_chi2(lens_ctx* ctx, const lens_potentials* pot, const lens_grid* grid, const lens_obs* obs,
                    const lens_chi2_opts* opts, lens_chi2_out* out, hipStream_t stream)
{
    if (!ctx) return LENS_ERR_INVALID;
    int rc = chi2_check(pot, grid, obs, opts, out);
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    Chi2Plan pl;
    if ((rc = chi2_plan(ctx, pot, grid, obs, opts, kFlagScratch, pl))) return rc;
    Chi2Bufs b;
    for (int k = 0; k < CB_N; k++) {
        if ((rc = ensure(ctx, kCtxBuf[k], pl.bytes[k]))) return rc;
        b.p[k] = ctx->buf[kCtxBuf[k]];
    }
    return chi2_run(ctx, pl, b, pot, opts, out, stream);
}

}  // extern "C"

// ------------------------------------------------------------ no-allocation chi^2

// Fixed scratch of lens_image_chi2_noalloc: one copy per device, held until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: only the address that hipGetSymbolAddress returns for the
// current device is ever passed to a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[LENS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoallocDevices = 64;

struct NoallocSlot {
    std::once_flag once;
    void* ptr = nullptr;
};
NoallocSlot g_noalloc[kNoallocDevices];

// Device address of device `dev`'s copy of the fixed scratch, looked up once
// per device with that device current (null if the lookup failed).
void* noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= kNoallocDevices) return nullptr;
    NoallocSlot& slot = g_noalloc[dev];
    std::call_once(slot.once, [&slot] {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) slot.ptr = p;
    });
    return slot.ptr;
}

}  // namespace

extern "C" {

int lens_image_chi2_noalloc(const lens_potentials* pot, const lens_grid* grid, const lens_obs* obs,
                            const lens_chi2_opts* opts, lens_chi2_out* out, hipStream_t stream)
{
    int rc = chi2_check(pot, grid, obs, opts, out);
    if (rc) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LENS_ERR_DEVICE;
    unsigned char* base = (unsigned char*)noalloc_scratch(dev);
    if (!base) return LENS_ERR_DEVICE;
    Chi2Plan pl;
    if ((rc = chi2_plan(nullptr, pot, grid, obs, opts, kFlagScratch, pl))) return rc;
    // the context path's buffers, carved in order from the fixed array
    Chi2Bufs b;
    size_t off = 0;
    for (int k = 0; k < CB_N; k++) {
        b.p[k] = base + off;
        off += (std::max(pl.bytes[k], (size_t)1) + 255) & ~(size_t)255;
        if (off > (size_t)LENS_NOALLOC_SCRATCH_BYTES) return LENS_ERR_SCRATCH;
    }
    // The evaluation state sits at the start of the array in every call; its
    // head ticket must be zero when the head kernel starts.  The fused path's
    // prep kernel clears it; otherwise a one-wave kernel does (no memset node
    // in a captured graph).
    EvalState* st = (EvalState*)b.p[CB_STATE];
    if (!pl.fused && launch_zero_u32(&st->head_ticket, 1, stream) != hipSuccess) return LENS_ERR_DEVICE;
    return chi2_run(nullptr, pl, b, pot, opts, out, stream);
}

}  // extern "C"

namespace {

size_t align8(size_t v) { return (v + 7) & ~(size_t)7; }


// Bytes of field scratch per chunk (env LENS_BATCH_FIELD_BYTES, default 16 GiB).
long long batch_field_budget()
{
    const char* env = getenv("LENS_BATCH_FIELD_BYTES");
    const long long v = env ? atoll(env) : 0;
    return v > 0 ? v : (16ll << 30);
}

// Builds (or finds) the plan of a batch: chunks of consecutive samples within
// the field-memory budget; inside a chunk the samples are ordered by cost
// P * nx * ny, heaviest first, and the work items of the field (row segments)
// and triangle (tile) stages are enumerated in that order.  New plans are
// uploaded on `s` from pinned staging that stays alive with the plan.
int batch_plan(lens_ctx* c, int n_samples, const int32_t* pot_off, const lens_grid* grids, int npl, int shape,
               bool fp32, hipStream_t s, PlanEntry** out)
{
    for (PlanEntry* e : *c->plans) {
        if (e->npl != npl || e->shape != shape || e->fp32 != (int)fp32 ||
            (int)e->pot_off.size() != n_samples + 1)
            continue;
        if (memcmp(e->pot_off.data(), pot_off, sizeof(int32_t) * (n_samples + 1)) != 0) continue;
        bool same = true;
        for (int i = 0; i < n_samples && same; i++) {
            const double* gv = &e->grids[5 * (size_t)i];
            same = gv[0] == grids[i].x0 && gv[1] == grids[i].y0 && gv[2] == grids[i].h && gv[3] == grids[i].nx &&
                   gv[4] == grids[i].ny;
        }
        if (same) {
            // most recently used last
            std::vector<PlanEntry*>& v = *c->plans;
            v.erase(std::find(v.begin(), v.end(), e));
            v.push_back(e);
            *out = e;
            return LENS_OK;
        }
    }
    if ((int)c->plans->size() >= kMaxPlans) {
        // release the least recently used plan once no queued work can read it
        if (hipDeviceSynchronize() != hipSuccess) return LENS_ERR_DEVICE;
        release_plan(c->plans->front());
        c->plans->erase(c->plans->begin());
    }
    PlanEntry* e = new (std::nothrow) PlanEntry();
    if (!e) return LENS_ERR_DEVICE;
    e->npl = npl;
    e->shape = shape;
    e->fp32 = (int)fp32;
    e->pot_off.assign(pot_off, pot_off + n_samples + 1);
    e->grids.resize(5 * (size_t)n_samples);
    for (int i = 0; i < n_samples; i++) {
        double* gv = &e->grids[5 * (size_t)i];
        gv[0] = grids[i].x0;
        gv[1] = grids[i].y0;
        gv[2] = grids[i].h;
        gv[3] = grids[i].nx;
        gv[4] = grids[i].ny;
    }
    int tx, ty;
    tile_dims(shape, tx, ty);
    const int seg_nodes = 256 * (fp32 ? field_cols(npl) : 1), seg_rows = fp32 ? field_rows(npl) : 1;
    const long long elem = fp32 ? 8 : 16;  // two planes
    const long long budget = batch_field_budget();
    int s0 = 0;
    int rc = LENS_OK;
    while (s0 < n_samples && rc == LENS_OK) {
        int s1 = s0;
        long long nodes = 0;
        while (s1 < n_samples && s1 - s0 < (1 << 19)) {
            const long long add = (long long)grids[s1].nx * grids[s1].ny;
            if (s1 > s0 && (nodes + add) * elem > budget) break;
            nodes += add;
            s1++;
        }
        PlanChunk ch;
        memset(&ch, 0, sizeof ch);
        ch.s0 = s0;
        ch.n = s1 - s0;
        ch.np = pot_off[s1] - pot_off[s0];
        const int n = ch.n;
        std::vector<int> perm(n);
        for (int k = 0; k < n; k++) perm[k] = k;
        auto cost = [&](int k) {
            const lens_grid& g = grids[s0 + k];
            return (double)(pot_off[s0 + k + 1] - pot_off[s0 + k] + 1) * g.nx * g.ny;
        };
        std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return cost(x) > cost(y); });
        const size_t o_pot = 0, o_grid = align8(o_pot + 4 * (size_t)(n + 1)),
                     o_perm = align8(o_grid + sizeof(GridDesc) * (size_t)n), o_fo = align8(o_perm + 4 * (size_t)n),
                     o_to = o_fo + 8 * (size_t)(n + 1), o_no = o_to + 8 * (size_t)(n + 1),
                     o_rr = o_no + 8 * (size_t)n, bytes = o_rr + 8 * (size_t)n;
        if (hipHostMalloc(&ch.host_stage, bytes, hipHostMallocDefault) != hipSuccess) {
            rc = LENS_ERR_DEVICE;
            break;
        }
        char* hb = (char*)ch.host_stage;
        int32_t* h_pot = (int32_t*)(hb + o_pot);
        GridDesc* h_grid = (GridDesc*)(hb + o_grid);
        int32_t* h_perm = (int32_t*)(hb + o_perm);
        long long* h_fo = (long long*)(hb + o_fo);
        long long* h_to = (long long*)(hb + o_to);
        long long* h_no = (long long*)(hb + o_no);
        long long* h_rr = (long long*)(hb + o_rr);
        for (int k = 0; k <= n; k++) h_pot[k] = pot_off[s0 + k];
        long long node = 0, nrr = 0;
        for (int k = 0; k < n; k++) {
            const lens_grid& g = grids[s0 + k];
            h_grid[k] = grid_desc(&g);
            h_no[k] = node;
            h_rr[k] = nrr;
            node += (long long)g.nx * g.ny;
            nrr += (long long)g.ny * ((g.nx - 2) / tx + 2) * kRR;
            ch.n_tests += 2ll * (g.nx - 1) * (g.ny - 1);
        }
        ch.n_rr = nrr;
        h_fo[0] = 0;
        h_to[0] = 0;
        for (int k = 0; k < n; k++) {
            const lens_grid& g = grids[s0 + perm[k]];
            h_perm[k] = perm[k];
            h_fo[k + 1] = h_fo[k] + (long long)((g.ny + seg_rows - 1) / seg_rows) * ((g.nx + seg_nodes - 1) / seg_nodes);
            // triangle stage: one item per (tile row, block of 64 tile columns)
            h_to[k + 1] = h_to[k] + (long long)(((g.nx - 2) / tx + 1 + 63) / 64) * ((g.ny - 2) / ty + 1);
        }
        ch.n_nodes = node;
        ch.n_fitems = h_fo[n];
        ch.n_tiles = h_to[n];
        if (ch.n_fitems >= (1ll << 31) || ch.n_tiles >= (1ll << 31)) {
            rc = LENS_ERR_INVALID;
            (void)hipHostFree(ch.host_stage);
            break;
        }
        if (hipMalloc(&ch.dev_plan, bytes) != hipSuccess || hipMalloc((void**)&ch.fmap, 4 * ch.n_fitems) != hipSuccess ||
            hipMalloc((void**)&ch.tmap, 4 * ch.n_tiles) != hipSuccess) {
            rc = LENS_ERR_DEVICE;
            e->chunks.push_back(ch);
            break;
        }
        char* db = (char*)ch.dev_plan;
        ch.bp.n = n;
        ch.bp.pot_off = (const int*)(db + o_pot);
        ch.bp.grid = (const GridDesc*)(db + o_grid);
        ch.bp.perm = (const int*)(db + o_perm);
        ch.bp.fitem_off = (const long long*)(db + o_fo);
        ch.bp.titem_off = (const long long*)(db + o_to);
        ch.bp.node_off = (const long long*)(db + o_no);
        ch.bp.rr_off = (const long long*)(db + o_rr);
        ch.bp.tx_shift = tx == 64 ? 6 : 5;
        if (hipMemcpyAsync(ch.dev_plan, ch.host_stage, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            launch_bmap(ch.bp, ch.fmap, ch.tmap, s) != hipSuccess)
            rc = LENS_ERR_DEVICE;
        e->chunks.push_back(ch);
        s0 = s1;
    }
    c->plans->push_back(e);  // kept even on failure so that destroy frees it
    if (rc) {
        e->pot_off.clear();  // never matches again
        return rc;
    }
    *out = e;
    return LENS_OK;
}

}  // namespace

extern "C" int lens_image_chi2_batched(lens_ctx* ctx, const lens_potentials* all, int32_t n_samples,
                                       const int32_t* pot_off, const lens_grid* grids, const lens_obs* obs,
                                       const lens_chi2_opts* opts, lens_batch_out* out, hipStream_t stream)
{
    if (!ctx || check_pot(all) || n_samples < 1 || !pot_off || !grids || check_obs(obs) || !opts || !out)
        return LENS_ERR_INVALID;
    if (!out->chi2 || !out->chi2_sys || !out->n_pred || !out->status || !out->stats) return LENS_ERR_INVALID;
    const bool want_hits = out->n_hits || out->hits || out->img_xy;
    if (want_hits && !(out->n_hits && out->hits && out->img_xy)) return LENS_ERR_INVALID;
    if (obs->n_img > kBatchMax || obs->n_sys > kBatchMax) return LENS_ERR_INVALID;
    if (opts->prec != LENS_FP64 && opts->prec != LENS_MIXED) return LENS_ERR_INVALID;
    if (opts->hit_capacity < 1 || opts->hit_capacity > kBatchMax) return LENS_ERR_INVALID;
    if (opts->prec == LENS_MIXED && (opts->fb_mode < 0 || opts->fb_mode > 1)) return LENS_ERR_INVALID;
    if (opts->prec == LENS_MIXED && opts->fb_mode == 1 && !(opts->fb_tau >= 0.0 && is_fin(opts->fb_tau)))
        return LENS_ERR_INVALID;
    if (!(opts->field_npl == 0 || bfield_code_ok(opts->field_npl)) || opts->tile < 0 || opts->tile > 4)
        return LENS_ERR_INVALID;
    if (pot_off[0] != 0 || pot_off[n_samples] != all->n) return LENS_ERR_INVALID;
    for (int i = 0; i < n_samples; i++) {
        if (pot_off[i + 1] < pot_off[i] || check_grid(&grids[i])) return LENS_ERR_INVALID;
    }
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    const bool mixed = opts->prec == LENS_MIXED;
    int shape = opts->tile, npl = opts->field_npl;
    int side = 1;
    for (int i = 0; i < n_samples; i++) side = std::max(side, std::max(grids[i].nx, grids[i].ny));
    resolve_tuned(ctx, opts->prec, 1, side, ((long long)all->n + n_samples - 1) / n_samples, shape, npl);
    if (!shape) shape = 1;
    npl = mixed ? (npl ? npl : 0x41) : 1;  // FP32 field: 1 column x 4 rows per thread (measured fastest)
    PlanEntry* plan = nullptr;
    int rc = batch_plan(ctx, n_samples, pot_off, grids, npl, shape, mixed, stream, &plan);
    if (rc) return rc;

    // scratch sized for the largest chunk
    long long max_n = 0, max_np = 0, max_nodes = 0, max_tiles = 0, n_tests = 0, max_rr = 0;
    for (const PlanChunk& ch : plan->chunks) {
        max_n = std::max(max_n, (long long)ch.n);
        max_np = std::max(max_np, (long long)ch.np);
        max_nodes = std::max(max_nodes, ch.n_nodes);
        max_tiles = std::max(max_tiles, ch.n_tiles);
        max_rr = std::max(max_rr, ch.n_rr);
        n_tests += ch.n_tests * obs->n_sys;
    }
    const int hcap = opts->hit_capacity;
    const long long flag_cap = mixed ? kFlagScratch : 0;
    const size_t per_sample_hits = (size_t)max_n * hcap;
    if ((rc = ensure(ctx, B_TAB64, (size_t)max_np * T64_STRIDE * 8)) ||
        (rc = ensure(ctx, B_TAB32, (size_t)max_np * T32_STRIDE * 4)) ||
        (rc = ensure(ctx, B_BTERM, (size_t)max_np * 3 * 8)) ||
        (rc = ensure(ctx, B_FIELD, (size_t)max_nodes * (mixed ? 8 : 16))) ||
        (rc = ensure(ctx, B_BX, (size_t)max_n * obs->n_img * 8)) ||
        (rc = ensure(ctx, B_BY, (size_t)max_n * obs->n_img * 8)) ||
        (rc = ensure(ctx, B_SYS, (size_t)max_n * obs->n_sys * SYS_STRIDE * 8)) ||
        (rc = ensure(ctx, B_HITS, per_sample_hits * 2 * 8)) ||
        (rc = ensure(ctx, B_FLAGS, (size_t)(mixed ? kFlagScratch : 1) * 8)) ||
        (rc = ensure(ctx, B_POS, per_sample_hits * 4 * 8)) || (rc = ensure(ctx, B_PART, (size_t)(max_tiles / 4 + 1) * 2 * 4)) ||
        (rc = ensure(ctx, B_RR, (size_t)max_rr * (mixed ? 4 : 8))) ||
        (rc = ensure(ctx, B_BCOUNT, (size_t)max_n * 20 + 8 * 16)))
        return rc;
    unsigned long long* hits = (unsigned long long*)ctx->buf[B_HITS];
    unsigned long long* fb = hits + per_sample_hits;
    double* pos = (double*)ctx->buf[B_POS];
    double* fb_pos = pos + 2 * per_sample_hits;
    unsigned long long* flags = (unsigned long long*)ctx->buf[B_FLAGS];
    unsigned long long* agg = (unsigned long long*)ctx->buf[B_BCOUNT];
    BatchState bs;
    bs.n_flags = agg + 8;
    bs.n_hits = agg + 16;
    bs.n_fb = bs.n_hits + max_n;
    bs.status = (int*)(bs.n_fb + max_n);
    const ObsPtrs o = obs_ptrs(obs);
    const PotPtrs p = pot_ptrs(all);
    double* bx = (double*)ctx->buf[B_BX];
    double* by = (double*)ctx->buf[B_BY];
    double* sysrow = (double*)ctx->buf[B_SYS];
    void* field = ctx->buf[B_FIELD];
    unsigned* part = (unsigned*)ctx->buf[B_PART];
    if (launch_zero_u64(agg, 8, stream) != hipSuccess) return LENS_ERR_DEVICE;
    for (const PlanChunk& ch : plan->chunks) {
        const BatchPlan& bp = ch.bp;
        hipError_t e = launch_bhead(bp, p, o, (double*)ctx->buf[B_TAB64], (float*)ctx->buf[B_TAB32],
                                    (double*)ctx->buf[B_BTERM], bx, by, ch.np, stream);
        if (e == hipSuccess) e = launch_bsys(bp, o, (double*)ctx->buf[B_BTERM], bx, by, sysrow, bs, stream);
        int slot;
        KernelEvents kev;
        const KernelEvents* ev;
        if ((rc = timing_begin(ctx, &kev, &ev, &slot))) return rc;
        if (e == hipSuccess) {
            if (mixed)
                e = launch_bfield32(bp, ch.fmap, ch.n_fitems, (const float*)ctx->buf[B_TAB32], (float*)field,
                                    (float*)field + ch.n_nodes, (float*)ctx->buf[B_RR], npl, ev, stream);
            else
                e = launch_bfield64(bp, ch.fmap, ch.n_fitems, (const double*)ctx->buf[B_TAB64], (double*)field,
                                    (double*)field + ch.n_nodes, (double*)ctx->buf[B_RR], ev, stream);
        }
        if (e != hipSuccess) return LENS_ERR_DEVICE;
        timing_end(ctx, slot);
        const void* fx = field;
        const void* fy = mixed ? (const void*)((float*)field + ch.n_nodes) : (const void*)((double*)field + ch.n_nodes);
        e = launch_btri(bp, ch.tmap, ch.n_tiles, o.n_sys, sysrow, fx, fy, ctx->buf[B_RR], mixed, bs, opts->fb_mode,
                        opts->fb_tau, hcap, hits, flags, flag_cap, part, shape, stream);
        if (e == hipSuccess)
            e = launch_bfbpos(bp, o.n_sys, (const double*)ctx->buf[B_TAB64], sysrow, bs, hcap, hits, flags, flag_cap,
                              fb, pos, fb_pos, stream);
        if (e == hipSuccess)
            e = launch_btail(bp, o, bs, hcap, flag_cap, hits, fb, pos, fb_pos, out->chi2 + ch.s0,
                             out->chi2_sys + (size_t)ch.s0 * o.n_sys, out->n_pred + (size_t)ch.s0 * o.n_sys,
                             out->status + ch.s0, agg, part, (ch.n_tiles + 3) / 4,
                             want_hits ? out->n_hits + ch.s0 : nullptr,
                             want_hits ? out->hits + (size_t)ch.s0 * 2 * hcap : nullptr,
                             want_hits ? out->img_xy + (size_t)ch.s0 * 2 * hcap : nullptr, stream);
        if (e != hipSuccess) return LENS_ERR_DEVICE;
    }
    return launch_bstats(agg, n_tests, (long long*)out->stats, stream) == hipSuccess ? LENS_OK : LENS_ERR_DEVICE;
}

// ---------------------------------------------------------------- backward form

extern "C" int lens_deflect_backward(lens_ctx* ctx, const lens_potentials* pot, const lens_grid* grid,
                                     lens_precision prec, const double* g_ax, const double* g_ay, double* grad,
                                     int32_t* status, hipStream_t stream)
{
    if (!ctx || check_pot(pot) || check_grid(grid) || !g_ax || !g_ay || (pot->n > 0 && !grad))
        return LENS_ERR_INVALID;
    if (prec != LENS_FP64 && prec != LENS_FP32) return LENS_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    const GridDesc g = grid_desc(grid);
    int rc = ensure(ctx, B_VJP, vjp_scratch(pot->n, g));
    if (rc) return rc;
    int slot;
    KernelEvents kev;
    const KernelEvents* ev;
    if ((rc = timing_begin(ctx, &kev, &ev, &slot))) return rc;
    if (launch_vjp(pot_ptrs(pot), g, prec == LENS_FP32, g_ax, g_ay, (double*)ctx->buf[B_VJP], grad, status, ev,
                   stream) != hipSuccess)
        return LENS_ERR_DEVICE;
    timing_end(ctx, slot);
    return LENS_OK;
}

namespace {

int src_common(lens_ctx* ctx, const lens_potentials* pot, const lens_obs* obs, double* chi2, int32_t* status,
               const double* g_chi2, double* grad, hipStream_t stream, const HmcUpdate* upd = nullptr)
{
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    int rc;
    const size_t ni = obs->n_img > 0 ? obs->n_img : 1;
    if ((rc = ensure(ctx, B_SRC, (4 * ni + obs->n_sys) * 8)) || (rc = ensure(ctx, B_SRCST, sizeof(SrcState))))
        return rc;
    double* beta = (double*)ctx->buf[B_SRC];
    if (launch_src(pot_ptrs(pot), obs_ptrs(obs), beta, beta + 2 * ni, beta + 4 * ni, (SrcState*)ctx->buf[B_SRCST],
                   chi2, status, g_chi2, grad, upd, stream) != hipSuccess)
        return LENS_ERR_DEVICE;
    return LENS_OK;
}

}  // namespace

extern "C" int lens_src_chi2(lens_ctx* ctx, const lens_potentials* pot, const lens_obs* obs, double* chi2,
                             int32_t* status, hipStream_t stream)
{
    if (!ctx || check_pot(pot) || check_obs(obs) || !chi2) return LENS_ERR_INVALID;
    return src_common(ctx, pot, obs, chi2, status, nullptr, nullptr, stream);
}

extern "C" int lens_src_chi2_backward(lens_ctx* ctx, const lens_potentials* pot, const lens_obs* obs,
                                      const double* g_chi2, double* grad, int32_t* status, hipStream_t stream)
{
    if (!ctx || check_pot(pot) || check_obs(obs) || (pot->n > 0 && !grad)) return LENS_ERR_INVALID;
    return src_common(ctx, pot, obs, nullptr, status, g_chi2, grad, stream);
}

// ---------------------------------------------------------------- sampler steps

namespace {

lens_potentials table_pots(double* t, int n)
{
    lens_potentials p;
    p.n = n;
    p.x = t;
    p.y = t + (size_t)n;
    p.eps = t + 2 * (size_t)n;
    p.phi = t + 3 * (size_t)n;
    p.r_core = t + 4 * (size_t)n;
    p.r_cut = t + 5 * (size_t)n;
    p.sigma_v = t + 6 * (size_t)n;
    return p;
}

}  // namespace

extern "C" int lens_hmc_step(lens_ctx* ctx, double* state, int32_t n, const lens_obs* obs, const double* step,
                             int32_t n_leapfrog, const double* momentum, const double* u, double* chi2,
                             int32_t* accepted, hipStream_t stream)
{
    if (!ctx || !state || n < 1 || check_obs(obs) || !step || !momentum || !u || !chi2 || !accepted ||
        n_leapfrog < 1 || n_leapfrog > 1000 || n > (1 << 24))
        return LENS_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    const int n7 = 7 * n;
    int rc;
    if ((rc = ensure(ctx, B_HMC, (size_t)3 * n7 * 8 + 64))) return rc;
    double* q = (double*)ctx->buf[B_HMC];
    double* pm = q + n7;
    double* g = pm + n7;
    double* chi2_pair = g + n7;                      // [2]
    int* status_pair = (int*)(chi2_pair + 2);        // [2]
    const lens_potentials qp = table_pots(q, n);
    if (launch_hmc_begin(state, momentum, step, n7, q, pm, stream) != hipSuccess) return LENS_ERR_DEVICE;
    // leapfrog: half kick and drift after the gradient at the start, full kick
    // and drift after each inner gradient, half kick after the last one
    HmcUpdate upd = {pm, q, step, 0.5, 1};
    if ((rc = src_common(ctx, &qp, obs, chi2_pair, status_pair, nullptr, g, stream, &upd))) return rc;
    for (int l = 1; l <= n_leapfrog; l++) {
        upd.kick = l < n_leapfrog ? 1.0 : 0.5;
        upd.drift = l < n_leapfrog ? 1 : 0;
        if ((rc = src_common(ctx, &qp, obs, chi2_pair + 1, status_pair + 1, nullptr, g, stream, &upd))) return rc;
    }
    if (launch_hmc_accept(state, q, momentum, pm, step, n7, chi2_pair, status_pair, u, chi2, accepted, stream) !=
        hipSuccess)
        return LENS_ERR_DEVICE;
    return LENS_OK;
}

extern "C" int lens_mh_step_batched(lens_ctx* ctx, double* states, int32_t n_chains, int32_t n,
                                    const lens_grid* grid, const lens_obs* obs, const lens_chi2_opts* opts,
                                    const double* step, const double* noise, const double* u, double* chi2,
                                    int32_t* accepted, hipStream_t stream)
{
    if (!ctx || !states || n_chains < 1 || n_chains > (1 << 20) || n < 1 || check_grid(grid) || check_obs(obs) ||
        !opts || !step || !noise || !u || !chi2 || !accepted)
        return LENS_ERR_INVALID;
    const long long bn = (long long)n_chains * n;
    if (bn > (1ll << 28)) return LENS_ERR_INVALID;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return LENS_ERR_DEVICE;
    const size_t ns = obs->n_sys > 0 ? obs->n_sys : 1;
    const size_t bytes = (size_t)7 * bn * 8 + (size_t)n_chains * (8 + 8 * ns + 4 * ns + 4) + 8 * LENS_STAT_N + 256;
    int rc;
    if ((rc = ensure(ctx, B_MHP, bytes))) return rc;
    double* prop = (double*)ctx->buf[B_MHP];
    double* chi2_new = prop + 7 * bn;
    double* chi2_sys = chi2_new + n_chains;
    int64_t* stats = (int64_t*)(chi2_sys + (size_t)n_chains * ns);
    int32_t* n_pred = (int32_t*)(stats + LENS_STAT_N);
    int32_t* status = n_pred + (size_t)n_chains * ns;
    if (launch_mh_propose(states, step, noise, n, n_chains, prop, stream) != hipSuccess) return LENS_ERR_DEVICE;
    std::vector<int32_t> pot_off((size_t)n_chains + 1);
    for (int b = 0; b <= n_chains; b++) pot_off[b] = (int32_t)((long long)b * n);
    std::vector<lens_grid> grids((size_t)n_chains, *grid);
    const lens_potentials all = table_pots(prop, (int)bn);
    lens_batch_out bo = {};
    bo.chi2 = chi2_new;
    bo.chi2_sys = chi2_sys;
    bo.n_pred = n_pred;
    bo.status = status;
    bo.stats = stats;
    if ((rc = lens_image_chi2_batched(ctx, &all, n_chains, pot_off.data(), grids.data(), obs, opts, &bo, stream)))
        return rc;
    if (launch_mh_accept(states, prop, n, n_chains, chi2_new, status, u, chi2, accepted, stream) != hipSuccess)
        return LENS_ERR_DEVICE;
    return LENS_OK;
}
