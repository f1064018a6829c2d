// Autotuner of the batched and single chi^2 evaluation: times the candidate
// triangle-stage tile shapes and FP32 field nodes per thread on the caller's
// problem, keeps the fastest per bucket in the context's table and persists
// the table as JSON.  Host code only.  No C++ exception crosses the extern "C"
// functions.
#include "lens_tune.hpp"
#include "lens_internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace lens {

struct TuneEntry {
    int prec, batched, n_log2, p_log2, tile, npl;
    double ms;
};

struct TuneTable {
    std::vector<TuneEntry> entries;
};

TuneTable* tune_new() { return new (std::nothrow) TuneTable(); }

void tune_delete(TuneTable* t) { delete t; }

int tune_log2(long long v)
{
    int k = 0;
    while (k < 62 && (1ll << k) < v) k++;
    return k;
}

static TuneEntry* find(TuneTable* t, int prec, int batched, int n_log2, int p_log2)
{
    for (TuneEntry& e : t->entries)
        if (e.prec == prec && e.batched == batched && e.n_log2 == n_log2 && e.p_log2 == p_log2) return &e;
    return nullptr;
}

bool tune_lookup(const TuneTable* t, int prec, int batched, int n_log2, int p_log2, int* tile, int* npl)
{
    if (!t) return false;
    const TuneEntry* e = find(const_cast<TuneTable*>(t), prec, batched, n_log2, p_log2);
    if (!e) return false;
    *tile = e->tile;
    *npl = e->npl;
    return true;
}

static void record(TuneTable* t, const TuneEntry& v)
{
    if (TuneEntry* e = find(t, v.prec, v.batched, v.n_log2, v.p_log2))
        *e = v;
    else
        t->entries.push_back(v);
}

static bool valid_entry(const TuneEntry& e)
{
    const bool npl_ok = e.npl == 0 || (e.batched ? bfield_code_ok(e.npl) : field_code_ok(e.npl));
    return (e.prec == LENS_FP64 || e.prec == LENS_MIXED) && (e.batched == 0 || e.batched == 1) && e.n_log2 >= 0 &&
           e.n_log2 <= 62 && e.p_log2 >= 0 && e.p_log2 <= 62 && e.tile >= 1 && e.tile <= 4 && npl_ok;
}

// ---------------------------------------------------------------- JSON (the subset this file writes)

namespace {

struct Reader {
    const char* p;
    const char* end;
    bool ok = true;
    int depth = 0;  // nesting of skipped objects and arrays, at most kMaxDepth
    static constexpr int kMaxDepth = 64;

    void ws()
    {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) p++;
    }
    bool eat(char c)
    {
        ws();
        if (p < end && *p == c) {
            p++;
            return true;
        }
        return false;
    }
    void expect(char c)
    {
        if (!eat(c)) ok = false;
    }
    std::string str()
    {
        ws();
        std::string s;
        if (p >= end || *p != '"') {
            ok = false;
            return s;
        }
        p++;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                ok = false;
                return s;
            }
            s.push_back(*p++);
        }
        if (p >= end) {
            ok = false;
            return s;
        }
        p++;
        return s;
    }
    double num()
    {
        ws();
        char buf[64];
        int n = 0;
        while (p < end && n < 63 && (strchr("+-.eE", *p) || (*p >= '0' && *p <= '9'))) buf[n++] = *p++;
        buf[n] = 0;
        char* q = nullptr;
        const double v = strtod(buf, &q);
        if (n == 0 || q != buf + n || !std::isfinite(v)) ok = false;
        return v;
    }
    void skip()
    {
        ws();
        if (p >= end) {
            ok = false;
            return;
        }
        if (*p == '"') {
            (void)str();
        } else if (*p == '{' || *p == '[') {
            if (depth >= kMaxDepth) {  // a table file nests two levels; deeper input is malformed
                ok = false;
                return;
            }
            const char close = *p == '{' ? '}' : ']';
            const bool obj = *p == '{';
            p++;
            depth++;
            if (!eat(close)) {
                do {
                    if (obj) {
                        (void)str();
                        expect(':');
                    }
                    skip();
                } while (ok && eat(','));
                expect(close);
            }
            depth--;
        } else if (end - p >= 4 && (!strncmp(p, "true", 4) || !strncmp(p, "null", 4))) {
            p += 4;
        } else if (end - p >= 5 && !strncmp(p, "false", 5)) {
            p += 5;
        } else {
            (void)num();
        }
    }
};

bool as_int(double v, int* out)
{
    if (!(v >= -1e9 && v <= 1e9) || v != std::floor(v)) return false;
    *out = (int)v;
    return true;
}

// Parses one entry object.
bool parse_entry(Reader& r, TuneEntry& e)
{
    e = TuneEntry{-1, -1, -1, -1, -1, -1, 0.0};
    r.expect('{');
    if (r.eat('}')) return false;
    do {
        const std::string k = r.str();
        r.expect(':');
        if (!r.ok) return false;
        if (k == "ms") {
            e.ms = r.num();
            continue;
        }
        int* dst = k == "prec" ? &e.prec : k == "batched" ? &e.batched : k == "n_log2" ? &e.n_log2
                 : k == "p_log2" ? &e.p_log2 : k == "tile" ? &e.tile : k == "field_npl" ? &e.npl : nullptr;
        if (!dst) {
            r.skip();
            continue;
        }
        if (!as_int(r.num(), dst)) r.ok = false;
    } while (r.ok && r.eat(','));
    r.expect('}');
    return r.ok && valid_entry(e);
}

// Architecture name up to the first ':' (the target features differ by driver).
std::string arch_base(const char* a)
{
    std::string s(a ? a : "");
    const size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
}

}  // namespace

int tune_load(TuneTable* t, const char* path, const char* arch)
{
    if (!t || !path) return LENS_ERR_INVALID;
    FILE* f = fopen(path, "rb");
    if (!f) return LENS_ERR_INVALID;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 24)) text.append(buf, n);
    fclose(f);
    Reader r{text.data(), text.data() + text.size()};
    std::string file_arch;
    std::vector<TuneEntry> got;
    r.expect('{');
    if (!r.eat('}')) {
        do {
            const std::string k = r.str();
            r.expect(':');
            if (!r.ok) break;
            if (k == "arch") {
                file_arch = r.str();
            } else if (k == "entries") {
                r.expect('[');
                if (!r.eat(']')) {
                    do {
                        TuneEntry e;
                        if (!parse_entry(r, e)) r.ok = false;
                        got.push_back(e);
                    } while (r.ok && r.eat(','));
                    r.expect(']');
                }
            } else {
                r.skip();
            }
        } while (r.ok && r.eat(','));
        r.expect('}');
    }
    r.ws();
    if (!r.ok || r.p != r.end || file_arch.empty()) return LENS_ERR_INVALID;
    if (arch_base(file_arch.c_str()) != arch_base(arch)) return LENS_OK;  // another GPU: nothing applies
    for (const TuneEntry& e : got) record(t, e);
    return LENS_OK;
}

static int save(const TuneTable* t, const char* path, const char* arch)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return LENS_ERR_INVALID;
    fprintf(f, "{\n  \"arch\": \"%s\",\n  \"entries\": [", arch_base(arch).c_str());
    for (size_t i = 0; i < t->entries.size(); i++) {
        const TuneEntry& e = t->entries[i];
        fprintf(f,
                "%s\n    {\"prec\": %d, \"batched\": %d, \"n_log2\": %d, \"p_log2\": %d, \"tile\": %d, "
                "\"field_npl\": %d, \"ms\": %.6f}",
                i ? "," : "", e.prec, e.batched, e.n_log2, e.p_log2, e.tile, e.npl, e.ms);
    }
    fprintf(f, "\n  ]\n}\n");
    const bool ok = fflush(f) == 0;
    if (fclose(f) != 0 || !ok) {
        remove(tmp.c_str());
        return LENS_ERR_INVALID;
    }
    if (rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return LENS_ERR_INVALID;
    }
    return LENS_OK;
}

// ---------------------------------------------------------------- timing of candidates

namespace {

struct Device {
    int prev = -1;
    bool ok = false;
    explicit Device(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~Device()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool device_arch(int dev, std::string& arch)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    arch = prop.gcnArchName;
    return true;
}

// Median wall time (ms, on the stream) of `reps` calls after one warm-up.
// rc receives the call's first error; a candidate that does not fit
// (LENS_ERR_CAPACITY from the call itself) is reported as such.
template <typename Call>
int time_call(Call call, int reps, hipStream_t s, hipEvent_t a, hipEvent_t b, double* ms)
{
    int rc = call();
    if (rc) return rc;
    std::vector<double> t;
    for (int k = 0; k < reps; k++) {
        if (hipEventRecord(a, s) != hipSuccess) return LENS_ERR_DEVICE;
        if ((rc = call())) return rc;
        if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return LENS_ERR_DEVICE;
        float v = 0.0f;
        if (hipEventElapsedTime(&v, a, b) != hipSuccess) return LENS_ERR_DEVICE;
        t.push_back(v);
    }
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return LENS_OK;
}

// Tries the default configuration first, then the other nodes per thread
// (mixed only) with the default tile, then the other tile shapes with the
// best nodes per thread.  A candidate replaces the best so far only when it is
// faster by more than kMargin, so timing noise leaves the default in place;
// records and returns the choice.
constexpr double kMargin = 0.02;

template <typename Run>
int tune(lens_ctx* ctx, int prec, int batched, int n_log2, int p_log2, int default_npl, int reps, hipStream_t s,
         Run run, int32_t* tile_out, int32_t* npl_out)
{
    if (reps < 1 || reps > 100) return LENS_ERR_INVALID;
    TuneTable* table = lens_ctx_tune(ctx);
    if (!table) return LENS_ERR_DEVICE;
    Device dev(lens_ctx_device(ctx));
    std::string arch;
    if (!dev.ok || !device_arch(lens_ctx_device(ctx), arch)) return LENS_ERR_DEVICE;
    const int timing = lens_ctx_timing(ctx);
    if (timing) lens_set_timing(ctx, 0);
    hipEvent_t a = nullptr, b = nullptr;
    int rc = LENS_OK;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = LENS_ERR_DEVICE;
    const bool mixed = prec == LENS_MIXED;
    int best_tile = 1, best_npl = mixed ? default_npl : 0;
    double best = INFINITY;
    auto trial = [&](int tile, int npl) {
        if (rc) return;
        double ms = 0.0;
        const int r = time_call([&] { return run(tile, npl); }, reps, s, a, b, &ms);
        if (r == LENS_ERR_CAPACITY) return;  // this shape's scratch bound is exceeded: not a candidate
        if (r) {
            rc = r;
            return;
        }
        if (ms < best * (1.0 - kMargin)) {
            best = ms;
            best_tile = tile;
            best_npl = npl;
        }
    };
    trial(best_tile, best_npl);
    if (mixed) {  // FP32 field layouts: nodes of one row, then blocks of rows x columns
        const int npls[9] = {1, 2, 4, 8, 0x21, 0x22, 0x24, 0x41, 0x42};
        for (int k = 0; k < 9; k++)
            if (npls[k] != default_npl && (batched ? bfield_code_ok(npls[k]) : field_code_ok(npls[k])))
                trial(1, npls[k]);
    }
    const int npl = best_npl;
    for (int tile = 2; tile <= 4; tile++) trial(tile, npl);
    if (!rc && !std::isfinite(best)) rc = LENS_ERR_CAPACITY;
    if (!rc) {
        record(table, TuneEntry{prec, batched, n_log2, p_log2, best_tile, best_npl, best});
        rc = run(best_tile, best_npl);  // leaves the caller's outputs from the chosen configuration
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (timing) lens_set_timing(ctx, 1);
    if (!rc) {
        if (tile_out) *tile_out = best_tile;
        if (npl_out) *npl_out = best_npl;
    }
    return rc;
}

}  // namespace

}  // namespace lens

using namespace lens;

extern "C" {

int lens_autotune_chi2(lens_ctx* ctx, const lens_potentials* pot, const lens_grid* grid, const lens_obs* obs,
                       const lens_chi2_opts* opts, lens_chi2_out* out, int32_t reps, int32_t* tile,
                       int32_t* field_npl, hipStream_t stream)
{
    try {
        if (!ctx || !pot || !grid || !opts) return LENS_ERR_INVALID;
        const int n_log2 = tune_log2(std::max(grid->nx, grid->ny));
        const int p_log2 = tune_log2(pot->n);
        auto run = [&](int t, int npl) {
            lens_chi2_opts o = *opts;
            o.tile = t;
            o.field_npl = npl;
            return lens_image_chi2(ctx, pot, grid, obs, &o, out, stream);
        };
        return tune(ctx, opts->prec, 0, n_log2, p_log2, lens_default_field_npl(grid->nx, grid->ny), reps, stream, run,
                    tile, field_npl);
    } catch (...) {
        return LENS_ERR_DEVICE;
    }
}

int lens_autotune_chi2_batched(lens_ctx* ctx, const lens_potentials* all, int32_t n_samples, const int32_t* pot_off,
                               const lens_grid* grids, const lens_obs* obs, const lens_chi2_opts* opts,
                               lens_batch_out* out, int32_t reps, int32_t* tile, int32_t* field_npl,
                               hipStream_t stream)
{
    try {
        if (!ctx || !all || n_samples < 1 || !pot_off || !grids || !opts) return LENS_ERR_INVALID;
        int side = 1;
        for (int i = 0; i < n_samples; i++) side = std::max(side, std::max(grids[i].nx, grids[i].ny));
        const long long mean_p = ((long long)all->n + n_samples - 1) / n_samples;
        auto run = [&](int t, int npl) {
            lens_chi2_opts o = *opts;
            o.tile = t;
            o.field_npl = npl;
            return lens_image_chi2_batched(ctx, all, n_samples, pot_off, grids, obs, &o, out, stream);
        };
        return tune(ctx, opts->prec, 1, tune_log2(side), tune_log2(mean_p), 0x41, reps, stream, run, tile, field_npl);
    } catch (...) {
        return LENS_ERR_DEVICE;
    }
}

int lens_autotune_lookup(lens_ctx* ctx, lens_precision prec, int32_t batched, int32_t n_side, int32_t n_pot,
                         int32_t* tile, int32_t* field_npl)
{
    if (!ctx || !tile || !field_npl || n_side < 1 || n_pot < 0 || (batched != 0 && batched != 1))
        return LENS_ERR_INVALID;
    int t = 0, n = 0;
    if (!tune_lookup(lens_ctx_tune(ctx), prec, batched, tune_log2(n_side), tune_log2(n_pot), &t, &n)) t = n = 0;
    *tile = t;
    *field_npl = n;
    return LENS_OK;
}

int lens_autotune_save(lens_ctx* ctx, const char* path)
{
    try {
        if (!ctx || !path || !lens_ctx_tune(ctx)) return LENS_ERR_INVALID;
        std::string arch;
        if (!device_arch(lens_ctx_device(ctx), arch)) return LENS_ERR_DEVICE;
        return save(lens_ctx_tune(ctx), path, arch.c_str());
    } catch (...) {
        return LENS_ERR_DEVICE;
    }
}

int lens_autotune_load(lens_ctx* ctx, const char* path)
{
    try {
        if (!ctx || !path || !lens_ctx_tune(ctx)) return LENS_ERR_INVALID;
        std::string arch;
        if (!device_arch(lens_ctx_device(ctx), arch)) return LENS_ERR_DEVICE;
        return tune_load(lens_ctx_tune(ctx), path, arch.c_str());
    } catch (...) {
        return LENS_ERR_DEVICE;
    }
}

}  // extern "C"
