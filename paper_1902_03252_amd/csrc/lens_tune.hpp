// Autotuning table of a context (internal interface between lens_api.hip and
// lens_tune.hip).  One entry per bucket
//     (precision, single or batched call, ceil(log2 grid side), ceil(log2 P))
// holds the fastest measured triangle-stage tile shape and FP32 field nodes
// per thread.
#pragma once

#include "lens.h"

namespace lens {

struct TuneTable;

TuneTable* tune_new();
void tune_delete(TuneTable* t);

// Bucket of a problem: grid side = max(nx, ny) (largest over a batch), P =
// potentials (rounded-up mean over a batch).
int tune_log2(long long v);

// The table's choice for a bucket; false if it holds none.
bool tune_lookup(const TuneTable* t, int prec, int batched, int n_log2, int p_log2, int* tile, int* npl);

// Merges the JSON file `path` (entries of other GPU architectures skipped).
// LENS_OK, or LENS_ERR_INVALID for a missing or malformed file (table unchanged).
int tune_load(TuneTable* t, const char* path, const char* arch);

}  // namespace lens

// Context accessors (defined in lens_api.hip).
lens::TuneTable* lens_ctx_tune(lens_ctx* ctx);
int lens_ctx_device(lens_ctx* ctx);
int lens_ctx_timing(lens_ctx* ctx);  // whether field-kernel timing is on
int lens_default_field_npl(int nx, int ny);  // FP32 field nodes per thread of an untuned single call
