// Host helpers shared by the single-simulation and batched C ABI sources.
#pragma once

#include "../../include/gs.h"

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gsapi {

gs_status fail(gs_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
gs_status hip_fail(hipError_t e, const char *what);
size_t storage_bytes(int32_t storage);
bool aligned(const void *p, size_t a);
// Validates a problem statement (grid, coefficients, init, tiling fields).
gs_status validate(const gs_params *p);
// Synchronising copies between a device field of `storage` type and host FP64.
gs_status read_field(const void *dev, int32_t storage, size_t n, double *host, hipStream_t st, int field);
gs_status write_field(void *dev, int32_t storage, size_t n, const double *host, hipStream_t st, int field);
// Synchronising diagnostics of a (u, v) pair using the workspace's partials.
gs_status diagnostics(int32_t storage, const void *u, const void *v, size_t n, void *ws, hipStream_t st,
                      gs_diag *out);
// Byte offset of the graph-replay step counter inside a workspace.
size_t counter_offset();

// Autotuner cache (file named by GS_TUNE_CACHE; see gs_tunecache.cpp).
enum { TUNE_SINGLE = 0, TUNE_BATCH = 1 };
struct TuneKey {
    int kind;          // TUNE_SINGLE or TUNE_BATCH
    int storage;
    int nx, ny, nz;
    int noisy;         // noise != 0
};
struct TuneVal {
    int tile, tblock, zchunk;
    double ms_per_step;
};
const char *tune_cache_path();
bool tune_cache_lookup(const TuneKey &key, TuneVal *val);
bool tune_cache_store(const TuneKey &key, const TuneVal &val); // false if the table could not be written

} // namespace gsapi
