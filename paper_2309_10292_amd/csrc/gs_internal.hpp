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
gs_status read_field(const void *dev, int32_t storage, size_t n, double *host, hipStream_t st);
gs_status write_field(void *dev, int32_t storage, size_t n, const double *host, hipStream_t st);
// Synchronising diagnostics of a (u, v) pair using the workspace's partials.
gs_status diagnostics(int32_t storage, const void *u, const void *v, size_t n, void *ws, hipStream_t st,
                      gs_diag *out);
// Byte offset of the graph-replay step counter inside a workspace.
size_t counter_offset();

} // namespace gsapi
