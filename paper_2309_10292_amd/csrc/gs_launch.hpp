// Internal interface between the C ABI (gs_api.cpp) and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gs {

// Everything a step launch needs, by value (kernel argument).
struct StepArgs {
    int nx, ny, nz;
    int zc;              // planes per z-chunk
    int ntx, nty;        // tiles per row / column (set by the launcher)
    double Du, Dv, F, FK, dt, noise;   // FK = F + k, rounded once
    double noise_s, noise_h;           // noise 2^-31 and noise 2^-32 (exact: |noise| >= 2^-990 or 0)
    float Du_f, Dv_f, F_f, FK_f, dt_f, noise_f;
    float noise_s_f, noise_h_f;        // RN(noise 2^-31), RN(noise 2^-32) in FP32
    uint64_t seed;
    uint64_t t;          // global index of the step being taken (noise key)
    // When non-null, the step index is *t_dev + t (graph replays read the
    // base step from device memory so one captured graph serves every start).
    const uint64_t *t_dev;
};

__host__ __device__ inline uint64_t step_index(const StepArgs &a) { return a.t_dev ? *a.t_dev + a.t : a.t; }

template <typename C> struct Coef;
template <> struct Coef<double> {
    static __host__ __device__ double Du(const StepArgs &a) { return a.Du; }
    static __host__ __device__ double Dv(const StepArgs &a) { return a.Dv; }
    static __host__ __device__ double F(const StepArgs &a) { return a.F; }
    static __host__ __device__ double FK(const StepArgs &a) { return a.FK; }
    static __host__ __device__ double dt(const StepArgs &a) { return a.dt; }
    static __host__ __device__ double noise(const StepArgs &a) { return a.noise; }
};
template <> struct Coef<float> {
    static __host__ __device__ float Du(const StepArgs &a) { return a.Du_f; }
    static __host__ __device__ float Dv(const StepArgs &a) { return a.Dv_f; }
    static __host__ __device__ float F(const StepArgs &a) { return a.F_f; }
    static __host__ __device__ float FK(const StepArgs &a) { return a.FK_f; }
    static __host__ __device__ float dt(const StepArgs &a) { return a.dt_f; }
    static __host__ __device__ float noise(const StepArgs &a) { return a.noise_f; }
};

struct TileShape {
    int tx, ty;
};

int num_tiles();
TileShape tile_shape(int tile, int storage);

// One step (u, v) -> (un, vn) with the given tile (1..num_tiles()).
hipError_t launch_step(int storage, int tile, const void *u, const void *v, void *un, void *vn,
                       const StepArgs &a, hipStream_t st);
// Resident workgroups per CU of the single-step kernel (0 when unknown).
int step_occupancy(int storage, int tile, bool noise);

hipError_t launch_laplacian7(const double *f, double *out, int nx, int ny, int nz, hipStream_t st);

// Cube initial state in the storage type.
hipError_t launch_init_cube(int storage, void *u, void *v, int nx, int ny, int nz, int side,
                            double cu, double cv, hipStream_t st);

// Periodic cube at an arbitrary corner (u, v) = (cu, cv) in a (1, 0) background.
hipError_t launch_init_box(int storage, void *u, void *v, int nx, int ny, int nz, int x0, int y0, int z0, int side,
                           double cu, double cv, hipStream_t st);

// Per-workgroup FP64 partial sums of (a - b)^2 (sqdiff_blocks() doubles).
int sqdiff_blocks();
hipError_t launch_sqdiff(int storage, const void *a, const void *b, size_t n, double *part, hipStream_t st);

// Diagnostics: per-block partials into `ws`, then one block folds them.
// Result (9 doubles: sum_u, comp_u, sum_v, comp_v, min_u, max_u, min_v,
// max_v, nonfinite as double) lands at ws + diag_result_offset().
hipError_t launch_diagnostics(int storage, const void *u, const void *v, size_t n, void *ws, hipStream_t st);
size_t diag_workspace_bytes();
size_t diag_result_offset();

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st);

// Writes `value` to *dst with a one-lane kernel (graph-safe; no memset node).
hipError_t launch_set_u64(uint64_t *dst, uint64_t value, hipStream_t st);

} // namespace gs

namespace gs {
// Temporally blocked sweep: T steps (u, v) -> (un, vn) in one launch with
// tile shape 1..num_tb_shapes().
int num_tb_shapes();
TileShape tb_shape(int shape, int T);
// Largest number of fused steps the temporally blocked shape runs for a
// storage type (its registers fit the shape's lanes without spills), in the
// single-grid kernel and in the persistent batched kernel (0: the shape is
// not available).
int tb_max_T(int shape, int storage);
int tb_batch_max_T(int shape, int storage);
hipError_t launch_tblock(int storage, int T, int shape, const void *u, const void *v, void *un, void *vn,
                         const StepArgs &a, hipStream_t st);

// Batched sweep over independent simulations (device tables).
struct SimDesc {
    void *buf[2][2];    // [parity][field] device buffers
    int nx, ny, nz, zc;
    double F, FK;       // per-simulation feed and F + k
    float F_f, FK_f;
    uint64_t seed;
};

struct WorkItem {
    int sim, bx, by, bz;
};

struct BatchArgs {
    StepArgs coef;       // shared coefficients (Du, Dv, dt, noise); per-sim fields overwritten
    const SimDesc *sims;
    const WorkItem *items;
    int n_items;
    int parity;          // buffers holding the current state of every simulation of this launch
    uint64_t t;          // step index of the first fused step (offset when t_dev is set)
    const uint64_t *t_dev;
};

hipError_t launch_tblock_batch(int storage, int T, int shape, const BatchArgs &b, int grid, hipStream_t st);
int tb_shape_lanes(int shape);
// Resident workgroups per CU of the batched kernel (at least 1).
int tb_batch_occupancy(int storage, int T, int shape);
// Resident workgroups per CU of the single-grid blocked kernel (0 when unknown).
int tb_occupancy(int storage, int T, int shape, bool noise);
} // namespace gs
