/*
 * gs.h -- C ABI of the MI355X (gfx950) Gray-Scott library, libgs.so.
 *
 * The library advances the two coupled Gray-Scott fields u, v of the paper's
 * Section 3.1 on a periodic 3-D grid:
 *   Eq. 1a/1b  dU/dt = Du lap(U) - U V^2 + F (1 - U) + n r
 *              dV/dt = Dv lap(V) + U V^2 - (F + k) V
 *   Eq. 2a/2b  forward Euler in time, Jacobi (level t+1 from level t only)
 *   Eq. 3      7-point Laplacian in normalised units: (sum of six neighbours - 6 c) / 6
 *
 * Conventions shared by every entry point:
 *   - Layout: a field is nz*ny*nx contiguous elements, x fastest:
 *     idx = x + nx * (y + ny * z). Boundaries are periodic in x, y and z.
 *   - Device pointers are HIP device allocations (hipMalloc or PyTorch's
 *     allocator) on the current HIP device, aligned to 256 bytes. The caller
 *     owns all field and workspace memory; the library never frees it.
 *   - Host pointers are ordinary host memory.
 *   - `hip_stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it; calls documented as
 *     synchronising wait for that stream only.
 *   - Every call returns a gs_status. Arguments are validated before any HIP
 *     call is made, so validation errors leave device state untouched.
 *     gs_last_error() returns a thread-local message for the last failure.
 *   - A handle is used from one host thread at a time; distinct handles are
 *     independent.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gs_status {
    GS_OK = 0,
    GS_ERR_INVALID_ARG = -1, /* NULL/misaligned pointer, non-finite or negative coefficient, bad size */
    GS_ERR_UNSUPPORTED = -2, /* well-formed request outside what the kernels handle (e.g. nx % 8 != 0) */
    GS_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed (message has hipGetErrorString) */
    GS_ERR_NONFINITE = -4,   /* gs_diagnostics found NaN or Inf in the fields */
    GS_ERR_STATE = -5        /* NULL or destroyed handle */
} gs_status;

/* Storage type of the fields in device memory. GS_F64 computes in FP64 and
 * reproduces the FP64 definition of the step bit for bit; the other types
 * compute in FP32 (Laplacian neighbour sum compensated) and round each stored
 * value to nearest-even. GS_BF16C is BF16 storage that keeps 1 - u in place
 * of u (v as it is): where u is near 1, most of a Gray-Scott state, 1 - u is
 * small and BF16 keeps eight significant bits of it, where plain BF16 steps
 * u by 2^-8. Its u buffers hold 1 - u (gs_read, gs_write and gs_diagnostics
 * convert; gs_current hands out the raw buffers); not for batched sweeps. */
typedef enum gs_dtype { GS_F64 = 0, GS_F32 = 1, GS_BF16 = 2, GS_F16 = 3, GS_BF16C = 4 } gs_dtype;

typedef enum gs_init_mode {
    GS_INIT_NONE = 0, /* the caller has filled u0, v0 (storage type) */
    GS_INIT_CUBE = 1  /* u = 1, v = 0, and the axis-aligned cube of side cube_side with lower
                         corner floor((n - cube_side) / 2) per axis set to (cube_u, cube_v) */
} gs_init_mode;

/* Problem statement (Eq. 1-3; parameter names as in the paper's provenance
 * record, Listing 1). */
typedef struct gs_params {
    int32_t nx, ny, nz;   /* grid; each >= 4, nx % 8 == 0 (else GS_ERR_UNSUPPORTED) */
    int32_t storage;      /* gs_dtype */
    double Du, Dv;        /* diffusion rates, finite, >= 0 */
    double F, k;          /* feed and kill rates, finite */
    double dt;            /* time step, finite */
    double noise;         /* magnitude n of the noise term n r on U; finite, 0 (disables it) or in
                             [2^-990, inf) (GS_ERR_UNSUPPORTED below) */
    uint64_t seed;        /* Philox4x32-10 key for r */
    uint64_t step0;       /* global index of the initial state's step (resume) */
    int32_t init_mode;    /* gs_init_mode */
    int32_t cube_side;    /* GS_INIT_CUBE only: 1 <= cube_side <= min(nx, ny, nz) */
    double cube_u, cube_v;
    int32_t tblock;       /* time steps fused per sweep: 0 = library choice, else 1..GS_MAX_TBLOCK */
    int32_t tile;         /* tile shape index: 0 = library choice, else 1..gs_num_tiles() */
    int32_t zchunk;       /* planes per z-chunk of one workgroup: 0 = library choice, else >= 1 */
    int32_t reserved;     /* must be 0 */
} gs_params;

#define GS_MAX_TBLOCK 4

/* The noise r(seed, t, idx) of step t (0-based index of the step being taken,
 * i.e. step0 + steps already done) at cell idx is word (idx % 4) of the
 * Philox4x32-10 block with counter (low, high halves of idx / 4, low, high
 * halves of t) and key (low, high halves of seed), read as a signed 32-bit
 * integer w and mapped to (w + 0.5) * 2^-31, an exact FP64 value in (-1, 1).
 * It is added to U's bracket in Eq. 2a, i.e. multiplied by dt. */

typedef struct gs_sim gs_sim; /* opaque handle */

typedef struct gs_diag {
    double sum_u, sum_v;      /* compensated FP64 sums over all cells */
    double min_u, max_u, min_v, max_v; /* over the finite cells */
    int64_t nonfinite;        /* number of NaN or Inf values in u and v together */
} gs_diag;

/* Library version string (static storage). */
const char *gs_version(void);

/* Thread-local message describing the last failed call on this thread. */
const char *gs_last_error(void);

/* Bytes of device workspace gs_init needs for this problem (diagnostic
 * partials and the graph-replay step counter); 0 for invalid params. The
 * caller allocates it. */
size_t gs_workspace_bytes(const gs_params *p);

/* Tile shapes (valid gs_params.tile values are 1..gs_num_tiles()). The first
 * four select the single-step z-streaming kernel (tblock must be 1); the
 * others select the temporally blocked kernel, which fuses tblock steps per
 * pass (workgroups of 256 to 1024 lanes; the larger ones fuse fewer steps in
 * FP64, whose registers are twice as many). gs_tile_info reports the output
 * tile (tx cells by ty rows) of `tile` for a storage type and tblock, and the
 * largest tblock the tile accepts for that storage type. */
int32_t gs_num_tiles(void);
gs_status gs_tile_info(int32_t tile, int32_t storage, int32_t tblock, int32_t *tx, int32_t *ty,
                       int32_t *max_tblock);

/* Binds four caller-owned device buffers of nx*ny*nz elements of the storage
 * type. (u0, v0) hold the state at step p->step0; (u1, v1) are the second
 * allocation of both fields that receives the next time level (the
 * temporaries of Sec. 3.2, On-Node Parallelization); the library ping-pongs
 * between the pairs. `workspace` holds
 * gs_workspace_bytes(p) bytes. If p->init_mode == GS_INIT_CUBE the init
 * kernel fills (u0, v0) on `hip_stream`. Does not allocate device memory.
 * On success *out is a new handle; on failure *out is NULL. */
gs_status gs_init(const gs_params *p, void *u0, void *v0, void *u1, void *v1,
                  void *workspace, void *hip_stream, gs_sim **out);

/* Advances the state by n_steps >= 0 steps (Eq. 2a/2b), enqueued on the
 * handle's stream; returns after the launches. n_steps == 0 is a no-op.
 * Launch failures return GS_ERR_HIP; faults inside kernels surface at the
 * next synchronising call. */
gs_status gs_step(gs_sim *s, int64_t n_steps);

/* Synchronising. Copies the current u and/or v, widened to FP64, into host
 * arrays of nx*ny*nz doubles (NULL skips that field): the state the paper's
 * workflow hands to output and analysis (Sec. 3.4). x varies fastest:
 * element x + nx*(y + ny*z). */
gs_status gs_read(gs_sim *s, double *u_host, double *v_host);

/* Synchronising. Replaces the current u and/or v by host FP64 arrays of
 * nx*ny*nz doubles, rounded to the storage type (to FP32 first, then to the
 * 16-bit type; nearest-even). NULL leaves that field unchanged. */
gs_status gs_write(gs_sim *s, const double *u_host, const double *v_host);

/* Zero-copy view: device pointers of the buffers holding the current state
 * (which of the two allocations of Sec. 3.2 holds the newest time level),
 * and the global step index of that state. Any output pointer may be NULL.
 * The pointers stay owned by the caller; they change after each step. */
gs_status gs_current(gs_sim *s, void **u_dev, void **v_dev, uint64_t *step);

/* Synchronising. Per-field min/max of the current state, as the paper's
 * provenance record reports them for U and V at each output step
 * (Listing 1), with FP64 compensated sums (the mass sum(u + v) is
 * sum_u + sum_v) and the non-finite count. Returns GS_ERR_NONFINITE (with
 * *out filled) when nonfinite > 0. */
gs_status gs_diagnostics(gs_sim *s, gs_diag *out);

/* Sets the global step index of the current state (the noise key of the
 * next step), for callers that replace the state by other means, such as a
 * learned surrogate's jump. */
gs_status gs_set_step(gs_sim *s, uint64_t step);

/* Replaces the current state by u = 1, v = 0 and the periodic cube of side
 * `side` with lower corner (x0, y0, z0) (wrapping around the grid) set to
 * (cu, cv). Asynchronous. */
gs_status gs_fill_cube(gs_sim *s, int32_t x0, int32_t y0, int32_t z0, int32_t side, double cu, double cv);

/* Synchronising: *out = sum over i < n of (a_i - b_i)^2 in FP64 for two
 * device arrays of the storage type; `workspace` holds
 * gs_sqdiff_workspace_bytes() device bytes. */
size_t gs_sqdiff_workspace_bytes(void);
gs_status gs_sqdiff(const void *a, const void *b, size_t n, int32_t storage, void *workspace, void *hip_stream,
                    double *out);

/* gs_sqdiff without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc). Same arguments, kernel and result (bit for bit) as gs_sqdiff.
 * The partial sums live in a static device array of the library (4 KiB per
 * GPU, held until the process ends), found on first use on each device; the
 * call allocates nothing. n <= 2^40 (GS_ERR_UNSUPPORTED beyond). Calls that
 * overlap on one GPU (several host threads, or streams of one device) share
 * that array and race: serialise them. Synchronising. */
gs_status gs_sqdiff_noalloc(const void *a, const void *b, size_t n, int32_t storage, void *hip_stream,
                            double *out);

/* Waits for all work enqueued by this handle. */
gs_status gs_sync(gs_sim *s);

/* Frees the handle only (not the caller's buffers); waits for its work first.
 * Any later call with this handle returns GS_ERR_STATE. */
gs_status gs_destroy(gs_sim *s);

/* ------------------------------------------------------------------ */
/* Launch configuration, autotuning and graph replay. */

typedef struct gs_tune_entry {
    int32_t tile, tblock, zchunk, reserved;
    double ms_per_step;   /* measured time per time step (ms) */
} gs_tune_entry;

/* Sets the launch configuration of later steps: tile 1..gs_num_tiles(),
 * tblock 1..max for that tile (see gs_tile_info), zchunk >= 1 (clamped to nz). */
gs_status gs_set_config(gs_sim *s, int32_t tile, int32_t tblock, int32_t zchunk);
gs_status gs_get_config(gs_sim *s, int32_t *tile, int32_t *tblock, int32_t *zchunk);

/* Synchronising autotuner. Times every (tile, tblock, zchunk) candidate with
 * `reps` >= 1 launches after one warm-up on the handle's own buffers: each
 * launch reads the current pair and writes the other, so the state and the
 * step index are unchanged. Selects the fastest (time per step) for later
 * gs_step / gs_step_graph calls. If `table` is non-NULL the first `capacity`
 * measurements are written there; *n_entries (if non-NULL) receives the
 * number of candidates measured.
 * Tuning cache: when the environment variable GS_TUNE_CACHE names a file, the
 * choice is recorded there (one JSON object per line, keyed by storage type,
 * nx, ny, nz and whether noise is on; an existing entry for the key is
 * replaced), and gs_init uses a recorded choice for the same key when
 * gs_params leaves tile, tblock and zchunk all 0. If the file cannot be
 * written, gs_tune returns GS_ERR_INVALID_ARG and the handle keeps the tuned
 * configuration. gs_batch_tune and gs_batch_init do the same per grid class
 * ("kind":"batch" entries). */
gs_status gs_tune(gs_sim *s, int32_t reps, gs_tune_entry *table, int32_t capacity, int32_t *n_entries);

/* Same result as gs_step(s, n_steps), enqueued as one HIP graph replay. The
 * graph is captured on first use for this (n_steps, current buffer pair,
 * configuration) and reused while those stay the same; every replay reads its
 * start step from a counter in the workspace, set by a one-lane kernel just
 * before the replay (no memset nodes). */
gs_status gs_step_graph(gs_sim *s, int64_t n_steps);

/* ------------------------------------------------------------------ */
/* Batched sweeps: many independent simulations (own grid and own F, k; shared
 * Du, Dv, dt, noise, storage) advanced together by persistent launches of the
 * temporally blocked kernel. Simulation i draws its noise with key seed + i.
 * Every simulation has a launch configuration (tile among the temporally
 * blocked tiles, tblock, zchunk >= 8); simulations sharing (tile, tblock) are
 * advanced by one persistent launch per tblock steps. */

typedef struct gs_batch gs_batch; /* opaque handle */

typedef struct gs_batch_tune_entry {
    int32_t nx, ny, nz, n_sims;       /* the grid class and how many simulations have it */
    int32_t tile, tblock, zchunk, reserved; /* the configuration chosen for it */
    double ms_per_step;               /* time per step of all its simulations together */
    double gcells;                    /* their cell-updates per second, in units of 1e9 */
} gs_batch_tune_entry;

/* Largest tblock a temporally blocked tile accepts in batched sweeps for a
 * storage type (the persistent kernel needs a few more registers than the
 * single-grid one); 0 when the tile is not available to batches or the
 * arguments are invalid. */
int32_t gs_batch_max_tblock(int32_t tile, int32_t storage);

/* Device bytes of the fields of all simulations (4 buffers each, 256-byte
 * aligned) and of the batch workspace (descriptors, work lists, diagnostic
 * partials); 0 for invalid arguments. */
size_t gs_batch_arena_bytes(int32_t storage, int32_t n_sims, const int32_t *nx, const int32_t *ny,
                            const int32_t *nz);
size_t gs_batch_workspace_bytes(int32_t n_sims, const int32_t *nx, const int32_t *ny, const int32_t *nz);

/* `base` gives storage, Du, Dv, dt, noise, seed, step0, init (the cube of
 * cube_side centred in every grid) and optionally tile/tblock/zchunk for all
 * simulations (0 = library choice); its nx, ny, nz, F and k are ignored.
 * nx, ny, nz, F, k are host arrays of n_sims entries; each grid follows the
 * gs_params rules. `arena` and `workspace` are caller-owned device memory of
 * at least the sizes above. Synchronising (uploads the work lists). */
gs_status gs_batch_init(const gs_params *base, int32_t n_sims, const int32_t *nx, const int32_t *ny,
                        const int32_t *nz, const double *F, const double *k, void *arena, size_t arena_bytes,
                        void *workspace, size_t workspace_bytes, void *hip_stream, gs_batch **out);

/* Advance every simulation by n_steps (asynchronous), directly or as one
 * captured HIP graph replay (same result). */
gs_status gs_batch_step(gs_batch *b, int64_t n_steps);
gs_status gs_batch_step_graph(gs_batch *b, int64_t n_steps);

/* Configuration of one simulation (sim >= 0) or of all (sim == -1); applied
 * at the next step call. */
gs_status gs_batch_set_config(gs_batch *b, int32_t sim, int32_t tile, int32_t tblock, int32_t zchunk);
gs_status gs_batch_get_config(gs_batch *b, int32_t sim, int32_t *tile, int32_t *tblock, int32_t *zchunk);

/* Synchronising autotuner: for every distinct grid size, times each
 * (tile, tblock, zchunk) candidate on the simulations of that size (their
 * states and the step index stay unchanged) and assigns the fastest to them.
 * One entry per grid size is written to `table` (up to `capacity`);
 * *n_entries receives the number of grid sizes. */
gs_status gs_batch_tune(gs_batch *b, int32_t reps, gs_batch_tune_entry *table, int32_t capacity,
                        int32_t *n_entries);

/* Per-simulation access, as gs_current / gs_read / gs_write / gs_diagnostics. */
gs_status gs_batch_current(gs_batch *b, int32_t sim, void **u_dev, void **v_dev, uint64_t *step);
gs_status gs_batch_read(gs_batch *b, int32_t sim, double *u_host, double *v_host);
gs_status gs_batch_write(gs_batch *b, int32_t sim, const double *u_host, const double *v_host);
gs_status gs_batch_diagnostics(gs_batch *b, int32_t sim, gs_diag *out);

/* As gs_fill_cube, for one simulation of a batch. */
gs_status gs_batch_fill_cube(gs_batch *b, int32_t sim, int32_t x0, int32_t y0, int32_t z0, int32_t side, double cu,
                             double cv);

gs_status gs_batch_sync(gs_batch *b);
gs_status gs_batch_destroy(gs_batch *b);

/* ------------------------------------------------------------------ */
/* Learned surrogate of 16 steps: a network of four circular 3x3x3
 * convolutions (channels 4 -> 32 -> 32 -> 32 -> 2, GELU after the first
 * three, bias everywhere) mapping (u, v, (F - 0.035) / 0.025, (k - 0.055) /
 * 0.015) to a correction added to (u, v). BF16 weights and activations, FP32
 * accumulation on the matrix cores, FP32 master weights for Adam. The network
 * reads u and v as BF16 pairs (high part plus the BF16 rounding of the rest,
 * about 16 significant bits) that share one weight, so the 16-step change it
 * predicts is not swamped by BF16 rounding of fields near 1.
 * Parameters are a flat FP32 host array of GS_SURR_NPARAMS values: for each
 * layer W[c_out][c_in][3][3][3] (row-major; W[o][i][dz][dy][dx] multiplies
 * the input at (z + dz - 1, y + dy - 1, x + dx - 1), periodic), then b[c_out].
 * Fields are planar device arrays, sample-major: nsamp * nx * ny * nz values,
 * x fastest. Grids need nx % 16 == 0 and a cell count divisible by 32. */

#define GS_SURR_NPARAMS 60578

typedef struct gs_surrogate gs_surrogate;

size_t gs_surrogate_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t max_batch);

/* Binds a caller-owned workspace for batches of up to max_batch samples and
 * uploads `params` (synchronising). */
gs_status gs_surrogate_init(int32_t nx, int32_t ny, int32_t nz, int32_t max_batch, const float *params,
                            void *workspace, size_t workspace_bytes, void *hip_stream, gs_surrogate **out);

/* Replaces the parameters (and resets the Adam moments), or reads them back.
 * Both synchronise. */
gs_status gs_surrogate_set_params(gs_surrogate *s, const float *params);
gs_status gs_surrogate_get_params(gs_surrogate *s, float *params);

/* Prediction of nsamp <= max_batch samples; io_storage is GS_F64 or GS_F32
 * for u, v, u_out, v_out (device, must not alias); F and k are host arrays of
 * nsamp values. Asynchronous after the upload of F and k. */
gs_status gs_surrogate_predict(gs_surrogate *s, int32_t nsamp, int32_t io_storage, const void *u, const void *v,
                               const double *F, const double *k, void *u_out, void *v_out);

/* Mean squared error of the prediction against (u_target, v_target) over all
 * samples, both fields and all cells (FP32 device inputs), and its gradient
 * with respect to every parameter, kept on the device for gs_surrogate_adam
 * and copied to grad_host (GS_SURR_NPARAMS floats) when it is non-NULL.
 * Synchronising; *loss receives the loss. */
gs_status gs_surrogate_loss_grad(gs_surrogate *s, int32_t nsamp, const float *u, const float *v,
                                 const float *u_target, const float *v_target, const double *F, const double *k,
                                 double *loss, float *grad_host);

/* One Adam step with the last gradient (bias-corrected moments). */
gs_status gs_surrogate_adam(gs_surrogate *s, float lr, float beta1, float beta2, float eps);

/* Inspection of the last forward pass (gs_surrogate_predict or
 * gs_surrogate_loss_grad) and of the last backward pass, for tests: copies
 * one workspace tensor, as stored, to `host` (at least the bytes given;
 * rows = samples of that pass times nx*ny*nz, sample-major, x fastest):
 *   GS_SURR_INPUT (layer 0)   the packed network input, BF16, 8 channels per
 *                             row: (u_hi, v_hi, f, k, u_lo, v_lo, 0, 0), u and
 *                             v as the BF16 pairs that share one weight;
 *   GS_SURR_PRE (layer 0..2)  pre-activation z = conv + bias, BF16, 32 channels;
 *                             loss_grad's forward pass only (a prediction
 *                             stores no pre-activations: GS_ERR_STATE);
 *   GS_SURR_ACT (layer 0..2)  GELU of the FP32 pre-activation, BF16, 32 channels;
 *   GS_SURR_PRED (layer 3)    the FP32 prediction u then v (2 * rows floats);
 *                             loss_grad's forward pass only (predict writes the
 *                             caller's outputs);
 *   GS_SURR_DOUT (layer 3)    dloss/dprediction, BF16, 8 channels (u, v, 0...);
 *   GS_SURR_DPRE (layer 0..2) dloss/dz of that layer, BF16, 32 channels.
 * Synchronising. GS_ERR_STATE when the pass has not run. */
typedef enum gs_surr_tensor {
    GS_SURR_INPUT = 0,
    GS_SURR_PRE = 1,
    GS_SURR_ACT = 2,
    GS_SURR_PRED = 3,
    GS_SURR_DOUT = 4,
    GS_SURR_DPRE = 5
} gs_surr_tensor;
gs_status gs_surrogate_read_tensor(gs_surrogate *s, int32_t tensor, int32_t layer, void *host, size_t host_bytes);

gs_status gs_surrogate_destroy(gs_surrogate *s);

/* ------------------------------------------------------------------ */
/* Calibration kernels (measure the single-field stencil and plain streaming
 * on the same device, the analogue of the paper's Table 2 / Table 3 rows). */

/* Single-field FP64 7-point periodic Laplacian (Eq. 3): out = (sum of six
 * neighbours - 6 f) / 6, bitwise equal to the IEEE division. f and out are
 * device arrays of nx*ny*nz doubles (must not overlap); nx % 8 == 0. */
gs_status gs_laplacian7(const double *f, double *out, int32_t nx, int32_t ny, int32_t nz,
                        void *hip_stream);

/* Plain device-to-device copy of `bytes` bytes (multiple of 16) with the
 * library's own streaming kernel: the achievable-bandwidth reference. */
gs_status gs_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
