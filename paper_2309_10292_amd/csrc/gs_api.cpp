// C ABI of libgs (declared in include/gs.h): validation, handle state,
// ping-pong parity, host <-> device conversion, launch selection.
#include "../../include/gs.h"
#include "gs_launch.hpp"
#include "gs_internal.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace gsapi {

thread_local std::string g_err;

gs_status fail(gs_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
gs_status fail(gs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

gs_status hip_fail(hipError_t e, const char *what)
{
    return fail(GS_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

const uint32_t k_magic = 0x47534d49u; // "GSMI"

size_t storage_bytes(int32_t s)
{
    switch (s) {
    case GS_F64: return 8;
    case GS_F32: return 4;
    case GS_BF16: return 2;
    case GS_F16: return 2;
    case GS_BF16C: return 2;
    }
    return 0;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Tile indices: 1..num_tiles() select the single-step z-streaming kernel's
// shapes; the next num_tb_shapes() indices select the temporally blocked
// kernel's shapes (any tblock).
int total_tiles() { return gs::num_tiles() + gs::num_tb_shapes(); }
bool is_tb_tile(int tile) { return tile > gs::num_tiles(); }
int tile_max_tblock(int tile, int storage) { return is_tb_tile(tile) ? gs::tb_max_T(tile - gs::num_tiles(), storage) : 1; }

gs_status validate(const gs_params *p)
{
    if (!p) return fail(GS_ERR_INVALID_ARG, "params is NULL");
    if (storage_bytes(p->storage) == 0) return fail(GS_ERR_INVALID_ARG, "unknown storage type %d", p->storage);
    if (p->nx < 4 || p->ny < 4 || p->nz < 4)
        return fail(GS_ERR_UNSUPPORTED, "grid %dx%dx%d: every dimension must be >= 4", p->nx, p->ny, p->nz);
    if (p->nx % 8 != 0) return fail(GS_ERR_UNSUPPORTED, "nx = %d must be a multiple of 8", p->nx);
    const double n = (double)p->nx * p->ny * p->nz;
    if (n * 16.0 > 9.0e18) return fail(GS_ERR_UNSUPPORTED, "grid too large");
    const double c[6] = {p->Du, p->Dv, p->F, p->k, p->dt, p->noise};
    const char *nm[6] = {"Du", "Dv", "F", "k", "dt", "noise"};
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(c[i])) return fail(GS_ERR_INVALID_ARG, "%s is not finite", nm[i]);
    if (p->Du < 0 || p->Dv < 0) return fail(GS_ERR_INVALID_ARG, "diffusion rates must be >= 0");
    if (p->noise < 0) return fail(GS_ERR_INVALID_ARG, "noise must be >= 0");
    // The FP64 kernels scale the noise by 2^-32 exactly; below this bound the
    // scaled value would be subnormal.
    if (p->noise != 0 && p->noise < 0x1p-990)
        return fail(GS_ERR_UNSUPPORTED, "noise %g below 2^-990 is not supported", p->noise);
    if (p->init_mode != GS_INIT_NONE && p->init_mode != GS_INIT_CUBE)
        return fail(GS_ERR_INVALID_ARG, "unknown init_mode %d", p->init_mode);
    if (p->init_mode == GS_INIT_CUBE) {
        int mn = p->nx < p->ny ? p->nx : p->ny;
        mn = mn < p->nz ? mn : p->nz;
        if (p->cube_side < 1 || p->cube_side > mn)
            return fail(GS_ERR_INVALID_ARG, "cube_side %d outside [1, %d]", p->cube_side, mn);
        if (!std::isfinite(p->cube_u) || !std::isfinite(p->cube_v))
            return fail(GS_ERR_INVALID_ARG, "cube values must be finite");
    }
    if (p->tblock < 0 || p->tblock > GS_MAX_TBLOCK)
        return fail(GS_ERR_INVALID_ARG, "tblock %d outside [0, %d]", p->tblock, GS_MAX_TBLOCK);
    if (p->tile < 0 || p->tile > total_tiles())
        return fail(GS_ERR_INVALID_ARG, "tile %d outside [0, %d]", p->tile, total_tiles());
    if (p->tile >= 1 && p->tile <= gs::num_tiles() && p->tblock > 1)
        return fail(GS_ERR_INVALID_ARG, "tile %d is a single-step tile; tblock must be 0 or 1", p->tile);
    if (p->tile >= 1 && p->tblock > tile_max_tblock(p->tile, p->storage))
        return fail(GS_ERR_INVALID_ARG, "tile %d fuses at most %d steps for this storage type", p->tile,
                    tile_max_tblock(p->tile, p->storage));
    if (p->zchunk < 0) return fail(GS_ERR_INVALID_ARG, "zchunk %d < 0", p->zchunk);
    if (p->reserved != 0) return fail(GS_ERR_INVALID_ARG, "reserved field must be 0");
    return GS_OK;
}

// Host rounding used by gs_write: FP64 -> FP32 (nearest-even, the C cast),
// then FP32 -> 16-bit nearest-even.
uint16_t host_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float host_from_bf16(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// field: 0 = u, 1 = v (GS_BF16C stores 1 - u).
gs_status read_field(const void *dev, int32_t storage, size_t n, double *host, hipStream_t st, int field)
{
    const size_t es = storage_bytes(storage);
    if (storage == GS_F64) {
        hipError_t e = hipMemcpyAsync(host, dev, n * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e == hipSuccess ? GS_OK : hip_fail(e, "device-to-host copy");
    }
    std::vector<unsigned char> stage(n * es);
    hipError_t e = hipMemcpyAsync(stage.data(), dev, n * es, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "device-to-host copy");
    if (storage == GS_F32) {
        const float *x = (const float *)stage.data();
        for (size_t i = 0; i < n; ++i) host[i] = x[i];
    } else if (storage == GS_BF16) {
        const uint16_t *x = (const uint16_t *)stage.data();
        for (size_t i = 0; i < n; ++i) host[i] = host_from_bf16(x[i]);
    } else if (storage == GS_BF16C) {
        const uint16_t *x = (const uint16_t *)stage.data();
        if (field == 0)
            for (size_t i = 0; i < n; ++i) host[i] = 1.0 - (double)host_from_bf16(x[i]);
        else
            for (size_t i = 0; i < n; ++i) host[i] = host_from_bf16(x[i]);
    } else {
        const _Float16 *x = (const _Float16 *)stage.data();
        for (size_t i = 0; i < n; ++i) host[i] = (double)(float)x[i];
    }
    return GS_OK;
}

gs_status write_field(void *dev, int32_t storage, size_t n, const double *host, hipStream_t st, int field)
{
    const size_t es = storage_bytes(storage);
    std::vector<unsigned char> stage;
    const void *src = host;
    if (storage != GS_F64) {
        stage.resize(n * es);
        if (storage == GS_F32) {
            float *d = (float *)stage.data();
            for (size_t i = 0; i < n; ++i) d[i] = (float)host[i];
        } else if (storage == GS_BF16) {
            uint16_t *d = (uint16_t *)stage.data();
            for (size_t i = 0; i < n; ++i) d[i] = host_bf16((float)host[i]);
        } else if (storage == GS_BF16C) {
            // u: 1 - u formed in FP64, then rounded to FP32 and to BF16
            uint16_t *d = (uint16_t *)stage.data();
            if (field == 0)
                for (size_t i = 0; i < n; ++i) d[i] = host_bf16((float)(1.0 - host[i]));
            else
                for (size_t i = 0; i < n; ++i) d[i] = host_bf16((float)host[i]);
        } else {
            _Float16 *d = (_Float16 *)stage.data();
            for (size_t i = 0; i < n; ++i) d[i] = (_Float16)(float)host[i];
        }
        src = stage.data();
    }
    hipError_t e = hipMemcpyAsync(dev, src, n * es, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? GS_OK : hip_fail(e, "host-to-device copy");
}

gs_status diagnostics(int32_t storage, const void *u, const void *v, size_t n, void *ws, hipStream_t st,
                      gs_diag *out)
{
    hipError_t e = gs::launch_diagnostics(storage, u, v, n, ws, st);
    if (e != hipSuccess) return hip_fail(e, "diagnostics launch");
    double r[9];
    e = hipMemcpyAsync(r, (char *)ws + gs::diag_result_offset(), sizeof r, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "diagnostics copy");
    out->sum_u = r[0] + r[1];
    out->sum_v = r[2] + r[3];
    out->min_u = r[4];
    out->max_u = r[5];
    out->min_v = r[6];
    out->max_v = r[7];
    out->nonfinite = (int64_t)r[8];
    if (out->nonfinite > 0) return fail(GS_ERR_NONFINITE, "%lld non-finite values", (long long)out->nonfinite);
    return GS_OK;
}

size_t counter_offset() { return (gs::diag_workspace_bytes() + 255) / 256 * 256; }

} // namespace gsapi

using namespace gsapi;

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    int64_t n = -1;
    int parity = -1;
    int tile = 0, tblock = 0, zc = 0;
};

struct gs_sim {
    uint32_t magic;
    gs_params p;
    void *buf[2][2]; // [parity][field]
    int parity;      // buffers holding the current state
    uint64_t step;   // global step index of the current state
    void *ws;
    hipStream_t stream;
    int tile;
    int zc;
    int tblock;
    size_t n;
    GraphCache graph;
    hipStream_t capture_stream;
};

namespace {

gs_status check(gs_sim *s)
{
    if (!s || s->magic != k_magic) return fail(GS_ERR_STATE, "invalid or destroyed handle");
    return GS_OK;
}

// Library choice of the launch configuration before any tuning (from the
// MI355X autotuner sweeps at 64^3 .. 1024^3, with and without noise): the
// temporally blocked kernel at every size. Large grids (>= 64 M cells): FP64
// fuses three steps in the 512-lane 64 x 22 tile; with noise the other
// storage types fuse two steps in the same tile (the Philox blocks of deeper
// fusion cost more than the traffic they save); without noise FP32 fuses two
// steps in the 1024-lane tile and the 16-bit types two in the 512-lane one.
// Smaller grids fuse two steps: in 256-lane workgroups below 4 M cells (more
// workgroups for 256 CUs), above that in the 768-lane tile for FP64 and the
// 512-lane one for the others. The single-step kernel (tiles 1..4) runs when
// asked for.
double grid_cells(const gs_params &p) { return (double)p.nx * p.ny * p.nz; }
bool large_grid(const gs_params &p) { return grid_cells(p) >= 64.0 * 1024 * 1024; }

int default_tile(const gs_params &p)
{
    const int tb = gs::num_tiles(); // tiles tb + 1 .. tb + 5 are the blocked shapes 1..5
    if (grid_cells(p) < 4.0 * 1024 * 1024) return tb + 1;
    if (!large_grid(p)) return p.storage == GS_F64 ? tb + 4 : tb + 2;
    if (p.storage == GS_F32 && p.noise == 0.0) return tb + 5;
    return tb + 2;
}

int default_tblock(const gs_params &p, int tile)
{
    if (tile <= gs::num_tiles()) return 1;
    int T = 2;
    if (large_grid(p) && p.storage == GS_F64) T = 3;
    const int mt = tile_max_tblock(tile, p.storage);
    return T < mt ? T : mt;
}

// z-chunks the autotuner sweeps.
const int k_zchunks[] = {4, 8, 16, 32, 64, 128, 256, 512};

// Default z-chunk: a workgroup of a chunk of zc output planes streams
// zc + 2T planes, and nb workgroups on `slots` resident places (CUs times
// workgroups per CU) take ceil(nb / slots) rounds, so the sweep costs about
// ceil(nb / slots) (zc + 2T) plane times; the partly filled last round costs
// up to a fifth of the throughput at 512^3 with a fixed chunk. Chunks that
// leave fewer than three rounds are slower than this predicts on large grids
// (every CU then starts and drains its workgroups at once), so the cheapest
// chunk with at least three rounds (two below 64 M cells, where longer
// chunks measured faster) is taken (the larger one on ties), else the
// shortest chunk. The single-step kernel keeps chunks of at most 32 planes (longer
// ones measured slower at 1024^3 although the estimate favours them).
// Without the occupancy figures it falls back to fixed chunks.
int default_zc(const gs_params &p, int tile, int tblock)
{
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    const bool tb = is_tb_tile(tile);
    const int occ = tb ? gs::tb_occupancy(p.storage, tblock, tile - gs::num_tiles(), p.noise != 0.0)
                       : gs::step_occupancy(p.storage, tile, p.noise != 0.0);
    const gs::TileShape t = tb ? gs::tb_shape(tile - gs::num_tiles(), tblock) : gs::tile_shape(tile, p.storage);
    if (cus > 0 && occ > 0 && t.tx > 0 && t.ty > 0) {
        const double slots = (double)cus * occ;
        const double tiles = (double)((p.nx + t.tx - 1) / t.tx) * (double)((p.ny + t.ty - 1) / t.ty);
        const int T = tb ? tblock : 1;
        const double min_rounds = large_grid(p) ? 3.0 : 2.0;
        double best = 1e300;
        int bz = 0;
        for (int z : k_zchunks) {
            const int zc = z < p.nz ? z : p.nz;
            const double nb = tiles * (double)((p.nz + zc - 1) / zc);
            if (nb < min_rounds * slots || (!tb && z > 32)) continue;
            const double cost = std::ceil(nb / slots) * (double)(zc + 2 * T);
            if (cost <= best) {
                best = cost;
                bz = zc;
            }
        }
        if (bz == 0) bz = k_zchunks[0] < p.nz ? k_zchunks[0] : p.nz;
        return bz;
    }
    int z = 16;
    if (large_grid(p))
        z = tile <= gs::num_tiles() ? 32 : p.storage == GS_F64 ? 128 : p.storage == GS_F32 ? 32 : 64;
    return p.nz < z ? p.nz : z;
}

gs::StepArgs make_args(const gs_sim *s)
{
    gs::StepArgs a = {};
    a.nx = s->p.nx;
    a.ny = s->p.ny;
    a.nz = s->p.nz;
    a.zc = s->zc;
    a.Du = s->p.Du;
    a.Dv = s->p.Dv;
    a.F = s->p.F;
    a.FK = s->p.F + s->p.k;
    a.dt = s->p.dt;
    a.noise = s->p.noise;
    a.noise_s = std::ldexp(a.noise, -31);
    a.noise_h = std::ldexp(a.noise, -32);
    a.Du_f = (float)a.Du;
    a.Dv_f = (float)a.Dv;
    a.F_f = (float)a.F;
    a.FK_f = (float)a.FK;
    a.dt_f = (float)a.dt;
    a.noise_f = (float)a.noise;
    a.noise_s_f = (float)a.noise_s;
    a.noise_h_f = (float)a.noise_h;
    a.seed = s->p.seed;
    a.t = s->step;
    a.t_dev = nullptr;
    return a;
}

// Enqueues n steps starting from buffer pair *parity on stream st; with
// t_dev set, kernels read the base step index from device memory and take
// their offset from it. Leaves the final parity in *parity.
hipError_t enqueue_steps(gs_sim *s, int64_t n, hipStream_t st, const uint64_t *t_dev, int *parity)
{
    int64_t left = n, off = 0;
    while (left > 0) {
        gs::StepArgs a = make_args(s);
        if (t_dev) {
            a.t = (uint64_t)off;
            a.t_dev = t_dev;
        } else {
            a.t = s->step + (uint64_t)off;
        }
        const int q = *parity;
        hipError_t e;
        int done = 1;
        if (is_tb_tile(s->tile)) {
            done = (int)(left < s->tblock ? left : s->tblock);
            e = gs::launch_tblock(s->p.storage, done, s->tile - gs::num_tiles(), s->buf[q][0], s->buf[q][1],
                                  s->buf[q ^ 1][0], s->buf[q ^ 1][1], a, st);
        } else {
            e = gs::launch_step(s->p.storage, s->tile, s->buf[q][0], s->buf[q][1], s->buf[q ^ 1][0],
                                s->buf[q ^ 1][1], a, st);
        }
        if (e != hipSuccess) return e;
        *parity ^= 1;
        left -= done;
        off += done;
    }
    return hipSuccess;
}

void drop_graph(gs_sim *s)
{
    if (s->graph.exec) (void)hipGraphExecDestroy(s->graph.exec);
    s->graph = GraphCache();
}

} // namespace

extern "C" {

const char *gs_version(void) { return "gs-mi355x 0.1 (gfx950)"; }

const char *gs_last_error(void) { return g_err.c_str(); }

// Workspace layout: diagnostic partials, then (256-byte aligned) the step
// counter read by graph replays.
size_t gs_workspace_bytes(const gs_params *p)
{
    if (validate(p) != GS_OK) return 0;
    return counter_offset() + 256;
}

int32_t gs_num_tiles(void) { return total_tiles(); }

gs_status gs_tile_info(int32_t tile, int32_t storage, int32_t tblock, int32_t *tx, int32_t *ty, int32_t *max_tblock)
{
    if (tile < 1 || tile > total_tiles()) return fail(GS_ERR_INVALID_ARG, "tile %d out of range", tile);
    if (storage_bytes(storage) == 0) return fail(GS_ERR_INVALID_ARG, "unknown storage type %d", storage);
    const int mt = tile_max_tblock(tile, storage);
    if (tblock < 1 || tblock > mt) return fail(GS_ERR_INVALID_ARG, "tblock %d outside [1, %d] for tile %d", tblock, mt, tile);
    gs::TileShape t = is_tb_tile(tile) ? gs::tb_shape(tile - gs::num_tiles(), tblock) : gs::tile_shape(tile, storage);
    if (tx) *tx = t.tx;
    if (ty) *ty = t.ty;
    if (max_tblock) *max_tblock = mt;
    return GS_OK;
}

gs_status gs_init(const gs_params *p, void *u0, void *v0, void *u1, void *v1, void *workspace,
                  void *hip_stream, gs_sim **out)
{
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    gs_status st = validate(p);
    if (st != GS_OK) return st;
    void *b[4] = {u0, v0, u1, v1};
    const char *nm[4] = {"u0", "v0", "u1", "v1"};
    for (int i = 0; i < 4; ++i) {
        if (!b[i]) return fail(GS_ERR_INVALID_ARG, "%s is NULL", nm[i]);
        if (!aligned(b[i], 256)) return fail(GS_ERR_INVALID_ARG, "%s is not 256-byte aligned", nm[i]);
        for (int j = 0; j < i; ++j)
            if (b[i] == b[j]) return fail(GS_ERR_INVALID_ARG, "%s aliases %s", nm[i], nm[j]);
    }
    if (!workspace) return fail(GS_ERR_INVALID_ARG, "workspace is NULL");
    if (!aligned(workspace, 256)) return fail(GS_ERR_INVALID_ARG, "workspace is not 256-byte aligned");

    gs_sim *s = new (std::nothrow) gs_sim();
    if (!s) return fail(GS_ERR_INVALID_ARG, "out of host memory");
    s->magic = k_magic;
    s->p = *p;
    s->buf[0][0] = u0;
    s->buf[0][1] = v0;
    s->buf[1][0] = u1;
    s->buf[1][1] = v1;
    s->parity = 0;
    s->step = p->step0;
    s->ws = workspace;
    s->stream = (hipStream_t)hip_stream;
    s->tile = p->tile ? p->tile : default_tile(*p);
    s->tblock = p->tblock ? p->tblock : default_tblock(*p, s->tile);
    s->zc = p->zchunk ? (p->zchunk < p->nz ? p->zchunk : p->nz) : default_zc(*p, s->tile, s->tblock);
    if (p->tile == 0 && p->tblock == 0 && p->zchunk == 0) {
        // a configuration recorded by gs_tune for this grid class, if any
        TuneVal v;
        const TuneKey key = {TUNE_SINGLE, p->storage, p->nx, p->ny, p->nz, p->noise != 0.0};
        if (tune_cache_lookup(key, &v) && v.tile >= 1 && v.tile <= total_tiles() && v.tblock >= 1 &&
            v.tblock <= tile_max_tblock(v.tile, p->storage) && v.zchunk >= 1) {
            s->tile = v.tile;
            s->tblock = v.tblock;
            s->zc = v.zchunk < p->nz ? v.zchunk : p->nz;
        }
    }
    s->n = (size_t)p->nx * p->ny * p->nz;
    s->graph = GraphCache();
    s->capture_stream = nullptr;

    if (p->init_mode == GS_INIT_CUBE) {
        hipError_t e = gs::launch_init_cube(p->storage, u0, v0, p->nx, p->ny, p->nz, p->cube_side, p->cube_u,
                                            p->cube_v, s->stream);
        if (e != hipSuccess) {
            s->magic = 0;
            delete s;
            return hip_fail(e, "init kernel launch");
        }
    }
    *out = s;
    return GS_OK;
}

gs_status gs_step(gs_sim *s, int64_t n_steps)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    if (n_steps < 0) return fail(GS_ERR_INVALID_ARG, "n_steps = %lld < 0", (long long)n_steps);
    int parity = s->parity;
    hipError_t e = enqueue_steps(s, n_steps, s->stream, nullptr, &parity);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    s->parity = parity;
    s->step += (uint64_t)n_steps;
    return GS_OK;
}

gs_status gs_read(gs_sim *s, double *u_host, double *v_host)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    double *dst[2] = {u_host, v_host};
    for (int f = 0; f < 2; ++f) {
        if (!dst[f]) continue;
        st = read_field(s->buf[s->parity][f], s->p.storage, s->n, dst[f], s->stream, f);
        if (st != GS_OK) return st;
    }
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "gs_read sync");
    return GS_OK;
}

gs_status gs_write(gs_sim *s, const double *u_host, const double *v_host)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    const double *srcs[2] = {u_host, v_host};
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "gs_write sync");
    for (int f = 0; f < 2; ++f) {
        if (!srcs[f]) continue;
        st = write_field(s->buf[s->parity][f], s->p.storage, s->n, srcs[f], s->stream, f);
        if (st != GS_OK) return st;
    }
    return GS_OK;
}

gs_status gs_current(gs_sim *s, void **u_dev, void **v_dev, uint64_t *step)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    if (u_dev) *u_dev = s->buf[s->parity][0];
    if (v_dev) *v_dev = s->buf[s->parity][1];
    if (step) *step = s->step;
    return GS_OK;
}

gs_status gs_diagnostics(gs_sim *s, gs_diag *out)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    return diagnostics(s->p.storage, s->buf[s->parity][0], s->buf[s->parity][1], s->n, s->ws, s->stream, out);
}

gs_status gs_sync(gs_sim *s)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "gs_sync");
    return GS_OK;
}

gs_status gs_destroy(gs_sim *s)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    hipError_t e = hipStreamSynchronize(s->stream);
    drop_graph(s);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    s->magic = 0;
    delete s;
    if (e != hipSuccess) return hip_fail(e, "gs_destroy sync");
    return GS_OK;
}

gs_status gs_set_config(gs_sim *s, int32_t tile, int32_t tblock, int32_t zchunk)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    if (tile < 1 || tile > total_tiles()) return fail(GS_ERR_INVALID_ARG, "tile %d out of range", tile);
    const int mt = tile_max_tblock(tile, s->p.storage);
    if (tblock < 1 || tblock > mt) return fail(GS_ERR_INVALID_ARG, "tblock %d outside [1, %d] for tile %d", tblock, mt, tile);
    if (zchunk < 1) return fail(GS_ERR_INVALID_ARG, "zchunk %d < 1", zchunk);
    s->tile = tile;
    s->tblock = tblock;
    s->zc = zchunk < s->p.nz ? zchunk : s->p.nz;
    return GS_OK;
}

gs_status gs_get_config(gs_sim *s, int32_t *tile, int32_t *tblock, int32_t *zchunk)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    if (tile) *tile = s->tile;
    if (tblock) *tblock = s->tblock;
    if (zchunk) *zchunk = s->zc;
    return GS_OK;
}

gs_status gs_tune(gs_sim *s, int32_t reps, gs_tune_entry *table, int32_t capacity, int32_t *n_entries)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    if (reps < 1) return fail(GS_ERR_INVALID_ARG, "reps %d < 1", reps);
    if (capacity < 0 || (capacity > 0 && !table)) return fail(GS_ERR_INVALID_ARG, "bad table/capacity");
    const int *zcs = k_zchunks;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "gs_tune events");
    }
    const int save_tile = s->tile, save_tb = s->tblock, save_zc = s->zc;
    double best = 1e300;
    int bt = save_tile, bT = save_tb, bz = save_zc;
    int count = 0;
    for (int tile = 1; tile <= total_tiles() && e == hipSuccess; ++tile) {
        for (int T = 1; T <= tile_max_tblock(tile, s->p.storage) && e == hipSuccess; ++T) {
            int last_zc = -1;
            for (int zi = 0; zi < (int)(sizeof k_zchunks / sizeof k_zchunks[0]) && e == hipSuccess; ++zi) {
                const int zc = zcs[zi] < s->p.nz ? zcs[zi] : s->p.nz;
                if (zc == last_zc) continue;
                last_zc = zc;
                s->tile = tile;
                s->tblock = T;
                s->zc = zc;
                // Reads the current pair and writes the other one; the state
                // and the step index are left unchanged.
                int par = s->parity;
                e = enqueue_steps(s, T, s->stream, nullptr, &par); // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
                for (int r = 0; r < reps && e == hipSuccess; ++r) {
                    par = s->parity;
                    e = enqueue_steps(s, T, s->stream, nullptr, &par);
                }
                if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) break;
                const double per_step = (double)ms / (reps * T);
                if (count < capacity) {
                    table[count].tile = tile;
                    table[count].tblock = T;
                    table[count].zchunk = zc;
                    table[count].reserved = 0;
                    table[count].ms_per_step = per_step;
                }
                ++count;
                if (per_step < best) {
                    best = per_step;
                    bt = tile;
                    bT = T;
                    bz = zc;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        s->tile = save_tile;
        s->tblock = save_tb;
        s->zc = save_zc;
        return hip_fail(e, "gs_tune");
    }
    s->tile = bt;
    s->tblock = bT;
    s->zc = bz;
    if (n_entries) *n_entries = count;
    const TuneKey key = {TUNE_SINGLE, s->p.storage, s->p.nx, s->p.ny, s->p.nz, s->p.noise != 0.0};
    if (!tune_cache_store(key, TuneVal{bt, bT, bz, best}))
        return fail(GS_ERR_INVALID_ARG, "tuned, but the table %s could not be written", tune_cache_path());
    return GS_OK;
}

gs_status gs_step_graph(gs_sim *s, int64_t n_steps)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    if (n_steps < 0) return fail(GS_ERR_INVALID_ARG, "n_steps = %lld < 0", (long long)n_steps);
    if (n_steps == 0) return GS_OK;
    GraphCache &g = s->graph;
    uint64_t *t_dev = (uint64_t *)((char *)s->ws + counter_offset());
    hipError_t e = hipSuccess;
    int end_parity = s->parity;
    if (!(g.exec && g.n == n_steps && g.parity == s->parity && g.tile == s->tile && g.tblock == s->tblock &&
          g.zc == s->zc)) {
        drop_graph(s);
        if (!s->capture_stream) {
            e = hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "capture stream");
        }
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "begin capture");
        int par = s->parity;
        hipError_t le = enqueue_steps(s, n_steps, s->capture_stream, t_dev, &par);
        e = hipStreamEndCapture(s->capture_stream, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le, "capture launches");
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g = GraphCache();
            return hip_fail(e, "graph instantiate");
        }
        g.n = n_steps;
        g.parity = s->parity;
        g.tile = s->tile;
        g.tblock = s->tblock;
        g.zc = s->zc;
    }
    // The captured kernels take their step index from the device counter.
    e = gs::launch_set_u64(t_dev, s->step, s->stream);
    if (e != hipSuccess) return hip_fail(e, "step counter");
    e = hipGraphLaunch(g.exec, s->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    const int64_t launches = is_tb_tile(s->tile) ? (n_steps + s->tblock - 1) / s->tblock : n_steps;
    if (launches & 1) end_parity ^= 1;
    s->parity = end_parity;
    s->step += (uint64_t)n_steps;
    return GS_OK;
}

gs_status gs_set_step(gs_sim *s, uint64_t step)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    s->step = step;
    return GS_OK;
}

gs_status gs_fill_cube(gs_sim *s, int32_t x0, int32_t y0, int32_t z0, int32_t side, double cu, double cv)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    int mn = s->p.nx < s->p.ny ? s->p.nx : s->p.ny;
    mn = mn < s->p.nz ? mn : s->p.nz;
    if (side < 1 || side > mn) return fail(GS_ERR_INVALID_ARG, "side %d outside [1, %d]", side, mn);
    if (x0 < 0 || y0 < 0 || z0 < 0 || x0 >= s->p.nx || y0 >= s->p.ny || z0 >= s->p.nz)
        return fail(GS_ERR_INVALID_ARG, "corner outside the grid");
    if (!std::isfinite(cu) || !std::isfinite(cv)) return fail(GS_ERR_INVALID_ARG, "cube values must be finite");
    hipError_t e = gs::launch_init_box(s->p.storage, s->buf[s->parity][0], s->buf[s->parity][1], s->p.nx, s->p.ny,
                                       s->p.nz, x0, y0, z0, side, cu, cv, s->stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "fill kernel launch");
}

size_t gs_sqdiff_workspace_bytes(void) { return (size_t)gs::sqdiff_blocks() * sizeof(double); }

gs_status gs_sqdiff(const void *a, const void *b, size_t n, int32_t storage, void *workspace, void *hip_stream,
                    double *out)
{
    if (!a || !b || !workspace || !out) return fail(GS_ERR_INVALID_ARG, "NULL pointer");
    if (storage_bytes(storage) == 0) return fail(GS_ERR_INVALID_ARG, "unknown storage type %d", storage);
    if (!aligned(workspace, 8)) return fail(GS_ERR_INVALID_ARG, "workspace must be 8-byte aligned");
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<double> part(gs::sqdiff_blocks());
    hipError_t e = gs::launch_sqdiff(storage, a, b, n, (double *)workspace, st);
    if (e == hipSuccess) e = hipMemcpyAsync(part.data(), workspace, part.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "gs_sqdiff");
    double sum = 0.0;
    for (double x : part) sum += x;
    *out = sum;
    return GS_OK;
}

gs_status gs_laplacian7(const double *f, double *out, int32_t nx, int32_t ny, int32_t nz, void *hip_stream)
{
    if (!f || !out) return fail(GS_ERR_INVALID_ARG, "NULL pointer");
    if (!aligned(f, 256) || !aligned(out, 256)) return fail(GS_ERR_INVALID_ARG, "pointers must be 256-byte aligned");
    if (f == out) return fail(GS_ERR_INVALID_ARG, "in-place Laplacian is not supported");
    if (nx < 4 || ny < 4 || nz < 4 || nx % 8 != 0)
        return fail(GS_ERR_UNSUPPORTED, "grid %dx%dx%d unsupported (>= 4 each, nx %% 8 == 0)", nx, ny, nz);
    hipError_t e = gs::launch_laplacian7(f, out, nx, ny, nz, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "laplacian launch");
    return GS_OK;
}

gs_status gs_copy(const void *src, void *dst, size_t bytes, void *hip_stream)
{
    if (!src || !dst) return fail(GS_ERR_INVALID_ARG, "NULL pointer");
    if (bytes % 16 != 0) return fail(GS_ERR_INVALID_ARG, "bytes must be a multiple of 16");
    if (!aligned(src, 16) || !aligned(dst, 16)) return fail(GS_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    if (bytes == 0) return GS_OK;
    hipError_t e = gs::launch_copy(src, dst, bytes, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return GS_OK;
}

} // extern "C"
