// C ABI of libgs (declared in include/gs.h): validation, handle state,
// ping-pong parity, host <-> device conversion, launch selection.
#include "../../include/gs.h"
#include "gs_launch.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace {

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
    }
    return 0;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

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
    if (p->tile < 0 || p->tile > gs::num_tiles())
        return fail(GS_ERR_INVALID_ARG, "tile %d outside [0, %d]", p->tile, gs::num_tiles());
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

} // namespace

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
};

namespace {

gs_status check(gs_sim *s)
{
    if (!s || s->magic != k_magic) return fail(GS_ERR_STATE, "invalid or destroyed handle");
    return GS_OK;
}

// Library choice of tile shape and z-chunk (measured on MI355X; see the
// benchmark's tile sweep).
int default_tile(const gs_params &p)
{
    (void)p;
    return 1;
}

int default_zc(const gs_params &p)
{
    const int z = 64;
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
    a.Du_f = (float)a.Du;
    a.Dv_f = (float)a.Dv;
    a.F_f = (float)a.F;
    a.FK_f = (float)a.FK;
    a.dt_f = (float)a.dt;
    a.noise_f = (float)a.noise;
    a.seed = s->p.seed;
    a.t = s->step;
    return a;
}

} // namespace

extern "C" {

const char *gs_version(void) { return "gs-mi355x 0.1 (gfx950)"; }

const char *gs_last_error(void) { return g_err.c_str(); }

size_t gs_workspace_bytes(const gs_params *p)
{
    if (validate(p) != GS_OK) return 0;
    return gs::diag_workspace_bytes();
}

int32_t gs_num_tiles(void) { return gs::num_tiles(); }

gs_status gs_tile_info(int32_t tile, int32_t storage, int32_t *tx, int32_t *ty, int32_t *zc)
{
    if (tile < 1 || tile > gs::num_tiles()) return fail(GS_ERR_INVALID_ARG, "tile %d out of range", tile);
    if (storage_bytes(storage) == 0) return fail(GS_ERR_INVALID_ARG, "unknown storage type %d", storage);
    gs::TileShape t = gs::tile_shape(tile, storage);
    if (tx) *tx = t.tx;
    if (ty) *ty = t.ty;
    if (zc) *zc = 64;
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
    s->zc = default_zc(*p);
    s->tblock = p->tblock ? p->tblock : 1;
    s->n = (size_t)p->nx * p->ny * p->nz;

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
    for (int64_t i = 0; i < n_steps; ++i) {
        gs::StepArgs a = make_args(s);
        const int q = s->parity;
        hipError_t e = gs::launch_step(s->p.storage, s->tile, s->buf[q][0], s->buf[q][1], s->buf[q ^ 1][0],
                                       s->buf[q ^ 1][1], a, s->stream);
        if (e != hipSuccess) return hip_fail(e, "step kernel launch");
        s->parity ^= 1;
        s->step += 1;
    }
    return GS_OK;
}

gs_status gs_read(gs_sim *s, double *u_host, double *v_host)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    double *dst[2] = {u_host, v_host};
    const size_t es = storage_bytes(s->p.storage);
    std::vector<unsigned char> stage;
    for (int f = 0; f < 2; ++f) {
        if (!dst[f]) continue;
        const void *src = s->buf[s->parity][f];
        if (s->p.storage == GS_F64) {
            hipError_t e = hipMemcpyAsync(dst[f], src, s->n * 8, hipMemcpyDeviceToHost, s->stream);
            if (e != hipSuccess) return hip_fail(e, "gs_read copy");
            e = hipStreamSynchronize(s->stream);
            if (e != hipSuccess) return hip_fail(e, "gs_read sync");
            continue;
        }
        stage.resize(s->n * es);
        hipError_t e = hipMemcpyAsync(stage.data(), src, s->n * es, hipMemcpyDeviceToHost, s->stream);
        if (e != hipSuccess) return hip_fail(e, "gs_read copy");
        e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(e, "gs_read sync");
        double *d = dst[f];
        if (s->p.storage == GS_F32) {
            const float *x = (const float *)stage.data();
            for (size_t i = 0; i < s->n; ++i) d[i] = x[i];
        } else if (s->p.storage == GS_BF16) {
            const uint16_t *x = (const uint16_t *)stage.data();
            for (size_t i = 0; i < s->n; ++i) d[i] = host_from_bf16(x[i]);
        } else {
            const _Float16 *x = (const _Float16 *)stage.data();
            for (size_t i = 0; i < s->n; ++i) d[i] = (double)(float)x[i];
        }
    }
    if (!u_host && !v_host) {
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(e, "gs_read sync");
    }
    return GS_OK;
}

gs_status gs_write(gs_sim *s, const double *u_host, const double *v_host)
{
    gs_status st = check(s);
    if (st != GS_OK) return st;
    const double *srcs[2] = {u_host, v_host};
    const size_t es = storage_bytes(s->p.storage);
    std::vector<unsigned char> stage;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "gs_write sync");
    for (int f = 0; f < 2; ++f) {
        if (!srcs[f]) continue;
        const double *x = srcs[f];
        const void *host = x;
        if (s->p.storage != GS_F64) {
            stage.resize(s->n * es);
            if (s->p.storage == GS_F32) {
                float *d = (float *)stage.data();
                for (size_t i = 0; i < s->n; ++i) d[i] = (float)x[i];
            } else if (s->p.storage == GS_BF16) {
                uint16_t *d = (uint16_t *)stage.data();
                for (size_t i = 0; i < s->n; ++i) d[i] = host_bf16((float)x[i]);
            } else {
                _Float16 *d = (_Float16 *)stage.data();
                for (size_t i = 0; i < s->n; ++i) d[i] = (_Float16)(float)x[i];
            }
            host = stage.data();
        }
        e = hipMemcpyAsync(s->buf[s->parity][f], host, s->n * es, hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return hip_fail(e, "gs_write copy");
        e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(e, "gs_write sync");
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
    hipError_t e = gs::launch_diagnostics(s->p.storage, s->buf[s->parity][0], s->buf[s->parity][1], s->n, s->ws,
                                          s->stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics launch");
    double r[9];
    e = hipMemcpyAsync(r, (char *)s->ws + gs::diag_result_offset(), sizeof r, hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics copy");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics sync");
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
    s->magic = 0;
    delete s;
    if (e != hipSuccess) return hip_fail(e, "gs_destroy sync");
    return GS_OK;
}

gs_status gs_laplacian7(const double *f, double *out, int32_t nx, int32_t ny, int32_t nz, void *hip_stream)
{
    if (!f || !out) return fail(GS_ERR_INVALID_ARG, "NULL pointer");
    if (!aligned(f, 256) || !aligned(out, 256)) return fail(GS_ERR_INVALID_ARG, "pointers must be 256-byte aligned");
    if (f == out) return fail(GS_ERR_INVALID_ARG, "in-place Laplacian is not supported");
    if (nx < 4 || ny < 4 || nz < 4 || nx % 8 != 0)
        return fail(GS_ERR_UNSUPPORTED, "grid %dx%dx%d unsupported (>= 4 each, nx % 8 == 0)", nx, ny, nz);
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
