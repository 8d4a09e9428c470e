// Batched C ABI: many independent Gray-Scott simulations (own grid size, F
// and k; shared Du, Dv, dt, noise) advanced together by persistent launches
// of the temporally blocked kernel.
//
// Each simulation has a launch configuration (tile shape, fused steps T,
// z-chunk); simulations with the same (shape, T) form a group that one
// persistent launch per T steps advances. Work items (one tile x z-chunk of
// one simulation) are listed per group, longest first, and every workgroup
// of the persistent grid walks the list with a stride of the grid size.
#include "../../include/gs.h"
#include "gs_internal.hpp"
#include "gs_launch.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

using namespace gsapi;

namespace {

const uint32_t k_batch_magic = 0x47534254u; // "GSBT"
const int k_min_batch_zc = 8;

struct BSim {
    int nx, ny, nz;
    double F, k;
    void *buf[2][2];
    int parity;  // pair holding the current state
    int group;   // index into gs_batch::groups after the last rebuild
    int shape, T, zc;
    size_t n;
};

// A group advances its simulations with sweeps of depth T; a call whose step
// count is not a multiple of T ends with one sweep of the remaining depth d,
// whose output tiles differ, so the group keeps one work list per depth.
struct BGroup {
    int shape, T;
    int parity;
    int off[GS_MAX_TBLOCK + 1], cnt[GS_MAX_TBLOCK + 1], grid[GS_MAX_TBLOCK + 1];
};

struct BGraph {
    hipGraphExec_t exec = nullptr;
    int64_t n = -1;
    int version = -1;
    std::vector<int> parities;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int tiles_along(int n, int t) { return (n + t - 1) / t; }

size_t items_for(int nx, int ny, int nz, int shape, int T, int zc)
{
    const gs::TileShape ts = gs::tb_shape(shape, T);
    return (size_t)tiles_along(nx, ts.tx) * tiles_along(ny, ts.ty) * tiles_along(nz, zc);
}

// Upper bound of the items of one simulation over every allowed configuration
// (smallest tile: 64 x 6 cells at T = 4; smallest chunk k_min_batch_zc).
size_t max_items(int nx, int ny, int nz) { return items_for(nx, ny, nz, 1, 4, k_min_batch_zc); }

} // namespace

struct gs_batch {
    uint32_t magic;
    gs_params base;
    std::vector<BSim> sims;
    std::vector<BGroup> groups;
    std::vector<gs::SimDesc> h_desc;
    std::vector<gs::WorkItem> h_items;
    gs::SimDesc *d_desc;
    gs::WorkItem *d_items;
    size_t item_capacity;  // items of the group lists
    size_t scratch_items;  // start of the tuning scratch list (after the group lists)
    void *ws;
    hipStream_t stream;
    hipStream_t capture_stream;
    uint64_t step;
    int cus;
    int version;
    bool dirty;
    BGraph graph;
};

namespace {

gs_status bcheck(gs_batch *b)
{
    if (!b || b->magic != k_batch_magic) return fail(GS_ERR_STATE, "invalid or destroyed batch handle");
    return GS_OK;
}

gs_status sim_index(gs_batch *b, int32_t i)
{
    if (i < 0 || (size_t)i >= b->sims.size()) return fail(GS_ERR_INVALID_ARG, "simulation index %d out of range", i);
    return GS_OK;
}

size_t desc_offset() { return align256(counter_offset() + 256); }
size_t items_offset(int32_t n_sims) { return align256(desc_offset() + (size_t)n_sims * sizeof(gs::SimDesc)); }

gs::StepArgs shared_coef(const gs_batch *b)
{
    gs::StepArgs a = {};
    a.Du = b->base.Du;
    a.Dv = b->base.Dv;
    a.dt = b->base.dt;
    a.noise = b->base.noise;
    a.noise_s = std::ldexp(a.noise, -31);
    a.noise_h = std::ldexp(a.noise, -32);
    a.Du_f = (float)a.Du;
    a.Dv_f = (float)a.Dv;
    a.dt_f = (float)a.dt;
    a.noise_f = (float)a.noise;
    a.noise_s_f = (float)a.noise_s;
    a.noise_h_f = (float)a.noise_h;
    return a;
}

void drop_graph(gs_batch *b)
{
    if (b->graph.exec) (void)hipGraphExecDestroy(b->graph.exec);
    b->graph = BGraph();
}

// Builds groups, descriptors and work items for the current per-simulation
// configurations and uploads them (synchronising). Simulations whose current
// state sits in their second buffer pair get their pairs swapped, so that
// every group starts with its state in pair 0.
gs_status rebuild(gs_batch *b)
{
    for (BSim &s : b->sims) {
        if (s.parity == 1) {
            std::swap(s.buf[0][0], s.buf[1][0]);
            std::swap(s.buf[0][1], s.buf[1][1]);
            s.parity = 0;
        }
    }
    b->groups.clear();
    b->h_items.clear();
    b->h_desc.resize(b->sims.size());
    for (size_t i = 0; i < b->sims.size(); ++i) {
        const BSim &s = b->sims[i];
        gs::SimDesc &d = b->h_desc[i];
        std::memcpy(d.buf, s.buf, sizeof d.buf);
        d.nx = s.nx;
        d.ny = s.ny;
        d.nz = s.nz;
        d.zc = s.zc;
        d.F = s.F;
        d.FK = s.F + s.k;
        d.F_f = (float)d.F;
        d.FK_f = (float)d.FK;
        d.seed = b->base.seed + (uint64_t)i;
    }
    for (int shape = 1; shape <= gs::num_tb_shapes(); ++shape) {
        for (int T = 1; T <= GS_MAX_TBLOCK; ++T) {
            bool any = false;
            for (const BSim &s : b->sims) any = any || (s.shape == shape && s.T == T);
            if (!any) continue;
            BGroup g;
            g.shape = shape;
            g.T = T;
            g.parity = 0;
            for (int d = 0; d <= GS_MAX_TBLOCK; ++d) g.off[d] = g.cnt[d] = g.grid[d] = 0;
            for (int d = 1; d <= T; ++d) {
                struct Tmp {
                    gs::WorkItem w;
                    int len;
                };
                std::vector<Tmp> items;
                const gs::TileShape ts = gs::tb_shape(shape, d);
                for (size_t i = 0; i < b->sims.size(); ++i) {
                    const BSim &s = b->sims[i];
                    if (s.shape != shape || s.T != T) continue;
                    const int ntx = tiles_along(s.nx, ts.tx), nty = tiles_along(s.ny, ts.ty);
                    const int nzc = tiles_along(s.nz, s.zc);
                    for (int bz = 0; bz < nzc; ++bz) {
                        const int len = std::min(s.zc, s.nz - bz * s.zc) + 2 * d - 2;
                        for (int by = 0; by < nty; ++by)
                            for (int bx = 0; bx < ntx; ++bx)
                                items.push_back(Tmp{gs::WorkItem{(int)i, bx, by, bz}, len});
                    }
                }
                // Longest chunks first; ties keep simulation-major order, so a
                // simulation's tiles run side by side (shared halos in L2).
                std::stable_sort(items.begin(), items.end(),
                                 [](const Tmp &x, const Tmp &y) { return x.len > y.len; });
                g.off[d] = (int)b->h_items.size();
                g.cnt[d] = (int)items.size();
                const int occ = gs::tb_batch_occupancy(b->base.storage, d, shape);
                g.grid[d] = std::max(1, std::min(g.cnt[d], b->cus * occ));
                for (const Tmp &t : items) b->h_items.push_back(t.w);
            }
            for (BSim &s : b->sims)
                if (s.shape == shape && s.T == T) s.group = (int)b->groups.size();
            b->groups.push_back(g);
        }
    }
    if (b->h_items.size() > b->item_capacity)
        return fail(GS_ERR_INVALID_ARG, "work list of %zu items exceeds the workspace capacity %zu", b->h_items.size(),
                    b->item_capacity);
    hipError_t e = hipMemcpyAsync(b->d_desc, b->h_desc.data(), b->h_desc.size() * sizeof(gs::SimDesc),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !b->h_items.empty())
        e = hipMemcpyAsync(b->d_items, b->h_items.data(), b->h_items.size() * sizeof(gs::WorkItem),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    drop_graph(b);
    b->version += 1;
    b->dirty = false;
    return GS_OK;
}

// Enqueues n steps of every group on stream st: n / T sweeps of depth T and,
// if n % T != 0, one sweep of the remaining depth. Group parities advance in
// `par` (one per group). With t_dev set the kernels take the base step index
// from device memory and their offset from it.
hipError_t enqueue_batch(gs_batch *b, int64_t n, hipStream_t st, const uint64_t *t_dev, std::vector<int> &par)
{
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const BGroup &g = b->groups[gi];
        int64_t left = n;
        uint64_t off = 0;
        while (left > 0) {
            const int d = (int)std::min<int64_t>(left, g.T);
            gs::BatchArgs a = {};
            a.coef = shared_coef(b);
            a.sims = b->d_desc;
            a.items = b->d_items + g.off[d];
            a.n_items = g.cnt[d];
            a.parity = par[gi];
            a.t = t_dev ? off : b->step + off;
            a.t_dev = t_dev;
            hipError_t e = gs::launch_tblock_batch(b->base.storage, d, g.shape, a, g.grid[d], st);
            if (e != hipSuccess) return e;
            par[gi] ^= 1;
            left -= d;
            off += (uint64_t)d;
        }
    }
    return hipSuccess;
}

void commit_parities(gs_batch *b, const std::vector<int> &par)
{
    for (size_t i = 0; i < par.size(); ++i) b->groups[i].parity = par[i];
    for (BSim &s : b->sims) s.parity = b->groups[s.group].parity;
}

} // namespace

extern "C" {

size_t gs_batch_arena_bytes(int32_t storage, int32_t n_sims, const int32_t *nx, const int32_t *ny, const int32_t *nz)
{
    const size_t es = storage_bytes(storage);
    if (es == 0 || n_sims < 1 || !nx || !ny || !nz) return 0;
    size_t total = 0;
    for (int32_t i = 0; i < n_sims; ++i) {
        if (nx[i] < 4 || ny[i] < 4 || nz[i] < 4) return 0;
        total += 4 * align256((size_t)nx[i] * ny[i] * nz[i] * es);
    }
    return total;
}

size_t gs_batch_workspace_bytes(int32_t n_sims, const int32_t *nx, const int32_t *ny, const int32_t *nz)
{
    if (n_sims < 1 || !nx || !ny || !nz) return 0;
    size_t items = 0;
    for (int32_t i = 0; i < n_sims; ++i) {
        if (nx[i] < 4 || ny[i] < 4 || nz[i] < 4) return 0;
        items += (GS_MAX_TBLOCK + 1) * max_items(nx[i], ny[i], nz[i]);
    }
    return items_offset(n_sims) + items * sizeof(gs::WorkItem);
}

gs_status gs_batch_init(const gs_params *base, int32_t n_sims, const int32_t *nx, const int32_t *ny,
                        const int32_t *nz, const double *F, const double *k, void *arena, size_t arena_bytes,
                        void *workspace, size_t workspace_bytes, void *hip_stream, gs_batch **out)
{
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!base) return fail(GS_ERR_INVALID_ARG, "base params are NULL");
    if (n_sims < 1) return fail(GS_ERR_INVALID_ARG, "n_sims = %d < 1", n_sims);
    if (!nx || !ny || !nz || !F || !k) return fail(GS_ERR_INVALID_ARG, "NULL per-simulation array");
    for (int32_t i = 0; i < n_sims; ++i) {
        gs_params p = *base;
        p.nx = nx[i];
        p.ny = ny[i];
        p.nz = nz[i];
        p.F = F[i];
        p.k = k[i];
        p.tile = 0;
        p.tblock = 0;
        p.zchunk = 0;
        gs_status st = validate(&p);
        if (st != GS_OK) return fail(st, "simulation %d: %s", i, gs_last_error());
    }
    if (base->tile != 0 && base->tile <= gs::num_tiles())
        return fail(GS_ERR_INVALID_ARG, "batched sweeps use the temporally blocked tiles (%d..%d)", gs::num_tiles() + 1,
                    gs::num_tiles() + gs::num_tb_shapes());
    if (base->tile > gs::num_tiles() + gs::num_tb_shapes() || base->tile < 0)
        return fail(GS_ERR_INVALID_ARG, "tile %d out of range", base->tile);
    if (base->tblock < 0 || base->tblock > GS_MAX_TBLOCK) return fail(GS_ERR_INVALID_ARG, "tblock out of range");
    if (base->storage == GS_BF16C)
        return fail(GS_ERR_UNSUPPORTED, "batched sweeps do not take the complemented BF16 storage");
    if (gs::tb_batch_max_T(base->tile ? base->tile - gs::num_tiles() : 2, base->storage) < 1)
        return fail(GS_ERR_UNSUPPORTED, "tile %d is not available to batched sweeps of this storage type", base->tile);
    if (base->tblock > gs::tb_batch_max_T(base->tile ? base->tile - gs::num_tiles() : 2, base->storage))
        return fail(GS_ERR_INVALID_ARG, "tile %d fuses at most %d steps for this storage type", base->tile,
                    gs::tb_batch_max_T(base->tile ? base->tile - gs::num_tiles() : 2, base->storage));
    if (base->zchunk != 0 && base->zchunk < k_min_batch_zc)
        return fail(GS_ERR_INVALID_ARG, "batched zchunk must be 0 or >= %d", k_min_batch_zc);
    const size_t need_arena = gs_batch_arena_bytes(base->storage, n_sims, nx, ny, nz);
    const size_t need_ws = gs_batch_workspace_bytes(n_sims, nx, ny, nz);
    if (!arena || !aligned(arena, 256)) return fail(GS_ERR_INVALID_ARG, "arena must be a 256-byte aligned device pointer");
    if (arena_bytes < need_arena) return fail(GS_ERR_INVALID_ARG, "arena holds %zu bytes, needs %zu", arena_bytes, need_arena);
    if (!workspace || !aligned(workspace, 256)) return fail(GS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < need_ws)
        return fail(GS_ERR_INVALID_ARG, "workspace holds %zu bytes, needs %zu", workspace_bytes, need_ws);

    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");

    gs_batch *b = new (std::nothrow) gs_batch();
    if (!b) return fail(GS_ERR_INVALID_ARG, "out of host memory");
    b->magic = k_batch_magic;
    b->base = *base;
    b->ws = workspace;
    b->stream = (hipStream_t)hip_stream;
    b->capture_stream = nullptr;
    b->step = base->step0;
    b->cus = cus > 0 ? cus : 1;
    b->version = 0;
    b->d_desc = (gs::SimDesc *)((char *)workspace + desc_offset());
    b->d_items = (gs::WorkItem *)((char *)workspace + items_offset(n_sims));
    {
        size_t bound = 0;
        for (int32_t i = 0; i < n_sims; ++i) bound += max_items(nx[i], ny[i], nz[i]);
        b->item_capacity = GS_MAX_TBLOCK * bound;
        b->scratch_items = b->item_capacity;
    }
    const size_t es = storage_bytes(base->storage);
    const int shape = base->tile ? base->tile - gs::num_tiles() : 2;
    const int T = base->tblock ? base->tblock
                               : std::min(gs::tb_batch_max_T(shape, base->storage),
                                          (base->storage == GS_F64 || base->storage == GS_F32) ? 3 : 1);
    char *p = (char *)arena;
    for (int32_t i = 0; i < n_sims; ++i) {
        BSim s;
        s.nx = nx[i];
        s.ny = ny[i];
        s.nz = nz[i];
        s.F = F[i];
        s.k = k[i];
        s.n = (size_t)s.nx * s.ny * s.nz;
        const size_t fb = align256(s.n * es);
        s.buf[0][0] = p;
        s.buf[0][1] = p + fb;
        s.buf[1][0] = p + 2 * fb;
        s.buf[1][1] = p + 3 * fb;
        p += 4 * fb;
        s.parity = 0;
        s.group = 0;
        s.shape = shape;
        s.T = T;
        const int zc = base->zchunk ? base->zchunk : 32;
        s.zc = std::min(zc, s.nz);
        if (base->tile == 0 && base->tblock == 0 && base->zchunk == 0) {
            // a configuration recorded by gs_batch_tune for this grid class, if any
            TuneVal v;
            const TuneKey key = {TUNE_BATCH, base->storage, s.nx, s.ny, s.nz, base->noise != 0.0};
            if (tune_cache_lookup(key, &v) && v.tile > gs::num_tiles() &&
                v.tile <= gs::num_tiles() + gs::num_tb_shapes() && v.tblock >= 1 &&
                v.tblock <= gs::tb_batch_max_T(v.tile - gs::num_tiles(), base->storage) && v.zchunk >= k_min_batch_zc) {
                s.shape = v.tile - gs::num_tiles();
                s.T = v.tblock;
                s.zc = std::min(v.zchunk, s.nz);
            }
        }
        b->sims.push_back(s);
        if (base->init_mode == GS_INIT_CUBE) {
            e = gs::launch_init_cube(base->storage, s.buf[0][0], s.buf[0][1], s.nx, s.ny, s.nz, base->cube_side,
                                     base->cube_u, base->cube_v, b->stream);
            if (e != hipSuccess) {
                b->magic = 0;
                delete b;
                return hip_fail(e, "init kernel launch");
            }
        }
    }
    gs_status st = rebuild(b);
    if (st != GS_OK) {
        b->magic = 0;
        delete b;
        return st;
    }
    *out = b;
    return GS_OK;
}

int32_t gs_batch_max_tblock(int32_t tile, int32_t storage)
{
    if (tile <= gs::num_tiles() || tile > gs::num_tiles() + gs::num_tb_shapes()) return 0;
    if (storage < GS_F64 || storage > GS_F16) return 0;
    return gs::tb_batch_max_T(tile - gs::num_tiles(), storage);
}

gs_status gs_batch_set_config(gs_batch *b, int32_t sim, int32_t tile, int32_t tblock, int32_t zchunk)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if (sim != -1 && (st = sim_index(b, sim)) != GS_OK) return st;
    if (tile <= gs::num_tiles() || tile > gs::num_tiles() + gs::num_tb_shapes())
        return fail(GS_ERR_INVALID_ARG, "batched tile must be in %d..%d", gs::num_tiles() + 1,
                    gs::num_tiles() + gs::num_tb_shapes());
    const int mt = gs::tb_batch_max_T(tile - gs::num_tiles(), b->base.storage);
    if (tblock < 1 || tblock > mt) return fail(GS_ERR_INVALID_ARG, "tblock %d outside [1, %d] for tile %d", tblock, mt, tile);
    if (zchunk < k_min_batch_zc) return fail(GS_ERR_INVALID_ARG, "zchunk %d < %d", zchunk, k_min_batch_zc);
    for (size_t i = 0; i < b->sims.size(); ++i) {
        if (sim != -1 && (int32_t)i != sim) continue;
        BSim &s = b->sims[i];
        s.shape = tile - gs::num_tiles();
        s.T = tblock;
        s.zc = std::min(zchunk, s.nz);
    }
    b->dirty = true;
    return GS_OK;
}

gs_status gs_batch_get_config(gs_batch *b, int32_t sim, int32_t *tile, int32_t *tblock, int32_t *zchunk)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if ((st = sim_index(b, sim)) != GS_OK) return st;
    const BSim &s = b->sims[sim];
    if (tile) *tile = s.shape + gs::num_tiles();
    if (tblock) *tblock = s.T;
    if (zchunk) *zchunk = s.zc;
    return GS_OK;
}

gs_status gs_batch_step(gs_batch *b, int64_t n_steps)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if (n_steps < 0) return fail(GS_ERR_INVALID_ARG, "n_steps < 0");
    if (b->dirty && (st = rebuild(b)) != GS_OK) return st;
    std::vector<int> par(b->groups.size());
    for (size_t i = 0; i < par.size(); ++i) par[i] = b->groups[i].parity;
    hipError_t e = enqueue_batch(b, n_steps, b->stream, nullptr, par);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    commit_parities(b, par);
    b->step += (uint64_t)n_steps;
    return GS_OK;
}

gs_status gs_batch_step_graph(gs_batch *b, int64_t n_steps)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if (n_steps < 0) return fail(GS_ERR_INVALID_ARG, "n_steps < 0");
    if (n_steps == 0) return GS_OK;
    if (b->dirty && (st = rebuild(b)) != GS_OK) return st;
    std::vector<int> par(b->groups.size());
    for (size_t i = 0; i < par.size(); ++i) par[i] = b->groups[i].parity;
    uint64_t *t_dev = (uint64_t *)((char *)b->ws + counter_offset());
    BGraph &g = b->graph;
    hipError_t e = hipSuccess;
    if (!(g.exec && g.n == n_steps && g.version == b->version && g.parities == par)) {
        drop_graph(b);
        if (!b->capture_stream) {
            e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "capture stream");
        }
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "begin capture");
        std::vector<int> cpar = par;
        hipError_t le = enqueue_batch(b, n_steps, b->capture_stream, t_dev, cpar);
        e = hipStreamEndCapture(b->capture_stream, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le, "capture launches");
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g = BGraph();
            return hip_fail(e, "graph instantiate");
        }
        g.n = n_steps;
        g.version = b->version;
        g.parities = par;
    }
    e = gs::launch_set_u64(t_dev, b->step, b->stream);
    if (e != hipSuccess) return hip_fail(e, "step counter");
    e = hipGraphLaunch(g.exec, b->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const BGroup &grp = b->groups[gi];
        const int64_t launches = (n_steps + grp.T - 1) / grp.T;
        if (launches & 1) par[gi] ^= 1;
    }
    commit_parities(b, par);
    b->step += (uint64_t)n_steps;
    return GS_OK;
}

gs_status gs_batch_tune(gs_batch *b, int32_t reps, gs_batch_tune_entry *table, int32_t capacity,
                        int32_t *n_entries)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if (reps < 1) return fail(GS_ERR_INVALID_ARG, "reps %d < 1", reps);
    if (capacity < 0 || (capacity > 0 && !table)) return fail(GS_ERR_INVALID_ARG, "bad table/capacity");
    // Every simulation's state into pair 0; the timed sweeps read pair 0 and
    // write pair 1, so states and the step index stay unchanged.
    b->dirty = true;
    if ((st = rebuild(b)) != GS_OK) return st;
    struct Key {
        int nx, ny, nz;
        bool operator==(const Key &o) const { return nx == o.nx && ny == o.ny && nz == o.nz; }
    };
    std::vector<Key> classes;
    for (const BSim &s : b->sims) {
        Key k{s.nx, s.ny, s.nz};
        if (std::find(classes.begin(), classes.end(), k) == classes.end()) classes.push_back(k);
    }
    static const int zcs[] = {k_min_batch_zc, 16, 32, 64, 128};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool cache_ok = true;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "tune events");
    }
    std::vector<gs::SimDesc> desc = b->h_desc;
    std::vector<gs::WorkItem> items;
    int count = 0;
    for (size_t c = 0; c < classes.size() && e == hipSuccess; ++c) {
        const Key k = classes[c];
        std::vector<int> members;
        double cells = 0;
        for (size_t i = 0; i < b->sims.size(); ++i)
            if (Key{b->sims[i].nx, b->sims[i].ny, b->sims[i].nz} == k) {
                members.push_back((int)i);
                cells += (double)b->sims[i].n;
            }
        double best = 1e300;
        int bs = b->sims[members[0]].shape, bT = b->sims[members[0]].T, bz = b->sims[members[0]].zc;
        for (int shape = 1; shape <= gs::num_tb_shapes() && e == hipSuccess; ++shape) {
            for (int T = 1; T <= gs::tb_batch_max_T(shape, b->base.storage) && e == hipSuccess; ++T) {
                int last = -1;
                for (int zi = 0; zi < 4 && e == hipSuccess; ++zi) {
                    const int zc = std::min(zcs[zi], k.nz);
                    if (zc == last) continue;
                    last = zc;
                    items.clear();
                    const gs::TileShape ts = gs::tb_shape(shape, T);
                    for (int i : members) {
                        desc[i].zc = zc;
                        const int ntx = tiles_along(k.nx, ts.tx), nty = tiles_along(k.ny, ts.ty), nzc = tiles_along(k.nz, zc);
                        for (int z = 0; z < nzc; ++z)
                            for (int y = 0; y < nty; ++y)
                                for (int x = 0; x < ntx; ++x) items.push_back(gs::WorkItem{i, x, y, z});
                    }
                    e = hipMemcpyAsync(b->d_desc, desc.data(), desc.size() * sizeof(gs::SimDesc),
                                       hipMemcpyHostToDevice, b->stream);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(b->d_items + b->scratch_items, items.data(),
                                           items.size() * sizeof(gs::WorkItem), hipMemcpyHostToDevice, b->stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
                    gs::BatchArgs a = {};
                    a.coef = shared_coef(b);
                    a.sims = b->d_desc;
                    a.items = b->d_items + b->scratch_items;
                    a.n_items = (int)items.size();
                    a.parity = 0;
                    a.t = b->step;
                    a.t_dev = nullptr;
                    const int grid = std::max(
                        1, std::min(a.n_items, b->cus * gs::tb_batch_occupancy(b->base.storage, T, shape)));
                    if (e == hipSuccess) e = gs::launch_tblock_batch(b->base.storage, T, shape, a, grid, b->stream);
                    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
                    for (int r = 0; r < reps && e == hipSuccess; ++r)
                        e = gs::launch_tblock_batch(b->base.storage, T, shape, a, grid, b->stream);
                    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) break;
                    ++count;
                    const double per_step = (double)ms / (reps * T);
                    if (per_step < best) {
                        best = per_step;
                        bs = shape;
                        bT = T;
                        bz = zc;
                    }
                }
            }
        }
        for (int i : members) {
            b->sims[i].shape = bs;
            b->sims[i].T = bT;
            b->sims[i].zc = bz;
            desc[i].zc = bz;
        }
        if (e == hipSuccess &&
            !tune_cache_store(TuneKey{TUNE_BATCH, b->base.storage, k.nx, k.ny, k.nz, b->base.noise != 0.0},
                              TuneVal{bs + gs::num_tiles(), bT, bz, best}))
            cache_ok = false;
        if ((int32_t)c < capacity) {
            gs_batch_tune_entry &t = table[c];
            t.nx = k.nx;
            t.ny = k.ny;
            t.nz = k.nz;
            t.n_sims = (int32_t)members.size();
            t.tile = bs + gs::num_tiles();
            t.tblock = bT;
            t.zchunk = bz;
            t.reserved = 0;
            t.ms_per_step = best;
            t.gcells = cells / (best * 1e-3) / 1e9;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "gs_batch_tune");
    if (n_entries) *n_entries = (int32_t)classes.size();
    (void)count;
    b->dirty = true;
    st = rebuild(b);
    if (st == GS_OK && !cache_ok)
        return fail(GS_ERR_INVALID_ARG, "tuned, but the table %s could not be written", tune_cache_path());
    return st;
}

gs_status gs_batch_current(gs_batch *b, int32_t sim, void **u_dev, void **v_dev, uint64_t *step)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if ((st = sim_index(b, sim)) != GS_OK) return st;
    const BSim &s = b->sims[sim];
    if (u_dev) *u_dev = s.buf[s.parity][0];
    if (v_dev) *v_dev = s.buf[s.parity][1];
    if (step) *step = b->step;
    return GS_OK;
}

gs_status gs_batch_read(gs_batch *b, int32_t sim, double *u_host, double *v_host)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if ((st = sim_index(b, sim)) != GS_OK) return st;
    const BSim &s = b->sims[sim];
    double *dst[2] = {u_host, v_host};
    for (int f = 0; f < 2; ++f) {
        if (!dst[f]) continue;
        if ((st = read_field(s.buf[s.parity][f], b->base.storage, s.n, dst[f], b->stream, f)) != GS_OK) return st;
    }
    hipError_t e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_batch_read sync");
}

gs_status gs_batch_write(gs_batch *b, int32_t sim, const double *u_host, const double *v_host)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if ((st = sim_index(b, sim)) != GS_OK) return st;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "gs_batch_write sync");
    const BSim &s = b->sims[sim];
    const double *srcs[2] = {u_host, v_host};
    for (int f = 0; f < 2; ++f) {
        if (!srcs[f]) continue;
        if ((st = write_field(s.buf[s.parity][f], b->base.storage, s.n, srcs[f], b->stream, f)) != GS_OK) return st;
    }
    return GS_OK;
}

gs_status gs_batch_diagnostics(gs_batch *b, int32_t sim, gs_diag *out)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if ((st = sim_index(b, sim)) != GS_OK) return st;
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    const BSim &s = b->sims[sim];
    return diagnostics(b->base.storage, s.buf[s.parity][0], s.buf[s.parity][1], s.n, b->ws, b->stream, out);
}

gs_status gs_batch_fill_cube(gs_batch *b, int32_t sim, int32_t x0, int32_t y0, int32_t z0, int32_t side, double cu,
                             double cv)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    if ((st = sim_index(b, sim)) != GS_OK) return st;
    const BSim &s = b->sims[sim];
    const int mn = std::min(s.nx, std::min(s.ny, s.nz));
    if (side < 1 || side > mn) return fail(GS_ERR_INVALID_ARG, "side %d outside [1, %d]", side, mn);
    if (x0 < 0 || y0 < 0 || z0 < 0 || x0 >= s.nx || y0 >= s.ny || z0 >= s.nz)
        return fail(GS_ERR_INVALID_ARG, "corner outside the grid");
    if (!std::isfinite(cu) || !std::isfinite(cv)) return fail(GS_ERR_INVALID_ARG, "cube values must be finite");
    hipError_t e = gs::launch_init_box(b->base.storage, s.buf[s.parity][0], s.buf[s.parity][1], s.nx, s.ny, s.nz, x0,
                                       y0, z0, side, cu, cv, b->stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "fill kernel launch");
}

gs_status gs_batch_sync(gs_batch *b)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    hipError_t e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_batch_sync");
}

gs_status gs_batch_destroy(gs_batch *b)
{
    gs_status st = bcheck(b);
    if (st != GS_OK) return st;
    hipError_t e = hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    b->magic = 0;
    delete b;
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_batch_destroy sync");
}

} // extern "C"
