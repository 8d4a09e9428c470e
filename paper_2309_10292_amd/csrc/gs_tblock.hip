// Temporally blocked Gray-Scott sweep for gfx950: T = 1..4 time steps per
// pass over HBM (Eq. 2a/2b applied T times with the Eq. 1a/1b sources and the
// Eq. 3 Laplacian; periodic in x, y, z).
//
// One workgroup of NT lanes owns an output tile of TXG x-groups (4 cells
// each) by TY rows and marches through a chunk of z planes. Level k (k = 0..T)
// is the state after k of the T steps; level k is needed on the output tile
// widened by T - k rows in y and by one x-group on each side in x (enough for
// T <= 4). Every lane owns one x-group of the level-0 region and the same
// position in every level. The depth of a position is the last level that
// needs it; lanes are ordered by decreasing depth, so a wave whose positions
// are all shallower than level k skips level k as a whole.
//
// Per z iteration i (a wavefront in z):
//   - level-0 plane i+1 enters (prefetched one iteration earlier, into
//     registers or, in the FP64 kernel with noise at three fused steps,
//     straight into a lane-private LDS area);
//   - for k = 1..T, level k computes plane i-k+1 from level k-1's planes
//     i-k, i-k+1, i-k+2: z neighbours from the lane's registers (three plane
//     slots per level; plane z sits in slot (z - i0) mod 3, and the loop is
//     unrolled by three so that slots are fixed registers), x and y neighbours
//     from level k-1's current plane staged in LDS;
//   - level T's plane is stored if it lies in the workgroup's chunk;
//   - each level's newest plane is staged in LDS for the next iteration.
// Every cell-update rounds exactly as the single-step kernel's (the same
// operation sequence; in FP64 the noise term n r is one fused operation on the
// same exact real), so results are bitwise independent of T and of the tile.
// The noise of level k uses step index t + k - 1.
#include "gs_device.hpp"
#include "gs_launch.hpp"
#include "gs_tblock_common.hpp"

namespace gs {

// The FP64 kernel with noise at three fused steps and 512 lanes prefetches
// level 0 through LDS (global_load_lds, 16 bytes per lane and load) instead
// of registers, and makes the next iteration's Philox blocks between the two
// barriers of an iteration, where the vector units otherwise wait for the
// LDS stores: the registers this frees keep its straight-line levels free of
// spills.
template <typename S, int T, int NT, bool NOISE, bool BATCH> constexpr bool tb_dma()
{
    return sizeof(S) == 8 && NOISE && !BATCH && T == 3 && NT == 512;
}
// A workgroup barrier that waits for the LDS operations only: the LDS-DMA
// prefetch stays in flight across it (each wave reads only the area its own
// loads fill, after waiting for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F); // lgkmcnt(0)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename S, int TXG, int TY, int T, int NT> struct TbGeom {
    typedef typename Traits<S>::C C;
    static constexpr int GX = TXG + 2;          // x-groups per region row
    static constexpr int RW = GX * 4;           // region row width (cells)
    static constexpr int H = 16 / (int)sizeof(C);  // LDS row pad (>= 1; keeps rows 16-byte aligned)
    static constexpr int RY0 = TY + 2 * T;      // level-0 rows
    static constexpr int NSLOT = GX * RY0;      // lanes with a level-0 position
    // LDS rows of levels 0..T-1: RY0 - 2k each.
    static constexpr int LDS_ROWS = T * RY0 - T * (T - 1);
    // FP64 rows are split in two half-rows: cells 0-1 of every x-group, then
    // cells 2-3. A lane's four cells are 32 bytes, and 16-byte LDS accesses at
    // a 32-byte lane stride conflict in the banks; in half-rows every 16-byte
    // access of a row of lanes is contiguous. Each half-row has a pad group on
    // either side for the x-neighbours at the region's edges. FP32 rows (16
    // bytes per lane) are contiguous as they are.
    static constexpr bool SPLIT = sizeof(C) == 8;
    static constexpr int HS = 2 * (GX + 2);     // half-row length
    static constexpr int RS_MIN = SPLIT ? 2 * HS : RW + 2 * H;
    // A wave holds several rows of 16 lanes; their 16-byte reads are free of
    // bank conflicts on gfx950 only when the rows start a multiple of 256
    // bytes apart (measured with the LDS counters; 640- and 320-byte strides
    // conflict two ways). Rows are padded to that where the padded planes fit
    // the LDS of a CU.
    static constexpr int RS_PAD = (int)((RS_MIN * sizeof(C) + 255) / 256 * 256 / sizeof(C));
    static constexpr int RS = 2 * LDS_ROWS * RS_PAD * sizeof(C) <= 160 * 1024 ? RS_PAD : RS_MIN; // row stride
    // Offset within a row of column 4 gx + e of the region (e = -1 .. 4):
    // a per-lane base plus a constant, so every access of a lane shares one
    // address register.
    static __host__ __device__ constexpr int lane_base(int gx) { return SPLIT ? 2 * (gx + 1) : H + 4 * gx; }
    static __host__ __device__ constexpr int cell_off(int e)
    {
        return SPLIT ? (e < 0 ? HS - 1 : e < 2 ? e : e < 4 ? HS + e - 2 : 2) : e;
    }
    static constexpr int FIELD = LDS_ROWS * RS; // elements per field
    static_assert(T >= 1 && T <= 4, "one pad group covers at most 4 levels");
    static_assert(NSLOT <= NT, "every level-0 position needs a lane");
    static_assert(2 * FIELD * sizeof(C) <= 160 * 1024, "staged planes fit the LDS of a CU");
    static constexpr int row_base(int k) { return k * RY0 - k * (k - 1); }
};

// One output tile [x0, x0 + 4 TXG) x [y0, y0 + TY) x [z0, ze) of a grid
// (a.nx, a.ny, a.nz), T steps from (u, v) into (un, vn); t0 is the step index
// of the first of the T steps. `lds` holds 2 * TbGeom::FIELD elements and
// `pre_lds` 4 * NT 16-byte slots where tb_dma() holds (else it is unused).
// Every lane of the workgroup must call it (it contains barriers).
template <typename S, int TXG, int TY, int T, int NT, bool NOISE, bool BATCH, bool UNIT_DT>
__device__ __forceinline__ void tb_tile(const S *__restrict__ u, const S *__restrict__ v, S *__restrict__ un,
                                        S *__restrict__ vn, const StepArgs &a, int x0, int y0, int z0, int ze,
                                        uint64_t t0, typename Traits<S>::C *__restrict__ lds,
                                        uint4 *__restrict__ pre_lds)
{
    typedef TbGeom<S, TXG, TY, T, NT> G;
    typedef typename G::C C;
    constexpr bool DMA = tb_dma<S, T, NT, NOISE, BATCH>();
    static_assert(!DMA || 2 * G::FIELD * sizeof(C) + 4 * NT * 16 <= 160 * 1024, "staged planes and prefetch fit");
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t plane = (size_t)nx * (size_t)ny;

    // This lane's position (x-group gxs, level-0 row rys) and depth dep
    // (-1: none). Order: the output tile (depth T, row-major), the x-halo
    // groups beside the output rows (depth T-1), then rows d and RY0-1-d for
    // d = T-1 down to 0 (depth d).
    int gxs = 0, rys = 0, dep = -1;
    {
        constexpr int nA = TXG * TY, nH = 2 * TY;
        const int s = threadIdx.x;
        if (s < nA) {
            rys = T + s / TXG;
            gxs = 1 + s % TXG;
            dep = T;
        } else if (s < nA + nH) {
            const int r = s - nA;
            rys = T + (r >> 1);
            gxs = (r & 1) ? G::GX - 1 : 0;
            dep = T - 1;
        } else {
            const int r = s - nA - nH;
            const int d = T - 1 - r / (2 * G::GX);
            if (d >= 0) {
                const int q = r % (2 * G::GX);
                rys = q < G::GX ? d : G::RY0 - 1 - d;
                gxs = q % G::GX;
                dep = d;
            }
        }
    }
    const bool has = dep >= 0;
    const int gx = (((x0 - 4 + 4 * gxs) % nx) + nx) % nx;
    const int gy = (((y0 - T + rys) % ny) + ny) % ny;
    const size_t xy = (size_t)gy * nx + gx;
    // Output positions are exactly the depth-T ones.
    const bool out_ok = dep == T && (x0 + 4 * (gxs - 1) < nx) && (y0 + rys - T < ny);

    C win[T][3][2][4]; // [level][slot][field][cell]
#pragma unroll
    for (int k = 0; k < T; ++k)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int e = 0; e < 4; ++e) win[k][q][f][e] = (C)0;

    const S *src[2] = {u, v};
    auto load_plane = [&](int z, Vec<S, 4> (&o)[2]) {
        const size_t off = (size_t)wrap(z, nz) * plane + xy;
#pragma unroll
        for (int f = 0; f < 2; ++f) o[f] = *reinterpret_cast<const Vec<S, 4> *>(src[f] + off);
    };
    const int lbase = G::lane_base(gxs);
    // Element e (-1 .. 4, column 4 gxs + e) of row `row` of level k's plane.
    auto lds_at = [&](int f, int k, int row, int e) -> C & {
        return lds[f * G::FIELD + (G::row_base(k) + row) * G::RS + lbase + G::cell_off(e)];
    };
    auto in_level = [&](int k) { return dep >= k; };

    // LDS-DMA prefetch (tb_dma): slot 2 f + hh of a lane holds cells
    // 2 hh, 2 hh + 1 of field f; a wave's 64 lanes fill 64 consecutive slots.
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    auto dma_plane = [&](int z) {
        const size_t off = (size_t)wrap(z, nz) * plane + xy;
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
                __builtin_amdgcn_global_load_lds((const void *)(src[f] + off + 2 * hh),
                                                 (__attribute__((address_space(3))) void *)(pre_lds + (2 * f + hh) * NT +
                                                                                            64 * wave),
                                                 16, 0, 0);
    };
    auto read_pre = [&](C (&o)[2][4]) {
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const double2 q = *reinterpret_cast<const double2 *>(pre_lds + (2 * f + hh) * NT + threadIdx.x);
                o[f][2 * hh] = q.x;
                o[f][2 * hh + 1] = q.y;
            }
    };
    // Philox blocks of the next iteration's levels (tb_dma), made ahead.
    uint32_t wq[T][4];
    auto make_noise = [&](const int i, auto full) {
        constexpr bool FULL = decltype(full)::value;
#pragma unroll
        for (int k = 1; k <= T; ++k) {
            if (!FULL && !in_level(k)) continue;
            const size_t idx = (size_t)wrap(i - k + 1, nz) * plane + xy;
            const Philox4 w = noise_block(idx, t0 + (uint64_t)(k - 1), a.seed);
#pragma unroll
            for (int e = 0; e < 4; ++e) wq[k - 1][e] = w.w[e];
        }
    };

    // Prologue: level-0 slots hold planes i0-1 (slot 2) and i0 (slot 0); plane
    // i0+1 is in flight; LDS holds level-0 plane i0.
    const int i0 = z0 - T + 1;
    const int i_end = ze + T - 2; // inclusive
    Vec<S, 4> pre[2];
    if constexpr (DMA) dma_plane(i0 + 1);
    if (has) {
        Vec<S, 4> q0[2], q1[2];
        load_plane(i0 - 1, q0);
        load_plane(i0, q1);
        if constexpr (!DMA) load_plane(i0 + 1, pre);
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                win[0][2][f][e] = fload<S>(f, q0[f].e[e]);
                win[0][0][f][e] = fload<S>(f, q1[f].e[e]);
            }
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int e = 0; e < 4; ++e) lds_at(f, 0, rys, e) = win[0][0][f][e];
    }
    if constexpr (DMA) {
        make_noise(i0, Full<true>{});
        lds_barrier();
    } else {
        __syncthreads();
    }

    // One z iteration at phase P = (i - i0) mod 3. A wave whose first lane
    // (the deepest position of the wave) has depth T runs every level on all
    // of its lanes without per-lane branches (FULL): the lanes that a level
    // does not need compute values nobody reads, from clamped LDS rows, and
    // only the stores stay per-lane. Straight-line levels let the scheduler
    // overlap the Philox chains with LDS reads and arithmetic. Other waves
    // skip, per lane, the levels their positions do not need.
    auto iteration = [&](const int i, auto phase, auto full) {
        constexpr int P = decltype(phase)::value;
        constexpr bool FULL = decltype(full)::value;
        // Level 0: plane i+1 enters its slot; prefetch plane i+2.
        if constexpr (DMA) {
            __builtin_amdgcn_s_waitcnt(0x0F70); // vmcnt(0): this wave's prefetch has landed
            read_pre(win[0][slot3(P + 1)]);
            __builtin_amdgcn_s_waitcnt(0xC07F); // lgkmcnt(0): read before it is overwritten
            if (i + 2 <= ze + T - 1) dma_plane(i + 2);
        } else {
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int e = 0; e < 4; ++e) win[0][slot3(P + 1)][f][e] = fload<S>(f, pre[f].e[e]);
            if (has && i + 2 <= ze + T - 1) load_plane(i + 2, pre);
        }

        // Levels 1..T, in order; level k computes plane i-k+1.
#pragma unroll
        for (int k = 1; k <= T; ++k) {
            if (!FULL && !in_level(k)) continue;
            const int zk = i - k + 1;
            const int sm = slot3(P - k), sc = slot3(P - k + 1), sp = slot3(P - k + 2);
            // Row of this position in level k-1's LDS plane (clamped for
            // positions outside level k, whose results are not used).
            const int ry = FULL ? min(max(rys, k), G::RY0 - 1 - k) : rys;
            const int row = ry - (k - 1);
            C xm[2][4], xp[2][4], ym[2][4], yp[2][4];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const C *c = win[k - 1][sc][f];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xm[f][e] = e > 0 ? c[e - 1] : lds_at(f, k - 1, row, -1);
                    xp[f][e] = e < 3 ? c[e + 1] : lds_at(f, k - 1, row, 4);
                    ym[f][e] = lds_at(f, k - 1, row - 1, e);
                    yp[f][e] = lds_at(f, k - 1, row + 1, e);
                }
            }
            C r[4] = {(C)0, (C)0, (C)0, (C)0}; // the noise term n r
            if constexpr (NOISE) {
                Philox4 w;
                if constexpr (DMA) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) w.w[e] = wq[k - 1][e];
                } else {
                    w = noise_block((size_t)wrap(zk, nz) * plane + xy, t0 + (uint64_t)(k - 1), a.seed);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // FP64: n r with r = (w + 1/2) 2^-31 is the exact real
                    // (n 2^-31) w + n 2^-32, so one fused operation rounds it
                    // once, as the product n r does.
                    if constexpr (sizeof(C) == 8)
                        r[e] = __builtin_fma(a.noise_s, (double)(int32_t)w.w[e], a.noise_h);
                    else
                        r[e] = noise_term_f32(w.w[e], a.noise_s_f, a.noise_h_f);
                }
            }
            C res[2][4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const C uc = win[k - 1][sc][0][e], vc = win[k - 1][sc][1][e];
                C lu, lv;
                if constexpr (sizeof(C) == 8) {
                    lu = lap_f64(uc, xm[0][e], xp[0][e], ym[0][e], yp[0][e], win[k - 1][sm][0][e], win[k - 1][sp][0][e]);
                    lv = lap_f64(vc, xm[1][e], xp[1][e], ym[1][e], yp[1][e], win[k - 1][sm][1][e], win[k - 1][sp][1][e]);
                } else {
                    lu = lap_f32<S>(uc, xm[0][e], xp[0][e], ym[0][e], yp[0][e], win[k - 1][sm][0][e],
                                      win[k - 1][sp][0][e]);
                    lv = lap_f32<S>(vc, xm[1][e], xp[1][e], ym[1][e], yp[1][e], win[k - 1][sm][1][e],
                                      win[k - 1][sp][1][e]);
                }
                C uo, vo;
                cell_update<C, UNIT_DT, NOISE>(a, uc, vc, lu, lv, r[e], uo, vo);
                // Intermediate levels carry the stored precision of the state.
                res[0][e] = fload<S>(0, fstore<S>(0, uo));
                res[1][e] = fload<S>(1, fstore<S>(1, vo));
            }
            if (k < T) {
#pragma unroll
                for (int f = 0; f < 2; ++f)
#pragma unroll
                    for (int e = 0; e < 4; ++e) win[k][sc][f][e] = res[f][e];
            } else if (out_ok && zk >= z0) {
                Vec<S, 4> ou, ov;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ou.e[e] = fstore<S>(0, res[0][e]);
                    ov.e[e] = fstore<S>(1, res[1][e]);
                }
                const size_t off = (size_t)zk * plane + xy;
                NtStore<S>::put(un + off, ou);
                NtStore<S>::put(vn + off, ov);
            }
        }
        if constexpr (DMA) lds_barrier(); // all reads of the staged planes are done
        else __syncthreads();
        // Stage the newest plane of levels 0..T-1 (the centre plane of the next iteration).
        if (has) {
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int e = 0; e < 4; ++e) lds_at(f, 0, rys, e) = win[0][slot3(P + 1)][f][e];
        }
#pragma unroll
        for (int k = 1; k < T; ++k) {
            if (in_level(k)) {
#pragma unroll
                for (int f = 0; f < 2; ++f)
#pragma unroll
                    for (int e = 0; e < 4; ++e) lds_at(f, k, rys - k, e) = win[k][slot3(P - k + 1)][f][e];
            }
        }
        if constexpr (DMA) {
            make_noise(i + 1, full);
            lds_barrier();
        } else {
            __syncthreads();
        }
    };

    // The straight-line variant needs more registers; it is used where they
    // fit the budget (up to 512 lanes; FP64 up to 3 levels, and not in the
    // persistent batched kernel).
    constexpr bool full_ok = NT <= 512 && (sizeof(C) == 4 || (T <= 3 && !BATCH));
    const int wave_depth = __builtin_amdgcn_readfirstlane(dep);
    if (full_ok && wave_depth == T) {
        for (int i = i0; i <= i_end; i += 3) {
            iteration(i, Phase<0>{}, Full<true>{});
            if (i + 1 <= i_end) iteration(i + 1, Phase<1>{}, Full<true>{});
            if (i + 2 <= i_end) iteration(i + 2, Phase<2>{}, Full<true>{});
        }
    } else {
        for (int i = i0; i <= i_end; i += 3) {
            iteration(i, Phase<0>{}, Full<false>{});
            if (i + 1 <= i_end) iteration(i + 1, Phase<1>{}, Full<false>{});
            if (i + 2 <= i_end) iteration(i + 2, Phase<2>{}, Full<false>{});
        }
    }
}

// Waves per SIMD the single-grid kernel is compiled for (its register
// budget): with FP32 arithmetic and up to two fused steps the kernel fits 128
// registers, so 256- and 512-lane workgroups keep four waves per SIMD (two
// 512-lane workgroups per CU; one register more would leave one); other
// kernels take what their lane count allows.
template <typename S, int T, int NT> constexpr int tb_min_waves()
{
    return (sizeof(typename Traits<S>::C) == 4 && T <= 2 && NT <= 512) ? 4 : 1;
}

template <typename S, int TXG, int TY, int T, int NT, bool NOISE>
__global__ __launch_bounds__(NT, (tb_min_waves<S, T, NT>())) void stencil_tb(const S *__restrict__ u,
                                                                           const S *__restrict__ v,
                                                                           S *__restrict__ un, S *__restrict__ vn,
                                                                           StepArgs a)
{
    typedef TbGeom<S, TXG, TY, T, NT> G;
    __shared__ typename G::C lds[2 * G::FIELD];
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int bx = (int)(lb % (uint32_t)a.ntx);
    const uint32_t rest = lb / (uint32_t)a.ntx;
    const int by = (int)(rest % (uint32_t)a.nty);
    const int bz = (int)(rest / (uint32_t)a.nty);
    const int z0 = bz * a.zc;
    const uint64_t t0 = NOISE ? step_index(a) : 0;
    const int ze = min(z0 + a.zc, a.nz);
    auto run = [&](uint4 *pre_lds) {
        // FP64 runs with dt = 1 (the workload of the paper) take the variant
        // without the dt products.
        if constexpr (sizeof(S) == 8) {
            if (a.dt == 1.0) {
                tb_tile<S, TXG, TY, T, NT, NOISE, false, true>(u, v, un, vn, a, bx * (TXG * 4), by * TY, z0, ze, t0,
                                                               lds, pre_lds);
                return;
            }
        }
        tb_tile<S, TXG, TY, T, NT, NOISE, false, false>(u, v, un, vn, a, bx * (TXG * 4), by * TY, z0, ze, t0, lds,
                                                        pre_lds);
    };
    if constexpr (tb_dma<S, T, NT, NOISE, false>()) {
        __shared__ uint4 pre_lds[4 * NT];
        run(pre_lds);
    } else {
        run(nullptr);
    }
}

// Persistent sweep over many independent simulations: each workgroup walks
// the work list (items sorted by decreasing cost) with a stride of the grid
// size; an item is one tile x z-chunk of one simulation.
template <typename S, int TXG, int TY, int T, int NT, bool NOISE>
__global__ __launch_bounds__(NT) void stencil_tb_batch(BatchArgs b)
{
    typedef TbGeom<S, TXG, TY, T, NT> G;
    __shared__ typename G::C lds[2 * G::FIELD];
    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const uint64_t t0 = NOISE ? (b.t_dev ? *b.t_dev + b.t : b.t) : 0;
    for (uint32_t it = lb; it < (uint32_t)b.n_items; it += gridDim.x) {
        const WorkItem w = b.items[it];
        const SimDesc &d = b.sims[w.sim];
        StepArgs a = b.coef;
        a.nx = d.nx;
        a.ny = d.ny;
        a.nz = d.nz;
        a.F = d.F;
        a.FK = d.FK;
        a.F_f = d.F_f;
        a.FK_f = d.FK_f;
        a.seed = d.seed;
        const int z0 = w.bz * d.zc;
        const S *u = (const S *)d.buf[b.parity][0];
        const S *v = (const S *)d.buf[b.parity][1];
        S *un = (S *)d.buf[b.parity ^ 1][0];
        S *vn = (S *)d.buf[b.parity ^ 1][1];
        const int ze = min(z0 + d.zc, d.nz);
        if constexpr (sizeof(S) == 8) {
            if (a.dt == 1.0) {
                tb_tile<S, TXG, TY, T, NT, NOISE, true, true>(u, v, un, vn, a, w.bx * (TXG * 4), w.by * TY, z0, ze,
                                                              t0, lds, nullptr);
                continue;
            }
        }
        tb_tile<S, TXG, TY, T, NT, NOISE, true, false>(u, v, un, vn, a, w.bx * (TXG * 4), w.by * TY, z0, ze, t0,
                                                       lds, nullptr);
    }
}

// ------------------------------------------------------------------ launch
template <typename S, int TXG, int TY, int T, int NT>
static hipError_t launch_tb_t(const void *u, const void *v, void *un, void *vn, StepArgs a, hipStream_t st)
{
    a.ntx = (a.nx + TXG * 4 - 1) / (TXG * 4);
    a.nty = (a.ny + TY - 1) / TY;
    const int nzc = (a.nz + a.zc - 1) / a.zc;
    const size_t nb = (size_t)a.ntx * a.nty * nzc;
    if (nb == 0 || nb > 0x7fffffffu) return hipErrorInvalidConfiguration;
    if (a.noise != 0.0)
        hipLaunchKernelGGL((stencil_tb<S, TXG, TY, T, NT, true>), dim3((unsigned)nb), dim3(NT), 0, st,
                           (const S *)u, (const S *)v, (S *)un, (S *)vn, a);
    else
        hipLaunchKernelGGL((stencil_tb<S, TXG, TY, T, NT, false>), dim3((unsigned)nb), dim3(NT), 0, st,
                           (const S *)u, (const S *)v, (S *)un, (S *)vn, a);
    return hipGetLastError();
}

// Shapes per T (output x-groups, rows, lanes): the level-0 region
// (TXG + 2) x (TY + 2T) fills the workgroup.
//   shape 1: TXG=16,  256 lanes, region 18 x 14
//   shape 2: TXG=16,  512 lanes, region 18 x 28
//   shape 3: TXG=32,  512 lanes, region 34 x 14
//   shape 4: TXG=16,  768 lanes, region 18 x 42
//   shape 5: TXG=16, 1024 lanes, region 18 x 56
// One workgroup per CU: NT lanes leave 512 / ceil(NT / 256) registers per
// lane. The deepest fusion whose registers fit that budget without spills
// (the persistent batched kernel holds a few more registers for its work
// list):
template <typename S, int NT, bool BATCH> constexpr int tb_max_T_of()
{
    if (NT <= 512) return 4;
    if (NT <= 768) return sizeof(S) == 8 ? (BATCH ? 1 : 2) : (BATCH ? 3 : 4);
    return sizeof(S) == 8 ? (BATCH ? 0 : 1) : (BATCH ? 2 : 3);
}
constexpr int shape_lanes(int shape) { return shape == 1 ? 256 : shape <= 3 ? 512 : shape == 4 ? 768 : 1024; }
template <typename S, bool BATCH> constexpr int tb_max_T_shape(int shape)
{
    return shape <= 3   ? tb_max_T_of<S, 512, BATCH>()
           : shape == 4 ? tb_max_T_of<S, 768, BATCH>()
                        : tb_max_T_of<S, 1024, BATCH>();
}

template <typename S, int T>
static hipError_t dispatch_tb_shape(int shape, const void *u, const void *v, void *un, void *vn, const StepArgs &a,
                                    hipStream_t st)
{
    switch (shape) {
    case 1: return launch_tb_t<S, 16, 14 - 2 * T, T, 256>(u, v, un, vn, a, st);
    case 2: return launch_tb_t<S, 16, 28 - 2 * T, T, 512>(u, v, un, vn, a, st);
    case 3: return launch_tb_t<S, 32, 14 - 2 * T, T, 512>(u, v, un, vn, a, st);
    case 4:
        if constexpr (T <= tb_max_T_of<S, 768, false>())
            return launch_tb_t<S, 16, 42 - 2 * T, T, 768>(u, v, un, vn, a, st);
        break;
    case 5:
        if constexpr (T <= tb_max_T_of<S, 1024, false>())
            return launch_tb_t<S, 16, 56 - 2 * T, T, 1024>(u, v, un, vn, a, st);
        break;
    }
    return hipErrorInvalidValue;
}

template <typename S>
static hipError_t dispatch_tb_T(int T, int shape, const void *u, const void *v, void *un, void *vn,
                                const StepArgs &a, hipStream_t st)
{
    switch (T) {
    case 1: return dispatch_tb_shape<S, 1>(shape, u, v, un, vn, a, st);
    case 2: return dispatch_tb_shape<S, 2>(shape, u, v, un, vn, a, st);
    case 3: return dispatch_tb_shape<S, 3>(shape, u, v, un, vn, a, st);
    case 4: return dispatch_tb_shape<S, 4>(shape, u, v, un, vn, a, st);
    }
    return hipErrorInvalidValue;
}

int num_tb_shapes() { return 5; }

TileShape tb_shape(int shape, int T)
{
    switch (shape) {
    case 1: return TileShape{64, 14 - 2 * T};
    case 2: return TileShape{64, 28 - 2 * T};
    case 3: return TileShape{128, 14 - 2 * T};
    case 4: return TileShape{64, 42 - 2 * T};
    case 5: return TileShape{64, 56 - 2 * T};
    }
    return TileShape{0, 0};
}

template <bool BATCH> static int max_T_for(int shape, int storage)
{
    if (shape < 1 || shape > 5) return 0;
    switch (storage) {
    case 0: return tb_max_T_shape<double, BATCH>(shape);
    case 1: return tb_max_T_shape<float, BATCH>(shape);
    case 2: return tb_max_T_shape<bf16, BATCH>(shape);
    case 3: return tb_max_T_shape<f16, BATCH>(shape);
    case 4: return BATCH ? 0 : tb_max_T_shape<bf16c, false>(shape);
    }
    return 0;
}

int tb_max_T(int shape, int storage) { return max_T_for<false>(shape, storage); }
int tb_batch_max_T(int shape, int storage) { return max_T_for<true>(shape, storage); }

template <typename S, int TXG, int TY, int T, int NT>
static hipError_t launch_tb_batch_t(const BatchArgs &b, int grid, hipStream_t st)
{
    if (grid < 1) return hipErrorInvalidConfiguration;
    if (b.coef.noise != 0.0)
        hipLaunchKernelGGL((stencil_tb_batch<S, TXG, TY, T, NT, true>), dim3(grid), dim3(NT), 0, st, b);
    else
        hipLaunchKernelGGL((stencil_tb_batch<S, TXG, TY, T, NT, false>), dim3(grid), dim3(NT), 0, st, b);
    return hipGetLastError();
}

template <typename S, int T>
static hipError_t batch_shape(int shape, const BatchArgs &b, int grid, hipStream_t st)
{
    switch (shape) {
    case 1: return launch_tb_batch_t<S, 16, 14 - 2 * T, T, 256>(b, grid, st);
    case 2: return launch_tb_batch_t<S, 16, 28 - 2 * T, T, 512>(b, grid, st);
    case 3: return launch_tb_batch_t<S, 32, 14 - 2 * T, T, 512>(b, grid, st);
    case 4:
        if constexpr (T <= tb_max_T_of<S, 768, true>()) return launch_tb_batch_t<S, 16, 42 - 2 * T, T, 768>(b, grid, st);
        break;
    case 5:
        if constexpr (T <= tb_max_T_of<S, 1024, true>())
            return launch_tb_batch_t<S, 16, 56 - 2 * T, T, 1024>(b, grid, st);
        break;
    }
    return hipErrorInvalidValue;
}

template <typename S>
static hipError_t batch_T(int T, int shape, const BatchArgs &b, int grid, hipStream_t st)
{
    switch (T) {
    case 1: return batch_shape<S, 1>(shape, b, grid, st);
    case 2: return batch_shape<S, 2>(shape, b, grid, st);
    case 3: return batch_shape<S, 3>(shape, b, grid, st);
    case 4: return batch_shape<S, 4>(shape, b, grid, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tblock_batch(int storage, int T, int shape, const BatchArgs &b, int grid, hipStream_t st)
{
    switch (storage) {
    case 0: return batch_T<double>(T, shape, b, grid, st);
    case 1: return batch_T<float>(T, shape, b, grid, st);
    case 2: return batch_T<bf16>(T, shape, b, grid, st);
    case 3: return batch_T<f16>(T, shape, b, grid, st);
    }
    return hipErrorInvalidValue;
}

int tb_shape_lanes(int shape) { return shape_lanes(shape); }

template <typename S, int TXG, int TY, int T, int NT>
static int occ_t()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stencil_tb_batch<S, TXG, TY, T, NT, false>, NT, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <typename S, int T>
static int occ_shape(int shape)
{
    switch (shape) {
    case 1: return occ_t<S, 16, 14 - 2 * T, T, 256>();
    case 2: return occ_t<S, 16, 28 - 2 * T, T, 512>();
    case 3: return occ_t<S, 32, 14 - 2 * T, T, 512>();
    case 4:
        if constexpr (T <= tb_max_T_of<S, 768, true>()) return occ_t<S, 16, 42 - 2 * T, T, 768>();
        break;
    case 5:
        if constexpr (T <= tb_max_T_of<S, 1024, true>()) return occ_t<S, 16, 56 - 2 * T, T, 1024>();
        break;
    }
    return 1;
}

template <typename S>
static int occ_T(int T, int shape)
{
    switch (T) {
    case 1: return occ_shape<S, 1>(shape);
    case 2: return occ_shape<S, 2>(shape);
    case 3: return occ_shape<S, 3>(shape);
    case 4: return occ_shape<S, 4>(shape);
    }
    return 1;
}

template <typename S, int TXG, int TY, int T, int NT>
static int occ_single_t(bool noise)
{
    int n = 0;
    const hipError_t e = noise
                             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stencil_tb<S, TXG, TY, T, NT, true>, NT, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stencil_tb<S, TXG, TY, T, NT, false>, NT, 0);
    return e == hipSuccess && n > 0 ? n : 0;
}

template <typename S, int T>
static int occ_single_shape(int shape, bool noise)
{
    switch (shape) {
    case 1: return occ_single_t<S, 16, 14 - 2 * T, T, 256>(noise);
    case 2: return occ_single_t<S, 16, 28 - 2 * T, T, 512>(noise);
    case 3: return occ_single_t<S, 32, 14 - 2 * T, T, 512>(noise);
    case 4:
        if constexpr (T <= tb_max_T_of<S, 768, false>()) return occ_single_t<S, 16, 42 - 2 * T, T, 768>(noise);
        break;
    case 5:
        if constexpr (T <= tb_max_T_of<S, 1024, false>()) return occ_single_t<S, 16, 56 - 2 * T, T, 1024>(noise);
        break;
    }
    return 0;
}

template <typename S>
static int occ_single_T(int T, int shape, bool noise)
{
    switch (T) {
    case 1: return occ_single_shape<S, 1>(shape, noise);
    case 2: return occ_single_shape<S, 2>(shape, noise);
    case 3: return occ_single_shape<S, 3>(shape, noise);
    case 4: return occ_single_shape<S, 4>(shape, noise);
    }
    return 0;
}

int tb_occupancy(int storage, int T, int shape, bool noise)
{
    switch (storage) {
    case 0: return occ_single_T<double>(T, shape, noise);
    case 1: return occ_single_T<float>(T, shape, noise);
    case 2: return occ_single_T<bf16>(T, shape, noise);
    case 3: return occ_single_T<f16>(T, shape, noise);
    case 4: return occ_single_T<bf16c>(T, shape, noise);
    }
    return 0;
}

int tb_batch_occupancy(int storage, int T, int shape)
{
    switch (storage) {
    case 0: return occ_T<double>(T, shape);
    case 1: return occ_T<float>(T, shape);
    case 2: return occ_T<bf16>(T, shape);
    case 3: return occ_T<f16>(T, shape);
    }
    return 1;
}

hipError_t launch_tblock(int storage, int T, int shape, const void *u, const void *v, void *un, void *vn,
                         const StepArgs &a, hipStream_t st)
{
    switch (storage) {
    case 0: return dispatch_tb_T<double>(T, shape, u, v, un, vn, a, st);
    case 1: return dispatch_tb_T<float>(T, shape, u, v, un, vn, a, st);
    case 2: return dispatch_tb_T<bf16>(T, shape, u, v, un, vn, a, st);
    case 3: return dispatch_tb_T<f16>(T, shape, u, v, un, vn, a, st);
    case 4: return dispatch_tb_T<bf16c>(T, shape, u, v, un, vn, a, st);
    }
    return hipErrorInvalidValue;
}

} // namespace gs
