// Fused Gray-Scott step for gfx950 (Eq. 1a/1b source terms, Eq. 2a/2b
// forward-Euler Jacobi update, Eq. 3 Laplacian; periodic in x, y, z).
//
// Design: 2.5-D z-streaming. A workgroup of 256 lanes owns a TX x TY tile of
// an xy plane and marches through a chunk of ZC planes. Each lane owns V
// x-consecutive cells (one 16- or 32-byte access per field). Per plane:
//   - the lane's own cells of planes z-1, z, z+1 are held in registers (the
//     z neighbours never leave registers);
//   - plane z with a one-cell ring is staged in LDS (double-buffered, one
//     barrier per plane) and gives the x and y neighbours;
//   - the loads of plane z+2 (own cells and ring) are issued before the
//     arithmetic of plane z, so a whole plane of work covers their latency.
// Every field value is therefore fetched from HBM about once per step; only
// the ring cells and the two planes at each chunk end are re-read, mostly
// from L2 (tiles are laid out so one XCD works on one contiguous region).
//
// FP64 storage evaluates exactly the operation sequence of the FP64 definition
// (pairwise neighbour sum, (s - 6c) / 6, source terms left to right, no
// contraction), so results are bitwise equal to it. Other storage types
// compute in FP32 (the Laplacian's sum in FP64 for FP32 storage, plain for
// 2-byte storage) and round on store.
#include "gs_device.hpp"
#include "gs_launch.hpp"

namespace gs {

template <typename S, int TX, int TY, int V> struct Geom {
    typedef typename Traits<S>::C C;
    static constexpr int TXV = TX / V;           // lanes per tile row
    static constexpr int NT = TXV * TY;          // lanes per workgroup
    static constexpr int H = 16 / (int)sizeof(C);  // left pad: interior 16-byte aligned in LDS
    static constexpr int RS = TX + 2 * H;         // LDS row stride in elements
    static constexpr int PLANE = (TY + 2) * RS;   // LDS elements per staged plane
    static constexpr int NYH = 2 * TXV;           // ring rows above/below: vector loads
    static constexpr int NXH = 2 * TY;            // ring columns left/right: scalar loads
    static_assert(NT == 256, "tiles are sized for 256-lane workgroups");
    static_assert(NYH + NXH <= NT, "ring loads must fit one lane each");
};

// Per-lane addressing of one tile, fixed for the whole z march.
struct LaneMap {
    size_t own_off;   // offset of the lane's first own cell inside a plane
    size_t halo_off;  // offset of the lane's ring element(s) inside a plane
    int lds_own;      // LDS index of the lane's first own cell
    int lds_halo;     // LDS index of the lane's ring element(s)
    int hkind;        // 0: no ring role, 1: ring row vector, 2: ring column scalar
    bool valid;       // own cells inside the grid (ragged tiles store nothing else)
};

template <typename S, int TX, int TY, int V>
__device__ __forceinline__ LaneMap make_lane_map(int x0, int y0, int nx, int ny)
{
    typedef Geom<S, TX, TY, V> G;
    LaneMap m;
    const int tid = threadIdx.x;
    const int tx = tid % G::TXV, ty = tid / G::TXV;
    const int gx = (x0 + tx * V) % nx;
    const int gy = (y0 + ty) % ny;
    m.own_off = (size_t)gy * nx + gx;
    m.lds_own = (ty + 1) * G::RS + G::H + tx * V;
    m.valid = (x0 + tx * V < nx) && (y0 + ty < ny);
    m.hkind = 0;
    m.halo_off = 0;
    m.lds_halo = 0;
    if (tid < G::NYH) {
        const int row = tid < G::TXV ? 0 : TY + 1;
        const int col = tid % G::TXV;
        const int hy = ((y0 + row - 1) % ny + ny) % ny;
        const int hx = (x0 + col * V) % nx;
        m.hkind = 1;
        m.halo_off = (size_t)hy * nx + hx;
        m.lds_halo = row * G::RS + G::H + col * V;
    } else if (tid < G::NYH + G::NXH) {
        const int j = tid - G::NYH;
        const int row = 1 + (j >> 1);
        const int right = j & 1;
        const int hy = (y0 + row - 1) % ny;
        const int hx = right ? (x0 + TX) % nx : (x0 - 1 + nx) % nx;
        m.hkind = 2;
        m.halo_off = (size_t)hy * nx + hx;
        m.lds_halo = row * G::RS + G::H + (right ? TX : -1);
    }
    return m;
}

template <typename S, int V>
__device__ __forceinline__ Vec<S, V> load_vec(const S *__restrict__ f, size_t off)
{
    return *reinterpret_cast<const Vec<S, V> *>(f + off);
}

template <typename S, int V>
__device__ __forceinline__ void load_ring(const S *__restrict__ f, size_t plane_off, const LaneMap &m,
                                          Vec<S, V> &out)
{
    if (m.hkind == 1)
        out = load_vec<S, V>(f, plane_off + m.halo_off);
    else if (m.hkind == 2)
        out.e[0] = f[plane_off + m.halo_off];
}

// f: field index (0 = u, 1 = v), for the storage types that keep u complemented.
template <typename S, int V, typename C>
__device__ __forceinline__ void stage(int f, C *__restrict__ L, const LaneMap &m, const C (&own)[V],
                                      const Vec<S, V> &ring)
{
#pragma unroll
    for (int i = 0; i < V; ++i) L[m.lds_own + i] = own[i];
    if (m.hkind == 1) {
#pragma unroll
        for (int i = 0; i < V; ++i) L[m.lds_halo + i] = fload<S>(f, ring.e[i]);
    } else if (m.hkind == 2) {
        L[m.lds_halo] = fload<S>(f, ring.e[0]);
    }
}

template <typename S, int V, typename C>
__device__ __forceinline__ void widen(int f, const Vec<S, V> &a, C (&out)[V])
{
#pragma unroll
    for (int i = 0; i < V; ++i) out[i] = fload<S>(f, a.e[i]);
}

// NF = 2: the Gray-Scott step on (u, v). NF = 1 with LAPLACE: out = lap(f)
// of a single FP64 field (calibration kernel).
template <typename S, int TX, int TY, int V, int NF, bool NOISE, bool LAPLACE>
__global__ __launch_bounds__(256) void stencil_tile(const S *__restrict__ u, const S *__restrict__ v,
                                                    S *__restrict__ un, S *__restrict__ vn, StepArgs a)
{
    typedef Geom<S, TX, TY, V> G;
    typedef typename G::C C;
    __shared__ C lds[2][NF][G::PLANE];

    const uint32_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int bx = (int)(lb % (uint32_t)a.ntx);
    const uint32_t rest = lb / (uint32_t)a.ntx;
    const int by = (int)(rest % (uint32_t)a.nty);
    const int bz = (int)(rest / (uint32_t)a.nty);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * a.zc;
    const int ze = min(z0 + a.zc, nz);
    const size_t plane = (size_t)nx * (size_t)ny;
    const LaneMap m = make_lane_map<S, TX, TY, V>(x0, y0, nx, ny);

    const S *src[2] = {u, v};
    C zm[NF][V], zc[NF][V], zp[NF][V];
    Vec<S, V> pre[NF], ring[NF], ring_next[NF];

#pragma unroll
    for (int f = 0; f < NF; ++f) {
        widen<S, V>(f, load_vec<S, V>(src[f], (size_t)wrap(z0 - 1, nz) * plane + m.own_off), zm[f]);
        widen<S, V>(f, load_vec<S, V>(src[f], (size_t)z0 * plane + m.own_off), zc[f]);
        widen<S, V>(f, load_vec<S, V>(src[f], (size_t)wrap(z0 + 1, nz) * plane + m.own_off), zp[f]);
        Vec<S, V> r0;
        load_ring<S, V>(src[f], (size_t)z0 * plane, m, r0);
        stage<S, V, C>(f, lds[0][f], m, zc[f], r0);
        if (z0 + 1 < ze) load_ring<S, V>(src[f], (size_t)wrap(z0 + 1, nz) * plane, m, ring[f]);
    }
    __syncthreads();

    int buf = 0;
    for (int z = z0; z < ze; ++z) {
        // Prefetch plane z+2: own cells (needed as the z+1 neighbour next
        // plane) and ring (staged next plane for use two planes on).
        const size_t p2 = (size_t)wrap(z + 2, nz) * plane;
        if (z + 2 <= ze) {
#pragma unroll
            for (int f = 0; f < NF; ++f) pre[f] = load_vec<S, V>(src[f], p2 + m.own_off);
        }
        if (z + 2 < ze) {
#pragma unroll
            for (int f = 0; f < NF; ++f) load_ring<S, V>(src[f], p2, m, ring_next[f]);
        }

        // Neighbours of the own cells of plane z.
        C xm[NF][V], xp[NF][V], ym[NF][V], yp[NF][V];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const C *L = lds[buf][f];
#pragma unroll
            for (int i = 0; i < V; ++i) {
                xm[f][i] = i > 0 ? zc[f][i - 1] : L[m.lds_own - 1];
                xp[f][i] = i < V - 1 ? zc[f][i + 1] : L[m.lds_own + V];
                ym[f][i] = L[m.lds_own - G::RS + i];
                yp[f][i] = L[m.lds_own + G::RS + i];
            }
        }

        const size_t out_off = (size_t)z * plane + m.own_off;
        if constexpr (LAPLACE) {
            Vec<S, V> o;
#pragma unroll
            for (int i = 0; i < V; ++i)
                o.e[i] = Traits<S>::store(lap_f64(zc[0][i], xm[0][i], xp[0][i], ym[0][i], yp[0][i],
                                                  zm[0][i], zp[0][i]));
            if (m.valid) *reinterpret_cast<Vec<S, V> *>(un + out_off) = o;
        } else {
            C r[V];
            if constexpr (NOISE) {
#pragma unroll
                for (int b = 0; b < V / 4; ++b) {
                    const Philox4 w = noise_block(out_off + 4 * b, step_index(a), a.seed);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if constexpr (sizeof(C) == 8)
                            r[4 * b + j] = noise_word_f64(w.w[j]);
                        else
                            r[4 * b + j] = noise_term_f32(w.w[j], a.noise_s_f, a.noise_h_f);
                    }
                }
            }
            Vec<S, V> ou, ov;
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const C uc = zc[0][i], vc = zc[1][i];
                C lu, lv;
                if constexpr (sizeof(C) == 8) {
                    lu = lap_f64(uc, xm[0][i], xp[0][i], ym[0][i], yp[0][i], zm[0][i], zp[0][i]);
                    lv = lap_f64(vc, xm[1][i], xp[1][i], ym[1][i], yp[1][i], zm[1][i], zp[1][i]);
                } else {
                    lu = lap_f32<S>(uc, xm[0][i], xp[0][i], ym[0][i], yp[0][i], zm[0][i], zp[0][i]);
                    lv = lap_f32<S>(vc, xm[1][i], xp[1][i], ym[1][i], yp[1][i], zm[1][i], zp[1][i]);
                }
                if constexpr (sizeof(C) == 4) {
                    // the FP32 sequence shared with the blocked kernels; r is n r
                    float uo, vo;
                    euler_f32<NOISE>(a.Du_f, a.Dv_f, a.F_f, a.FK_f, a.dt_f, uc, vc, lu, lv, r[i], uo, vo);
                    ou.e[i] = fstore<S>(0, uo);
                    ov.e[i] = fstore<S>(1, vo);
                } else {
                    const C Du = Coef<C>::Du(a), Dv = Coef<C>::Dv(a), F = Coef<C>::F(a);
                    const C FK = Coef<C>::FK(a), dt = Coef<C>::dt(a);
                    const C uvv = uc * (vc * vc);
                    C du = (Du * lu - uvv) + F * ((C)1 - uc);
                    if constexpr (NOISE) du = du + Coef<C>::noise(a) * r[i];
                    const C dv = (Dv * lv + uvv) - FK * vc;
                    ou.e[i] = Traits<S>::store(uc + du * dt);
                    ov.e[i] = Traits<S>::store(vc + dv * dt);
                }
            }
            if (m.valid) {
                *reinterpret_cast<Vec<S, V> *>(un + out_off) = ou;
                *reinterpret_cast<Vec<S, V> *>(vn + out_off) = ov;
            }
        }

        // Stage plane z+1 for the next iteration, then rotate the z window.
        if (z + 1 < ze) {
#pragma unroll
            for (int f = 0; f < NF; ++f) stage<S, V, C>(f, lds[buf ^ 1][f], m, zp[f], ring[f]);
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int i = 0; i < V; ++i) {
                zm[f][i] = zc[f][i];
                zc[f][i] = zp[f][i];
            }
            widen<S, V>(f, pre[f], zp[f]);
            ring[f] = ring_next[f];
        }
        buf ^= 1;
    }
}

// ------------------------------------------------------------------ launch
template <typename S, int TX, int TY, int V, int NF, bool NOISE, bool LAPLACE>
static hipError_t launch_tile(const void *u, const void *v, void *un, void *vn, StepArgs a,
                              hipStream_t st)
{
    a.ntx = (a.nx + TX - 1) / TX;
    a.nty = (a.ny + TY - 1) / TY;
    const int nzc = (a.nz + a.zc - 1) / a.zc;
    const size_t nb = (size_t)a.ntx * a.nty * nzc;
    if (nb == 0 || nb > 0x7fffffffu) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((stencil_tile<S, TX, TY, V, NF, NOISE, LAPLACE>), dim3((unsigned)nb), dim3(256), 0, st,
                       (const S *)u, (const S *)v, (S *)un, (S *)vn, a);
    return hipGetLastError();
}

template <typename S, int TX, int TY, int V>
static hipError_t launch_step_t(const void *u, const void *v, void *un, void *vn, const StepArgs &a,
                                hipStream_t st)
{
    if (a.noise != 0.0) return launch_tile<S, TX, TY, V, 2, true, false>(u, v, un, vn, a, st);
    return launch_tile<S, TX, TY, V, 2, false, false>(u, v, un, vn, a, st);
}

// Tile table: index 1..4. V = 16 bytes of FP32 or 32 bytes of FP64 per lane
// (4 cells), 8 cells for the 16-bit types; 256 lanes per workgroup.
static const TileShape k_tiles_w4[] = {{64, 16}, {128, 8}, {32, 32}, {256, 4}};
static const TileShape k_tiles_w8[] = {{128, 16}, {64, 32}, {256, 8}, {32, 64}};

int num_tiles() { return 4; }

TileShape tile_shape(int tile, int storage)
{
    if (tile < 1 || tile > 4) return TileShape{0, 0};
    return (storage == 2 || storage == 3 || storage == 4) ? k_tiles_w8[tile - 1] : k_tiles_w4[tile - 1];
}

template <typename S>
static hipError_t dispatch_w4(int tile, const void *u, const void *v, void *un, void *vn, const StepArgs &a,
                              hipStream_t st)
{
    switch (tile) {
    case 1: return launch_step_t<S, 64, 16, 4>(u, v, un, vn, a, st);
    case 2: return launch_step_t<S, 128, 8, 4>(u, v, un, vn, a, st);
    case 3: return launch_step_t<S, 32, 32, 4>(u, v, un, vn, a, st);
    case 4: return launch_step_t<S, 256, 4, 4>(u, v, un, vn, a, st);
    }
    return hipErrorInvalidValue;
}

template <typename S>
static hipError_t dispatch_w8(int tile, const void *u, const void *v, void *un, void *vn, const StepArgs &a,
                              hipStream_t st)
{
    switch (tile) {
    case 1: return launch_step_t<S, 128, 16, 8>(u, v, un, vn, a, st);
    case 2: return launch_step_t<S, 64, 32, 8>(u, v, un, vn, a, st);
    case 3: return launch_step_t<S, 256, 8, 8>(u, v, un, vn, a, st);
    case 4: return launch_step_t<S, 32, 64, 8>(u, v, un, vn, a, st);
    }
    return hipErrorInvalidValue;
}

template <typename S, int TX, int TY, int V>
static int occ_step_t(bool noise)
{
    int n = 0;
    const hipError_t e =
        noise ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stencil_tile<S, TX, TY, V, 2, true, false>, 256, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stencil_tile<S, TX, TY, V, 2, false, false>, 256, 0);
    return e == hipSuccess && n > 0 ? n : 0;
}

template <typename S> static int occ_w4(int tile, bool noise)
{
    switch (tile) {
    case 1: return occ_step_t<S, 64, 16, 4>(noise);
    case 2: return occ_step_t<S, 128, 8, 4>(noise);
    case 3: return occ_step_t<S, 32, 32, 4>(noise);
    case 4: return occ_step_t<S, 256, 4, 4>(noise);
    }
    return 0;
}

template <typename S> static int occ_w8(int tile, bool noise)
{
    switch (tile) {
    case 1: return occ_step_t<S, 128, 16, 8>(noise);
    case 2: return occ_step_t<S, 64, 32, 8>(noise);
    case 3: return occ_step_t<S, 256, 8, 8>(noise);
    case 4: return occ_step_t<S, 32, 64, 8>(noise);
    }
    return 0;
}

int step_occupancy(int storage, int tile, bool noise)
{
    switch (storage) {
    case 0: return occ_w4<double>(tile, noise);
    case 1: return occ_w4<float>(tile, noise);
    case 2: return occ_w8<bf16>(tile, noise);
    case 3: return occ_w8<f16>(tile, noise);
    case 4: return occ_w8<bf16c>(tile, noise);
    }
    return 0;
}

hipError_t launch_step(int storage, int tile, const void *u, const void *v, void *un, void *vn,
                       const StepArgs &a, hipStream_t st)
{
    switch (storage) {
    case 0: return dispatch_w4<double>(tile, u, v, un, vn, a, st);
    case 1: return dispatch_w4<float>(tile, u, v, un, vn, a, st);
    case 2: return dispatch_w8<bf16>(tile, u, v, un, vn, a, st);
    case 3: return dispatch_w8<f16>(tile, u, v, un, vn, a, st);
    case 4: return dispatch_w8<bf16c>(tile, u, v, un, vn, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_laplacian7(const double *f, double *out, int nx, int ny, int nz, hipStream_t st)
{
    StepArgs a = {};
    a.nx = nx; a.ny = ny; a.nz = nz;
    a.zc = nz < 64 ? nz : 64;
    return launch_tile<double, 64, 16, 4, 1, false, true>(f, nullptr, out, nullptr, a, st);
}

} // namespace gs
