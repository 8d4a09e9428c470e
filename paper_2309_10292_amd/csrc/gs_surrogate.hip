// Learned 16-step surrogate: a 4-layer 3x3x3 circular convolution network
// (channels 4 -> 32 -> 32 -> 32 -> 2, GELU, residual output) on gfx950 with
// BF16 weights and activations and FP32 accumulation on the matrix cores.
//
// Activations are channels-last (cell-major, channels contiguous: 8 channels
// for the input layer, 32 for hidden layers), so one lane's K fragment of an
// implicit GEMM (8 consecutive channels of one neighbour cell) is one 16-byte
// load. Convolutions are implicit GEMMs with M = cells (tiles of 16 cells of
// one x-row), N = output channels (tiles of 16) and K = 27 offsets x input
// channels, walked in chunks of 32 with v_mfma_f32_16x16x32_bf16; the packed
// weights of a layer sit in LDS. The data gradient is the same convolution
// with the weights transposed and the offsets mirrored; the weight gradient
// is a GEMM with K = cells, reduced per workgroup into FP32 partials.
#include "gs_device.hpp"
#include "gs_surrogate.hpp"

namespace gs {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ u16 f2bf(float f) { return bf16_rne(f).bits; }

// erf by Abramowitz and Stegun 7.1.26 (Hastings' rational approximation,
// |error| <= 1.5e-7, far below the BF16 rounding of the activations),
// without branches; e receives exp(-x^2), which the GELU's derivative reuses.
__device__ __forceinline__ float erf_as(float x, float &e)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, ax, 1.0f));
    float p = __builtin_fmaf(1.061405429f, t, -1.453152027f);
    p = __builtin_fmaf(p, t, 1.421413741f);
    p = __builtin_fmaf(p, t, -0.284496736f);
    p = __builtin_fmaf(p, t, 0.254829592f);
    p *= t;
    e = __expf(-ax * ax);
    return copysignf(__builtin_fmaf(-p, e, 1.0f), x);
}

// GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 and its derivative
// Phi(z) + z phi(z), phi(z) = exp(-z^2 / 2) / sqrt(2 pi).
__device__ __forceinline__ float gelu(float z)
{
    float e;
    return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f, e));
}
__device__ __forceinline__ float gelu_grad(float z)
{
    float e;
    const float er = erf_as(z * 0.70710678118654752f, e);
    return __builtin_fmaf(0.5f, 1.0f + er, z * e * 0.39894228040143268f);
}

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ bf16x8 load8(const u16 *p)
{
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, q);
}

// ------------------------------------------------------------------ convolution
// MODE_HIDDEN: z = acc + bias, writes z and GELU(z) (32 channels, BF16).
// MODE_ACT:    the same, writing GELU(z) only (inference keeps no z).
// MODE_OUT:    pred = residual input + acc + bias for output channels 0, 1.
// MODE_DGRAD:  writes acc * GELU'(zprev) (the gradient of the layer below's
//              pre-activation, 32 channels, BF16).
//
// A workgroup (4 wavefronts) owns a patch of 16 x-cells by 4 y-rows of one
// sample and marches through a chunk of z planes; wavefront w computes row w
// (one 16-cell M tile per plane). The input planes z-1, z, z+1 of the patch
// with a one-cell ring (18 x 6 cells) sit in an LDS ring of three planes next
// to the packed weights, so every input value is fetched from L2 once per
// chunk instead of once per offset; the plane z+2 is loaded into registers
// while plane z is computed. Every MFMA operand is read from LDS: the ring is
// stored channel group major so that a fragment read is 256 contiguous bytes
// per 16 lanes (no bank conflicts), and the K loop keeps its reads a few
// chunks ahead of the MFMAs that use them.
constexpr int PX = 16, PY = 4;               // patch (x, y)
constexpr int RX = PX + 2, RY = PY + 2;      // ring plane (x, y)
constexpr int RCELLS = RX * RY;              // cells per ring plane

template <int CIN, int NT, int MODE, typename IO>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a)
{
    constexpr int NCH = (27 * CIN + 31) / 32;
    constexpr int VPC = CIN / 8;              // 16-byte vectors per cell
    // Ring layout: channel group major, cells contiguous within a group, so
    // the 16 lanes of a channel group read 16 consecutive cells (256
    // contiguous bytes, free of bank conflicts); each group's cells are padded
    // to a multiple of 16 vectors (256 bytes).
    constexpr int GCELLS = (RCELLS + 15) / 16 * 16;
    constexpr int PLANE_V = GCELLS * VPC;     // 16-byte vectors per ring plane
    constexpr int LOAD_V = RCELLS * VPC;      // vectors loaded per plane
    constexpr int LOADS = (LOAD_V + 255) / 256;
    // ring position of loaded vector v (cell v / VPC, channel group v % VPC)
    auto ring_pos = [](int v) { return (v % VPC) * GCELLS + v / VPC; };
    __shared__ uint4 wl[NCH * NT * 64];
    __shared__ uint4 ring[3 * PLANE_V];
    const uint4 *wg = reinterpret_cast<const uint4 *>(a.wpack);
    for (int i = threadIdx.x; i < NCH * NT * 64; i += 256) wl[i] = wg[i];

    const Geo g = a.geo;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, quad = lane >> 4;
    const int tx = g.nx / PX, ty = (g.ny + PY - 1) / PY, tzc = (g.nz + a.zc - 1) / a.zc;
    int b = blockIdx.x;
    const int bx = b % tx;
    b /= tx;
    const int by = b % ty;
    b /= ty;
    const int bz = b % tzc;
    const int s = b / tzc;
    const int x0 = bx * PX, y0 = by * PY, z0 = bz * a.zc;
    const int ze = min(z0 + a.zc, g.nz);
    const size_t sbase = (size_t)s * g.ncell;

    // global address of ring vector v (cell (rx, ry) of plane z, channel group cg)
    auto ring_src = [&](int v, int z) -> const uint4 * {
        const int cell = v / VPC, cg = v % VPC;
        const int rx = cell % RX, ry = cell / RX;
        const int gx = wrapc(x0 + rx - 1, g.nx), gy = wrapc(y0 + ry - 1, g.ny), gz = wrapc(z, g.nz);
        const size_t row = sbase + (size_t)gx + (size_t)g.nx * ((size_t)gy + (size_t)g.ny * gz);
        return reinterpret_cast<const uint4 *>(a.in + row * CIN) + cg;
    };
    for (int p = 0; p < 3; ++p) {
        const int z = z0 - 1 + p; // ring slot of plane z is (z mod 3)
        const int slot = ((z % 3) + 3) % 3;
        for (int v = threadIdx.x; v < LOAD_V; v += 256) ring[slot * PLANE_V + ring_pos(v)] = *ring_src(v, z);
    }
    __syncthreads();

    // One output-channel tile with 32 input channels (the output layer): its
    // 27 weight fragments stay in registers, so the K loop reads only the
    // activation fragments from LDS.
    constexpr bool WREG = CIN == 32 && NT == 1;
    bf16x8 wreg[WREG ? 27 : 1];
    if constexpr (WREG) {
#pragma unroll
        for (int c = 0; c < 27; ++c) wreg[c] = __builtin_bit_cast(bf16x8, wl[c * 64 + lane]);
    }

    const int yrow = y0 + wave;
    const bool row_ok = yrow < g.ny;
    for (int z = z0; z < ze; ++z) {
        // prefetch plane z+2 (needed from the next plane on); every lane loads
        // an in-range vector (indices clamped) and only the LDS store is masked
        const bool more = z + 1 < ze;
        static_assert(LOADS <= 2, "a ring plane is at most two vectors per lane");
        const uint4 pre0 = *ring_src(min((int)threadIdx.x, LOAD_V - 1), z + 2);
        const uint4 pre1 = LOADS > 1 ? *ring_src(min((int)threadIdx.x + 256, LOAD_V - 1), z + 2) : pre0;
        f32x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        // A = weights (rows: output channels), B = activations (columns:
        // cells), so a lane's accumulators are 4 consecutive output channels
        // of one cell.
        if constexpr (CIN == 32) {
            // K chunk c is offset d = c with all 32 input channels. The 27
            // chunks are unrolled with the fragments of the next KD chunks in
            // flight (a register ring), so each MFMA's LDS reads were issued
            // KD chunks earlier.
            constexpr int KD = 3;
            bf16x8 avr[KD], wvr[KD][NT];
            auto load = [&](int c, int sl) {
                const int dz = c / 9, dy = (c / 3) % 3, dx = c % 3;
                const uint4 *rs = ring + ((z + dz + 2) % 3) * PLANE_V; // slot of plane z + dz - 1
                avr[sl] = __builtin_bit_cast(bf16x8, rs[quad * GCELLS + (wave + dy) * RX + col + dx]);
                if constexpr (!WREG) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) wvr[sl][t] = __builtin_bit_cast(bf16x8, wl[(c * NT + t) * 64 + lane]);
                }
            };
#pragma unroll
            for (int c = 0; c < KD; ++c) load(c, c);
#pragma unroll
            for (int c = 0; c < 27; ++c) {
                const int sl = c % KD;
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(WREG ? wreg[c] : wvr[sl][t], avr[sl], acc[t], 0, 0, 0);
                if (c + KD < 27) load(c + KD, sl);
                // keep the reads KD chunks ahead of their MFMAs
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll 9
            for (int c = 0; c < NCH; ++c) {
                const int k0 = 32 * c + 8 * quad;
                const int d = k0 / CIN, ci0 = k0 % CIN;
                bf16x8 av;
                if (d < 27) {
                    const int dz = d / 9, dy = (d / 3) % 3, dx = d % 3;
                    const int slot = (((z + dz - 1) % 3) + 3) % 3;
                    const int cell = (wave + dy) * RX + col + dx;
                    av = __builtin_bit_cast(bf16x8, ring[slot * PLANE_V + (ci0 / 8) * GCELLS + cell]);
                } else {
                    av = __builtin_bit_cast(bf16x8, uint4{0u, 0u, 0u, 0u});
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const bf16x8 wv = __builtin_bit_cast(bf16x8, wl[(c * NT + t) * 64 + lane]);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv, av, acc[t], 0, 0, 0);
                }
            }
        }
        // acc[t][j]: output channel 16 t + 4 quad + j of cell (x0 + col, yrow, z).
        const size_t r = sbase + (size_t)(x0 + col) + (size_t)g.nx * ((size_t)yrow + (size_t)g.ny * z);
        if (row_ok) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int co0 = 16 * t + 4 * quad;
                if constexpr (MODE == MODE_HIDDEN) {
                    uint2 zq, aq;
                    u16 zb[4], ab[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float zz = acc[t][j] + a.bias[co0 + j];
                        zb[j] = f2bf(zz);
                        ab[j] = f2bf(gelu(zz));
                    }
                    zq.x = (uint32_t)zb[0] | ((uint32_t)zb[1] << 16);
                    zq.y = (uint32_t)zb[2] | ((uint32_t)zb[3] << 16);
                    aq.x = (uint32_t)ab[0] | ((uint32_t)ab[1] << 16);
                    aq.y = (uint32_t)ab[2] | ((uint32_t)ab[3] << 16);
                    *reinterpret_cast<uint2 *>(a.zout + r * 32 + co0) = zq;
                    *reinterpret_cast<uint2 *>(a.aout + r * 32 + co0) = aq;
                } else if constexpr (MODE == MODE_ACT) {
                    u16 ab[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) ab[j] = f2bf(gelu(acc[t][j] + a.bias[co0 + j]));
                    *reinterpret_cast<uint2 *>(a.aout + r * 32 + co0) =
                        uint2{(uint32_t)ab[0] | ((uint32_t)ab[1] << 16), (uint32_t)ab[2] | ((uint32_t)ab[3] << 16)};
                } else if constexpr (MODE == MODE_OUT) {
                    if (quad == 0) {
                        // r = s * ncell + cell indexes the planar (sample, cell) fields
                        const IO *ru = (const IO *)a.res_u, *rv = (const IO *)a.res_v;
                        ((IO *)a.out_u)[r] = ru[r] + (IO)(acc[t][0] + a.bias[0]);
                        ((IO *)a.out_v)[r] = rv[r] + (IO)(acc[t][1] + a.bias[1]);
                    }
                } else {
                    const uint2 zq = *reinterpret_cast<const uint2 *>(a.zprev + r * 32 + co0);
                    const float zp[4] = {bf2f((u16)(zq.x & 0xffffu)), bf2f((u16)(zq.x >> 16)),
                                         bf2f((u16)(zq.y & 0xffffu)), bf2f((u16)(zq.y >> 16))};
                    u16 gb[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) gb[j] = f2bf(acc[t][j] * gelu_grad(zp[j]));
                    uint2 gq;
                    gq.x = (uint32_t)gb[0] | ((uint32_t)gb[1] << 16);
                    gq.y = (uint32_t)gb[2] | ((uint32_t)gb[3] << 16);
                    *reinterpret_cast<uint2 *>(a.aout + r * 32 + co0) = gq;
                }
            }
        }
        __syncthreads(); // every read of plane z-1's slot is done
        if (more) {
            const int slot = ((z + 2) % 3 + 3) % 3;
            if ((int)threadIdx.x < LOAD_V) ring[slot * PLANE_V + ring_pos(threadIdx.x)] = pre0;
            if (LOADS > 1 && (int)threadIdx.x + 256 < LOAD_V) ring[slot * PLANE_V + ring_pos(threadIdx.x + 256)] = pre1;
        }
        __syncthreads();
    }
}

// 32 -> 32 convolutions of the forward hidden layer (with or without the
// pre-activation's store) and the data gradient. A wavefront owns RW rows of
// 16 cells and both 16-channel N tiles (four accumulator chains) of one
// sample and marches through a chunk of z planes with a private LDS ring of
// three input planes (rows y-1 .. y+RW, cells x-1 .. x+16, channel group
// major), so the wavefronts of a workgroup meet at one barrier only, after
// the weights are staged. The weight fragments of the first C32_CR K chunks
// sit in registers and the other chunks' in LDS (shared by the workgroup's
// eight wavefronts), which leaves room for two wavefronts per SIMD: one
// wavefront's vector work (the epilogue, the staging) then runs beside the
// other's MFMAs. The K loop reads the activation fragments (one per row and
// K chunk for two MFMAs) and the LDS weight fragments a few chunks ahead.
// Plane z's MFMAs and plane z-1's epilogue (bias, GELU or its derivative,
// BF16 rounding) sit in one basic block. The MFMAs accumulate each output
// over the 27 K chunks in the same order as conv_kernel, so the results are
// the same bit for bit.
constexpr int C32_RW = 2, C32_WAVES = 8, C32_CR = 8;
typedef unsigned u32x4 __attribute__((ext_vector_type(4))); // a native vector (no struct copies)
template <bool B> struct BoolC {
    static constexpr bool value = B;
};
template <int MODE>
__global__ __launch_bounds__(64 * C32_WAVES) __attribute__((amdgpu_waves_per_eu(2, 2))) void conv32p_kernel(ConvArgs a)
{
    constexpr int NT = 2, NCH = 27, VPC = 4, RW = C32_RW, PYW = RW * C32_WAVES;
    constexpr int RCELLS = RX * (RW + 2);              // ring cells per plane
    constexpr int GC = (RCELLS + 15) / 16 * 16;        // cells per channel group, padded to 256 bytes
    constexpr int SLOT_V = GC * VPC;                   // 16-byte vectors per plane slot
    constexpr int LOAD_V = RCELLS * VPC;               // vectors loaded per plane
    constexpr int LOADS = (LOAD_V + 63) / 64;
    constexpr int CR = C32_CR, CL = NCH - CR;          // weight chunks in registers / in LDS
    __shared__ u32x4 ring_all[C32_WAVES * 3 * SLOT_V];
    __shared__ uint4 wl[CL * NT * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    u32x4 *ring = ring_all + wave * 3 * SLOT_V;
    auto slot3 = [](int z) { return ((z % 3) + 3) % 3; };
    const int col = lane & 15, quad = lane >> 4;
    const Geo g = a.geo;

    bf16x8 wr[CR][NT];
    {
        const uint4 *wg = reinterpret_cast<const uint4 *>(a.wpack);
#pragma unroll
        for (int c = 0; c < CR; ++c)
#pragma unroll
            for (int t = 0; t < NT; ++t) wr[c][t] = __builtin_bit_cast(bf16x8, wg[(c * NT + t) * 64 + lane]);
        for (int i = threadIdx.x; i < CL * NT * 64; i += 64 * C32_WAVES) wl[i] = wg[CR * NT * 64 + i];
    }
    __syncthreads();
    const int tx = g.nx / PX, ty = (g.ny + PYW - 1) / PYW, tzc = (g.nz + a.zc - 1) / a.zc;
    int b = blockIdx.x;
    const int bx = b % tx;
    b /= tx;
    const int by = b % ty;
    b /= ty;
    const int bz = b % tzc;
    const int s = b / tzc;
    const int x0 = bx * PX, yw = by * PYW + RW * wave, z0 = bz * a.zc;
    const int ze = min(z0 + a.zc, g.nz);
    if (yw >= g.ny) return; // a wavefront below the grid (no barriers after this point)
    const size_t sbase = (size_t)s * g.ncell, plane = (size_t)g.nx * g.ny;

    // This lane's ring vectors: offset within an input plane (in channels)
    // and ring position; the lanes past the plane load a valid vector and
    // store nothing.
    size_t goff[LOADS];
    int rpos[LOADS];
#pragma unroll
    for (int l = 0; l < LOADS; ++l) {
        const int v = min(lane + 64 * l, LOAD_V - 1);
        const int cell = v / VPC, cg = v % VPC;
        const int rx = cell % RX, ry = cell / RX;
        int gy = yw + ry - 1;
        if (gy < 0) gy += g.ny;
        while (gy >= g.ny) gy -= g.ny;
        const int gx = wrapc(x0 + rx - 1, g.nx);
        goff[l] = ((size_t)gx + (size_t)g.nx * gy) * 32 + cg * 8;
        // lanes past the plane store into the padding cells of channel group 3
        rpos[l] = lane + 64 * l < LOAD_V ? cg * GC + cell : 3 * GC + RCELLS + (lane & (GC - RCELLS - 1));
    }
    auto load_plane = [&](int z, u32x4 (&o)[LOADS]) __attribute__((always_inline)) {
        const uint16_t *base = a.in + (sbase + (size_t)wrapc(z, g.nz) * plane) * 32;
#pragma unroll
        for (int l = 0; l < LOADS; ++l) o[l] = *reinterpret_cast<const u32x4 *>(base + goff[l]);
    };
    auto stage_plane = [&](int z, const u32x4 (&o)[LOADS]) __attribute__((always_inline)) {
        u32x4 *dst = ring + slot3(z) * SLOT_V;
#pragma unroll
        for (int l = 0; l < LOADS; ++l) dst[rpos[l]] = o[l];
    };
    // Epilogue values: the lane's biases are read once (the compiler cannot
    // move their loads past the output stores).
    float bias_r[NT][4] = {};
    if constexpr (MODE == MODE_HIDDEN || MODE == MODE_ACT) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) bias_r[t][j] = a.bias[16 * t + 4 * quad + j];
    }
    auto cell_of = [&](int r, int z) __attribute__((always_inline)) {
        const int yrow = min(yw + r, g.ny - 1);
        return sbase + (size_t)(x0 + col) + (size_t)g.nx * ((size_t)yrow + (size_t)g.ny * wrapc(z, g.nz));
    };
    // One plane: start loading plane z+2, run the 27 K chunks of plane z,
    // then stage plane z+2 into the ring; with PREV, the
    // previous plane's 16 epilogue values (2 rows x 2 tiles x 4 channels) are
    // computed one per chunk beside its MFMAs, and stored at the end.
    auto plane_step = [&](auto prev, int z, f32x4 (&acc)[RW][NT], const f32x4 (&accp)[RW][NT], u32x4 (&pre)[LOADS]) __attribute__((always_inline)) {
        constexpr bool PREV = decltype(prev)::value;
        load_plane(z + 2, pre);
        uint2 zq[RW][NT];
        if constexpr (PREV && MODE == MODE_DGRAD) {
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    zq[r][t] = *reinterpret_cast<const uint2 *>(a.zprev + cell_of(r, z - 1) * 32 + 16 * t + 4 * quad);
        }
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        constexpr int KD = 3;
        bf16x8 av[KD][RW], wv[KD][NT];
        auto frag = [&](int c, int sl) __attribute__((always_inline)) {
            const int dz = c / 9, dy = (c / 3) % 3, dx = c % 3;
            const u32x4 *rs = ring + slot3(z + dz - 1) * SLOT_V + quad * GC;
#pragma unroll
            for (int r = 0; r < RW; ++r) av[sl][r] = __builtin_bit_cast(bf16x8, rs[(r + dy) * RX + col + dx]);
            if (c >= CR) {
#pragma unroll
                for (int t = 0; t < NT; ++t) wv[sl][t] = __builtin_bit_cast(bf16x8, wl[((c - CR) * NT + t) * 64 + lane]);
            }
        };
#pragma unroll
        for (int c = 0; c < KD; ++c) frag(c, c);
        u16 e1[RW][NT][4], e2[RW][NT][4];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int sl = c % KD;
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < RW; ++r)
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c < CR ? wr[c < CR ? c : 0][t] : wv[sl][t], av[sl][r],
                                                                        acc[r][t], 0, 0, 0);
            if (c + KD < NCH) frag(c + KD, sl);
            if constexpr (PREV) {
                if (c < RW * NT * 4) {
                    const int r = c / (NT * 4), t = (c / 4) % NT, j = c % 4;
                    // the empty asm keeps each value's arithmetic at this chunk
                    // (pure arithmetic would otherwise sink to the stores)
                    if constexpr (MODE == MODE_HIDDEN) {
                        float zz = accp[r][t][j] + bias_r[t][j];
                        float gz = gelu(zz);
                        asm volatile("" : "+v"(zz), "+v"(gz));
                        e1[r][t][j] = f2bf(zz);
                        e2[r][t][j] = f2bf(gz);
                    } else if constexpr (MODE == MODE_ACT) {
                        float gz = gelu(accp[r][t][j] + bias_r[t][j]);
                        asm volatile("" : "+v"(gz));
                        e1[r][t][j] = f2bf(gz);
                    } else {
                        const uint32_t w = j < 2 ? zq[r][t].x : zq[r][t].y;
                        const float zp = bf2f((u16)((j & 1) ? (w >> 16) : (w & 0xffffu)));
                        float gd = accp[r][t][j] * gelu_grad(zp);
                        asm volatile("" : "+v"(gd));
                        e1[r][t][j] = f2bf(gd);
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // plane z+2 into its slot (last read as plane z-2), before the stores
        // so that the wait for its loads does not also wait for them
        stage_plane(z + 2, pre);
        if constexpr (PREV) {
            // rows last to first: a row past the grid (only when ny is odd) is
            // clamped onto row 0's cell, whose own store then follows it
#pragma unroll
            for (int r = RW - 1; r >= 0; --r) {
                const size_t cell = cell_of(r, z - 1);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int co0 = 16 * t + 4 * quad;
                    const uint2 q1{(uint32_t)e1[r][t][0] | ((uint32_t)e1[r][t][1] << 16),
                                   (uint32_t)e1[r][t][2] | ((uint32_t)e1[r][t][3] << 16)};
                    if constexpr (MODE == MODE_HIDDEN) {
                        const uint2 q2{(uint32_t)e2[r][t][0] | ((uint32_t)e2[r][t][1] << 16),
                                       (uint32_t)e2[r][t][2] | ((uint32_t)e2[r][t][3] << 16)};
                        *reinterpret_cast<uint2 *>(a.zout + cell * 32 + co0) = q1;
                        *reinterpret_cast<uint2 *>(a.aout + cell * 32 + co0) = q2;
                    } else {
                        *reinterpret_cast<uint2 *>(a.aout + cell * 32 + co0) = q1;
                    }
                }
            }
        }
    };
    // The last plane's epilogue on its own.
    auto last_epilogue = [&](int z, const f32x4 (&accp)[RW][NT]) __attribute__((always_inline)) {
#pragma unroll
        for (int r = RW - 1; r >= 0; --r) {
            const size_t cell = cell_of(r, z);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int co0 = 16 * t + 4 * quad;
                u16 e1[4], e2[4];
                if constexpr (MODE == MODE_HIDDEN) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float zz = accp[r][t][j] + bias_r[t][j];
                        e1[j] = f2bf(zz);
                        e2[j] = f2bf(gelu(zz));
                    }
                    *reinterpret_cast<uint2 *>(a.zout + cell * 32 + co0) =
                        uint2{(uint32_t)e1[0] | ((uint32_t)e1[1] << 16), (uint32_t)e1[2] | ((uint32_t)e1[3] << 16)};
                    *reinterpret_cast<uint2 *>(a.aout + cell * 32 + co0) =
                        uint2{(uint32_t)e2[0] | ((uint32_t)e2[1] << 16), (uint32_t)e2[2] | ((uint32_t)e2[3] << 16)};
                } else if constexpr (MODE == MODE_ACT) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) e1[j] = f2bf(gelu(accp[r][t][j] + bias_r[t][j]));
                    *reinterpret_cast<uint2 *>(a.aout + cell * 32 + co0) =
                        uint2{(uint32_t)e1[0] | ((uint32_t)e1[1] << 16), (uint32_t)e1[2] | ((uint32_t)e1[3] << 16)};
                } else {
                    const uint2 zq = *reinterpret_cast<const uint2 *>(a.zprev + cell * 32 + co0);
                    const float zp[4] = {bf2f((u16)(zq.x & 0xffffu)), bf2f((u16)(zq.x >> 16)),
                                         bf2f((u16)(zq.y & 0xffffu)), bf2f((u16)(zq.y >> 16))};
#pragma unroll
                    for (int j = 0; j < 4; ++j) e1[j] = f2bf(accp[r][t][j] * gelu_grad(zp[j]));
                    *reinterpret_cast<uint2 *>(a.aout + cell * 32 + co0) =
                        uint2{(uint32_t)e1[0] | ((uint32_t)e1[1] << 16), (uint32_t)e1[2] | ((uint32_t)e1[3] << 16)};
                }
            }
        }
    };

    u32x4 pre[LOADS];
    {
        u32x4 q[LOADS];
        for (int p = -1; p <= 1; ++p) {
            load_plane(z0 + p, q);
            stage_plane(z0 + p, q);
        }
    }
    f32x4 accA[RW][NT], accB[RW][NT];
    plane_step(BoolC<false>{}, z0, accA, accB, pre);
    int z = z0 + 1;
    for (; z + 1 < ze; z += 2) {
        plane_step(BoolC<true>{}, z, accB, accA, pre);
        plane_step(BoolC<true>{}, z + 1, accA, accB, pre);
    }
    if (z < ze) {
        plane_step(BoolC<true>{}, z, accB, accA, pre);
        last_epilogue(z, accB);
    } else {
        last_epilogue(ze - 1, accA);
    }
}
// Planes per workgroup of conv32p_kernel: one workgroup of eight wavefronts
// fills a CU (its registers and LDS), so the chunk is the longest that still
// gives at least two workgroups per CU, which amortises the weights' load and
// the ring's first planes.
int conv32p_zc(const Geo &g, int nsamp)
{
    const size_t cols = (size_t)(g.nx / PX) * ((g.ny + C32_RW * C32_WAVES - 1) / (C32_RW * C32_WAVES)) * (size_t)nsamp;
    int zc = 1;
    while (zc < g.nz) zc *= 2;
    while (zc > 4 && cols * ((g.nz + zc - 1) / zc) < 512) zc /= 2;
    return zc;
}

// ------------------------------------------------------------------ weight gradient
// dW[d][co][ci] = sum over cells of dz[cell][co] * act[cell + d][ci]: for each
// of the 27 offsets d a product A B with A = dz^T (rows co, K = cells) and
// B = act shifted by d (K = cells, columns ci), on 16x16x32 MFMAs whose K runs
// over 32 cells (two rows of 16).
//
// The workgroups are persistent: each walks work items (a patch of 16 x-cells
// by TR y-rows of one sample, through a chunk of WG_ZC planes) and keeps its
// sums in registers. TR is 8 for the layers with 32 input channels, whose
// staging of 32-channel activation planes costs the most: 8 rows load 10
// activation rows per 8 instead of 6 per 4 (the 32 -> 8 layer then runs one
// workgroup per CU, for its registers); the 8 -> 32 layer keeps 4. Act plane p
// meets dz planes p + 1, p and p - 1 (z offsets -1, 0, +1), so the loop runs
// over act planes: while plane p is in LDS, the dz fragments of the three
// planes it meets are held in registers, and every B fragment read from LDS
// feeds three MFMAs, one per z offset (a third of the LDS reads of a loop that
// takes the offsets one by one). For each offset the planes are still added in
// increasing z. Both operands stay channels-last in LDS, as in memory (16-byte
// chunks, no transposes on the way in): a fragment (8 cells of one channel per
// lane) is two transposing LDS reads. Cells 8 .. 15 of every 16 have their
// channel halves swapped (rows of 32 channels) or are moved 4 cells over (rows
// of 16), so that the two 16-lane groups of a half-wave read distinct banks.
//
// Wave w owns one 16 x 16 output tile (co x ci) for all 27 offsets: with four
// tiles (32 -> 32) for all K chunks of a plane (two rows of 16 cells each),
// with two tiles two waves share a tile, split the K chunks, and add their sums
// at the end. Staging is double-buffered with one barrier per plane: act plane
// p + 2 and dz plane p + 3 are loaded into registers while plane p is
// multiplied and stored into the free buffers at the start of the next plane.
// The bias gradient (the sum of dz over cells) is accumulated while dz is
// staged. Each workgroup writes its partial sums (padded 16*MT x 16*NT per
// offset, and 32 bias sums) once.
constexpr int WG_ZC = 64;

typedef short v4s __attribute__((ext_vector_type(4)));

// Offset (16-bit units) of channel ch of cell `cell` in an LDS row of
// channels-last cells of NC channels, with the bank swizzle described above.
template <int NC>
__device__ __forceinline__ int wg_pos(int cell, int ch)
{
    static_assert(NC == 16 || NC == 32, "rows of 16 or 32 channels");
    if constexpr (NC == 32)
        return cell * 32 + (ch ^ ((cell & 8) << 1));
    else
        return (cell ^ ((cell >> 1) & 4)) * 16 + ch;
}

// MFMA operand of cells cell0 .. cell0 + 7 and channels c0 .. c0 + 15 (one per
// lane of a 16-lane group) from an LDS row. In each group of 16 lanes the
// transposing read concatenates the 8-byte pieces the lanes address, in lane
// order, into 64 values X and hands lane t the values X[t], X[t + 16],
// X[t + 32] and X[t + 48]; so lane L addresses cell L / 4 (then 4 + L / 4)
// at channels c0 + 4 (L % 4) .. + 3, and receives channel c0 + L of the
// 8 cells.
template <int NC>
__device__ __forceinline__ bf16x8 frag_tr(const u16 *row, int cell0, int c0, int lane16)
{
    const int cell = cell0 + (lane16 >> 2), ch = c0 + 4 * (lane16 & 3);
    typedef __attribute__((address_space(3))) v4s *lds_v4s;
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(row + wg_pos<NC>(cell, ch)));
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(row + wg_pos<NC>(cell + 4, ch)));
    const v4s v[2] = {lo, hi};
    return __builtin_bit_cast(bf16x8, v);
}

// Workgroup barrier that waits for the wave's LDS operations only: global
// loads in flight (the next planes' staging) stay in flight across it.
__device__ __forceinline__ void wg_lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F); // lgkmcnt(0); vmcnt and expcnt not waited
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
template <int CIN, int COUTS, int MT, int NT, int TR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void wgrad_kernel(WgradArgs a)
{
    constexpr int NCI = 16 * NT, NCO = 16 * MT;
    constexpr int NCG = CIN / 8, NCGZ = COUTS / 8;
    constexpr int KS = MT * NT == 4 ? 1 : 2; // waves per output tile (splitting the K chunks)
    constexpr int NKC = TR / 2 / KS;         // K chunks (two rows of 16 cells) per wave and plane
    static_assert(TR % (2 * KS) == 0, "whole K chunks per wave");
    static_assert(MT * NT * KS == 4, "four waves");
    constexpr int AROW = (18 * NCI * 2 + 255) / 256 * 256 / 2; // u16 per act row: cells x0 - 1 .. x0 + 16
    constexpr int APL = (TR + 2) * AROW;                        // act rows y0 - 1 .. y0 + TR
    constexpr int DROW = 16 * NCO, DPL = TR * DROW;             // dz rows y0 .. y0 + TR - 1
    constexpr int T_ACT = (TR + 2) * 18 * NCG, RA = (T_ACT + 255) / 256; // 16-byte chunks of an act plane
    constexpr int T_DZ = TR * 16 * NCGZ;                                  // and of a dz plane
    constexpr int RD = (T_DZ + 255) / 256, TDL = T_DZ < 256 ? T_DZ : 256; // dz chunks per lane, lanes staging dz
    static_assert(T_DZ <= 256 || T_DZ % 256 == 0, "whole dz rounds");
    __shared__ __align__(16) u16 act_l[2 * APL];
    __shared__ __align__(16) u16 dz_l[2 * DPL];
    __shared__ float bsum_l[TDL][8];
    __shared__ float red_l[KS == 2 ? 2 * 27 * 4 * 64 : 1];
    const Geo g = a.geo;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, quad = lane >> 4;
    const int tile = KS == 1 ? wave : (wave & 1);
    const int mw = MT == 1 ? 0 : (NT == 1 ? tile : tile >> 1);
    const int nw = NT == 1 ? 0 : (MT == 1 ? tile : tile & 1);
    const int kc0 = KS == 1 ? 0 : (wave >> 1) * NKC;

    // Channels past CIN / COUTS stay zero.
    for (int e = tid; e < 2 * APL; e += 256) act_l[e] = 0;
    for (int e = tid; e < 2 * DPL; e += 256) dz_l[e] = 0;
    __syncthreads();

    f32x4 acc[27];
#pragma unroll
    for (int d = 0; d < 27; ++d) acc[d] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bs[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) bs[c] = 0.f;

    const int ntx = g.nx / 16, nty = (g.ny + TR - 1) / TR, ntz = (g.nz + WG_ZC - 1) / WG_ZC;
    const int nitems = ntx * nty * ntz * a.nsamp;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int r = it;
        const int tx = r % ntx;
        r /= ntx;
        const int ty = r % nty;
        r /= nty;
        const int tz = r % ntz;
        const int smp = r / ntz;
        const int x0 = tx * 16, y0 = ty * TR, z0 = tz * WG_ZC, ze = min(z0 + WG_ZC, g.nz);
        const size_t sbase = (size_t)smp * g.ncell;

        // Per item, each lane's staging chunks sit at fixed offsets within a
        // plane (global) and within a buffer (LDS); a plane adds its offset.
        // Chunk v of an act plane: channel group v % NCG of cell (v / NCG) % 18
        // (x0 - 1 + cell) in row v / (18 NCG) (y0 - 1 + row); chunk t of a dz
        // plane (lanes t < T_DZ): group t % NCGZ, cell (t / NCGZ) % 16, row
        // t / (16 NCGZ) (rows past ny contribute zero). Plane p goes to buffer p & 1.
        const size_t plane_a = (size_t)g.ny * g.nx * CIN, plane_d = (size_t)g.ny * g.nx * COUTS;
        const u16 *act_s = a.act + sbase * CIN, *dz_s = a.dz + sbase * COUTS;
        size_t goff_a[RA];
        int loff_a[RA];
#pragma unroll
        for (int k = 0; k < RA; ++k) {
            const int v = min(tid + 256 * k, T_ACT - 1);
            const int cg = v % NCG, cell = (v / NCG) % 18, row = v / (18 * NCG);
            const int x = wrapc(x0 + cell - 1, g.nx), y = wrapc(y0 + row - 1, g.ny);
            goff_a[k] = ((size_t)y * g.nx + x) * CIN + 8 * cg;
            loff_a[k] = row * AROW + wg_pos<NCI>(cell, 8 * cg);
        }
        // lanes with nothing to stage load a valid chunk of the plane and keep zero
        bool dz_lane[RD], dz_in[RD];
        size_t goff_d[RD];
        int loff_d[RD];
#pragma unroll
        for (int r = 0; r < RD; ++r) {
            const int t = tid + 256 * r;
            const int dcg = t % NCGZ, dcell = (t / NCGZ) % 16, drow = t / (16 * NCGZ);
            dz_lane[r] = t < T_DZ;
            dz_in[r] = dz_lane[r] && y0 + drow < g.ny;
            goff_d[r] = dz_in[r] ? ((size_t)(y0 + drow) * g.nx + x0 + dcell) * COUTS + 8 * dcg : (size_t)x0 * COUTS;
            loff_d[r] = drow * DROW + wg_pos<NCO>(dcell, 8 * dcg);
        }

        uint4 qa[RA], qd[RD];
        auto load_act = [&](int p) {
            const u16 *src = act_s + (size_t)wrapc(p, g.nz) * plane_a;
#pragma unroll
            for (int k = 0; k < RA; ++k) qa[k] = *reinterpret_cast<const uint4 *>(src + goff_a[k]);
        };
        auto store_act = [&](int p) {
            u16 *pl = act_l + (p & 1) * APL;
#pragma unroll
            for (int k = 0; k < RA; ++k)
                if (tid + 256 * k < T_ACT) *reinterpret_cast<uint4 *>(pl + loff_a[k]) = qa[k];
        };
        auto load_dz = [&](int z) {
#pragma unroll
            for (int r = 0; r < RD; ++r) {
                const uint4 t = *reinterpret_cast<const uint4 *>(dz_s + (size_t)z * plane_d + goff_d[r]);
                qd[r] = dz_in[r] ? t : uint4{0u, 0u, 0u, 0u};
            }
        };
        auto store_dz = [&](int z) {
#pragma unroll
            for (int r = 0; r < RD; ++r)
                if (dz_lane[r]) { // chunk r of this lane: channel group tid % NCGZ, as every r
                    const uint32_t *w = reinterpret_cast<const uint32_t *>(&qd[r]);
#pragma unroll
                    for (int c = 0; c < 8; ++c) bs[c] += bf2f((u16)((c & 1) ? (w[c >> 1] >> 16) : (w[c >> 1] & 0xffffu)));
                    *reinterpret_cast<uint4 *>(dz_l + (z & 1) * DPL + loff_d[r]) = qd[r];
                }
        };
        // dz fragments (K chunk kc0 + c) of planes p - 1, p, p + 1
        bf16x8 am[NKC], a0[NKC], ap[NKC];
#pragma unroll
        for (int c = 0; c < NKC; ++c) am[c] = a0[c] = ap[c] = bf16x8{};

        // B fragments of offset (dyo, dxo) from act plane p meet dz planes
        // p + 1 (z offset -1), p (0) and p - 1 (+1); the fragments of planes
        // outside [z0, ze) are zero (one code path: the two planes around a
        // chunk cost 2 / WG_ZC more MFMAs, adding exact zeros).
        auto mult = [&](int p) {
            const u16 *pl = act_l + (p & 1) * APL;
            auto read_b = [&](int e, bf16x8 *b) {
                const int dyo = e / 3 - 1, dxo = e % 3 - 1;
#pragma unroll
                for (int c = 0; c < NKC; ++c)
                    b[c] = frag_tr<NCI>(pl + (2 * (kc0 + c) + (quad >> 1) + dyo + 1) * AROW, 8 * (quad & 1) + dxo + 1, 16 * nw, col);
            };
            // the reads of offset pair e + LA are issued before the MFMAs of
            // pair e, and no earlier: LA + 1 pairs of B fragments are live
            // (fewer where a wave takes more K chunks, for the registers)
            constexpr int LA = NKC == 1 ? 3 : NKC == 2 ? 2 : 1;
            bf16x8 b[LA + 1][NKC];
#pragma unroll
            for (int e = 0; e < LA; ++e) read_b(e, b[e]);
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                if (e + LA < 9) read_b(e + LA, b[(e + LA) % (LA + 1)]);
#pragma unroll
                for (int c = 0; c < NKC; ++c) {
                    const bf16x8 bv = b[e % (LA + 1)][c];
                    acc[e] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[c], bv, acc[e], 0, 0, 0);
                    acc[9 + e] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[c], bv, acc[9 + e], 0, 0, 0);
                    acc[18 + e] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[c], bv, acc[18 + e], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        };

        // When plane p is multiplied the registers hold act plane p + 1 and
        // dz plane p + 2, loaded during plane p - 1. Every plane issues the
        // same loads (plane indices clamped to the chunk) and the barrier
        // waits for LDS operations only, so the loads stay in flight across
        // it until their stores.
        load_act(z0 - 1);
        load_dz(z0);
        store_act(z0 - 1);
        store_dz(z0);
        load_act(z0);
        load_dz(min(z0 + 1, ze - 1));
        __syncthreads();
        for (int p = z0 - 1; p <= ze; ++p) {
            if (p + 1 <= ze) store_act(p + 1);
            if (p + 2 < ze) store_dz(p + 2);
            if (p + 1 < ze) {
                const u16 *dl = dz_l + ((p + 1) & 1) * DPL;
#pragma unroll
                for (int c = 0; c < NKC; ++c)
                    ap[c] = frag_tr<NCO>(dl + (2 * (kc0 + c) + (quad >> 1)) * DROW, 8 * (quad & 1), 16 * mw, col);
            } else {
#pragma unroll
                for (int c = 0; c < NKC; ++c) ap[c] = bf16x8{};
            }
            load_act(min(p + 2, ze));
            load_dz(min(p + 3, ze - 1));
            mult(p);
            wg_lds_barrier();
#pragma unroll
            for (int c = 0; c < NKC; ++c) {
                am[c] = a0[c];
                a0[c] = ap[c];
            }
        }
        __syncthreads(); // the loads issued past the chunk's end have landed
    }

    // Bias partials: dz staging lane t summed channels 8 (t % NCGZ) + c (of
    // every chunk it stages); fold the lanes of each channel in lane order.
    if (tid < TDL)
#pragma unroll
        for (int c = 0; c < 8; ++c) bsum_l[tid][c] = bs[c];
    if constexpr (KS == 2) {
        // the waves of the second K chunk hand their sums to those of the first
        if (wave >= 2)
#pragma unroll
            for (int d = 0; d < 27; ++d)
#pragma unroll
                for (int j = 0; j < 4; ++j) red_l[(((wave & 1) * 27 + d) * 4 + j) * 64 + lane] = acc[d][j];
    }
    __syncthreads();
    if (tid < COUTS) {
        float t = 0.f;
        for (int l = tid / 8; l < TDL; l += NCGZ) t += bsum_l[l][tid % 8];
        a.bpart[(size_t)blockIdx.x * 32 + tid] = t;
    }
    if (KS == 2 && wave >= 2) return;
    if constexpr (KS == 2) {
#pragma unroll
        for (int d = 0; d < 27; ++d)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[d][j] += red_l[(((wave & 1) * 27 + d) * 4 + j) * 64 + lane];
    }
    // acc[d][j]: co = 16 mw + 4 quad + j, ci = 16 nw + col
    constexpr int PCO = 16 * MT, PCI = 16 * NT;
    float *part = a.part + (size_t)blockIdx.x * 27 * PCO * PCI;
#pragma unroll
    for (int d = 0; d < 27; ++d)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[((size_t)d * PCO + 16 * mw + 4 * quad + j) * PCI + 16 * nw + col] = acc[d][j];
}

// grad[W(co, ci, d)] = sum over workgroups of the partials; the first
// lo_pairs input channels add the partials of their low parts (stored
// channels cin ..). A workgroup handles 64 outputs (input channel fastest, so
// the loads of a wave are contiguous) with 4 slices each: slice j sums the
// workgroups b = j, j + 4, ... in order, and the 4 slice sums are added in
// a fixed order: the result does not depend on scheduling.
__global__ __launch_bounds__(256) void wgrad_reduce(const float *__restrict__ part, int nblk, int pco, int pci,
                                                    int cout, int cin, int lo_pairs, float *__restrict__ gW)
{
    __shared__ double red[4][64];
    const int n = cout * cin * 27;
    const int o = threadIdx.x & 63, j = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + o;
    double s = 0.0;
    int ci = 0, co = 0, d = 0;
    if (e < n) {
        ci = e % cin;
        co = (e / cin) % cout;
        d = e / (cin * cout);
        const size_t stride = (size_t)27 * pco * pci;
        const float *p = part + ((size_t)d * pco + co) * pci;
        // unrolled so that eight loads are in flight; the adds keep their order
#pragma unroll 8
        for (int b = j; b < nblk; b += 4) s += p[(size_t)b * stride + ci];
        if (ci < lo_pairs)
#pragma unroll 8
            for (int b = j; b < nblk; b += 4) s += p[(size_t)b * stride + cin + ci];
    }
    red[j][o] = s;
    __syncthreads();
    if (j == 0 && e < n) gW[((size_t)co * cin + ci) * 27 + d] = (float)((red[0][o] + red[1][o]) + (red[2][o] + red[3][o]));
}

// Bias gradient: fixed-order fold of the per-workgroup channel sums; 32
// groups of lanes each sum every 32nd workgroup in order, then lane c adds
// the 32 group sums of channel c in order.
__global__ __launch_bounds__(1024) void colsum_reduce(const float *__restrict__ part, int nblk, int cout,
                                                     float *__restrict__ gb)
{
    __shared__ double red[32][32];
    const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
    double s = 0.0;
    for (int b = g; b < nblk; b += 32) s += part[(size_t)b * 32 + c];
    red[g][c] = s;
    __syncthreads();
    if (g == 0 && c < cout) {
        double t = 0.0;
        for (int i = 0; i < 32; ++i) t += red[i][c];
        gb[c] = (float)t;
    }
}

// ------------------------------------------------------------------ input, loss, optimiser
template <typename IO>
__global__ __launch_bounds__(256) void pack_input(const IO *__restrict__ u, const IO *__restrict__ v,
                                                  const float *__restrict__ fk, int nsamp, int ncell,
                                                  u16 *__restrict__ x)
{
    const size_t rows = (size_t)nsamp * ncell;
    for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(r / ncell);
        // u and v as BF16 pairs hi + lo (about 16 significant bits); the first
        // layer applies the same weight to both parts.
        const float uf = (float)u[r], vf = (float)v[r];
        const u16 uh = f2bf(uf), vh = f2bf(vf);
        const u16 ul = f2bf(uf - bf2f(uh)), vl = f2bf(vf - bf2f(vh));
        uint4 q;
        q.x = (uint32_t)uh | ((uint32_t)vh << 16);
        q.y = (uint32_t)f2bf((fk[2 * s] - F_CENTER) / F_SCALE) | ((uint32_t)f2bf((fk[2 * s + 1] - K_CENTER) / K_SCALE) << 16);
        q.z = (uint32_t)ul | ((uint32_t)vl << 16);
        q.w = 0u;
        *reinterpret_cast<uint4 *>(x + r * 8) = q;
    }
}

// Residuals of the prediction, their squared sum per workgroup, and the loss
// gradient dL/dpred = 2 (pred - target) / n_terms (channels 0, 1 of 8).
__global__ __launch_bounds__(256) void loss_grad(const float *__restrict__ pu, const float *__restrict__ pv,
                                                 const float *__restrict__ tu, const float *__restrict__ tv,
                                                 size_t rows, float scale, u16 *__restrict__ dz4,
                                                 double *__restrict__ part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += (size_t)gridDim.x * blockDim.x) {
        const float ru = pu[r] - tu[r], rv = pv[r] - tv[r];
        acc += (double)ru * ru + (double)rv * rv;
        uint4 q;
        q.x = (uint32_t)f2bf(scale * ru) | ((uint32_t)f2bf(scale * rv) << 16);
        q.y = q.z = q.w = 0u;
        *reinterpret_cast<uint4 *>(dz4 + r * 8) = q;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, const float *__restrict__ gr,
                                                   float *__restrict__ m, float *__restrict__ v, int n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float g = gr[i];
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Packs layer weights (FP32, W[co][ci][d]) into the B-fragment order of the
// convolution kernel: chunk c, N-tile t, lane, 8 consecutive k = 32 c + 8
// (lane / 16) + j with k = d * cins + ci. DGRAD packs the mirrored, transposed
// weights W'[ci][co][d] = W[co][ci][26 - d] (input channels = co).
// lo_pairs: input channels cin .. cin + lo_pairs - 1 carry the low parts of
// channels 0 .. lo_pairs - 1 and take their weights.
__global__ __launch_bounds__(256) void repack(const float *__restrict__ W, int cout, int cin, int cins, int nt,
                                              int nch, int dgrad, int lo_pairs, u16 *__restrict__ out)
{
    const int total = nch * nt * 64 * 8;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int j = e % 8, lane = (e / 8) % 64, t = (e / 512) % nt, c = e / (512 * nt);
        const int k = 32 * c + 8 * (lane / 16) + j;
        const int d = k / cins, kc = k % cins, n = 16 * t + lane % 16;
        float w = 0.f;
        if (d < 27) {
            if (!dgrad) {
                const int src = kc < cin ? kc : (kc - cin < lo_pairs ? kc - cin : -1);
                if (src >= 0 && n < cout) w = W[((size_t)n * cin + src) * 27 + d];
            } else {
                // input channel kc = co of the layer, output channel n = ci of the layer
                if (kc < cout && n < cin) w = W[((size_t)kc * cin + n) * 27 + (26 - d)];
            }
        }
        out[e] = f2bf(w);
    }
}

// ------------------------------------------------------------------ launchers
static int grid_cap(size_t work, int per_block, int cap)
{
    size_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > (size_t)cap) b = cap;
    return (int)b;
}

hipError_t launch_conv(int cin, int nt, int mode, int io_f64, const ConvArgs &a, hipStream_t st)
{
    if (a.zc < 1 || a.geo.nx % PX != 0) return hipErrorInvalidValue;
    if (cin == 32 && nt == 2 && mode != MODE_OUT) {
        ConvArgs b = a;
        b.zc = conv32p_zc(a.geo, a.nsamp);
        const int py = C32_RW * C32_WAVES;
        const size_t nb = (size_t)(a.geo.nx / PX) * ((a.geo.ny + py - 1) / py) * ((a.geo.nz + b.zc - 1) / b.zc) * a.nsamp;
        if (nb == 0 || nb > 0x7fffffffu) return hipErrorInvalidConfiguration;
        if (mode == MODE_HIDDEN)
            hipLaunchKernelGGL(conv32p_kernel<MODE_HIDDEN>, dim3((unsigned)nb), dim3(64 * C32_WAVES), 0, st, b);
        else if (mode == MODE_ACT)
            hipLaunchKernelGGL(conv32p_kernel<MODE_ACT>, dim3((unsigned)nb), dim3(64 * C32_WAVES), 0, st, b);
        else
            hipLaunchKernelGGL(conv32p_kernel<MODE_DGRAD>, dim3((unsigned)nb), dim3(64 * C32_WAVES), 0, st, b);
        return hipGetLastError();
    }
    const size_t blocks = (size_t)(a.geo.nx / PX) * ((a.geo.ny + PY - 1) / PY) * ((a.geo.nz + a.zc - 1) / a.zc) * a.nsamp;
    if (blocks == 0 || blocks > 0x7fffffffu) return hipErrorInvalidConfiguration;
    const int grid = (int)blocks;
#define GS_CONV(CI, N, M, IO) hipLaunchKernelGGL((conv_kernel<CI, N, M, IO>), dim3(grid), dim3(256), 0, st, a)
    if (cin == 8 && nt == 2 && mode == MODE_HIDDEN) GS_CONV(8, 2, MODE_HIDDEN, float);
    else if (cin == 8 && nt == 2 && mode == MODE_ACT) GS_CONV(8, 2, MODE_ACT, float);
    else if (cin == 32 && nt == 1 && mode == MODE_OUT && io_f64) GS_CONV(32, 1, MODE_OUT, double);
    else if (cin == 32 && nt == 1 && mode == MODE_OUT) GS_CONV(32, 1, MODE_OUT, float);
    else if (cin == 8 && nt == 2 && mode == MODE_DGRAD) GS_CONV(8, 2, MODE_DGRAD, float);
    else return hipErrorInvalidValue;
#undef GS_CONV
    return hipGetLastError();
}

int wgrad_blocks() { return 512; }

hipError_t launch_wgrad(int cin, int couts, const WgradArgs &a, hipStream_t st)
{
    const int grid = wgrad_blocks();
    if (cin == 32 && couts == 32)
        hipLaunchKernelGGL((wgrad_kernel<32, 32, 2, 2, 8>), dim3(grid), dim3(256), 0, st, a);
    else if (cin == 32 && couts == 8)
        hipLaunchKernelGGL((wgrad_kernel<32, 8, 1, 2, 8>), dim3(grid), dim3(256), 0, st, a);
    else if (cin == 8 && couts == 32)
        hipLaunchKernelGGL((wgrad_kernel<8, 32, 2, 1, 4>), dim3(grid), dim3(256), 0, st, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const float *part, int pco, int pci, int cout, int cin, int lo_pairs, float *gW,
                               hipStream_t st)
{
    const int n = cout * cin * 27;
    hipLaunchKernelGGL(wgrad_reduce, dim3((n + 63) / 64), dim3(256), 0, st, part, wgrad_blocks(), pco, pci, cout, cin,
                       lo_pairs, gW);
    return hipGetLastError();
}

hipError_t launch_bias_reduce(const float *bpart, int cout, float *gb, hipStream_t st)
{
    hipLaunchKernelGGL(colsum_reduce, dim3(1), dim3(1024), 0, st, bpart, wgrad_blocks(), cout, gb);
    return hipGetLastError();
}

hipError_t launch_pack_input(int io_f64, const void *u, const void *v, const float *fk, int nsamp, int ncell,
                             uint16_t *x, hipStream_t st)
{
    const int grid = grid_cap((size_t)nsamp * ncell, 256, 65536);
    if (io_f64)
        hipLaunchKernelGGL(pack_input<double>, dim3(grid), dim3(256), 0, st, (const double *)u, (const double *)v, fk,
                           nsamp, ncell, x);
    else
        hipLaunchKernelGGL(pack_input<float>, dim3(grid), dim3(256), 0, st, (const float *)u, (const float *)v, fk,
                           nsamp, ncell, x);
    return hipGetLastError();
}

int loss_blocks() { return 1024; }

hipError_t launch_loss_grad(const float *pu, const float *pv, const float *tu, const float *tv, size_t rows,
                            float scale, uint16_t *dz4, double *part, hipStream_t st)
{
    hipLaunchKernelGGL(loss_grad, dim3(loss_blocks()), dim3(256), 0, st, pu, pv, tu, tv, rows, scale, dz4, part);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t st)
{
    hipLaunchKernelGGL(adam_kernel, dim3(grid_cap(n, 256, 1024)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_repack(const float *W, int cout, int cin, int cins, int nt, int nch, int dgrad, int lo_pairs,
                         uint16_t *out, hipStream_t st)
{
    const int total = nch * nt * 512;
    hipLaunchKernelGGL(repack, dim3(grid_cap(total, 256, 1024)), dim3(256), 0, st, W, cout, cin, cins, nt, nch, dgrad,
                       lo_pairs, out);
    return hipGetLastError();
}

} // namespace nn
} // namespace gs
