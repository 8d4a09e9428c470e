// Device-side building blocks of the Gray-Scott kernels for gfx950:
// storage-type conversion, Philox4x32-10 noise, FP64 division by 6, the
// compensated FP32 Laplacian, and a z-streaming tile of one field (global ->
// registers -> LDS) shared by the step and Laplacian kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

// ---------------------------------------------------------------- storage
struct bf16 {
    uint16_t bits;
};
typedef _Float16 f16;

__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(f16 x) { return (float)x; }
__device__ __forceinline__ float to_f32(bf16 x) { return __uint_as_float((uint32_t)x.bits << 16); }

// Round-to-nearest-even FP32 -> BF16 (NaN stays NaN): one gfx950
// conversion instruction.
__device__ __forceinline__ bf16 bf16_rne(float f)
{
    bf16 r;
    r.bits = __builtin_bit_cast(uint16_t, (__bf16)f);
    return r;
}

// Compute type C and conversions for each storage type S.
template <typename S> struct Traits;
template <> struct Traits<double> {
    typedef double C;
    static __device__ __forceinline__ double load(double s) { return s; }
    static __device__ __forceinline__ double store(double c) { return c; }
};
template <> struct Traits<float> {
    typedef float C;
    static __device__ __forceinline__ float load(float s) { return s; }
    static __device__ __forceinline__ float store(float c) { return c; }
};
template <> struct Traits<bf16> {
    typedef float C;
    static __device__ __forceinline__ float load(bf16 s) { return to_f32(s); }
    static __device__ __forceinline__ bf16 store(float c) { return bf16_rne(c); }
};
// BF16 storage with u kept as its complement 1 - u (v as it is). Most of a
// Gray-Scott state sits near u = 1, where BF16 steps are 2^-8 and the small
// updates of a step are rounded away; 1 - u is near 0 there and BF16 keeps
// eight significant bits of it. The same 2 bytes per value.
struct bf16c {
    uint16_t bits;
};
template <> struct Traits<bf16c> {
    typedef float C;
    static __device__ __forceinline__ float load(bf16c s) { return __uint_as_float((uint32_t)s.bits << 16); }
    static __device__ __forceinline__ bf16c store(float c)
    {
        bf16c r;
        r.bits = __builtin_bit_cast(uint16_t, (__bf16)c);
        return r;
    }
};
template <typename S> struct Complemented {
    static constexpr bool value = false;
};
template <> struct Complemented<bf16c> {
    static constexpr bool value = true;
};

template <> struct Traits<f16> {
    typedef float C;
    static __device__ __forceinline__ float load(f16 s) { return (float)s; }
    // The empty asm hides the FP32 value before the conversion (no
    // instruction): without it the compiler may fuse the conversion into the
    // fma that produced the value (an fma_mix with an FP16 result), which
    // rounds differently from the fma and then the conversion, and does so in
    // some kernels and not in others.
    static __device__ __forceinline__ f16 store(float c)
    {
        asm("" : "+v"(c));
        return (f16)c;
    }
};

// V consecutive storage elements moved as one aligned vector access.
template <typename S, int V> struct alignas(16) Vec {
    S e[V];
};

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds; each multiplies counter
// words 0 and 2 by the round multipliers into 64-bit products and recombines
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is
// advanced by the two Weyl increments between rounds. The key and the step
// words are uniform across the launch.
struct Philox4 {
    uint32_t w[4];
};

// a ^ b ^ c in one instruction (gfx950 three-input bit operation; truth
// table 0x96 is the odd-parity function).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // One 32x32 -> 64-bit multiply instruction per product (hi and lo together).
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        c0 = xor3((uint32_t)(pb >> 32), c1, k0);
        c1 = (uint32_t)pb;
        c2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c3 = (uint32_t)pa;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

// r = (w + 1/2) 2^-31 for the signed word w: exact in FP64, in (-1, 1).
__device__ __forceinline__ double noise_word_f64(uint32_t w)
{
    return ((double)(int32_t)w + 0.5) * 0x1p-31;
}
// FP32 noise term n r = (n 2^-31) w + n 2^-32 for the signed word w, as one
// fma of the word converted to FP32 with the FP32 scales s = RN(n 2^-31),
// h = RN(n 2^-32) (the word keeps 24 significant bits, below what FP32
// storage resolves in the step).
__device__ __forceinline__ float noise_term_f32(uint32_t w, float s, float h)
{
    return __builtin_fmaf((float)(int32_t)w, s, h);
}

// One Euler step of a cell in FP32 arithmetic (storage other than FP64):
// Eq. 1a/1b and 2a/2b with the products fused into the sums, so each field
// takes three operations after u v^2. nr is the noise term n r (NOISE).
// Every FP32 kernel uses this one sequence, so results do not depend on the
// kernel, the tile or the fused depth.
template <bool NOISE>
__device__ __forceinline__ void euler_f32(float Du, float Dv, float F, float FK, float dt, float uc, float vc,
                                          float lu, float lv, float nr, float &uo, float &vo)
{
    const float uvv = uc * (vc * vc);
    float du = __builtin_fmaf(F, 1.0f - uc, __builtin_fmaf(Du, lu, -uvv));
    if constexpr (NOISE) du = du + nr;
    const float dv = __builtin_fmaf(-FK, vc, __builtin_fmaf(Dv, lv, uvv));
    uo = __builtin_fmaf(du, dt, uc);
    vo = __builtin_fmaf(dv, dt, vc);
}

// Noise of the 4 cells idx4 .. idx4+3 (idx4 a multiple of 4) at step t.
__device__ __forceinline__ Philox4 noise_block(uint64_t idx4, uint64_t t, uint64_t seed)
{
    const uint64_t q = idx4 >> 2;
    return philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), (uint32_t)t, (uint32_t)(t >> 32),
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------- arithmetic
// Correctly rounded x / 6 without the FP64 divide sequence: the IEEE
// quotient, bit for bit, for every finite x (a zero gives +0).
//
// With h = RN(1/6) and q0 = RN(x h), the residual r = x - 6 q0 is a small
// multiple of ulp(q0) (|r| <= 3 ulp(q0) and a little) and so exact in one
// fma, and x / 6 = q0 + r / 6. The quotient is RN(q0 + r c) for any c close
// enough to 1/6, except on an exact tie:
//  - Away from ties. x is an integer multiple of an ulp at least four times
//    the quotient's (x / 6 < x / 4), and of 2^-1074 where the quotient is
//    subnormal, so x / 6 sits at a multiple of 1/6 of the quotient's grid
//    step from a grid point and at least 1/6 of a step from every rounding
//    boundary. r (c - 1/6) moves it by at most 3 |c - 1/6| steps, far less
//    for |c - 1/6| <= 2^-23.
//  - Ties. Only a subnormal quotient can lie exactly half-way between two
//    grid points (x an odd multiple of 3 2^-1074); q0 is one of the two and
//    r = +-3 steps. RN(q0 + r c) is q0 for c below 1/6 and the other point
//    for c above it, while the rule wants the even one.
// So c is taken just below 1/6 when q0's last significand bit is 0 and just
// above it when that bit is 1: its high word is 0x3FC55555 and its low word
// the same constant with q0's last bit moved to bit 31 (0x3FC55555 or
// 0xBFC55555, both within 2^-24 of 1/6), one shift-or. The same constant in
// both words lets one register serve as the shift-or's operand and as the
// multiplier's high half. A tiny negative x gives RN(-0 + r c) = -0, as the
// division does.
// A numerator of +-Inf (an infinite input, or a neighbour sum beyond the
// largest double) gives NaN where the division gives +-Inf.
__host__ __device__ __forceinline__ double div6(double x)
{
    const double h = 0x1.5555555555555p-3; // RN(1/6), just below 1/6
    const double q0 = x * h;
    const double r = __builtin_fma(-q0, 6.0, x);
    const uint32_t k = 0x3FC55555u;
    const uint32_t lo = ((uint32_t)__builtin_bit_cast(uint64_t, q0) << 31) | k;
    const double c = __builtin_bit_cast(double, ((uint64_t)k << 32) | lo);
    return __builtin_fma(r, c, q0);
}

// Field-aware conversions between storage and compute values (field 0 is u,
// field 1 is v): the complemented storage type stores 1 - u. In FP32 1 - u is
// exact for u in [1/2, 2], and the stored complement of a u below 1/2 (at
// least 1/2) is rounded far more finely than by the storage.
template <typename S> __device__ __forceinline__ typename Traits<S>::C fload(int f, S s)
{
    const typename Traits<S>::C c = Traits<S>::load(s);
    if constexpr (Complemented<S>::value) return f == 0 ? 1.0f - c : c;
    else return c;
}
template <typename S> __device__ __forceinline__ S fstore(int f, typename Traits<S>::C c)
{
    if constexpr (Complemented<S>::value) return Traits<S>::store(f == 0 ? 1.0f - c : c);
    else return Traits<S>::store(c);
}

// Laplacian in FP32 of values read from 2-byte storage: the six differences
// summed in three levels without compensation. A difference of two 16-bit
// values (for the complemented BF16 storage, of their complements) is exact
// in FP32 whenever their exponents are within 16 of each other (a BF16 or
// FP16 value has at most 11 significant bits), and the sum errs by at most
// 3 u sum |d_i| (u = 2^-24): below 2e-7 of the differences, while the state
// is rounded to 2^-9 (BF16) or 2^-12 (FP16) of itself after every step. The
// compensated sum buys nothing at this storage and costs 16 more operations
// per field.
__device__ __forceinline__ float lap_sum_f32(float c, float xm, float xp, float ym, float yp, float zm, float zp)
{
    const float s = ((xm - c) + (xp - c)) + ((ym - c) + (yp - c)) + ((zm - c) + (zp - c));
    return s * (1.0f / 6.0f);
}
// Laplacian in FP32 of values read from FP32 storage: the six FP32
// differences (exact where a neighbour is within a factor 2 of c) summed in
// FP64, which errs by at most 3 2^-53 sum |d_i|, then rounded once to FP32
// and scaled. A compensated FP32 sum (Kahan) errs by up to (2u + O(u^2))
// sum |d_i| (u = 2^-24), which exceeds a rounding of the sum itself wherever
// the differences cancel, and takes more operations.
__device__ __forceinline__ float lap_wide_f32(float c, float xm, float xp, float ym, float yp, float zm, float zp)
{
    const double s = (((double)(xm - c) + (double)(xp - c)) + ((double)(ym - c) + (double)(yp - c))) +
                     ((double)(zm - c) + (double)(zp - c));
    return (float)s * (1.0f / 6.0f);
}
// The FP32-arithmetic Laplacian of storage type S: the FP64 sum for FP32
// storage, the plain sum for 2-byte storage.
template <typename S>
__device__ __forceinline__ float lap_f32(float c, float xm, float xp, float ym, float yp, float zm, float zp)
{
    if constexpr (sizeof(S) == 2) return lap_sum_f32(c, xm, xp, ym, yp, zm, zp);
    else return lap_wide_f32(c, xm, xp, ym, yp, zm, zp);
}

// FP64 Laplacian in the canonical order: ((x- + x+) + (y- + y+)) + (z- + z+),
// then (sum - 6 c) / 6.
__host__ __device__ __forceinline__ double lap_f64(double c, double xm, double xp, double ym, double yp,
                                                   double zm, double zp)
{
    const double s = ((xm + xp) + (ym + yp)) + (zm + zp);
    const double c6 = 6.0 * c;
    return div6(s - c6);
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Block index -> logical tile index such that the blocks the dispatcher
// sends to one XCD (hardware block ids congruent mod 8) get one contiguous
// range of logical tiles, so halos and z-chunk edges are shared in that
// XCD's L2.
__device__ __forceinline__ uint32_t xcd_logical_block(uint32_t b, uint32_t nb)
{
    const uint32_t per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7u) * per + (b >> 3);
}

} // namespace gs
