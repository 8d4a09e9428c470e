// Host-side check of the library's FP64 division by 6 (gs::div6 and the
// Laplacian built on it, compiled for the host from the device header)
// against the IEEE quotient x / 6, bit for bit. Prints "ok" and the number of
// arguments checked, or the first mismatches.
#include "../../paper_2309_10292_amd/csrc/gs_device.hpp"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

static double from_bits(uint64_t b)
{
    double d;
    std::memcpy(&d, &b, 8);
    return d;
}
static uint64_t bits(double d)
{
    uint64_t b;
    std::memcpy(&b, &d, 8);
    return b;
}

static long checked = 0, bad = 0;

static void check(double x)
{
    ++checked;
    const double got = gs::div6(x), want = x / 6.0;
    bool ok = bits(got) == bits(want);
    if (x == 0.0) ok = got == 0.0 && !std::signbit(got); // both zeros give +0 (documented)
    if (std::isinf(x) || std::isnan(x)) ok = std::isnan(got); // +-Inf and NaN give NaN (documented)
    if (!ok && bad++ < 8) std::printf("mismatch x=%a div6=%a x/6=%a\n", x, got, want);
}

int main()
{
    // every subnormal argument m 2^-1074 with m < 2^20, both signs
    for (uint64_t m = 0; m < (1u << 20); ++m) {
        check(from_bits(m));
        check(-from_bits(m));
    }
    // subnormal arguments across the whole significand range (strided), and
    // the exact ties m = 6 j + 3 at every magnitude, both signs
    for (uint64_t i = 0; i < (1u << 21); ++i) {
        const uint64_t m = i * 2147483659ull % (1ull << 52);
        const uint64_t j = (i * 6700417ull) % ((1ull << 52) / 6);
        check(from_bits(m));
        check(-from_bits(m));
        check(from_bits(6 * j + 3));
        check(-from_bits(6 * j + 3));
    }
    // the normal arguments whose quotient is subnormal or just normal:
    // exponent fields 1..5, strided through the significand
    for (uint64_t e = 1; e <= 5; ++e)
        for (uint64_t i = 0; i < (1u << 20); ++i) {
            const double x = from_bits((e << 52) + i * 4294967291ull % (1ull << 52));
            check(x);
            check(-x);
        }
    // a band around 6 * 2^-1022, where the quotient becomes normal
    const uint64_t t = bits(0x1.8p-1020);
    for (int64_t i = -(1 << 20); i < (1 << 20); ++i) check(from_bits(t + i));
    // random finite doubles over all exponents (xorshift64)
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (long i = 0; i < 20000000; ++i) {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        const double x = from_bits(s);
        if (std::isfinite(x)) check(x);
    }
    // non-finite arguments
    check(INFINITY);
    check(-INFINITY);
    check(NAN);
    // the Laplacian's numerator and quotient: subnormal neighbours around a zero
    // centre, and neighbours that cancel to a tie of the subnormal grid
    for (uint64_t m = 1; m < 4096; ++m) {
        const double a = from_bits(m), b = from_bits(3 * m + 1);
        const double xs = ((a + b) + (a + 0.0)) + (b + a) - 6.0 * 0.0;
        ++checked;
        if (bits(gs::lap_f64(0.0, a, b, a, 0.0, b, a)) != bits(xs / 6.0) && bad++ < 8)
            std::printf("laplacian mismatch m=%llu\n", (unsigned long long)m);
    }
    if (bad) {
        std::printf("%ld mismatches of %ld\n", bad, checked);
        return 1;
    }
    std::printf("ok %ld\n", checked);
    return 0;
}
