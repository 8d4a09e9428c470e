// Host-only program: prints rocRAND's Philox4x32-10 output words for the
// (seed, subsequence = step t, offset = 4 q) triples given on stdin, one
// "seed t q" triple per line. rocRAND's engine seeds the key with the two
// halves of the seed, puts the subsequence in counter words 2..3 and adds
// offset/4 to counter words 0..1, so its four words are the Philox block at
// counter (q, t), key (seed): the same block the oracle's noise draws from.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long seed, t, q;
    while (std::scanf("%llu %llu %llu", &seed, &t, &q) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, t, 4ull * q, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
