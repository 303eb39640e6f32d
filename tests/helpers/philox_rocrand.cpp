// Philox4x32-10 outputs from the rocRAND library routine (host build of its
// header), used to pin the oracle's own Philox against an independent
// implementation.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) from stdin and
// prints the four 32-bit outputs of the block at that counter and key.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        // rocRAND: key = seed (lo, hi); counter = {offset/4 lo, hi, subsequence lo, hi}
        const unsigned long long seed = k0 | (k1 << 32);
        const unsigned long long subseq = c2 | (c3 << 32);
        const unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
