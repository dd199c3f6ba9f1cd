// Host-side reference words from rocRAND's philox4x32_10 engine, used by the
// test suite to pin the oracle's own Philox4x32-10 against an independent
// implementation.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin and
// prints the four output words of Philox(counter, key) per line.
//
// rocRAND's engine maps (seed, subsequence, offset) to key = seed,
// counter.zw += subsequence, counter.xy += offset / 4, so the block for
// counter (c0, c1, c2, c3) is the first four draws of
// engine(seed = k1:k0, subsequence = c3:c2, offset = 4 * (c1:c0)); the offset
// is a 64-bit count, so c1 must stay below 2^30.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (k1 << 32) | k0;
        unsigned long long sub = (c3 << 32) | c2;
        unsigned long long off = 4ull * ((c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
