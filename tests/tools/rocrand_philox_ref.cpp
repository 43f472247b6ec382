// Host-only reference: prints ROCm rocRAND's Philox4x32-10 output blocks for
// counters read from stdin ("c0 c1 c2 c3 k0 k1" per line, decimal).  The
// engine's (seed, subsequence, offset) map to key = (seed lo, seed hi) and
// counter = (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (k1 << 32) | k0;
        unsigned long long subseq = (c3 << 32) | c2;
        unsigned long long offset = 4ull * ((c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
