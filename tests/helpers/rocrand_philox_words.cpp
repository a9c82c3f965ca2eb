// Prints rocRAND's Philox4x32-10 output words for (seed, subsequence, counter)
// triples read from stdin, one "w0 w1 w2 w3" line per triple.  Host-only use of
// rocRAND's open-source device/host header; pins the oracle's Philox.
// rocrand_init(seed, subsequence, 0) sets key = (seed lo, seed hi) and
// counter = (0, 0, subsequence lo, subsequence hi); skipahead(4 c) then adds c
// to the low 64 counter bits.  A 64-bit c is added in pieces below 2^62.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main()
{
    unsigned long long seed, sub, c;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &c) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, 0, &st);
        const unsigned long long low = c & ((1ull << 60) - 1);
        skipahead(4ull * low, &st);
        for (unsigned long long k = 0; k < (c >> 60); ++k) skipahead(4ull << 60, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
