// Test pin: prints rocRAND's Philox4x32-10 block for given keys and counters.
// Reads lines "seed c0 c1 c2 c3" (c1 < 2^30) and writes "x0 x1 x2 x3".
// rocRAND addresses a block by (subsequence -> counter words 2,3) and
// (offset / 4 -> counter words 0,1), with key = (seed lo32, seed hi32).
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main()
{
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, c2 | (c3 << 32), 4ull * (c0 | (c1 << 32)), &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
