// Host-side harness that calls rocRAND's installed Philox4x32-10 engine
// (rocrand/rocrand_philox4x32_10.h) to pin the oracle's block function.
// Reads lines "seed c0 c1 c2 c3" (decimal) and prints the four output words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        // The engine's counter is (offset/4 as words 0-1, subsequence as words 2-3).
        unsigned long long subsequence = c2 | (c3 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0);
        // Advance words 0-1 of the counter by c0 + c1 * 2^32 blocks (4 numbers
        // per block) in pieces that do not overflow the 64-bit offset.
        eng.discard(4ull * c0);
        unsigned long long h = c1 >> 2, l = c1 & 3ull;
        for (int rep = 0; rep < 4; ++rep) eng.discard(h << 34);
        eng.discard(l << 34);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
