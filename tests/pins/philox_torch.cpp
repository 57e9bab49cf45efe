// Host-side harness that calls PyTorch's installed Philox4x32-10 engine
// (ATen/core/PhiloxRNGEngine.h) to pin the oracle's block function.
// Reads lines "seed c0 c1 c2 c3" (decimal) and prints the four output words.
#include <cstdio>
#include <cstdint>
#include <ATen/core/PhiloxRNGEngine.h>

int main()
{
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        // philox_engine(seed, subsequence -> words 2-3, offset -> words 0-1)
        at::philox_engine eng(seed, c2 | (c3 << 32), c0 | (c1 << 32));
        uint32_t a = eng(), b = eng(), c = eng(), d = eng();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
