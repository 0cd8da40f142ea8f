// Independent pin for the oracle's Philox4x32-10: prints raw blocks from
// rocRAND's host-callable philox4x32_10_engine for counters read from stdin.
// Input lines: c0 c1 c2 c3 k0 k1 (decimal).  Output lines: x0 x1 x2 x3.
// rocRAND's engine with seed = k1:k0, subsequence = c3:c2 and offset = 4*(c1:c0)
// starts exactly at Philox(counter = (c0, c1, c2, c3), key = (k0, k1)).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (k1 << 32) | k0;
        unsigned long long subseq = (c3 << 32) | c2;
        unsigned long long offset = 4ull * ((c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        unsigned int x0 = eng(), x1 = eng(), x2 = eng(), x3 = eng();
        std::printf("%u %u %u %u\n", x0, x1, x2, x3);
    }
    return 0;
}
