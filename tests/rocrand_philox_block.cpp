// Prints Philox4x32-10 blocks computed by rocRAND's host-callable engine, for
// cross-checking the oracle's independent implementation.  Reads lines of
// "ctr0 ctr1 ctr2 ctr3 seed64" (decimal) from stdin.  Host code only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned long long c0, c1, c2, c3, seed;
    while (std::scanf("%llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &seed) == 5) {
        // the engine's counter is (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi)
        unsigned long long subseq = c2 | (c3 << 32);
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
