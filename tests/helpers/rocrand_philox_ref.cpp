// Prints Philox4x32-10 blocks produced by rocRAND's own host-callable engine,
// used as an independent black-box reference for the oracle's generator.
// Usage: rocrand_philox_ref seed subsequence block   (one line per query on stdin)
// For each "seed subsequence block" line it prints the four 32-bit words of
// the block that rocRAND yields at offset 4*block of that subsequence.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long seed, subseq, block;
    while (std::scanf("%llu %llu %llu", &seed, &subseq, &block) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, 4ull * block, &st);
        unsigned int a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
