// Host-side driver around rocRAND's header implementation of Philox4x32-10,
// used only as an independent known-answer source for the oracle's Philox.
// Reads lines "seed c0 c1 c2 c3" on stdin and prints the four output words.
// rocRAND's state keeps the counter as (offset/4 low, high, subsequence low,
// high) and the key as (seed low, seed high).
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        const unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        // counter words 0-1 = number of 4-word blocks skipped; skip in chunks
        // below 2^62 blocks so that the byte offset never overflows 64 bits.
        unsigned long long blocks = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, 0, &st);
        const unsigned long long chunk = 1ull << 61;
        while (blocks >= chunk) {
            skipahead(4ull * chunk, &st);
            blocks -= chunk;
        }
        skipahead(4ull * blocks, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
