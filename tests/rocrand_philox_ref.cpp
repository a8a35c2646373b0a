// Independent reference for the Philox4x32-10 stream: rocRAND's header-only
// engine compiled for the host.  Reads lines "seed ctr0 ctr1 ctr2 ctr3" (hex)
// on stdin and prints the four 32-bit output words of that block (hex).
//
// rocRAND's engine keys Philox with (seed lo, seed hi); its counter is
// (offset/4 as 64 bits in words 0-1, subsequence as 64 bits in words 2-3), so
// the block with counter (c0, c1, c2, c3) is reached with
// subsequence = c2 | c3 << 32 and then advancing by c0 | c1 << 32 blocks of
// four numbers (in chunks, since four times a 64-bit block count overflows).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned long long seed;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llx %x %x %x %x", &seed, &c0, &c1, &c2, &c3) == 5) {
        const unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long blocks = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_device::philox4x32_10_engine e(seed, sub, 0);
        while (blocks) {
            const unsigned long long chunk = blocks < (1ULL << 60) ? blocks : (1ULL << 60);
            e.discard(4ULL * chunk);
            blocks -= chunk;
        }
        const unsigned int w0 = e.next(), w1 = e.next(), w2 = e.next(), w3 = e.next();
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
