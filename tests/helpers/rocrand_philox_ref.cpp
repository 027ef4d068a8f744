// Host-only reference for Philox-4x32-10 words, using AMD rocRAND's own
// engine (rocrand_philox4x32_10.h).  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on
// stdin and prints the four output words (hex) for counter (c0,c1,c2,c3) and
// key (k0,k1).  rocRAND's engine(seed, subsequence, offset) starts at counter
// (offset/4 low, high, subsequence low, high) with key (seed low, high).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long ctr = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, sub, 0);
        // advance the 64-bit counter by ctr in pieces that do not overflow
        // the engine's offset argument (offset = 4 x counter increment)
        for (int part = 0; part < 4; ++part) eng.discard((ctr / 4ull) * 4ull);
        eng.discard((ctr % 4ull) * 4ull);
        uint4 r = eng.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
