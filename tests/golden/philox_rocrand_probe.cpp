// Prints Philox4x32-10 blocks computed by rocRAND's header engine, for
// counters/keys read from stdin ("c0 c1 c2 c3 k0 k1" per line).  Host-only;
// used by the oracle tests as an independent implementation of the published
// Philox4x32-10 generator.  The engine maps (seed, subsequence, offset) to
// key = seed, counter = (offset/4 lo, offset/4 hi, subsequence lo, hi);
// discard(n) advances the counter by n/4 blocks.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        // advance by c0 + c1 * 2^32 blocks; split so every offset fits 64 bits
        rocrand_device::philox4x32_10_engine eng(seed, sub, 4ull * c0);
        for (int q = 0; q < 4; ++q) eng.discard((unsigned long long)c1 << 32);
        unsigned a = eng.next(), b = eng.next(), c = eng.next(), d = eng.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
