// Host-side dump of rocRAND's open-source Philox-4x32-10 engine, used only as
// an independent third-party cross-check of the oracle's generator.  Reads
// lines "c0 c1 c2 c3 k0 k1" (decimal) from stdin and prints the four output
// words of the block with that counter and key.  The engine's public API maps
// seed -> key, subsequence -> counter words 2..3 and offset/4 -> words 0..1.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subsequence = c2 | (c3 << 32);
        // Counter words 0..1 are reached through discard(), whose argument
        // counts 32-bit outputs (4 per block); it is split so that no
        // argument overflows 64 bits.
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 4ull * c0);
        for (int piece = 0; piece < 16; ++piece)
            eng.discard(4ull * (c1 << 28));
        unsigned int w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
