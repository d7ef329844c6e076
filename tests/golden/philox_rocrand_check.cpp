// Host-only program: prints rocRAND's Philox4x32-10 block for counters and
// keys read from stdin ("c0 c1 c2 c3 k0 k1" per line, decimal).  Used to pin
// the oracle's own Philox against an independent implementation.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subsequence = c2 | (c3 << 32);
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
