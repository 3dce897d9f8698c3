// Cross-check helper (host only): prints Philox4x32-10 outputs computed by
// rocRAND's header implementation for counters/keys read from stdin, one
// "c0 c1 c2 c3 k0 k1" line (hex) per query. Used by the oracle tests to pin
// the oracle's Philox against an independent implementation.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// ten_rounds is a protected member; expose it through a derived type.
struct exposed_engine : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main()
{
    unsigned c[4], k[2];
    exposed_engine eng;
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        uint4 ctr = {c[0], c[1], c[2], c[3]};
        uint2 key = {k[0], k[1]};
        uint4 r = eng.ten_rounds(ctr, key);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
