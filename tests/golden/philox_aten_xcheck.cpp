// Cross-check helper (host only): prints Philox4x32-10 outputs computed by
// PyTorch's ATen header engine. Counter (c0, c1, c2, c3) maps to
// offset = c0 | c1 << 32 and subsequence = c2 | c3 << 32; key = k0 | k1 << 32.
#include <cstdint>
#include <cstdio>
#include <ATen/core/PhiloxRNGEngine.h>

int main()
{
    unsigned c[4], k[2];
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        uint64_t seed = (uint64_t)k[0] | ((uint64_t)k[1] << 32);
        uint64_t sub = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
        at::Philox4_32 eng(seed, sub, 0);
        eng.set_offset((uint64_t)c[0] | ((uint64_t)c[1] << 32));
        unsigned r0 = eng(), r1 = eng(), r2 = eng(), r3 = eng();
        std::printf("%08x %08x %08x %08x\n", r0, r1, r2, r3);
    }
    return 0;
}
