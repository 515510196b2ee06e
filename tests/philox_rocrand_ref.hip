// A host-only reference for the tests: rocRAND's Philox4x32-10 bijection
// (the ten rounds its engine applies to a counter block under a key), read
// from ROCm's own header, so that the oracle's Philox is checked against an
// implementation written outside this project.  No kernel is launched and no
// HIP runtime call is made.
//
// stdin: lines "c0 c1 c2 c3 k0 k1" (hexadecimal 32-bit words)
// stdout: lines "r0 r1 r2 r3" (hexadecimal), one per input line
#include <cstdio>

#include <rocrand/rocrand_philox4x32_10.h>

struct PhiloxRef : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 counter, uint2 key) { return ten_rounds(counter, key); }
};

int main()
{
    PhiloxRef ref;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c;
        c.x = c0;
        c.y = c1;
        c.z = c2;
        c.w = c3;
        uint2 k;
        k.x = k0;
        k.y = k1;
        const uint4 r = ref.block(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
