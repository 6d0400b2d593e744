// Philox4x32-10 words computed by rocRAND's engine, an implementation that is
// independent of the oracle.  Test infrastructure: it pins the oracle's
// generator to the library's reading of the published definition.
// Input lines: "c0 c1 c2 c3 k0 k1" in hex; output lines: "w0 w1 w2 w3".
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 words(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    unsigned a, b, c, d, e, f;
    Probe p;
    while (std::scanf("%x %x %x %x %x %x", &a, &b, &c, &d, &e, &f) == 6) {
        uint4 r = p.words(make_uint4(a, b, c, d), make_uint2(e, f));
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
