// Prints Philox4x32-10 blocks computed by rocRAND's engine (an implementation
// independent of the oracle's) for counters and keys read from stdin, one
// "c0 c1 c2 c3 k0 k1" line per query, as "x0 x1 x2 x3" lines.  Built on the
// host only; used by the oracle's random-number pin.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    probe p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = p.block(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
