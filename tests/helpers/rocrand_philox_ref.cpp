// Independent reference for the oracle's Philox4x32-10: rocRAND's open-source
// host/device engine.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal uint32) on
// stdin and prints the four output words of ten rounds, decimal, one line each.
// Built and run on the CPU by the oracle tests; no GPU code is involved.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
