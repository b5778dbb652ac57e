// Test-only reference for the Philox4x32-10 block: the engine shipped in the
// rocRAND headers, driven through its protected ten-round function.  Reads
// lines "c0 c1 c2 c3 k0 k1" (hex) and prints the four output words (hex).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main()
{
    unsigned a[6];
    Probe p;
    while (std::scanf("%x %x %x %x %x %x", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
        uint4 c = {a[0], a[1], a[2], a[3]};
        uint2 k = {a[4], a[5]};
        uint4 r = p.run(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
