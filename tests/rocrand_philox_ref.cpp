// Independent comparator for the oracle's Philox4x32-10: rocRAND's engine,
// run on the host (no GPU needed).  Reads lines "seed c0 c1 c2 c3" (decimal)
// from stdin and prints the four output words of Philox4x32-10 applied to
// counter (c0, c1, c2, c3) under key (seed mod 2^32, seed >> 32).
//
// The engine's ten-round bijection is reached through a derived class, so
// any 128-bit counter can be fed to it directly.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

struct philox_ref : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};

int main()
{
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    philox_ref e;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        uint4 ctr = {c0, c1, c2, c3};
        uint2 key = {(unsigned)seed, (unsigned)(seed >> 32)};
        uint4 r = e.apply(ctr, key);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
