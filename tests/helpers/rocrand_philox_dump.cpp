// Test helper: prints rocRAND's Philox4x32-10 output for a list of
// (counter, key) pairs read from stdin, using rocRAND's own engine
// (rocrand_init / rocrand4 from <rocrand/rocrand_kernel.h>) on the host CPU.
// rocRAND maps (seed, subsequence, offset) to key = seed and
// counter = (offset/4 as 64 bits, subsequence as 64 bits); the low 64
// counter bits are reached by skipping ahead 4 times by that many outputs
// (4 outputs per counter step), so no 64-bit offset overflows.
// Input lines: c0 c1 c2 c3 k0 k1 (hex). Output lines: o0 o1 o2 o3 (hex).
#include <cstdio>
#include <cstdint>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long low = ((unsigned long long)c1 << 32) | c0;
        rocrand_init(seed, subseq, 0ull, &st);
        for (int r = 0; r < 4; r++) skipahead(low, &st);
        uint4 v = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
