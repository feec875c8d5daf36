// Prints raw rocRAND Philox4x32-10 output for counters (i, j, k, 0) under a
// 64-bit seed: rocrand_init(seed, subsequence = k, offset = 4 * (i + 2^32 j))
// positions the generator's 128-bit counter at (i, j, k, 0), and the first
// rocrand4() returns the ten-round output for that counter.  Built on the host
// only (no GPU needed) and used to pin the oracle's own Philox.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv)
{
    // argv: seed i j k  (repeated groups of four)
    for (int a = 1; a + 3 < argc; a += 4) {
        unsigned long long seed = strtoull(argv[a], nullptr, 0);
        unsigned long long i = strtoull(argv[a + 1], nullptr, 0);
        unsigned long long j = strtoull(argv[a + 2], nullptr, 0);
        unsigned long long k = strtoull(argv[a + 3], nullptr, 0);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, k, 4ull * (i + (j << 32)), &st);
        uint4 r = rocrand4(&st);
        printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
