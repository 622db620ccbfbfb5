// Third opinion on Philox4x32-10 for the tests: rocRAND's own engine, host side.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four output words.
// rocRAND maps key = seed, counter words 0-1 = offset / 4, words 2-3 = subsequence.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
