// Black-box reference for the Philox4x32-10 pin: reads lines
// "ctr0 ctr1 ctr2 ctr3 key0 key1" on stdin and prints the four output words of
// rocRAND's philox4x32_10 engine positioned at that counter and key
// (key = seed, counter words 2-3 = subsequence, counter words 0-1 = offset / 4).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = (((unsigned long long)c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
