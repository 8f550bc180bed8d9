// Reference Philox4x32-10 blocks from rocRAND's header-only engine, used by
// the test suite as an implementation independent of the oracle's.
// stdin: lines "seed c0 c1 c2 c3"; stdout: the four 32-bit output words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        // The engine's counter is (offset/4 lo, offset/4 hi, subsequence lo,
        // subsequence hi); its key is (seed lo, seed hi).
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long blk = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_device::philox4x32_10_engine e(seed, sub, blk * 4ull);
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
