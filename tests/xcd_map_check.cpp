// Host check of the walk kernel's workgroup -> chunk-block mapping: a
// bijection of [0, G) for every grid size, with each XCD's workgroups
// taking runs of consecutive blocks and each round's runs dealt to distinct
// XCDs; and of the treecode traversal's contiguous mapping.  Prints "ok" or
// the first failure.
#include <cstdio>
#include <vector>

#include "../paper_1210_1491_amd/csrc/dtn_device.h"
#include "../paper_1210_1491_amd/csrc/dtn_xcd.h"

int main()
{
    std::vector<long long> sizes;
    for (long long G = 1; G <= 4096; ++G) sizes.push_back(G);
    for (long long G : {204801LL, 819204LL, 1000003LL, 16777216LL}) sizes.push_back(G);
    for (long long G : sizes) {
        std::vector<char> hit(G, 0);
        for (long long i = 0; i < G; ++i) {
            const long long L = dtn::xcd_block(i, G);
            if (L < 0 || L >= G || hit[L]) {
                std::printf("not a bijection: G=%lld i=%lld L=%lld\n", G, i, L);
                return 1;
            }
            hit[L] = 1;
        }
        const long long run = dtn::kXcdStripe, round = dtn::kXcds * run;
        const long long full = G - G % round;
        for (long long i = 0; i < full; ++i) {
            // consecutive workgroups of one XCD (i, i + 8) inside a run take consecutive blocks
            const long long k = i / dtn::kXcds;
            if (k % run != run - 1 && i + dtn::kXcds < full &&
                dtn::xcd_block(i + dtn::kXcds, G) != dtn::xcd_block(i, G) + 1) {
                std::printf("run broken: G=%lld i=%lld\n", G, i);
                return 1;
            }
            // a round's blocks come from the workgroups of that round
            if (dtn::xcd_block(i, G) / round != i / round) {
                std::printf("round broken: G=%lld i=%lld\n", G, i);
                return 1;
            }
        }
    }
    // the traversal's contiguous mapping: a bijection of [0, n) for n a
    // multiple of 8 W, each XCD's blocks (ib, ib + 8, ...) taking one
    // eighth of the range in order
    for (int W : {1, 2, 4})
        for (long long n = 8LL * W; n <= 8LL * W * 300; n += 8LL * W) {
            std::vector<char> hit(n, 0);
            const long long blocks = n / W;
            for (long long ib = 0; ib < blocks; ++ib)
                for (int wv = 0; wv < W; ++wv) {
                    const long long g = dtn::xcd_contiguous(ib, wv, n, W);
                    const long long x = ib % dtn::kXcds, lo = x * (n / dtn::kXcds), hi = lo + n / dtn::kXcds;
                    if (g < lo || g >= hi || hit[g]) {
                        std::printf("contiguous map broken: n=%lld W=%d ib=%lld wv=%d g=%lld\n", n, W, ib, wv, g);
                        return 1;
                    }
                    hit[g] = 1;
                    if (ib >= dtn::kXcds && dtn::xcd_contiguous(ib - dtn::kXcds, wv, n, W) != g - W) {
                        std::printf("contiguous map out of order: n=%lld W=%d ib=%lld\n", n, W, ib);
                        return 1;
                    }
                }
        }
    std::printf("ok\n");
    return 0;
}
