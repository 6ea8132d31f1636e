// CPU check of the persistent launch's barrier-tree arithmetic
// (paper_1010_2592_amd/csrc/barrier_tree.h).  Reads "G nblocks seed" and the
// XCD of every block (the census), then replays three barriers with the
// blocks arriving in a seeded random order through the tree's monotone
// counters: group counter -> XCD counter -> global counter.  Prints "OK" if,
// in every barrier, every group and every XCD has exactly one leader (the
// arrival that completes it), the global counter reaches exactly
// number * (XCDs in use) and the last global arrival comes after every block
// has arrived; else a message.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "barrier_tree.h"

int main() {
    int G, nb;
    unsigned seed;
    if (std::scanf("%d %d %u", &G, &nb, &seed) != 3 || G < 1 || nb < 1) return 2;
    std::vector<int> xcd(nb), rank(nb);
    int count[8] = {};
    for (int b = 0; b < nb; ++b) {
        if (std::scanf("%d", &xcd[b]) != 1 || xcd[b] < 0 || xcd[b] >= 8) return 2;
        rank[b] = count[xcd[b]]++;            // census rank, in census order
    }
    int nxcd = 0;
    int ngmax = 0;
    for (int x = 0; x < 8; ++x) {
        if (count[x] > 0) ++nxcd;
        if (count[x] > 0) ngmax = std::max(ngmax, msb::tree::group_of(0, count[x], G).ng);
    }
    std::vector<unsigned long long> gbar(8 * ngmax + 8, 0), xbar(8, 0);
    unsigned long long bar = 0;
    std::mt19937 rng(seed);
    std::vector<int> order(nb);
    for (int b = 0; b < nb; ++b) order[b] = b;
    for (unsigned long long number = 1; number <= 3; ++number) {
        std::shuffle(order.begin(), order.end(), rng);
        std::vector<int> gleaders(8 * ngmax + 8, 0), xleaders(8, 0);
        int arrived = 0;
        for (int b : order) {
            ++arrived;
            const int x = xcd[b];
            const msb::tree::Group t = msb::tree::group_of(rank[b], count[x], G);
            if (t.g < 0 || t.g >= t.ng || t.gsize < 1 || t.gsize > G) {
                std::printf("bad group %d of %d size %d\n", t.g, t.ng, t.gsize);
                return 1;
            }
            const int gi = x * ngmax + t.g;
            if (++gbar[gi] == number * (unsigned long long)t.gsize) {
                ++gleaders[gi];
                if (++xbar[x] == number * (unsigned long long)t.ng) {
                    ++xleaders[x];
                    if (++bar == number * (unsigned long long)nxcd && arrived != nb) {
                        std::printf("global counter complete after %d of %d arrivals\n", arrived, nb);
                        return 1;
                    }
                }
            }
        }
        for (int x = 0; x < 8; ++x) {
            if (count[x] == 0) continue;
            const int ng = msb::tree::group_of(0, count[x], G).ng;
            if (xleaders[x] != 1) {
                std::printf("XCD %d: %d leaders\n", x, xleaders[x]);
                return 1;
            }
            for (int g = 0; g < ng; ++g)
                if (gleaders[x * ngmax + g] != 1) {
                    std::printf("XCD %d group %d: %d leaders\n", x, g, gleaders[x * ngmax + g]);
                    return 1;
                }
        }
        if (bar != number * (unsigned long long)nxcd) {
            std::printf("global counter %llu, expected %llu\n", bar, number * (unsigned long long)nxcd);
            return 1;
        }
    }
    std::printf("OK\n");
    return 0;
}
