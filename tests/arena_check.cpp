// Randomised check of the server arena's first-fit carving against a brute-force map of 256-B
// granules: a carve succeeds exactly when a run of free granules can hold it, carved ranges never
// overlap, and the holes are always exactly the free granules, disjoint and never adjacent.
#include <cstdint>
#include <cstdio>
#include <random>
#include <utility>
#include <vector>

#include "arena.h"

int main()
{
    std::mt19937 rng(1);
    for (int trial = 0; trial < 300; ++trial) {
        const int64_t n = 256 * (1 + rng() % 64);
        std::vector<char> buf(n);
        dpk::Arena a;
        a.reset(buf.data(), n);
        std::vector<int> used(n / 256, 0);
        std::vector<std::pair<int64_t, int64_t>> live;
        for (int step = 0; step < 400; ++step) {
            if (!live.empty() && rng() % 2) {
                const size_t k = rng() % live.size();
                const auto [off, b] = live[k];
                a.give_back(off, b);
                for (int64_t g = off / 256; g < off / 256 + (b + 255) / 256; ++g) used[g] = 0;
                live.erase(live.begin() + k);
            } else {
                const int64_t b = 1 + rng() % (n / 3 + 1), gb = (b + 255) / 256;
                const int64_t off = a.carve(b);
                bool fits = false;
                int run = 0;
                for (size_t g = 0; g < used.size() && !fits; ++g) {
                    run = used[g] ? 0 : run + 1;
                    fits = run >= gb;
                }
                if ((off >= 0) != fits) {
                    std::printf("carve of %lld bytes: %lld, brute force %d\n", (long long)b, (long long)off, fits);
                    return 1;
                }
                if (off >= 0) {
                    if (off % 256 || !a.owns(buf.data() + off)) return 2;
                    for (int64_t g = off / 256; g < off / 256 + gb; ++g) {
                        if (used[g]) return 3;
                        used[g] = 1;
                    }
                    live.push_back({off, b});
                }
            }
            std::vector<int> hole(n / 256, 0);
            int64_t end = -1;
            for (const auto& h : a.holes) {
                if (h.first <= end) return 4;   // overlapping or adjacent holes
                end = h.first + h.second;
                for (int64_t g = h.first / 256; g < end / 256; ++g) hole[g] = 1;
            }
            for (size_t g = 0; g < used.size(); ++g)
                if (hole[g] == used[g]) return 5;
        }
    }
    std::printf("arena ok\n");
    return 0;
}
