// Host check of the strip launch's bucket order (csrc/strip_pack.h): random
// buckets of problems with 1..10 strips; every strip exactly once, no more
// wavefronts than the strips need, a problem of four strips (or a multiple
// of four) never split, and a problem of two or three strips split only when
// no pairing was left for it.  Built with the address and undefined-behaviour
// sanitizers by tests/test_pack_cpu.py.
#include <cstdio>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "strip_pack.h"

struct Item {
    int prob, strip, ncols;
};

int main() {
    std::mt19937 rng(12345);
    for (int trial = 0; trial < 20000; ++trial) {
        const int np = (int)(rng() % 40) + 1;
        const int kmax = trial % 2 ? 4 : 10;
        std::vector<Item> v;
        std::vector<hsma::StripSpan> sp;
        for (int p = 0; p < np; ++p) {
            const int k = (int)(rng() % kmax) + 1;
            const int first = (int)v.size();
            for (int s = 0; s < k; ++s) v.push_back({p, s, 16});
            sp.push_back({first, k});
        }
        std::vector<Item> out;
        hsma::pack_bucket(v, sp, out);
        if (out.size() != v.size()) {
            std::printf("trial %d: %zu strips out, %zu in\n", trial, out.size(), v.size());
            return 1;
        }
        std::set<std::pair<int, int>> seen;
        for (const Item &x : out)
            if (!seen.insert({x.prob, x.strip}).second) {
                std::printf("trial %d: strip (%d, %d) twice\n", trial, x.prob, x.strip);
                return 1;
            }
        // wavefronts each problem's strips land in
        std::vector<std::set<size_t>> waves(np);
        for (size_t i = 0; i < out.size(); ++i) waves[out[i].prob].insert(i / 4);
        int r[4] = {0, 0, 0, 0};
        for (const hsma::StripSpan &s : sp) r[s.k % 4]++;
        for (int p = 0; p < np; ++p) {
            const int k = sp[p].k;
            const size_t need = (size_t)(k + 3) / 4;
            if (k % 4 == 0 && waves[p].size() != need) {
                std::printf("trial %d: problem of %d strips over %zu wavefronts\n", trial, k, waves[p].size());
                return 1;
            }
        }
        // With remainders that pair exactly (as many 3s as 1s, an even number
        // of 2s, a multiple of four 1s left), nothing is split beyond need.
        if (r[3] == r[1] && r[2] % 2 == 0) {
            for (int p = 0; p < np; ++p) {
                const size_t need = (size_t)(sp[p].k + 3) / 4;
                if (waves[p].size() != need) {
                    std::printf("trial %d: problem %d (%d strips) over %zu wavefronts\n", trial, p,
                                sp[p].k, waves[p].size());
                    return 1;
                }
            }
        }
    }
    std::printf("pack ok\n");
    return 0;
}
