// Host-side check of tile_run (iblb_internal.h): for every axis length,
// tile size, start and span in range, the tiles it lists are exactly the
// distinct tiles of the cells lo .. lo + span - 1 (wrapped on a periodic
// axis), each once.  Prints the number of cases and exits non-zero on the
// first mismatch.
#include "iblb_internal.h"

#include <cstdio>
#include <set>
#include <vector>

int main() {
    long cases = 0;
    for (int per = 0; per < 2; ++per)
        for (int sh : {0, 1, 2, 4, 5})
            for (int n = 1; n <= 70; ++n)
                for (int lo = 0; lo < n; ++lo)
                    for (int span = 0; span <= 80; ++span) {
                        if (!per && lo + span > n) continue;
                        std::set<int> want;
                        for (int k = 0; k < span; ++k) want.insert(((lo + k) % n) >> sh);
                        const iblb::TileRun r = iblb::tile_run(lo, span, n, sh, per != 0);
                        const int nt = (n + (1 << sh) - 1) >> sh;
                        std::vector<int> got;
                        for (int k = 0; k < r.count; ++k) {
                            int t = r.first + k;
                            if (per && t >= nt) t -= nt;
                            got.push_back(t);
                        }
                        const std::set<int> gs(got.begin(), got.end());
                        ++cases;
                        if (gs != want || got.size() != gs.size() || (int)want.size() != r.count) {
                            std::printf("mismatch: per %d sh %d n %d lo %d span %d: first %d count %d, want %zu tiles\n",
                                        per, sh, n, lo, span, r.first, r.count, want.size());
                            return 1;
                        }
                    }
    std::printf("tile_run: %ld cases ok\n", cases);
    return 0;
}
