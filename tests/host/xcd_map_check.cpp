// Host-side check of the XCD-aware work mappings (iblb_internal.h):
//  - xcd_item(w, n) is a bijection of [0, n), and the workgroups of each
//    XCD (w % 8) take one contiguous, increasing range of items;
//  - xcd_list_range over a grid of g workgroups (four waves each, g a
//    multiple of eight) visits every list position in [0, count) exactly
//    once, each wave staying inside its XCD's eighth of the list.
// Prints the number of cases and exits non-zero on the first mismatch.
#include "iblb_internal.h"

#include <cstdio>
#include <vector>

int main() {
    long cases = 0;
    for (int n = 1; n <= 4200; ++n) {
        std::vector<int> seen(n, 0);
        int prev[8];
        for (int x = 0; x < 8; ++x) prev[x] = -2;
        for (int w = 0; w < n; ++w) {
            const int it = iblb::xcd_item(w, n);
            if (it < 0 || it >= n || seen[it]++) {
                std::printf("xcd_item: n %d w %d -> %d (out of range or repeated)\n", n, w, it);
                return 1;
            }
            const int x = w & 7;
            if (prev[x] != -2 && it != prev[x] + 1) {
                std::printf("xcd_item: n %d w %d -> %d, previous item of XCD %d was %d\n", n, w, it, x, prev[x]);
                return 1;
            }
            prev[x] = it;
        }
        ++cases;
    }
    std::vector<int> counts;
    for (int c = 0; c <= 3000; ++c) counts.push_back(c);
    for (int c : {4095, 4096, 4097, 32767, 32768, 32769, 41568, 65536, 100003, 262144}) counts.push_back(c);
    for (int g : {8, 16, 24, 64, 1024, 8192})
        for (int count : counts) {
            if (g == 8192 && count > 3000 && count % 7 != 0 && count != 41568 && count != 262144) continue;
            std::vector<int> seen(count, 0);
            for (int b = 0; b < g; ++b)
                for (int v = 0; v < 4; ++v) {
                    const iblb::ListRange r = iblb::xcd_list_range(b, v, g, count);
                    const int x = b & 7;
                    const long lo = (long)count * x / 8, hi = (long)count * (x + 1) / 8;
                    if (r.end != hi || r.stride != g / 2) {
                        std::printf("xcd_list_range: g %d count %d b %d v %d: end %d stride %d\n", g, count, b, v,
                                    r.end, r.stride);
                        return 1;
                    }
                    for (int i = r.first; i < r.end; i += r.stride) {
                        if (i < lo || i >= count || seen[i]++) {
                            std::printf("xcd_list_range: g %d count %d b %d v %d visits %d twice or outside [%ld, %ld)\n",
                                        g, count, b, v, i, lo, hi);
                            return 1;
                        }
                    }
                }
            for (int i = 0; i < count; ++i)
                if (seen[i] != 1) {
                    std::printf("xcd_list_range: g %d count %d: position %d visited %d times\n", g, count, i, seen[i]);
                    return 1;
                }
            ++cases;
        }
    std::printf("xcd maps: %ld cases ok\n", cases);
    return 0;
}
