// Host check of the propagation's wave roles (csrc/roles.h): for every wave
// count, column-block count, row-block count and rotation, each (row block,
// column block) has exactly one owning wave, no SIMD carries more products
// than without the split, and the 80-orbital workgroup at M = 200 (16 waves,
// 13 column blocks, 5 row blocks) has at most 17 of its 65 products on one
// SIMD.  Prints "ok" and exits 0 when all hold.
#include <cstdio>
#include <vector>

#include "roles.h"

int main() {
    int fails = 0, worst_m200 = 0;
    for (int nwave : {4, 8, 16})
        for (int MB = 1; MB <= nwave; ++MB)
            for (int nrbv = 1; nrbv <= 5; ++nrbv)
                for (int L = 0; L < nwave; ++L) {
                    std::vector<int> owner(MB * nrbv, -1);
                    int simd[4] = {0, 0, 0, 0}, base[4] = {0, 0, 0, 0};
                    for (int w = 0; w < nwave; ++w) {
                        const int vw = (w + L) % nwave;
                        if (vw < MB) base[w % 4] += nrbv;
                        int col = vw, rlo = 0, rhi = nrbv;
                        afq::dev::balance_roles(nwave, MB, nrbv, vw, col, rlo, rhi);
                        if (col >= MB) continue;
                        if (rlo < 0 || rhi > nrbv || rlo > rhi) ++fails;
                        for (int r = rlo; r < rhi && r >= 0 && r < nrbv; ++r) {
                            if (owner[r * MB + col] >= 0) ++fails;
                            owner[r * MB + col] = w;
                        }
                        simd[w % 4] += rhi - rlo;
                    }
                    for (int o : owner)
                        if (o < 0) ++fails;
                    int mx = 0, mb = 0;
                    for (int k = 0; k < 4; ++k) {
                        mx = simd[k] > mx ? simd[k] : mx;
                        mb = base[k] > mb ? base[k] : mb;
                    }
                    if (mx > mb) ++fails;
                    if (nwave == 16 && MB == 13 && nrbv == 5 && mx > worst_m200) worst_m200 = mx;
                }
    if (worst_m200 != 17) ++fails;
    if (fails) {
        std::printf("FAIL %d (M = 200 busiest SIMD %d)\n", fails, worst_m200);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
