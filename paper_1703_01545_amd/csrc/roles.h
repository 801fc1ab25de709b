// Work split of the 80-orbital propagation workgroup over its waves.  Host
// and device: the kernel calls it per wave, and a host program checks its
// invariants.
#pragma once
#include <hip/hip_runtime.h>

namespace afq {
namespace dev {

// One column block per wave and fewer column blocks than waves: the idle
// waves take over the upper row blocks of some columns, so that the four
// SIMDs carry nearly equal numbers of (row block, column block) products
// (wave w runs on SIMD w mod 4; roles vw are the waves rotated, and with a
// wave count that is a multiple of 4 the roles vw mod 4 = k share one SIMD).
// Greedy and wave-uniform: each idle role in turn splits an unsplit column of
// the most loaded SIMD when that lowers the largest load; the column keeps its
// lower rs row blocks, the idle role takes the rest.  Every (row block, column
// block) keeps exactly one owner and the same order of products.
__host__ __device__ __forceinline__ void balance_roles(int nwave, int MB, int nrbv, int vw,
                                                      int& col, int& rlo, int& rhi) {
    const int moved = nrbv / 2, rs = nrbv - moved;
    if (moved == 0 || MB >= nwave) return;
    int load[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) load[k] = nrbv * ((MB - k + 3) / 4);
    unsigned split = 0;
    for (int u = MB; u < nwave; ++u) {
        int h = 0, hl = load[0], lu = load[0];
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            if (load[k] > hl) h = k, hl = load[k];
            if (k == (u & 3)) lu = load[k];
        }
        if (lu + moved >= hl) continue;  // no gain: the role stays idle
        int c = -1;
        for (int x = h; x < MB; x += 4)
            if (!((split >> x) & 1u)) {
                c = x;
                break;
            }
        if (c < 0) continue;
        split |= 1u << c;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k == h) load[k] -= moved;
            if (k == (u & 3)) load[k] += moved;
        }
        if (u == vw) col = c, rlo = rs;
    }
    if (vw < MB && ((split >> vw) & 1u)) rhi = rs;
}

}  // namespace dev
}  // namespace afq
