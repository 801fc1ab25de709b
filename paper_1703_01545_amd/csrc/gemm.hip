// Tiled MFMA contractions for gfx950 (CDNA4, 64-wide wavefronts).
//
// Every Cholesky contraction of the walker step is a real GEMM once the
// complex walker planes are laid out as extra rows or columns:
//   force bias     F[(w,p), g]   = sum_(i,m) Theta[(w,p), (i,m)] L^half[g, (i,m)]
//   field sum      A[(w,p), q]   = sum_g X[(w,p), g] Lpacked[q, g]
//   overlap        O[(w,p,i), j] = sum_m Phi[(w,p,i), m] PhiT[j, m]
// (all operands K-contiguous: the "TN" form C = A B^T).  The exchange term
// of the local energy needs whole N_s x N_s blocks of T = L^half Theta in
// one tile and has its own kernel on the same core.
#include "mfma.h"

namespace afq {
namespace {

using namespace dev;

template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int BK, int WGM,
          int WGN, int VA, int VB, bool AL>
__global__ __launch_bounds__(64 * WGM * WGN) void k_gemm(Gemm g) {
    typedef Core<TA, TB, TC, BM, BN, BK, WGM, WGN, VA, VB, AL> C;
    __shared__ __attribute__((aligned(16))) typename C::LT As[C::LDS_A];
    __shared__ __attribute__((aligned(16))) typename C::LT Bs[C::LDS_B];
    const int b = blockIdx.z;
    const long row0 = (long)blockIdx.y * BM, col0 = (long)blockIdx.x * BN;
    const TA* A = (const TA*)g.A + (long)b * g.a_bs;
    const TB* B = (const TB*)g.B + (long)b * g.b_bs;
    const int tid = threadIdx.x;
    long aoff[C::LA], boff[C::LB];
#pragma unroll
    for (int j = 0; j < C::LA; ++j) {
        const long r = row0 + C::arow(j);
        aoff[j] = r < g.m ? rowmap(g.ra, r) : -1;
    }
#pragma unroll
    for (int j = 0; j < C::LB; ++j) {
        const long r = col0 + C::brow(j);
        boff[j] = r < g.n ? rowmap(g.rb, r) : -1;
    }
    typename C::accv acc[C::TM][C::TN];
    C::run(A, aoff, B, boff, g.k, As, Bs, acc);

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    TO* out = (TO*)g.C + (long)b * g.c_bs;
    TO* out2 = g.C2 ? (TO*)g.C2 + (long)b * g.c_bs : nullptr;
    typedef typename std::conditional<std::is_same<TC, double>::value, double, float>::type AccS;
#pragma unroll
    for (int a = 0; a < C::TM; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long i = row0 + wm * C::TM * 16 + a * 16 + acc_row<AccS>(lane, r);
            if (i >= g.m) continue;
            const long ro = rowmap(g.rc, i);
#pragma unroll
            for (int bb = 0; bb < C::TN; ++bb) {
                const long j = col0 + wn * C::TN * 16 + bb * 16 + (lane & 15);
                if (j >= g.n) continue;
                double v = g.alpha * (double)acc[a][bb][r];
                if (out2) out2[ro + j] = (TO)v;
                if (g.beta != 0.0) v += g.beta * (double)out[ro + j];
                out[ro + j] = (TO)v;
            }
        }
    }
}

// Rows of an operand can be read with 16-byte loads: every row offset and
// the base pointer aligned to one vector.
bool rows_aligned(const void* p, const RowMap& r, long bs, int batch, int v, size_t es) {
    if (((uintptr_t)p) % 16) return false;
    if (r.base % v || r.s_out % v || (r.n_in != 1 && r.s_in % v)) return false;
    if (batch > 1 && bs % v) return false;
    (void)es;
    return true;
}

template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int BK, int WGM,
          int WGN>
hipError_t launch_tile(const Gemm& g, hipStream_t s) {
    dim3 grid((g.n + BN - 1) / BN, (g.m + BM - 1) / BM, g.batch);
    constexpr int VA = VW<TA>::v, VB = VW<TB>::v;
    const bool al = rows_aligned(g.A, g.ra, g.a_bs, g.batch, VA, sizeof(TA)) &&
                    rows_aligned(g.B, g.rb, g.b_bs, g.batch, VB, sizeof(TB));
    if (al)
        hipLaunchKernelGGL((k_gemm<TA, TB, TC, TO, BM, BN, BK, WGM, WGN, VA, VB, true>), grid,
                           dim3(64 * WGM * WGN), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm<TA, TB, TC, TO, BM, BN, BK, WGM, WGN, 1, 1, false>), grid,
                           dim3(64 * WGM * WGN), 0, s, g);
    return hipGetLastError();
}

template <typename TA, typename TB, typename TC, typename TO>
hipError_t launch_gemm(const Gemm& g, hipStream_t s) {
    const long tiles128 = ((long)(g.m + 127) / 128) * ((g.n + 127) / 128) * g.batch;
    constexpr int BK = Info<TC>::KM == 4 ? 16 : 32;
    const bool big = g.tile ? g.tile == 2 : (g.m >= 96 && g.n >= 96 && tiles128 >= 512);
    if (big) return launch_tile<TA, TB, TC, TO, 128, 128, BK, 2, 2>(g, s);
    return launch_tile<TA, TB, TC, TO, 64, 64, BK, 2, 2>(g, s);
}

// ---------------------------------------------------------------------------
// Exchange: tile rows = G whole gamma blocks (G * nsig rows of (gamma, i)),
// tile columns = W whole walkers (W * 2 nsig columns of (walker, plane, j)),
// K = M.  After the MFMA loop the tile T goes to LDS and each walker's
// sum_ij T_ij T_ji is reduced in a fixed order.  Tiles are ordered so that
// the workgroups one XCD runs back to back share a walker group (its Theta
// stays in that XCD's L2) and stream L^half.
template <typename TS, typename TC, int BM, int BN, int BK, int WGM, int WGN, int V, bool AL>
__global__ __launch_bounds__(64 * WGM * WGN) void k_exchange(
    const TS* __restrict__ lhalf, const TS* __restrict__ theta, double* __restrict__ out, int nw,
    int M, int N, int n_chol, int off, int nsig, int spin, int G, int W, int n_gt, int n_wt) {
    typedef Core<TS, TS, TC, BM, BN, BK, WGM, WGN, V, V, AL> C;
    constexpr int NT = C::NT;
    typedef typename std::conditional<std::is_same<TC, double>::value, double, float>::type accs;
    constexpr int SP = BN + 4;  // 4 SP = 16 (mod 64 banks): conflict-free tile stores
    constexpr int OPB = (C::LDS_A + C::LDS_B) * sizeof(typename C::LT);
    constexpr int SB = BM * SP * sizeof(accs);
    constexpr int SMEM = OPB > SB ? OPB : SB;
    __shared__ __attribute__((aligned(16))) char smem[SMEM];
    __shared__ double red[NT * 2];
    typename C::LT* As = reinterpret_cast<typename C::LT*>(smem);
    typename C::LT* Bs = As + C::LDS_A;
    accs* S = reinterpret_cast<accs*>(smem);

    // XCD-aware tile order: consecutive logical tiles on one XCD
    const long nblk = (long)n_gt * n_wt;
    const long per = (nblk + 7) / 8;
    const long L = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblk) return;
    const int wt = (int)(L / n_gt), gt = (int)(L % n_gt);

    const int tid = threadIdx.x;
    const long NM = (long)N * M;
    const int g0 = gt * G, w0 = wt * W;
    const int rows_valid = G * nsig, cols_valid = W * 2 * nsig;
    long aoff[C::LA], boff[C::LB];
#pragma unroll
    for (int j = 0; j < C::LA; ++j) {
        const int r = C::arow(j);
        const int g = g0 + r / nsig, i = r % nsig;
        aoff[j] = (r < rows_valid && g < n_chol) ? (long)g * NM + (long)(off + i) * M : -1;
    }
#pragma unroll
    for (int j = 0; j < C::LB; ++j) {
        const int c = C::brow(j);
        const int u = c / (2 * nsig), p = (c / nsig) & 1, jj = c % nsig;
        const int w = w0 + u;
        boff[j] = (c < cols_valid && w < nw) ? (long)(2 * w + p) * NM + (long)(off + jj) * M : -1;
    }
    typename C::accv acc[C::TM][C::TN];
    C::run(lhalf, aoff, theta, boff, M, As, Bs, acc);
    // the operand tiles are dead after the final barrier of run(): reuse as S
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
#pragma unroll
    for (int a = 0; a < C::TM; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = wm * C::TM * 16 + a * 16 + acc_row<accs>(lane, r);
#pragma unroll
            for (int b = 0; b < C::TN; ++b) {
                const int j = wn * C::TN * 16 + b * 16 + (lane & 15);
                S[i * SP + j] = acc[a][b][r];
            }
        }
    __syncthreads();
    const int tpu = NT / W;
    const int u = tid / tpu, sub = tid % tpu;
    double sr = 0.0, si = 0.0;
    if (u < W) {
        const int cb = u * 2 * nsig;
        for (int idx = sub; idx < G * nsig; idx += tpu) {
            const int g = idx / nsig, i = idx % nsig;
            if (g0 + g >= n_chol) break;
            const int rb = g * nsig;
            for (int j = 0; j < nsig; ++j) {
                const double tr_ij = S[(rb + i) * SP + cb + j];
                const double ti_ij = S[(rb + i) * SP + cb + nsig + j];
                const double tr_ji = S[(rb + j) * SP + cb + i];
                const double ti_ji = S[(rb + j) * SP + cb + nsig + i];
                sr += tr_ij * tr_ji - ti_ij * ti_ji;
                si += tr_ij * ti_ji + ti_ij * tr_ji;
            }
        }
    }
    red[2 * tid] = sr;
    red[2 * tid + 1] = si;
    __syncthreads();
    if (tid < W) {
        const int w = w0 + tid;
        if (w < nw) {
            double a = 0.0, b = 0.0;
            for (int t = tid * tpu; t < tid * tpu + tpu; ++t) {
                a += red[2 * t];
                b += red[2 * t + 1];
            }
            double* o = out + ((long)(w * 2 + spin) * n_gt + gt) * 2;
            o[0] = a;
            o[1] = b;
        }
    }
}

struct ExchCfg {
    int BM, BN;
};
ExchCfg exch_cfg(DType t) {
    if (t == DT_F64) return {128, 128};
    return {128, 256};
}

template <typename TS, typename TC, int BM, int BN, int BK, int WGM, int WGN>
hipError_t launch_exchange(const void* lhalf, const void* theta, double* out, int nw, int M, int N,
                           int n_chol, int off, int nsig, int spin, int n_gt, hipStream_t s) {
    const int G = BM / nsig, W = BN / (2 * nsig);
    const int n_wt = (nw + W - 1) / W;
    const long nblk = (long)n_gt * n_wt;
    const long grid = ((nblk + 7) / 8) * 8;
    constexpr int V = VW<TS>::v;
    const bool al = ((uintptr_t)lhalf % 16 == 0) && ((uintptr_t)theta % 16 == 0) && M % V == 0 &&
                    off * M % V == 0;
    if (al)
        hipLaunchKernelGGL((k_exchange<TS, TC, BM, BN, BK, WGM, WGN, V, true>), dim3(grid),
                           dim3(64 * WGM * WGN), 0, s, (const TS*)lhalf, (const TS*)theta, out, nw,
                           M, N, n_chol, off, nsig, spin, G, W, n_gt, n_wt);
    else
        hipLaunchKernelGGL((k_exchange<TS, TC, BM, BN, BK, WGM, WGN, 1, false>), dim3(grid),
                           dim3(64 * WGM * WGN), 0, s, (const TS*)lhalf, (const TS*)theta, out, nw,
                           M, N, n_chol, off, nsig, spin, G, W, n_gt, n_wt);
    return hipGetLastError();
}

template <typename T>
constexpr DType dt_of() {
    return std::is_same<T, double>::value
               ? DT_F64
               : (std::is_same<T, float>::value
                      ? DT_F32
                      : (std::is_same<T, bf16_t>::value ? DT_BF16 : DT_SPLIT));
}

}  // namespace

hipError_t gemm(const Gemm& g, DType compute, hipStream_t s) {
    if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return hipSuccess;
#define AFQ_G(TA_, TB_, TC_, TO_)                                                       \
    if (g.ta == dt_of<TA_>() && g.tb == dt_of<TB_>() && g.tc == dt_of<TO_>() &&         \
        compute == dt_of<TC_>())                                                         \
        return launch_gemm<TA_, TB_, TC_, TO_>(g, s);
    AFQ_G(double, double, double, double)
    AFQ_G(float, float, float, double)
    AFQ_G(float, float, float, float)
    AFQ_G(double, float, float, float)
    AFQ_G(double, float, float, double)
    AFQ_G(bf16_t, bf16_t, bf16_t, double)
    AFQ_G(bf16_t, bf16_t, bf16_t, float)
    AFQ_G(float, float, Split, double)
    AFQ_G(float, float, Split, float)
    AFQ_G(double, double, float, double)
    AFQ_G(double, double, bf16_t, double)
    AFQ_G(double, double, Split, double)
#undef AFQ_G
    return hipErrorInvalidValue;
}

int exchange_gtiles(int n_chol, int nsig, DType t) {
    if (nsig <= 0) return 0;
    const int G = exch_cfg(t).BM / nsig;
    return (n_chol + G - 1) / G;
}

hipError_t exchange(const void* lhalf, const void* theta, double* out, int nw, int M, int N,
                    int n_chol, int off, int nsig, int spin, int n_gt, DType t, hipStream_t s) {
    if (nsig <= 0 || nw <= 0 || n_chol <= 0) return hipSuccess;
    if (2 * nsig > exch_cfg(t).BN || nsig > exch_cfg(t).BM) return hipErrorInvalidValue;
    switch (t) {
        case DT_F64:
            return launch_exchange<double, double, 128, 128, 16, 2, 2>(lhalf, theta, out, nw, M, N,
                                                                      n_chol, off, nsig, spin,
                                                                      n_gt, s);
        case DT_F32:
            return launch_exchange<float, float, 128, 256, 16, 2, 4>(lhalf, theta, out, nw, M, N,
                                                                    n_chol, off, nsig, spin, n_gt,
                                                                    s);
        case DT_BF16:
            return launch_exchange<bf16_t, bf16_t, 128, 256, 32, 2, 4>(lhalf, theta, out, nw, M, N,
                                                                      n_chol, off, nsig, spin,
                                                                      n_gt, s);
        case DT_SPLIT:
            return launch_exchange<float, Split, 128, 256, 32, 2, 4>(lhalf, theta, out, nw, M, N,
                                                                    n_chol, off, nsig, spin, n_gt,
                                                                    s);
    }
    return hipErrorInvalidValue;
}

}  // namespace afq
