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

// K range length of a split GEMM: ceil(k / ksplit) rounded up to 32, so the
// ranges start on vector boundaries and do not depend on the tile shape.
__host__ __device__ inline int gemm_kchunk_dev(int k, int ksplit) {
    const int c = (k + ksplit - 1) / ksplit;
    return (c + 31) / 32 * 32;
}

// C = alpha sum_z ws[z] (+ beta C; C2 = alpha sum), z in order, in FP64.
template <typename AccS, typename TO>
__global__ __launch_bounds__(256) void k_ksum(Gemm g) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long)g.m * g.n) return;
    const long i = idx / g.n, j = idx % g.n;
    const AccS* w = (const AccS*)g.ws;
    double v = 0.0;
    for (int z = 0; z < g.ksplit; ++z) v += (double)w[(long)z * g.m * g.n + idx];
    v *= g.alpha;
    const long ro = rowmap(g.rc, i);
    TO* out = (TO*)g.C;
    if (g.C2) ((TO*)g.C2)[ro + j] = (TO)v;
    if (g.beta != 0.0) v += g.beta * (double)out[ro + j];
    out[ro + j] = (TO)v;
}

template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int BK, int WGM,
          int WGN, int VA, int VB, bool AL>
__global__ __launch_bounds__(64 * WGM * WGN) void k_gemm(Gemm g, int ntn, int ntm) {
    typedef Core<TA, TB, TC, BM, BN, BK, WGM, WGN, VA, VB, AL> C;
    // split-BF16 tiles of 128 rows or more: two LDS buffers (the split and
    // stores of the next K tile overlap the products); the others: one
    constexpr bool DB = std::is_same<TC, Split>::value && AL && BM >= 128;
    __shared__ __attribute__((aligned(16))) typename C::LT As[(DB ? 2 : 1) * C::LDS_A];
    __shared__ __attribute__((aligned(16))) typename C::LT Bs[(DB ? 2 : 1) * C::LDS_B];
    // XCD-aware order: workgroups are dealt to the eight XCDs in turn, so
    // logical tile L = (id mod 8) per + id / 8 gives each XCD a contiguous
    // run of tiles (column tiles fastest): the column tiles of one row block
    // share its A rows in one L2
    const int ks = g.ksplit > 1 ? g.ksplit : 1;
    const long nt = (long)ntn * ntm * ks * g.batch;
    const long per = (nt + 7) / 8;
    const long L = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nt) return;
    const long tpk = (long)ntn * ntm;
    const int b = (int)(L / (tpk * ks));
    const int kz = (int)((L / tpk) % ks);
    const long rem = L % tpk;
    const long row0 = (rem / ntn) * BM, col0 = (rem % ntn) * BN;
    // K range of this workgroup (whole K without split)
    const int kc = ks > 1 ? gemm_kchunk_dev(g.k, ks) : g.k;
    const int k_lo = kz * kc;
    const int k_len = k_lo < g.k ? (g.k - k_lo < kc ? g.k - k_lo : kc) : 0;
    const TA* A = (const TA*)g.A + (long)b * g.a_bs + k_lo;
    const TB* B = (const TB*)g.B + (long)b * g.b_bs + k_lo;
    const int tid = threadIdx.x;
    // rows past the operands: with two LDS buffers they repeat the last row
    // (their products land in outputs that are not stored), else read zero
    long aoff[C::LA], boff[C::LB];
#pragma unroll
    for (int j = 0; j < C::LA; ++j) {
        const long r = row0 + C::arow(j);
        aoff[j] = r < g.m ? rowmap(g.ra, r) : DB ? rowmap(g.ra, g.m - 1) : -1;
    }
#pragma unroll
    for (int j = 0; j < C::LB; ++j) {
        const long r = col0 + C::brow(j);
        boff[j] = r < g.n ? rowmap(g.rb, r) : DB ? rowmap(g.rb, g.n - 1) : -1;
    }
    typename C::accv acc[C::TM][C::TN];
    C::template run<DB, DB>(A, aoff, B, boff, k_len, As, Bs, acc);

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    TO* out = (TO*)g.C + (long)b * g.c_bs;
    TO* out2 = g.C2 ? (TO*)g.C2 + (long)b * g.c_bs : nullptr;
    typedef typename std::conditional<std::is_same<TC, double>::value, double, float>::type AccS;
    if (ks > 1) {
        // partial sums of this K range
        AccS* wsp = (AccS*)g.ws + (long)kz * g.m * g.n;
#pragma unroll
        for (int a = 0; a < C::TM; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long i = row0 + wm * C::TM * 16 + a * 16 + acc_row<AccS>(lane, r);
                if (i >= g.m) continue;
#pragma unroll
                for (int bb = 0; bb < C::TN; ++bb) {
                    const long j = col0 + wn * C::TN * 16 + bb * 16 + (lane & 15);
                    if (j < g.n) wsp[i * g.n + j] = acc[a][bb][r];
                }
            }
        return;
    }
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
    const int ntn = (g.n + BN - 1) / BN, ntm = (g.m + BM - 1) / BM;
    const long nt = (long)ntn * ntm * g.batch * (g.ksplit > 1 ? g.ksplit : 1);
    const dim3 grid((unsigned)(((nt + 7) / 8) * 8));
    constexpr int VA = VW<TA>::v, VB = VW<TB>::v;
    const bool al = rows_aligned(g.A, g.ra, g.a_bs, g.batch, VA, sizeof(TA)) &&
                    rows_aligned(g.B, g.rb, g.b_bs, g.batch, VB, sizeof(TB));
    if (al)
        hipLaunchKernelGGL((k_gemm<TA, TB, TC, TO, BM, BN, BK, WGM, WGN, VA, VB, true>), grid,
                           dim3(64 * WGM * WGN), 0, s, g, ntn, ntm);
    else
        hipLaunchKernelGGL((k_gemm<TA, TB, TC, TO, BM, BN, BK, WGM, WGN, 1, 1, false>), grid,
                           dim3(64 * WGM * WGN), 0, s, g, ntn, ntm);
    return hipGetLastError();
}

// Tile 4: the 256 x 128 tile over 16 wavefronts of 32 x 64 (four per SIMD in
// about 120 registers instead of two in 233, so more waves cover the barrier
// and LDS waits); split BF16 only, other types take the 8-wavefront tile.
template <typename TA, typename TB, typename TC, typename TO, int BK>
hipError_t launch_tile_256x128_16w(const Gemm& g, hipStream_t s) {
    if constexpr (std::is_same<TC, Split>::value)
        return launch_tile<TA, TB, TC, TO, 256, 128, BK, 8, 2>(g, s);
    else
        return launch_tile<TA, TB, TC, TO, 256, 128, BK, 4, 2>(g, s);
}

template <typename TA, typename TB, typename TC, typename TO>
hipError_t launch_gemm(const Gemm& g, hipStream_t s) {
    const long tiles128 = ((long)(g.m + 127) / 128) * ((g.n + 127) / 128) * g.batch;
    constexpr int BK = Info<TC>::KM == 4 ? 16 : 32;
    const bool big = g.tile ? g.tile == 2 : (g.m >= 96 && g.n >= 96 && tiles128 >= 512);
    hipError_t e;
    if (g.tile == 4)
        e = launch_tile_256x128_16w<TA, TB, TC, TO, BK>(g, s);
    else if (g.tile == 3)
        e = launch_tile<TA, TB, TC, TO, 256, 128, BK, 4, 2>(g, s);
    else if (big)
        e = launch_tile<TA, TB, TC, TO, 128, 128, BK, 2, 2>(g, s);
    else
        e = launch_tile<TA, TB, TC, TO, 64, 64, BK, 2, 2>(g, s);
    if (e != hipSuccess || g.ksplit <= 1) return e;
    typedef typename std::conditional<std::is_same<TC, double>::value, double, float>::type AccS;
    const long n = (long)g.m * g.n;
    hipLaunchKernelGGL((k_ksum<AccS, TO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g);
    return hipGetLastError();
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
#pragma unroll 4
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
    // walker u: the partial sums of its tpu threads, strided over one
    // wavefront's lanes and folded by a butterfly (fixed order)
    for (int uu = wave; uu < W; uu += NT / 64) {
        double a = 0.0, b = 0.0;
        for (int t = uu * tpu + lane; t < uu * tpu + tpu; t += 64) {
            a += red[2 * t];
            b += red[2 * t + 1];
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            a += __shfl_xor(a, o, 64);
            b += __shfl_xor(b, o, 64);
        }
        const int w = w0 + uu;
        if (lane == 0 && w < nw) {
            double* o = out + ((long)(w * 2 + spin) * n_gt + gt) * 2;
            o[0] = a;
            o[1] = b;
        }
    }
}

// Exchange with whole gamma blocks per wavefront, for spin blocks of 17..48
// orbitals padded to NB (a multiple of 8).  Wavefront (wm, wn) of the 2 x 2
// workgroup owns G gamma blocks (rows gamma, i: R = G NB, a multiple of 16)
// of one walker (columns plane, j: C = 2 NB), so its R x C tile holds whole
// N_s x N_s blocks and the pairing T_ij T_ji stays inside the wavefront: one
// gamma block at a time goes row-major to the wavefront's own LDS region, and
// each lane multiplies its accumulators T_ij (four consecutive i at one j)
// with the partners T_ji (four consecutive floats of row j, per plane).  The
// lane sums run over all ordered (i, j) and are folded by a butterfly.
// Output slot: walker, spin, gamma group gg (G blocks each).
template <int NB, int G>
struct ExchBlk {
    static constexpr int R = G * NB, C = 2 * NB, BM = 2 * R, BN = 2 * C;
    static constexpr int PW = C + 4;  // row pitch of a stored block (floats)
    typedef Core<float, float, Split, BM, BN, 32, 2, 2, 4, 4, true> Cr;
    // two operand buffers (the split of the next K tile overlaps the
    // products; 80 KB at N_s = 40, so two workgroups share a CU's 160 KB),
    // reused after the K loop for the four wavefronts' block regions
    static constexpr int OPB = 2 * (Cr::LDS_A + Cr::LDS_B) * (int)sizeof(bf16_t);
    static constexpr int EPB = 4 * NB * PW * (int)sizeof(float);
    static constexpr int SMEM = OPB > EPB ? OPB : EPB;
};

template <int NB, int G>
__global__ __launch_bounds__(256, 2) void k_exchange_blk(const float* __restrict__ lhalf,
                                                      const float* __restrict__ theta,
                                                      double* __restrict__ out, int nw, int M,
                                                      int N, int n_chol, int off, int nsig,
                                                      int spin, int n_gt, int n_gtw, int n_wt) {
    typedef ExchBlk<NB, G> E;
    typedef typename E::Cr Cr;
    __shared__ __attribute__((aligned(16))) char smem[E::SMEM];
    bf16_t* As = reinterpret_cast<bf16_t*>(smem);
    bf16_t* Bs = As + 2 * Cr::LDS_A;
    float* S = reinterpret_cast<float*>(smem);

    // XCD-aware tile order: each XCD takes a contiguous range of logical
    // tiles, walked in super-tiles of 8 gamma groups x 8 walker pairs, so the
    // workgroups one XCD runs together share 8 L^half and 8 Theta tiles in
    // its L2 instead of streaming one operand from memory
    const int n_sg = (n_gtw + 7) / 8, n_sw = (n_wt + 7) / 8;
    const long nblk = (long)n_sg * n_sw * 64;
    const long per = (nblk + 7) / 8;
    const long L = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblk) return;
    const long st = L / 64;
    const int loc = (int)(L % 64);
    const int gt = (int)(st % n_sg) * 8 + (loc & 7), wt = (int)(st / n_sg) * 8 + (loc >> 3);
    if (gt >= n_gtw || wt >= n_wt) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const long NM = (long)N * M;
    const int g0 = gt * 2 * G, w0 = wt * 2;
    long aoff[Cr::LA], boff[Cr::LB];
#pragma unroll
    for (int j = 0; j < Cr::LA; ++j) {
        const int r = Cr::arow(j);
        const int g = g0 + r / NB, i = r % NB;
        aoff[j] = (i < nsig && g < n_chol) ? (long)g * NM + (long)(off + i) * M : -1;
    }
#pragma unroll
    for (int j = 0; j < Cr::LB; ++j) {
        const int c = Cr::brow(j);
        const int u = c / (2 * NB), p = (c / NB) & 1, jj = c % NB;
        const int w = w0 + u;
        boff[j] = (jj < nsig && w < nw) ? (long)(2 * w + p) * NM + (long)(off + jj) * M : -1;
    }
    typename Cr::accv acc[Cr::TM][Cr::TN];
    Cr::template run<true>(lhalf, aoff, theta, boff, M, As, Bs, acc);
    // the operand buffers are free (the K loop ends on a barrier); this
    // wavefront's block region
    constexpr int PW = E::PW;
    float* Sw = S + wave * NB * PW;
    const int li = lane & 15, rq = 4 * (lane >> 4);
    float fr = 0.0f, fi = 0.0f;
#pragma unroll
    for (int gb = 0; gb < G; ++gb) {
        // block gb's rows (gamma, i), row-major (columns plane, j)
#pragma unroll
        for (int a = 0; a < Cr::TM; ++a) {
            const int r0 = a * 16 + rq;  // four rows r0 .. r0 + 3, one block
            if (r0 / NB != gb) continue;
#pragma unroll
            for (int b = 0; b < Cr::TN; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) Sw[(r0 - gb * NB + q) * PW + b * 16 + li] = acc[a][b][q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int a = 0; a < Cr::TM; ++a) {
            const int r0 = a * 16 + rq;
            if (r0 / NB != gb) continue;
            const int i0 = r0 - gb * NB;
#pragma unroll
            for (int b = 0; b < Cr::TN; ++b) {
                const int c = b * 16 + li, p = c / NB, j = c % NB;
                // partners of T_(i0+q) j: T_j(i0+q) in planes 0 (a) and 1 (b)
                const f4 pa = *reinterpret_cast<const f4*>(&Sw[j * PW + i0]);
                const f4 pb = *reinterpret_cast<const f4*>(&Sw[j * PW + NB + i0]);
                const f4 t = acc[a][b];
                if (p == 0) {  // t = Re T_ij: Re += a_ij a_ji, Im += a_ij b_ji
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        fr += t[q] * pa[q];
                        fi += t[q] * pb[q];
                    }
                } else {  // t = Im T_ij: Re -= b_ij b_ji, Im += b_ij a_ji
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        fr -= t[q] * pb[q];
                        fi += t[q] * pa[q];
                    }
                }
            }
        }
        // every lane's reads of this block before the next block's stores
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    double sr = fr, si = fi;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        sr += __shfl_xor(sr, o, 64);
        si += __shfl_xor(si, o, 64);
    }
    const int w = w0 + wn, gg = gt * 2 + wm;
    if (lane == 0 && w < nw && gg < n_gt) {
        double* o = out + ((long)(w * 2 + spin) * n_gt + gg) * 2;
        o[0] = sr;
        o[1] = si;
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

// Gamma blocks per wavefront of the block kernel (0: not used for this
// spin block): split-BF16 contractions, 17..48 orbitals, M a multiple of 4.
int exch_blk_g(int nsig, int M, DType t) {
    if (t != DT_SPLIT || M % 4 || nsig <= 16 || nsig > 48) return 0;
    const int nb = (nsig + 7) / 8 * 8;
    return nb == 48 ? 1 : 2;
}

template <int NB, int G>
hipError_t launch_exchange_blk(const void* lhalf, const void* theta, double* out, int nw, int M,
                               int N, int n_chol, int off, int nsig, int spin, int n_gt,
                               hipStream_t s) {
    const int n_gtw = (n_chol + 2 * G - 1) / (2 * G), n_wt = (nw + 1) / 2;
    const long nblk = (long)((n_gtw + 7) / 8) * ((n_wt + 7) / 8) * 64;
    const long grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_exchange_blk<NB, G>), dim3(grid), dim3(256), 0, s, (const float*)lhalf,
                       (const float*)theta, out, nw, M, N, n_chol, off, nsig, spin, n_gt, n_gtw,
                       n_wt);
    return hipGetLastError();
}

}  // namespace

int gemm_kchunk(int k, int ksplit) { return gemm_kchunk_dev(k, ksplit); }

size_t gemm_ws_bytes(int m, int n, int ksplit, DType compute) {
    if (ksplit <= 1) return 0;
    return (size_t)ksplit * m * n * (compute == DT_F64 ? 8 : 4);
}

hipError_t gemm(const Gemm& g, DType compute, hipStream_t s) {
    if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return hipSuccess;
    if (g.ksplit > 1 && (g.batch != 1 || !g.ws || g.k <= 0))
        return hipErrorInvalidValue;
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

int exchange_gtiles(int n_chol, int nsig, int M, DType t) {
    if (nsig <= 0) return 0;
    const int gb = exch_blk_g(nsig, M, t);
    const int G = gb ? gb : exch_cfg(t).BM / nsig;
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
            if (exch_blk_g(nsig, M, t) && (uintptr_t)lhalf % 16 == 0 &&
                (uintptr_t)theta % 16 == 0) {
                switch ((nsig + 7) / 8 * 8) {
                    case 24:
                        return launch_exchange_blk<24, 2>(lhalf, theta, out, nw, M, N, n_chol, off,
                                                          nsig, spin, n_gt, s);
                    case 32:
                        return launch_exchange_blk<32, 2>(lhalf, theta, out, nw, M, N, n_chol, off,
                                                          nsig, spin, n_gt, s);
                    case 40:
                        return launch_exchange_blk<40, 2>(lhalf, theta, out, nw, M, N, n_chol, off,
                                                          nsig, spin, n_gt, s);
                    default:
                        return launch_exchange_blk<48, 1>(lhalf, theta, out, nw, M, N, n_chol, off,
                                                          nsig, spin, n_gt, s);
                }
            }
            return launch_exchange<float, Split, 128, 256, 32, 2, 4>(lhalf, theta, out, nw, M, N,
                                                                    n_chol, off, nsig, spin, n_gt,
                                                                    s);
    }
    return hipErrorInvalidValue;
}

}  // namespace afq
