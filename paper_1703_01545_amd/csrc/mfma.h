// Device building blocks shared by the contraction kernels (gfx950):
// MFMA wrappers, storage conversions, split-BF16 operands, vector loads and
// the LDS-staged GEMM core.
//
// MFMA fragment layout (v_mfma_{f64,f32}_16x16x4 and v_mfma_f32_16x16x32_bf16):
// lane l supplies A[l % 16][kb + l / 16] and B^T[l % 16][kb + l / 16]
// (kb + 8 (l / 16) + e, e < 8, for bf16).  Accumulator element r of lane l
// is D[4 (l / 16) + r][l % 16] for the FP32-accumulating instructions and
// D[l / 16 + 4 r][l % 16] for v_mfma_f64_16x16x4.
//
// Split-BF16 ("x3"): an FP32 value x is carried as hi = bf16(x) and
// lo = bf16(x - hi); a product a b is evaluated as a_hi b_hi + a_hi b_lo +
// a_lo b_hi on the BF16 matrix cores with FP32 accumulation (the dropped
// a_lo b_lo term and the two roundings leave a relative error of a few
// 2^-17), three MFMAs where FP32 would need eight 16x16x4 instructions.
#pragma once

#include <type_traits>

#include "internal.h"

namespace afq {
namespace dev {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

// Compute-type tag of the split-BF16 scheme.
struct Split {};

template <typename TC>
struct AccT {
    typedef float s;
    typedef f4 v;
};
template <>
struct AccT<double> {
    typedef double s;
    typedef d4 v;
};

__device__ __forceinline__ d4 mma1(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma1(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma8(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
typedef short s4v __attribute__((ext_vector_type(4)));
// 16 x 16 x 16 BF16 product: lane l supplies k = 4 (l / 16) .. + 3
__device__ __forceinline__ f4 mma4(s4v a, s4v b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Double held by lane l (wave-uniform result).
__device__ __forceinline__ double rdlane(double v, int l) {
    const unsigned long long x = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Maximum of a 64-bit key over the wavefront: DPP prefix maxima within rows
// of 16 lanes (row_shr 1, 2, 4, 8), then across rows (row_bcast 15 into rows
// 1 and 3, row_bcast 31 into rows 2 and 3); lane 63 ends with the maximum.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_max_step(unsigned long long x) {
    const int lo = (int)(unsigned)x, hi = (int)(unsigned)(x >> 32);
    const unsigned l2 = (unsigned)__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
    const unsigned h2 = (unsigned)__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
    const unsigned long long y = ((unsigned long long)h2 << 32) | l2;
    return y > x ? y : x;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
    x = dpp_max_step<0x111, 0xF>(x);
    x = dpp_max_step<0x112, 0xF>(x);
    x = dpp_max_step<0x114, 0xF>(x);
    x = dpp_max_step<0x118, 0xF>(x);
    x = dpp_max_step<0x142, 0xA>(x);
    x = dpp_max_step<0x143, 0xC>(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// Row of accumulator element r held by lane l (see the layout note above).
template <typename TC>
__device__ __forceinline__ int acc_row(int lane, int r) {
    return 4 * (lane >> 4) + r;
}
template <>
__device__ __forceinline__ int acc_row<double>(int lane, int r) {
    return (lane >> 4) + 4 * r;
}

__device__ __forceinline__ long rowmap(const RowMap& r, long i) {
    if (r.n_in == 1) return r.base + i * r.s_out;
    return r.base + (i / r.n_in) * r.s_out + (i % r.n_in) * r.s_in;
}

// ---- storage element -> staging value (double for FP64 compute, else float)
template <typename ST, typename TS>
__device__ __forceinline__ ST stage(TS x) { return (ST)x; }
template <>
__device__ __forceinline__ float stage<float, bf16_t>(bf16_t x) { return (float)x; }
template <>
__device__ __forceinline__ double stage<double, bf16_t>(bf16_t x) { return (double)(float)x; }

__device__ __forceinline__ bf16_t to_bf(float x) { return (bf16_t)x; }

template <typename TC>
struct Info {
    typedef float ST;                // staging type
    static constexpr int KM = 32;    // k per MFMA
    static constexpr int PLANES = 1; // LDS planes per operand (hi/lo for Split)
    typedef bf16_t LT;               // LDS element type
};
template <>
struct Info<double> {
    typedef double ST;
    static constexpr int KM = 4;
    static constexpr int PLANES = 1;
    typedef double LT;
};
template <>
struct Info<float> {
    typedef float ST;
    static constexpr int KM = 4;
    static constexpr int PLANES = 1;
    typedef float LT;
};
template <>
struct Info<Split> {
    typedef float ST;
    static constexpr int KM = 32;
    static constexpr int PLANES = 2;
    typedef bf16_t LT;
};

// LDS row pitch in elements: odd word strides for 4/8-byte types; BF16 rows
// unpadded (BK = 32: 64 bytes), their 16-byte granules swizzled (see lds_index).
template <typename TC, int BK>
struct Pitch {
    static constexpr int v = BK + (sizeof(typename Info<TC>::LT) == 2 ? 0 : 1);
};

// LDS element index of (row r, k) in a tile of pitch PK.  BF16 tiles (PK =
// 32): granule k / 8 of row r is stored at granule (k / 8) ^ ((r / 4) % 4), so
// that 16 consecutive rows reading one granule (a fragment load, 16 lanes per
// LDS cycle) and four consecutive rows written 8 bytes per lane (32 lanes per
// cycle) each cover the 64 banks once.
template <typename LT, int PK>
__device__ __forceinline__ int lds_index(int r, int k) {
    if constexpr (sizeof(LT) == 2)
        return r * PK + ((((k >> 3) ^ (r >> 2)) & 3) << 3) + (k & 7);
    else
        return r * PK + k;
}

// Store one staged value into the LDS plane(s) of compute type TC.
template <typename TC>
__device__ __forceinline__ void lds_put(typename Info<TC>::LT* p, long plane, int idx,
                                        typename Info<TC>::ST v) {
    if constexpr (std::is_same<TC, Split>::value) {
        const bf16_t hi = to_bf(v);
        p[idx] = hi;
        p[plane + idx] = to_bf(v - (float)hi);
    } else if constexpr (std::is_same<TC, bf16_t>::value) {
        p[idx] = to_bf(v);
    } else {
        p[idx] = v;
    }
}

// Four consecutive staged values (idx a multiple of 4) into the BF16 LDS
// plane(s) of compute type TC with one 8-byte store per plane; the same
// values as four lds_put calls.
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
template <typename TC>
__device__ __forceinline__ void lds_put4(bf16_t* p, long plane, int idx, const float* v) {
    bf4 hi, lo;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        hi[e] = to_bf(v[e]);
        lo[e] = to_bf(v[e] - (float)hi[e]);
    }
    *reinterpret_cast<bf4*>(p + idx) = hi;
    if constexpr (std::is_same<TC, Split>::value) *reinterpret_cast<bf4*>(p + plane + idx) = lo;
}

// Vector width (elements) of one 16-byte global load of storage type TS.
template <typename TS>
struct VW {
    static constexpr int v = 16 / sizeof(TS);
};

// Load V consecutive elements starting at p[kg] into staging registers;
// vector load when the whole run is in range and aligned, else per element
// with k >= K reading as zero.
template <typename ST, typename TS, int V, bool ALIGNED, bool FULL = false>
__device__ __forceinline__ void gload_run(const TS* __restrict__ row, int kg, int K, ST* out) {
    static_assert(!FULL || ALIGNED, "whole-run loads are vector loads");
    if (FULL || (ALIGNED && kg + V <= K)) {
        if constexpr (sizeof(TS) == 8) {
            const d2 x = *reinterpret_cast<const d2*>(row + kg);
            out[0] = (ST)x[0];
            out[1] = (ST)x[1];
        } else if constexpr (sizeof(TS) == 4) {
            const f4 x = *reinterpret_cast<const f4*>(row + kg);
#pragma unroll
            for (int e = 0; e < 4; ++e) out[e] = (ST)x[e];
        } else {
            const bf8 x = *reinterpret_cast<const bf8*>(row + kg);
#pragma unroll
            for (int e = 0; e < 8; ++e) out[e] = stage<ST>(x[e]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) out[e] = (kg + e < K) ? stage<ST>(row[kg + e]) : (ST)0;
    }
}

// ---------------------------------------------------------------------------
// GEMM core.  C[i, j] = sum_k A(i, k) B(j, k), both operands K-contiguous
// rows resolved once per thread (aoff/boff; -1 = row out of range, reads
// zero).  BM x BK and BN x BK tiles are staged through LDS (one buffer, or
// two with the next tile's stores overlapping the products) with one
// register prefetch of the next K tile; each of the NT/64 waves accumulates TM x TN
// MFMA blocks of a (BM/WGM) x (BN/WGN) sub-tile.  V*: elements per global
// load of each operand (1 = scalar, else one 16-byte vector load).
template <typename TA, typename TB, typename TC, int BM, int BN, int BK, int WGM, int WGN, int VA,
          int VB, bool AL>
struct Core {
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int TM = BM / WGM / 16;
    static constexpr int TN = BN / WGN / 16;
    typedef typename Info<TC>::ST ST;
    typedef typename Info<TC>::LT LT;
    static constexpr int PK = Pitch<TC, BK>::v;
    static constexpr int PL = Info<TC>::PLANES;
    // threads per row and rows per pass for each operand
    static constexpr int TPRA = BK / VA, RPA = NT / TPRA, LA = BM / RPA;
    static constexpr int TPRB = BK / VB, RPB = NT / TPRB, LB = BN / RPB;
    static constexpr int LDS_A = PL * BM * PK, LDS_B = PL * BN * PK;  // elements
    typedef typename AccT<TC>::v accv;
    static_assert(BM % (WGM * 16) == 0 && BN % (WGN * 16) == 0, "tile");
    static_assert(BK % VA == 0 && BK % VB == 0 && NT % TPRA == 0 && NT % TPRB == 0, "loads");
    static_assert(LA >= 1 && LB >= 1 && BM % RPA == 0 && BN % RPB == 0, "loads");
    static_assert(BK % Info<TC>::KM == 0, "bk");
    static_assert(sizeof(LT) != 2 || BK == 32, "swizzled BF16 tiles hold 32 k");

    // per-thread rows: r = tid / TPR + j * RP
    static __device__ __forceinline__ int arow(int j) { return threadIdx.x / TPRA + j * RPA; }
    static __device__ __forceinline__ int brow(int j) { return threadIdx.x / TPRB + j * RPB; }

    // Split BF16, a last K tile whose valid k end at or below 16 (the rest
    // is zero): the products over its first 16 k only, 16 x 16 x 16 MFMAs.
    // Every path of run() takes such a tile this way, so all tile shapes
    // still sum alike.
    static __device__ __forceinline__ void compute_half(const LT* As, const LT* Bs,
                                                        accv (&acc)[TM][TN]) {
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int wm = wave / WGN, wn = wave % WGN;
        const int k4 = 4 * (lane >> 4);
        s4v ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a) {
            const int i = lds_index<LT, PK>(wm * TM * 16 + a * 16 + (lane & 15), k4);
            ah[a] = *reinterpret_cast<const s4v*>(&As[i]);
            al[a] = *reinterpret_cast<const s4v*>(&As[BM * PK + i]);
        }
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int i = lds_index<LT, PK>(wn * TN * 16 + b * 16 + (lane & 15), k4);
            bh[b] = *reinterpret_cast<const s4v*>(&Bs[i]);
            bl[b] = *reinterpret_cast<const s4v*>(&Bs[BN * PK + i]);
        }
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                acc[a][b] = mma4(al[a], bh[b], acc[a][b]);
                acc[a][b] = mma4(ah[a], bl[b], acc[a][b]);
                acc[a][b] = mma4(ah[a], bh[b], acc[a][b]);
            }
    }

    // acc += the products of one staged K tile (As, Bs: one buffer)
    static __device__ __forceinline__ void compute(const LT* As, const LT* Bs,
                                                   accv (&acc)[TM][TN]) {
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        const int wm = wave / WGN, wn = wave % WGN;
        if constexpr (Info<TC>::KM == 4) {
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                LT af[TM], bfr[TN];
#pragma unroll
                for (int a = 0; a < TM; ++a)
                    af[a] = As[(wm * TM * 16 + a * 16 + (lane & 15)) * PK + ks + (lane >> 4)];
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    bfr[b] = Bs[(wn * TN * 16 + b * 16 + (lane & 15)) * PK + ks + (lane >> 4)];
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b) acc[a][b] = mma1(af[a], bfr[b], acc[a][b]);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < BK; ks += 32) {
                bf8 ah[TM], bh[TN];
#pragma unroll
                for (int a = 0; a < TM; ++a)
                    ah[a] = *reinterpret_cast<const bf8*>(&As[lds_index<LT, PK>(
                        wm * TM * 16 + a * 16 + (lane & 15), ks + 8 * (lane >> 4))]);
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    bh[b] = *reinterpret_cast<const bf8*>(&Bs[lds_index<LT, PK>(
                        wn * TN * 16 + b * 16 + (lane & 15), ks + 8 * (lane >> 4))]);
                if constexpr (PL == 2) {
                    bf8 al[TM], bl[TN];
#pragma unroll
                    for (int a = 0; a < TM; ++a)
                        al[a] = *reinterpret_cast<const bf8*>(&As[BM * PK + lds_index<LT, PK>(
                            wm * TM * 16 + a * 16 + (lane & 15), ks + 8 * (lane >> 4))]);
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        bl[b] = *reinterpret_cast<const bf8*>(&Bs[BN * PK + lds_index<LT, PK>(
                            wn * TN * 16 + b * 16 + (lane & 15), ks + 8 * (lane >> 4))]);
#pragma unroll
                    for (int a = 0; a < TM; ++a)
#pragma unroll
                        for (int b = 0; b < TN; ++b) {
                            acc[a][b] = mma8(al[a], bh[b], acc[a][b]);
                            acc[a][b] = mma8(ah[a], bl[b], acc[a][b]);
                            acc[a][b] = mma8(ah[a], bh[b], acc[a][b]);
                        }
                } else {
#pragma unroll
                    for (int a = 0; a < TM; ++a)
#pragma unroll
                        for (int b = 0; b < TN; ++b) acc[a][b] = mma8(ah[a], bh[b], acc[a][b]);
                }
            }
        }
    }

    // DB = false: one LDS buffer, two barriers per K tile.  DB = true: As and
    // Bs hold two buffers each; tile t + 1 is split and stored into the other
    // buffer right after the products of tile t are issued, one barrier per
    // K tile.  The products and their order per accumulator are the same.
    // ROWS_VALID: every aoff / boff names a readable row (rows past the
    // operand repeat its last row; their results are never stored).
    template <bool DB = false, bool ROWS_VALID = false>
    static __device__ __forceinline__ void run(const TA* __restrict__ A, const long* aoff,
                                               const TB* __restrict__ B, const long* boff, int K,
                                               LT* As, LT* Bs, accv (&acc)[TM][TN]) {
        const int tid = threadIdx.x;
        const int ka = (tid % TPRA) * VA, kb = (tid % TPRB) * VB;
        ST ra[LA][VA], rb[LB][VB];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b)
                for (int e = 0; e < 4; ++e) acc[a][b][e] = 0;

        // staging sets: registers holding one K tile between its fetch and
        // its split into LDS
        auto gload = [&](int k0, ST (&xa)[LA][VA], ST (&xb)[LB][VB]) {
#pragma unroll
            for (int j = 0; j < LA; ++j) {
                if (aoff[j] >= 0)
                    gload_run<ST, TA, VA, AL>(A + aoff[j], k0 + ka, K, xa[j]);
                else
#pragma unroll
                    for (int e = 0; e < VA; ++e) xa[j][e] = (ST)0;
            }
#pragma unroll
            for (int j = 0; j < LB; ++j) {
                if (boff[j] >= 0)
                    gload_run<ST, TB, VB, AL>(B + boff[j], k0 + kb, K, xb[j]);
                else
#pragma unroll
                    for (int e = 0; e < VB; ++e) xb[j][e] = (ST)0;
            }
        };
        auto sstore = [&](LT* Ad, LT* Bd, ST (&xa)[LA][VA], ST (&xb)[LB][VB]) {
            if constexpr (sizeof(LT) == 2 && VA % 4 == 0 && VB % 4 == 0) {
                // BF16 planes: each thread's run of V consecutive k goes out as
                // 8-byte stores (4 elements per plane), rows 16-byte aligned
#pragma unroll
                for (int j = 0; j < LA; ++j)
#pragma unroll
                    for (int e = 0; e < VA; e += 4)
                        lds_put4<TC>(Ad, BM * PK, lds_index<LT, PK>(arow(j), ka + e), &xa[j][e]);
#pragma unroll
                for (int j = 0; j < LB; ++j)
#pragma unroll
                    for (int e = 0; e < VB; e += 4)
                        lds_put4<TC>(Bd, BN * PK, lds_index<LT, PK>(brow(j), kb + e), &xb[j][e]);
            } else {
#pragma unroll
                for (int j = 0; j < LA; ++j)
#pragma unroll
                    for (int e = 0; e < VA; ++e)
                        lds_put<TC>(Ad, BM * PK, lds_index<LT, PK>(arow(j), ka + e), xa[j][e]);
#pragma unroll
                for (int j = 0; j < LB; ++j)
#pragma unroll
                    for (int e = 0; e < VB; ++e)
                        lds_put<TC>(Bd, BN * PK, lds_index<LT, PK>(brow(j), kb + e), xb[j][e]);
            }
        };

        gload(0, ra, rb);
        sstore(As, Bs, ra, rb);
        // (operands staged as four-element runs, as FP32 storage gives them)
        if (DB && PL == 2 && VA % 4 == 0 && VB % 4 == 0 && ROWS_VALID && K > 0 && K % BK == 0) {
            // Split BF16 over whole K tiles: a second staging set, so that each
            // tile is fetched two tiles ahead of its split into LDS (the fetch
            // latency hides behind two tiles of products instead of one).  Tile
            // t + 1 waits in set (t + 1) & 1 (set 0 = ra/rb, set 1 = sa/sb).
            // Every step issues the same vector loads and LDS stores (past the
            // last tile it fetches the last tile again and stores it into the
            // buffer no later step reads), so the loop body has no branch and
            // the wait before a split counts only the older set.  Same products
            // in the same order as the other paths.
            const int nt = K / BK;
            ST sa[LA][VA], sb[LB][VB];
            auto fetch = [&](int t, ST (&xa)[LA][VA], ST (&xb)[LB][VB]) {
                const int k0 = (t < nt ? t : nt - 1) * BK;
#pragma unroll
                for (int j = 0; j < LA; ++j)
                    gload_run<ST, TA, VA, AL, AL>(A + aoff[j], k0 + ka, K, xa[j]);
#pragma unroll
                for (int j = 0; j < LB; ++j)
                    gload_run<ST, TB, VB, AL, AL>(B + boff[j], k0 + kb, K, xb[j]);
            };
            fetch(1, sa, sb);
            fetch(2, ra, rb);
            __syncthreads();
            auto step = [&](int t, ST (&xa)[LA][VA], ST (&xb)[LB][VB]) {
                compute(As + (t & 1) * LDS_A, Bs + (t & 1) * LDS_B, acc);
                sstore(As + ((t + 1) & 1) * LDS_A, Bs + ((t + 1) & 1) * LDS_B, xa, xb);
                fetch(t + 3, xa, xb);
                __syncthreads();
                // keep the next step's split of the other set below this
                // point (hoisted above, it would wait for that set's fetch)
                __builtin_amdgcn_sched_barrier(0);
            };
            int t = 0;
            for (; t + 1 < nt; t += 2) {
                step(t, sa, sb);
                step(t + 1, ra, rb);
            }
            if (t < nt) step(t, sa, sb);
        } else if constexpr (DB) {
            if (BK < K) gload(BK, ra, rb);
            __syncthreads();
            int cur = 0;
            // split BF16 with a last tile of at most 16 valid k: that tile
            // after the loop, with half the products
            const bool half = PL == 2 && BK == 32 && K > 0 && (K - 1) % BK < 16;
            const int kend = half ? (K - 1) / BK * BK : K;
            for (int k0 = 0; k0 < kend; k0 += BK) {
                compute(As + cur * LDS_A, Bs + cur * LDS_B, acc);
                if (k0 + BK < K) {
                    sstore(As + (cur ^ 1) * LDS_A, Bs + (cur ^ 1) * LDS_B, ra, rb);
                    if (k0 + 2 * BK < K) gload(k0 + 2 * BK, ra, rb);
                }
                __syncthreads();
                cur ^= 1;
            }
            if constexpr (PL == 2 && BK == 32) {
                if (half) {
                    compute_half(As + cur * LDS_A, Bs + cur * LDS_B, acc);
                    __syncthreads();  // callers may reuse the buffers after run()
                }
            }
        } else {
            __syncthreads();
            const bool half = PL == 2 && BK == 32 && K > 0 && (K - 1) % BK < 16;
            const int kend = half ? (K - 1) / BK * BK : K;
            for (int k0 = 0; k0 < kend; k0 += BK) {
                const bool more = k0 + BK < K;
                if (more) gload(k0 + BK, ra, rb);
                compute(As, Bs, acc);
                __syncthreads();
                if (more) {
                    sstore(As, Bs, ra, rb);
                    __syncthreads();
                }
            }
            if constexpr (PL == 2 && BK == 32) {
                if (half) {
                    compute_half(As, Bs, acc);
                    __syncthreads();
                }
            }
        }
    }
};

}  // namespace dev
}  // namespace afq
