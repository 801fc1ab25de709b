// Tiled MFMA contractions for gfx950 (CDNA4, 64-wide wavefronts).
//
// Every Cholesky contraction of the walker step is a real GEMM once the
// complex walker planes are laid out as extra rows or columns:
//   force bias     F[(w,p), g]   = sum_(i,m) Theta[(w,p), (i,m)] L^half[g, (i,m)]
//   field sum      A[(w,p), q]   = sum_g X[(w,p), g] Lpacked[q, g]
//   one-body half  Y[(w,p,i), m] = sum_m' Phi[(w,p,i), m'] P[m, m']
//   overlap        O[(w,p,i), j] = sum_m Phi[(w,p,i), m] PhiT[j, m]
// (all operands K-contiguous: the "TN" form C = A B^T).  The Taylor series
// of the HS factor is a complex product per walker (A_w differs per walker)
// and the exchange term of the local energy needs whole N_s x N_s blocks of
// T = L^half Theta in one tile; both have their own kernels built from the
// same LDS-staged MFMA loop.
//
// MFMA fragment layout (v_mfma_{f64,f32}_16x16x4 and v_mfma_f32_16x16x32_bf16):
// lane l supplies A[l % 16][kb + l / 16] and B^T[l % 16][kb + l / 16]
// (kb + 8 (l / 16) + e, e < 8, for bf16).  Accumulator element r of lane l
// is D[4 (l / 16) + r][l % 16] for the FP32-accumulating instructions and
// D[l / 16 + 4 r][l % 16] for v_mfma_f64_16x16x4.
#include "internal.h"

namespace afq {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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

template <typename T>
__device__ __forceinline__ T from_f(float x);
template <>
__device__ __forceinline__ float from_f<float>(float x) { return x; }
template <>
__device__ __forceinline__ bf16_t from_f<bf16_t>(float x) { return (bf16_t)x; }

// Storage -> compute conversions (round to nearest even).
template <typename TC, typename TS>
__device__ __forceinline__ TC to_c(TS x) { return (TC)x; }
template <>
__device__ __forceinline__ bf16_t to_c<bf16_t, double>(double x) { return (bf16_t)(float)x; }
template <>
__device__ __forceinline__ bf16_t to_c<bf16_t, float>(float x) { return (bf16_t)x; }
template <>
__device__ __forceinline__ bf16_t to_c<bf16_t, bf16_t>(bf16_t x) { return x; }
template <>
__device__ __forceinline__ double to_c<double, bf16_t>(bf16_t x) { return (double)(float)x; }
template <>
__device__ __forceinline__ float to_c<float, bf16_t>(bf16_t x) { return (float)x; }

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

template <typename TC>
struct KInfo {
    static constexpr int KPL = 1;  // k values per lane per MFMA
    static constexpr int KM = 4;   // k per MFMA
};
template <>
struct KInfo<bf16_t> {
    static constexpr int KPL = 8;
    static constexpr int KM = 32;
};

// LDS row pitch (elements) for a BK-wide tile: keeps rows on distinct banks.
template <typename TC, int BK>
struct Pitch {
    static constexpr int v = BK + (sizeof(TC) == 8 ? 1 : (sizeof(TC) == 4 ? 1 : 8));
};

// ---------------------------------------------------------------------------
// Core: stage BMxBK and BNxBK tiles through LDS, accumulate TMxTN MFMA blocks
// per wave.  Row pointers are resolved once per thread; out-of-range rows and
// k >= K read as zero.
template <typename TA, typename TB, typename TC, int BM, int BN, int BK, int WGM, int WGN>
struct Core {
    static constexpr int NT = 256;
    static constexpr int TM = BM / WGM / 16;
    static constexpr int TN = BN / WGN / 16;
    static constexpr int PK = Pitch<TC, BK>::v;
    static constexpr int LA = BM * BK / NT;
    static constexpr int LB = BN * BK / NT;
    static constexpr int RSTEP = NT / BK;
    typedef typename AccT<TC>::v accv;
    static_assert(BM % (WGM * 16) == 0 && BN % (WGN * 16) == 0, "tile");
    static_assert(WGM * WGN == 4, "4 waves");
    static_assert(NT % BK == 0 && LA >= 1 && LB >= 1, "loads");
    static_assert(BK % KInfo<TC>::KM == 0, "bk");

    static __device__ __forceinline__ void run(const TA* __restrict__ A, const long* aoff,
                                               const TB* __restrict__ B, const long* boff, int K,
                                               TC* As, TC* Bs, accv (&acc)[TM][TN]) {
        const int tid = threadIdx.x;
        const int lane = tid & 63;
        const int wave = tid >> 6;
        const int wm = wave / WGN, wn = wave % WGN;
        const int kk = tid % BK;
        const int rr = tid / BK;
        TC ra[LA], rb[LB];
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b)
                for (int e = 0; e < 4; ++e) acc[a][b][e] = 0;

        auto gload = [&](int k0) {
            const int kg = k0 + kk;
            const bool kin = kg < K;
#pragma unroll
            for (int j = 0; j < LA; ++j)
                ra[j] = (kin && aoff[j] >= 0) ? to_c<TC>(A[aoff[j] + kg]) : (TC)0;
#pragma unroll
            for (int j = 0; j < LB; ++j)
                rb[j] = (kin && boff[j] >= 0) ? to_c<TC>(B[boff[j] + kg]) : (TC)0;
        };
        auto sstore = [&]() {
#pragma unroll
            for (int j = 0; j < LA; ++j) As[(rr + j * RSTEP) * PK + kk] = ra[j];
#pragma unroll
            for (int j = 0; j < LB; ++j) Bs[(rr + j * RSTEP) * PK + kk] = rb[j];
        };

        gload(0);
        sstore();
        __syncthreads();
        for (int k0 = 0; k0 < K; k0 += BK) {
            const bool more = k0 + BK < K;
            if (more) gload(k0 + BK);
            if constexpr (KInfo<TC>::KPL == 1) {
#pragma unroll
                for (int ks = 0; ks < BK; ks += 4) {
                    TC af[TM], bfr[TN];
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
                    bf8 af[TM], bfr[TN];
#pragma unroll
                    for (int a = 0; a < TM; ++a)
                        af[a] = *reinterpret_cast<const bf8*>(
                            &As[(wm * TM * 16 + a * 16 + (lane & 15)) * PK + ks + 8 * (lane >> 4)]);
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        bfr[b] = *reinterpret_cast<const bf8*>(
                            &Bs[(wn * TN * 16 + b * 16 + (lane & 15)) * PK + ks + 8 * (lane >> 4)]);
#pragma unroll
                    for (int a = 0; a < TM; ++a)
#pragma unroll
                        for (int b = 0; b < TN; ++b) acc[a][b] = mma8(af[a], bfr[b], acc[a][b]);
                }
            }
            __syncthreads();
            if (more) {
                sstore();
                __syncthreads();
            }
        }
    }
};

// ---------------------------------------------------------------------------
template <typename TA, typename TB, typename TC, typename TO, int BM, int BN, int BK, int WGM,
          int WGN>
__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
    typedef Core<TA, TB, TC, BM, BN, BK, WGM, WGN> C;
    __shared__ __attribute__((aligned(16))) TC As[BM * C::PK];
    __shared__ __attribute__((aligned(16))) TC Bs[BN * C::PK];
    const int b = blockIdx.z;
    const long row0 = (long)blockIdx.y * BM, col0 = (long)blockIdx.x * BN;
    const TA* A = (const TA*)g.A + (long)b * g.a_bs;
    const TB* B = (const TB*)g.B + (long)b * g.b_bs;
    const int tid = threadIdx.x;
    long aoff[C::LA], boff[C::LB];
#pragma unroll
    for (int j = 0; j < C::LA; ++j) {
        long r = row0 + tid / BK + j * C::RSTEP;
        aoff[j] = r < g.m ? rowmap(g.ra, r) : -1;
    }
#pragma unroll
    for (int j = 0; j < C::LB; ++j) {
        long r = col0 + tid / BK + j * C::RSTEP;
        boff[j] = r < g.n ? rowmap(g.rb, r) : -1;
    }
    typename C::accv acc[C::TM][C::TN];
    C::run(A, aoff, B, boff, g.k, As, Bs, acc);

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    TO* out = (TO*)g.C + (long)b * g.c_bs;
    TO* out2 = g.C2 ? (TO*)g.C2 + (long)b * g.c_bs : nullptr;
#pragma unroll
    for (int a = 0; a < C::TM; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long i = row0 + wm * C::TM * 16 + a * 16 + acc_row<TC>(lane, r);
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

template <typename TA, typename TB, typename TC, typename TO>
hipError_t launch_gemm(const Gemm& g, hipStream_t s) {
    const long tiles128 = ((long)(g.m + 127) / 128) * ((g.n + 127) / 128) * g.batch;
    constexpr int BK = KInfo<TC>::KPL == 1 ? 16 : 32;
    if (g.m >= 96 && g.n >= 96 && tiles128 >= 512) {
        dim3 grid((g.n + 127) / 128, (g.m + 127) / 128, g.batch);
        hipLaunchKernelGGL((k_gemm<TA, TB, TC, TO, 128, 128, BK, 2, 2>), grid, dim3(256), 0, s, g);
    } else {
        dim3 grid((g.n + 63) / 64, (g.m + 63) / 64, g.batch);
        hipLaunchKernelGGL((k_gemm<TA, TB, TC, TO, 64, 64, BK, 2, 2>), grid, dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Taylor term of the HS factor, complex, one walker per blockIdx.z.
// Rows: walker orbitals i (N); columns: basis index m (M); K: m' (M).
template <typename T, int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(256) void k_taylor(const T* __restrict__ Tp, T* __restrict__ Tn,
                                                T* __restrict__ Z, const T* __restrict__ Apk,
                                                const uint8_t* __restrict__ live, int M, int N,
                                                T inv_n) {
    typedef typename AccT<T>::v accv;
    constexpr int TM = BM / WGM / 16, TN = BN / WGN / 16;
    constexpr int PK = BK + 1;
    constexpr int LA = BM * BK / 256, LB = BN * BK / 256, RSTEP = 256 / BK;
    __shared__ T Ar[BM * PK], Ai[BM * PK], Br[BN * PK], Bi[BN * PK];
    const int w = blockIdx.z;
    if (!live[w]) return;
    const long NM = (long)N * M;
    const long P = (long)M * (M + 1) / 2;
    const T* tr = Tp + (long)w * 2 * NM;
    const T* ti = tr + NM;
    const T* ar = Apk + (long)w * 2 * P;
    const T* ai = ar + P;
    const int row0 = blockIdx.y * BM, col0 = blockIdx.x * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int kk = tid % BK, rr = tid / BK;
    accv cr[TM][TN], ci[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
            for (int e = 0; e < 4; ++e) cr[a][b][e] = ci[a][b][e] = 0;
    T xa_r[LA], xa_i[LA], xb_r[LB], xb_i[LB];
    auto gload = [&](int k0) {
        const int kg = k0 + kk;
#pragma unroll
        for (int j = 0; j < LA; ++j) {
            const int i = row0 + rr + j * RSTEP;
            const bool ok = i < N && kg < M;
            xa_r[j] = ok ? tr[(long)i * M + kg] : (T)0;
            xa_i[j] = ok ? ti[(long)i * M + kg] : (T)0;
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            const int m = col0 + rr + j * RSTEP;
            const bool ok = m < M && kg < M;
            const int r = m < kg ? m : kg, c = m < kg ? kg : m;
            const long q = (long)r * (2 * M - r + 1) / 2 + (c - r);
            if (ok) {
                xb_r[j] = ar[q];
                xb_i[j] = ai[q];
            } else {
                xb_r[j] = xb_i[j] = (T)0;
            }
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int j = 0; j < LA; ++j) {
            Ar[(rr + j * RSTEP) * PK + kk] = xa_r[j];
            Ai[(rr + j * RSTEP) * PK + kk] = xa_i[j];
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            Br[(rr + j * RSTEP) * PK + kk] = xb_r[j];
            Bi[(rr + j * RSTEP) * PK + kk] = xb_i[j];
        }
    };
    gload(0);
    sstore();
    __syncthreads();
    for (int k0 = 0; k0 < M; k0 += BK) {
        const bool more = k0 + BK < M;
        if (more) gload(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            T a_r[TM], a_i[TM], a_n[TM], b_r[TN], b_i[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) {
                const int o = (wm * TM * 16 + a * 16 + (lane & 15)) * PK + ks + (lane >> 4);
                a_r[a] = Ar[o];
                a_i[a] = Ai[o];
                a_n[a] = -a_i[a];
            }
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                const int o = (wn * TN * 16 + b * 16 + (lane & 15)) * PK + ks + (lane >> 4);
                b_r[b] = Br[o];
                b_i[b] = Bi[o];
            }
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    cr[a][b] = mma1(a_r[a], b_r[b], cr[a][b]);
                    cr[a][b] = mma1(a_n[a], b_i[b], cr[a][b]);
                    ci[a][b] = mma1(a_r[a], b_i[b], ci[a][b]);
                    ci[a][b] = mma1(a_i[a], b_r[b], ci[a][b]);
                }
        }
        __syncthreads();
        if (more) {
            sstore();
            __syncthreads();
        }
    }
    T* onr = Tn + (long)w * 2 * NM;
    T* oni = onr + NM;
    T* zr = Z + (long)w * 2 * NM;
    T* zi = zr + NM;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = row0 + wm * TM * 16 + a * 16 + acc_row<T>(lane, r);
            if (i >= N) continue;
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                const int m = col0 + wn * TN * 16 + b * 16 + (lane & 15);
                if (m >= M) continue;
                const long o = (long)i * M + m;
                const T vr = cr[a][b][r] * inv_n, vi = ci[a][b][r] * inv_n;
                onr[o] = vr;
                oni[o] = vi;
                zr[o] += vr;
                zi[o] += vi;
            }
        }
}

// ---------------------------------------------------------------------------
// Exchange: tile rows = G whole gamma blocks (G * nsig rows of (gamma, i)),
// tile columns = W whole walkers (W * 2 nsig columns of (walker, plane, j)).
template <typename TS, typename TC, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void k_exchange(const TS* __restrict__ lhalf,
                                                  const TS* __restrict__ theta,
                                                  double* __restrict__ out, int nw, int M, int N,
                                                  int n_chol, int off, int nsig, int spin, int G,
                                                  int W, int n_gt) {
    typedef Core<TS, TS, TC, BM, BN, BK, 2, 2> C;
    typedef typename AccT<TC>::s accs;
    constexpr int SP = BN + 1;
    constexpr int OPB = (BM + BN) * C::PK * sizeof(TC);
    constexpr int SB = BM * SP * sizeof(accs);
    constexpr int SMEM = OPB > SB ? OPB : SB;
    __shared__ __attribute__((aligned(16))) char smem[SMEM];
    __shared__ double red[256 * 2];
    TC* As = reinterpret_cast<TC*>(smem);
    TC* Bs = As + BM * C::PK;
    accs* S = reinterpret_cast<accs*>(smem);

    const int tid = threadIdx.x;
    const long NM = (long)N * M;
    const int gt = blockIdx.y, wt = blockIdx.x;
    const int g0 = gt * G, w0 = wt * W;
    const int rows_valid = G * nsig, cols_valid = W * 2 * nsig;
    long aoff[C::LA], boff[C::LB];
#pragma unroll
    for (int j = 0; j < C::LA; ++j) {
        const int r = tid / BK + j * C::RSTEP;
        const int g = g0 + r / nsig, i = r % nsig;
        aoff[j] = (r < rows_valid && g < n_chol) ? (long)g * NM + (long)(off + i) * M : -1;
    }
#pragma unroll
    for (int j = 0; j < C::LB; ++j) {
        const int c = tid / BK + j * C::RSTEP;
        const int u = c / (2 * nsig), p = (c / nsig) & 1, jj = c % nsig;
        const int w = w0 + u;
        boff[j] = (c < cols_valid && w < nw) ? (long)(2 * w + p) * NM + (long)(off + jj) * M : -1;
    }
    typename C::accv acc[C::TM][C::TN];
    C::run(lhalf, aoff, theta, boff, M, As, Bs, acc);
    // operand tiles are dead after the final barrier of run(): reuse as S
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int a = 0; a < C::TM; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = wm * C::TM * 16 + a * 16 + acc_row<TC>(lane, r);
#pragma unroll
            for (int b = 0; b < C::TN; ++b) {
                const int j = wn * C::TN * 16 + b * 16 + (lane & 15);
                S[i * SP + j] = acc[a][b][r];
            }
        }
    __syncthreads();
    const int tpu = 256 / W;
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

}  // namespace

template <typename T>
constexpr DType dt_of() {
    return sizeof(T) == 8 ? DT_F64 : (sizeof(T) == 4 ? DT_F32 : DT_BF16);
}

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
    AFQ_G(double, double, float, double)
    AFQ_G(double, double, bf16_t, double)
#undef AFQ_G
    return hipErrorInvalidValue;
}

hipError_t taylor_term(const void* Tprev, void* Tn, void* Z, const void* Apk, const uint8_t* live,
                       int nw, int M, int N, double inv_n, DType t, hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    if (t == DT_F64) {
        constexpr int BM = 32, BN = 64;
        dim3 grid((M + BN - 1) / BN, (N + BM - 1) / BM, nw);
        hipLaunchKernelGGL((k_taylor<double, BM, BN, 16, 2, 2>), grid, dim3(256), 0, s,
                           (const double*)Tprev, (double*)Tn, (double*)Z, (const double*)Apk, live,
                           M, N, inv_n);
    } else if (t == DT_F32) {
        constexpr int BM = 32, BN = 64;
        dim3 grid((M + BN - 1) / BN, (N + BM - 1) / BM, nw);
        hipLaunchKernelGGL((k_taylor<float, BM, BN, 16, 2, 2>), grid, dim3(256), 0, s,
                           (const float*)Tprev, (float*)Tn, (float*)Z, (const float*)Apk, live, M,
                           N, (float)inv_n);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int exchange_gtiles(int n_chol, int nsig, DType t) {
    (void)t;
    const int BM = 128;
    if (nsig <= 0) return 0;
    const int G = BM / nsig;
    return (n_chol + G - 1) / G;
}

hipError_t exchange(const void* lhalf, const void* theta, double* out, int nw, int M, int N,
                    int n_chol, int off, int nsig, int spin, int n_gt, DType t, hipStream_t s) {
    if (nsig <= 0 || nw <= 0 || n_chol <= 0) return hipSuccess;
    constexpr int BM = 128, BN = 128;
    if (nsig > 64) return hipErrorInvalidValue;
    const int G = BM / nsig, W = BN / (2 * nsig);
    dim3 grid((nw + W - 1) / W, (n_chol + G - 1) / G, 1);
    if (t == DT_F64) {
        hipLaunchKernelGGL((k_exchange<double, double, BM, BN, 16>), grid, dim3(256), 0, s,
                           (const double*)lhalf, (const double*)theta, out, nw, M, N, n_chol, off,
                           nsig, spin, G, W, n_gt);
    } else if (t == DT_F32) {
        hipLaunchKernelGGL((k_exchange<float, float, BM, BN, 16>), grid, dim3(256), 0, s,
                           (const float*)lhalf, (const float*)theta, out, nw, M, N, n_chol, off,
                           nsig, spin, G, W, n_gt);
    } else {
        hipLaunchKernelGGL((k_exchange<bf16_t, bf16_t, BM, BN, 32>), grid, dim3(256), 0, s,
                           (const bf16_t*)lhalf, (const bf16_t*)theta, out, nw, M, N, n_chol, off,
                           nsig, spin, G, W, n_gt);
    }
    return hipGetLastError();
}

}  // namespace afq
