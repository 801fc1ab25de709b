// Complex products of the reverse pass through the Taylor series of the
// Hubbard-Stratonovich propagator (Eq. 8): per walker, the forward terms
// t_n = A t_{n-1} / n, the backward recursion t_bar_{n-1} = y_bar +
// conj(A) t_bar_n / n, and A_bar = sum_n (t_bar_n / n) t_{n-1}^H.
//
// Each complex product is one kernel on the matrix cores (v_mfma_f64_16x16x4
// for FP64 compute, v_mfma_f32_16x16x4 otherwise, both accumulating in their
// own type): the real and imaginary planes of both operands are staged once
// through LDS and a complex product takes three real ones (Gauss's
// (a + b)(c + d) - ac - bd for the imaginary part), accumulated side by side,
// so no operand is fetched once per real product, the terms stay in the
// walker row layout (no transpose), and the sums over terms happen in the
// epilogue.
#include "mfma.h"

namespace afq {
namespace dev {
namespace {

constexpr int BK = 16;   // contraction chunk staged per round
constexpr int BJ = 64;   // output columns per workgroup (16 per wave)

// XCD-aware order: workgroups are dealt to the eight XCDs in turn, so logical
// block L = (id mod 8) per + id / 8 gives each XCD a contiguous run of blocks
// (the column blocks of one walker share its rows in one L2).
__device__ __forceinline__ long xcd_block(long n) {
    const long per = (n + 7) / 8;
    return (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// Two consecutive doubles p[0], p[1] of a row into registers: one 16-byte load
// when the pair is aligned and in range (AL: even row lengths and strides),
// else element by element; out-of-range elements read as zero.
template <bool AL>
__device__ __forceinline__ d2 ld_pair(const double* __restrict__ p, bool ok0, bool ok1) {
    if (AL) return ok0 ? *reinterpret_cast<const d2*>(p) : d2{0.0, 0.0};
    return d2{ok0 ? p[0] : 0.0, ok1 ? p[1] : 0.0};
}

// One Taylor term for the rows of walker w (planes [2][N][M], row i holds
// orbital column i): C = in op(A)^T with op(A) = A_r + i sgn A_i (A complex
// symmetric, sgn = -1 for conj), o = (base + alpha C) oscale -> out, and
// acc_out = acc_in + o.  Workgroup: 16 RT rows x 64 columns of C; wave v owns
// columns 16 v .. 16 v + 15 of the block and all RT row tiles.  The
// contraction runs in BK chunks through two LDS buffers: while chunk c is
// multiplied, chunk c + 1 (fetched into registers during chunk c - 1) is
// stored into the other buffer and chunk c + 2 is fetched, one barrier per
// chunk; A is staged through its symmetry as rows k (columns j contiguous),
// so a chunk of it is BK runs of 64 consecutive elements.
template <typename TC, int RT, bool AL>
__global__ __launch_bounds__(256, 2) void k_cterm(CTerm c, int ncb, int nrb) {
    typedef typename Info<TC>::ST ST;
    typedef typename AccT<TC>::v accv;
    constexpr int BI = 16 * RT, PK = BK + 1;
    // A-chunk pitch: 80 = 16 (mod 32) doubles / (mod 64) floats, so the
    // fragment reads of lanes l and l + 16 fall in different banks
    constexpr int PJ = BJ + 16;
    constexpr int NIN = RT;  // pairs of the rows chunk per thread (2 BI BK / 2 / 256)
    constexpr int NA = 4;    // pairs of the A chunk per thread (2 BK BJ / 2 / 256)
    // two LDS buffers: chunk c + 1 is stored while chunk c is multiplied
    __shared__ ST s_in[2][2][BI][PK];
    __shared__ ST s_a[2][2][BK][PJ];
    const long nb = (long)ncb * nrb * c.nw;
    const long L = xcd_block(nb);
    if (L >= nb) return;
    const int w = (int)(L / ((long)ncb * nrb));
    const int rb = (int)((L / ncb) % nrb), cb = (int)(L % ncb);
    const int M = c.M, N = c.N;
    const long NM = (long)N * M, MM = (long)M * M;
    const int i0 = rb * BI, j0 = cb * BJ;
    const double* __restrict__ in = c.in + (long)w * c.in_bs;
    const double* __restrict__ A = c.A + (long)w * 2 * MM;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15;
    const ST sgn = c.conj ? (ST)-1 : (ST)1;
    // fixed parts of this thread's chunk elements: rows chunk pair e = tid +
    // 256 u -> plane, row, k pair (8 pairs per row); A chunk pair -> plane,
    // k row, j pair (32 pairs per row)
    int in_p[NIN], in_r[NIN], in_k[NIN], a_p[NA], a_k[NA], a_j[NA];
#pragma unroll
    for (int u = 0; u < NIN; ++u) {
        const int e = tid + 256 * u;
        in_p[u] = e / (BI * 8);
        in_r[u] = (e / 8) % BI;
        in_k[u] = 2 * (e % 8);
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        const int e = tid + 256 * u;
        a_p[u] = e / (BK * 32);
        a_k[u] = (e / 32) % BK;
        a_j[u] = 2 * (e % 32);
    }
    d2 rin[NIN], ra[NA];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < NIN; ++u) {
            const int i = i0 + in_r[u], k = k0 + in_k[u];
            const bool ok = i < N;
            rin[u] = ld_pair<AL>(in + in_p[u] * NM + (long)i * M + k, ok && k < M,
                                 ok && k + 1 < M);
        }
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int k = k0 + a_k[u], j = j0 + a_j[u];
            const bool ok = k < M;
            ra[u] = ld_pair<AL>(A + a_p[u] * MM + (long)k * M + j, ok && j < M, ok && j + 1 < M);
        }
    };
    // three real products per complex one (Gauss): rr = in_r A_r, ii = in_i B_i,
    // ss = (in_r + in_i)(A_r + B_i), B_i = sgn A_i; C = rr - ii + i (ss - rr - ii)
    accv acc_rr[RT], acc_ii[RT], acc_ss[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc_rr[t] = acc_ii[t] = acc_ss[t] = accv{0, 0, 0, 0};
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NIN; ++u) {
            s_in[buf][in_p[u]][in_r[u]][in_k[u]] = (ST)rin[u][0];
            s_in[buf][in_p[u]][in_r[u]][in_k[u] + 1] = (ST)rin[u][1];
        }
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const ST f = a_p[u] ? sgn : (ST)1;
            s_a[buf][a_p[u]][a_k[u]][a_j[u]] = f * (ST)ra[u][0];
            s_a[buf][a_p[u]][a_k[u]][a_j[u] + 1] = f * (ST)ra[u][1];
        }
    };
    fetch(0);
    stash(0);
    if (BK < M) fetch(BK);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < M; k0 += BK) {
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            const int kk = ks + (lane >> 4);
            const ST br = s_a[cur][0][kk][16 * wv + lr];
            const ST bi = s_a[cur][1][kk][16 * wv + lr];
            const ST bs = br + bi;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const ST ar = s_in[cur][0][16 * t + lr][kk];
                const ST ai = s_in[cur][1][16 * t + lr][kk];
                acc_rr[t] = mma1(ar, br, acc_rr[t]);
                acc_ii[t] = mma1(ai, bi, acc_ii[t]);
                acc_ss[t] = mma1(ar + ai, bs, acc_ss[t]);
            }
        }
        // the other buffer was last read before the previous barrier
        if (k0 + BK < M) {
            stash(cur ^ 1);
            if (k0 + 2 * BK < M) fetch(k0 + 2 * BK);
        }
        __syncthreads();
        cur ^= 1;
    }
    const int j = j0 + 16 * wv + lr;
    if (j >= M) return;
    const double* base = c.base ? c.base + (long)w * c.base_bs : nullptr;
    double* out = c.out ? c.out + (long)w * c.out_bs : nullptr;
    const double* ai_ = c.acc_out ? c.acc_in + (long)w * c.acc_in_bs : nullptr;
    double* ao = c.acc_out ? c.acc_out + (long)w * c.acc_out_bs : nullptr;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 16 * t + acc_row<TC>(lane, r);
            if (i >= N) continue;
            const long o = (long)i * M + j;
            const double rr = (double)acc_rr[t][r], ii = (double)acc_ii[t][r];
            double cr = c.alpha * (rr - ii), ci = c.alpha * ((double)acc_ss[t][r] - rr - ii);
            if (base) {
                cr += base[o];
                ci += base[NM + o];
            }
            cr *= c.oscale;
            ci *= c.oscale;
            if (out) {
                out[o] = cr;
                out[NM + o] = ci;
            }
            if (ao) {
                const double yr = ai_[o] + cr, yi = ai_[NM + o] + ci;
                ao[o] = yr;
                ao[NM + o] = yi;
            }
        }
}

// A_bar[w](j, m) = sum_{q < nq, i < N} S_q(i, j) conj(T_q(i, m)) over the
// slots q of two tapes ([w][q][2][N][M]), complex M x M per walker
// ([w][2][M][M]).  The contraction index runs over (q, i); workgroup: 64 x 64
// outputs, wave v rows 16 v .. 16 v + 15 and all four column tiles.  Chunks
// are fetched into registers while the previous one is multiplied.
template <typename TC, bool AL>
__global__ __launch_bounds__(256, 2) void k_cabar(CAbar c, int nb1) {
    typedef typename Info<TC>::ST ST;
    typedef typename AccT<TC>::v accv;
    constexpr int BO = 64, PJ = BO + 16;
    constexpr int NP = 4;  // pairs per thread per operand (2 BK BO / 2 / 256)
    __shared__ ST s_s[2][BK][PJ];
    __shared__ ST s_t[2][BK][PJ];
    const long nb = (long)nb1 * nb1 * c.nw;
    const long L = xcd_block(nb);
    if (L >= nb) return;
    const int w = (int)(L / ((long)nb1 * nb1));
    const int bj = (int)((L / nb1) % nb1), bm = (int)(L % nb1);
    const int M = c.M, N = c.N;
    const long NM = (long)N * M, MM = (long)M * M;
    const int j0 = bj * BO, m0 = bm * BO;
    const double* __restrict__ S = c.S + (long)w * c.bs;
    const double* __restrict__ T = c.T + (long)w * c.bs;
    const int KC = c.nq * N;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, lr = lane & 15;
    int e_p[NP], e_r[NP], e_c[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        const int e = tid + 256 * u;
        e_p[u] = e / (BK * 32);
        e_r[u] = (e / 32) % BK;
        e_c[u] = 2 * (e % 32);
    }
    d2 rs[NP], rt[NP];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int cc = c0 + e_r[u];
            const bool ok = cc < KC;
            const int q = ok ? cc / N : 0, i = ok ? cc % N : 0;
            const long ro = (long)q * 2 * NM + e_p[u] * NM + (long)i * M;
            const int j = j0 + e_c[u], m = m0 + e_c[u];
            rs[u] = ld_pair<AL>(S + ro + j, ok && j < M, ok && j + 1 < M);
            rt[u] = ld_pair<AL>(T + ro + m, ok && m < M, ok && m + 1 < M);
        }
    };
    // three real products per complex one: rr = S_r T_r, ii = S_i T_i,
    // ss = (S_r + S_i)(T_r - T_i); A_bar = rr + ii + i (ss - rr + ii)
    accv acc_rr[4], acc_ii[4], acc_ss[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc_rr[u] = acc_ii[u] = acc_ss[u] = accv{0, 0, 0, 0};
    if (KC > 0) fetch(0);
    for (int c0 = 0; c0 < KC; c0 += BK) {
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            s_s[e_p[u]][e_r[u]][e_c[u]] = (ST)rs[u][0];
            s_s[e_p[u]][e_r[u]][e_c[u] + 1] = (ST)rs[u][1];
            s_t[e_p[u]][e_r[u]][e_c[u]] = (ST)rt[u][0];
            s_t[e_p[u]][e_r[u]][e_c[u] + 1] = (ST)rt[u][1];
        }
        __syncthreads();
        if (c0 + BK < KC) fetch(c0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            const int kk = ks + (lane >> 4);
            const ST ar = s_s[0][kk][16 * wv + lr];
            const ST ai = s_s[1][kk][16 * wv + lr];
            const ST as = ar + ai;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const ST br = s_t[0][kk][16 * u + lr];
                const ST bi = s_t[1][kk][16 * u + lr];
                acc_rr[u] = mma1(ar, br, acc_rr[u]);
                acc_ii[u] = mma1(ai, bi, acc_ii[u]);
                acc_ss[u] = mma1(as, br - bi, acc_ss[u]);
            }
        }
        __syncthreads();
    }
    double* out = c.Abar + (long)w * 2 * MM;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int m = m0 + 16 * u + lr;
        if (m >= M) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = j0 + 16 * wv + acc_row<TC>(lane, r);
            if (j >= M) continue;
            const double rr = (double)acc_rr[u][r], ii = (double)acc_ii[u][r];
            out[(long)j * M + m] = rr + ii;
            out[MM + (long)j * M + m] = (double)acc_ss[u][r] - rr + ii;
        }
    }
}

// 16-byte pair loads: base 16-byte aligned, even row length and walker stride
// (every row start and every even offset in a row is then aligned)
inline bool aligned(const double* p, long bs, int M) {
    return ((uintptr_t)p % 16) == 0 && bs % 2 == 0 && M % 2 == 0;
}

template <typename TC>
hipError_t launch_cterm(const CTerm& c, hipStream_t s) {
    const int ncb = (c.M + BJ - 1) / BJ;
    const int rt = c.N <= 16 ? 1 : (c.N <= 32 ? 2 : 3);
    const int nrb = (c.N + 16 * rt - 1) / (16 * rt);
    const long nb = (long)ncb * nrb * c.nw;
    const dim3 grid((unsigned)((nb + 7) / 8 * 8));
    const bool al = aligned(c.in, c.in_bs, c.M) && aligned(c.A, 2L * c.M * c.M, c.M);
    if (al) {
        if (rt == 1)
            hipLaunchKernelGGL((k_cterm<TC, 1, true>), grid, dim3(256), 0, s, c, ncb, nrb);
        else if (rt == 2)
            hipLaunchKernelGGL((k_cterm<TC, 2, true>), grid, dim3(256), 0, s, c, ncb, nrb);
        else
            hipLaunchKernelGGL((k_cterm<TC, 3, true>), grid, dim3(256), 0, s, c, ncb, nrb);
    } else {
        if (rt == 1)
            hipLaunchKernelGGL((k_cterm<TC, 1, false>), grid, dim3(256), 0, s, c, ncb, nrb);
        else if (rt == 2)
            hipLaunchKernelGGL((k_cterm<TC, 2, false>), grid, dim3(256), 0, s, c, ncb, nrb);
        else
            hipLaunchKernelGGL((k_cterm<TC, 3, false>), grid, dim3(256), 0, s, c, ncb, nrb);
    }
    return hipGetLastError();
}

template <typename TC>
hipError_t launch_cabar(const CAbar& c, hipStream_t s) {
    const int nb1 = (c.M + 63) / 64;
    const long nb = (long)nb1 * nb1 * c.nw;
    const dim3 grid((unsigned)((nb + 7) / 8 * 8));
    if (aligned(c.S, c.bs, c.M) && aligned(c.T, c.bs, c.M))
        hipLaunchKernelGGL((k_cabar<TC, true>), grid, dim3(256), 0, s, c, nb1);
    else
        hipLaunchKernelGGL((k_cabar<TC, false>), grid, dim3(256), 0, s, c, nb1);
    return hipGetLastError();
}

}  // namespace
}  // namespace dev

hipError_t cterm(const CTerm& c, DType compute, hipStream_t s) {
    if (c.nw <= 0 || c.M <= 0 || c.N <= 0) return hipSuccess;
    if (!c.in || !c.A || (!c.out && !c.acc_out) || (c.acc_out && !c.acc_in))
        return hipErrorInvalidValue;
    return compute == DT_F64 ? dev::launch_cterm<double>(c, s) : dev::launch_cterm<float>(c, s);
}

hipError_t cabar(const CAbar& c, DType compute, hipStream_t s) {
    if (c.nw <= 0 || c.M <= 0) return hipSuccess;
    if (!c.S || !c.T || !c.Abar || c.nq < 0 || c.N < 0) return hipErrorInvalidValue;
    return compute == DT_F64 ? dev::launch_cabar<double>(c, s) : dev::launch_cabar<float>(c, s);
}

}  // namespace afq
