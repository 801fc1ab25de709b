// Fused walker propagation (Eq. 11 between one-body halves, Eq. 3):
//   Phi' = P T_K(A_w) P Phi,   T_K(A) = sum_{n <= K} A^n / n!,
// evaluated term by term (term_n = A term_{n-1} / n) for every walker.
//
// Each workgroup owns R orbital columns of one walker for the whole
// propagation: the orbitals never couple (every factor multiplies from the
// left), so the R x M complex state stays resident in LDS across the
// 2 + K dense products and only P, A_w and the walker itself stream from
// HBM/L2.  The running sum Z of the Taylor terms lives in registers (in LDS
// for two of the shapes).  The products run on the matrix cores: FP64 or
// FP32 MFMA 16x16x4, or split BF16 (MFMA 16x16x32, three per product).
#include <atomic>

#include "mfma.h"
#include "roles.h"

// No contraction of a multiply and an add into one fused operation anywhere
// in this file: the Taylor-term scaling and the running sum must round the
// same way in every workgroup shape.
#pragma clang fp contract(off)

namespace afq {
namespace {

using namespace dev;

// Packed upper triangle (row-major, P = M(M+1)/2 per plane) -> full
// symmetric M x M, through a 32 x 33 LDS tile so both the direct and the
// mirrored writes are coalesced.  grid: (planes, row bands of 32): the plane
// count (2 per walker) on x, whose limit is 2^31 - 1 blocks.
template <typename T>
__global__ __launch_bounds__(256) void k_unpack(const T* __restrict__ pk, T* __restrict__ full,
                                                int M) {
    __shared__ T tile[32][33];
    const long P = (long)M * (M + 1) / 2;
    const long plane = blockIdx.x;
    const int ti = blockIdx.y;
    const T* src = pk + plane * P;
    T* dst = full + plane * (long)M * M;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int nt = (M + 31) / 32;
    for (int tj = ti; tj < nt; ++tj) {
        // load rows i in band ti, columns j in band tj with j >= i
        for (int r = ty; r < 32; r += 8) {
            const int i = ti * 32 + r, j = tj * 32 + tx;
            T v = (T)0;
            if (i < M && j < M && j >= i) v = src[(long)i * (2 * M - i + 1) / 2 + (j - i)];
            tile[r][tx] = v;
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = ti * 32 + r, j = tj * 32 + tx;
            if (i < M && j < M) {
                // direct element (i, j): upper part from the tile, lower part of a
                // diagonal tile from its mirror
                dst[(long)i * M + j] = (j >= i) ? tile[r][tx] : tile[tx][r];
            }
            if (tj != ti) {
                // mirrored element (j', i') with j' = tj*32 + r, i' = ti*32 + tx
                const int jm = tj * 32 + r, im = ti * 32 + tx;
                if (jm < M && im < M) dst[(long)jm * M + im] = tile[tx][r];
            }
        }
        __syncthreads();
    }
}

// Raw buffer loads: 32-bit byte offsets against a descriptor of the operand
// (no 64-bit address registers; offsets past the end read as zero).
// LDS row pitches of the propagation state for M <= 256 (elements): 16-byte
// aligned rows whose starts step across the banks.
constexpr int kPitchF = 260, kPitchB = 264;
// BF16 row pitch of the five-row-block shape (M <= 224): 80 rows fit in LDS
constexpr int kPitchB5 = 232;
constexpr int rb_pitch(int rb) { return rb == 5 ? kPitchB5 : kPitchB; }

constexpr int kBufFlags = 0x00020000;  // gfx9-family raw buffer descriptor word 3
constexpr int kOutOfRange = 0x40000000;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const T* p, long n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, (int)(n * sizeof(T)),
                                             kBufFlags);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, int off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Raw buffer load of 4 consecutive elements of T (float: one dwordx4;
// double: two dwordx4).  The loaded vector is bit-cast as a whole.
__device__ __forceinline__ void bload4(__amdgpu_buffer_rsrc_t r, int off, float* v) {
    const f4 x = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = x[e];
}
__device__ __forceinline__ void bload4(__amdgpu_buffer_rsrc_t r, int off, double* v) {
    const d2 x = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    const d2 y = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0));
    v[0] = x[0];
    v[1] = x[1];
    v[2] = y[0];
    v[3] = y[1];
}

// 1 / n as a compile-time table (correctly rounded by the compiler), so
// every kernel shape scales the Taylor terms by the same value.
__device__ __forceinline__ double inv_n_d(int n) {
    constexpr double t[17] = {0.0,        1.0,        1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,
                              1.0 / 6,    1.0 / 7,    1.0 / 8,  1.0 / 9,  1.0 / 10, 1.0 / 11,
                              1.0 / 12,   1.0 / 13,   1.0 / 14, 1.0 / 15, 1.0 / 16};
    return n <= 16 ? t[n] : 1.0 / n;
}
__device__ __forceinline__ float inv_n_f(int n) {
    constexpr float t[17] = {0.0f,        1.0f,        1.0f / 2,  1.0f / 3,  1.0f / 4,  1.0f / 5,
                             1.0f / 6,    1.0f / 7,    1.0f / 8,  1.0f / 9,  1.0f / 10, 1.0f / 11,
                             1.0f / 12,   1.0f / 13,   1.0f / 14, 1.0f / 15, 1.0f / 16};
    return n <= 16 ? t[n] : 1.0f / n;
}

// acc <- acc / n and z <- z + acc with separate roundings (no contraction
// into a fused multiply-add, so every workgroup shape rounds alike).
template <typename V, typename S_>
__device__ __forceinline__ void term_update(V& acc, V& z, S_ inv) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        acc[e] = acc[e] * inv;  // contraction is off in this file
        z[e] = z[e] + acc[e];
    }
}

// One pass: acc[s] = S (16 x Mp, 2 planes in LDS) x B^T for this wave's
// column blocks cb[s] (skipped when >= MB, a wave-uniform test), B = M x M
// (rows m, K-contiguous), real (NPB = 1) or complex (NPB = 2, planes M*M
// apart), read through descriptor rb.
// Inside each 16-wide K chunk the MFMA k-order is permuted: for sub-step j
// lane group g = lane / 16 supplies k = k0 + 4 g + j.  Every lane's operand
// run is then 4 contiguous elements: one LDS read of S and one 16-byte
// buffer load of B per chunk, straight into registers (each B column block
// belongs to one wave, so no staging and no barrier inside the pass).  B
// loads run one chunk ahead.  Columns >= M of B multiply zero columns of S.
template <typename T, int MAXB, int NPB, bool PF, int SPT>
__device__ __forceinline__ void pass(__amdgpu_buffer_rsrc_t rb, int M, int Mp, int MB,
                                     const T* S, const int* cb,
                                     typename AccT<T>::v (&acc)[MAXB][2]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, li = lane & 15;
    const int plane_b = M * M * (int)sizeof(T);
    const long splane = 16L * SPT;
    const T* srow_r = S + li * SPT + 4 * g;
    const T* srow_i = srow_r + splane;
    int boff[MAXB];
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        const int m = cb[s] * 16 + li;
        boff[s] = m < M ? (m * M + 4 * g) * (int)sizeof(T) : kOutOfRange;
        acc[s][0] = acc[s][1] = typename AccT<T>::v{0, 0, 0, 0};
    }
    T bc[MAXB][NPB][4], bn[MAXB][NPB][4];
    // Loads are unconditional (straight-line code lets the compiler count
    // them exactly): blocks >= MB read through an out-of-range offset (zeros)
    // and the prefetch past the last chunk reads values that are never used.
    // PF: B runs one chunk ahead; else each chunk loads its own B (fewer
    // registers, more waves to hide the latency).
    if constexpr (PF) {
#pragma unroll
        for (int s = 0; s < MAXB; ++s)
#pragma unroll
            for (int p = 0; p < NPB; ++p) bload4(rb, boff[s] + p * plane_b, bc[s][p]);
    }
    for (int k0 = 0; k0 < Mp; k0 += 16) {
        const int kb = (k0 + (PF ? 16 : 0)) * (int)sizeof(T);
#pragma unroll
        for (int s = 0; s < MAXB; ++s)
#pragma unroll
            for (int p = 0; p < NPB; ++p)
                bload4(rb, boff[s] + kb + p * plane_b, PF ? bn[s][p] : bc[s][p]);
        T sr[4], si[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sr[j] = srow_r[k0 + j];
            si[j] = srow_i[k0 + j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int s = 0; s < MAXB; ++s) {
                if (cb[s] >= MB) continue;  // wave-uniform
                if constexpr (NPB == 1) {
                    acc[s][0] = mma1(sr[j], bc[s][0][j], acc[s][0]);
                    acc[s][1] = mma1(si[j], bc[s][0][j], acc[s][1]);
                } else {
                    acc[s][0] = mma1(sr[j], bc[s][0][j], acc[s][0]);
                    acc[s][0] = mma1(-si[j], bc[s][1][j], acc[s][0]);
                    acc[s][1] = mma1(sr[j], bc[s][1][j], acc[s][1]);
                    acc[s][1] = mma1(si[j], bc[s][0][j], acc[s][1]);
                }
            }
        }
        if constexpr (PF) {
#pragma unroll
            for (int s = 0; s < MAXB; ++s)
#pragma unroll
                for (int p = 0; p < NPB; ++p)
#pragma unroll
                    for (int e = 0; e < 4; ++e) bc[s][p][e] = bn[s][p][e];
        }
    }
}

// One workgroup = 16 orbitals (one MFMA row block) of one walker for the
// whole propagation.  Workgroups are ordered so that the row blocks of a
// walker run back to back on one XCD and A_w streams through its L2; the
// assignment of column blocks to waves rotates between workgroups so the
// waves holding an extra block land on different SIMDs.
// REC: also record the Taylor terms and their sum (rec; see Record).
template <typename T, int NWAVE, int MAXB, bool PF, bool REC>
__global__ __launch_bounds__(64 * NWAVE, 2) void k_propagate(
    const double* __restrict__ phi, double* __restrict__ phi_out, const T* __restrict__ Pm,
    const T* __restrict__ Af, const uint8_t* __restrict__ live, int nw, int M, int N, int K,
    int nrb, Record rec) {
    typedef typename AccT<T>::v accv;
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    T* S = reinterpret_cast<T*>(smem_raw);
    constexpr int NT = 64 * NWAVE;
    const int Mp = (M + 15) / 16 * 16;
    const int MB = Mp / 16;
    // fixed row pitch for M <= 256 (16-byte aligned rows, staggered banks):
    // LDS offsets become instruction immediates
    constexpr int SPT = kPitchF;
    constexpr long splane = 16L * SPT;
    const long nblk = (long)nw * nrb;
    const long per = (nblk + 7) / 8;
    const long L = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblk) return;
    const int w = (int)(L / nrb), row0 = (int)(L % nrb) * 16;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const long NM = (long)N * M;
    const double* src = phi + (long)w * 2 * NM;
    double* dst = phi_out + (long)w * 2 * NM;
    const int nrow = min(16, N - row0);
    if (nrow <= 0) return;
    // recorded terms of this walker: slot n at rt + n rec.bs_slot (planes NM apart)
    double* rt = REC ? rec.terms + (long)w * rec.bs_walker : nullptr;
    double* ry = REC ? rec.y + (long)w * 2 * NM : nullptr;
    if (!live[w]) {  // frozen walker: carried over unchanged (recorded terms zero)
        for (int e = tid; e < 2 * nrow * M; e += NT) {
            const int p = e / (nrow * M), rem = e % (nrow * M);
            const long o = p * NM + (long)(row0 + rem / M) * M + rem % M;
            dst[o] = src[o];
            if constexpr (REC) {
                ry[o] = 0.0;
                for (int n = 0; n < K; ++n) rt[n * rec.bs_slot + o] = 0.0;
            }
        }
        return;
    }
    for (int e = tid; e < 2 * 16 * Mp; e += NT) {
        const int p = e / (16 * Mp), rem = e % (16 * Mp);
        const int r = rem / Mp, m = rem % Mp;
        double v = 0.0;
        if (r < nrow && m < M) v = src[p * NM + (long)(row0 + r) * M + m];
        S[p * splane + r * SPT + m] = (T)v;
    }
    const int vw = (wave + (int)(L % NWAVE)) % NWAVE;  // rotated wave slot
    int cb[MAXB];
#pragma unroll
    for (int s = 0; s < MAXB; ++s) cb[s] = vw + s * NWAVE;
    __syncthreads();
    accv acc[MAXB][2], z[MAXB][2];
    const long Aplane = (long)M * M;
    const __amdgpu_buffer_rsrc_t rP = make_rsrc(Pm, Aplane);
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(Af + (long)w * 2 * Aplane, 2 * Aplane);
    // write a block of the running state into S; columns >= M stay zero
    auto put = [&](int s, const accv& vr, const accv& vi) {
        const int col = cb[s] * 16 + (lane & 15);
        const bool ok = col < M;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int off = acc_row<T>(lane, r) * SPT + col;
            S[off] = ok ? vr[r] : (T)0;
            S[splane + off] = ok ? vi[r] : (T)0;
        }
    };
    // a block of this walker's rows in the walker layout (recording)
    auto keep = [&](double* base, int s, const accv& vr, const accv& vi) {
        const int col = cb[s] * 16 + (lane & 15);
        if (cb[s] >= MB || col >= M) return;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = acc_row<T>(lane, r);
            if (row < nrow) {
                const long o = (long)(row0 + row) * M + col;
                base[o] = (double)vr[r];
                base[NM + o] = (double)vi[r];
            }
        }
    };
    // first one-body half
    pass<T, MAXB, 1, PF, SPT>(rP, M, Mp, MB, S, cb, acc);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        z[s][0] = acc[s][0];
        z[s][1] = acc[s][1];
        if (cb[s] < MB) put(s, acc[s][0], acc[s][1]);
        if constexpr (REC)
            if (K > 0) keep(rt, s, acc[s][0], acc[s][1]);
    }
    __syncthreads();
    // Taylor series of exp(A): term_n = A term_{n-1} / n, z = sum of terms
    for (int n = 1; n <= K; ++n) {
        pass<T, MAXB, 2, PF, SPT>(rA, M, Mp, MB, S, cb, acc);
        __syncthreads();
        const T inv = sizeof(T) == 8 ? (T)inv_n_d(n) : (T)inv_n_f(n);
#pragma unroll
        for (int s = 0; s < MAXB; ++s) {
            term_update(acc[s][0], z[s][0], inv);
            term_update(acc[s][1], z[s][1], inv);
            if (cb[s] < MB) {
                if (n == K)
                    put(s, z[s][0], z[s][1]);
                else
                    put(s, acc[s][0], acc[s][1]);
            }
            if constexpr (REC) {
                if (n < K) keep(rt + n * rec.bs_slot, s, acc[s][0], acc[s][1]);
                if (n == K) keep(ry, s, z[s][0], z[s][1]);
            }
        }
        __syncthreads();
    }
    // second one-body half, FP64 result
    pass<T, MAXB, 1, PF, SPT>(rP, M, Mp, MB, S, cb, acc);
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        const int col = cb[s] * 16 + (lane & 15);
        if (cb[s] >= MB || col >= M) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = acc_row<T>(lane, r);
            if (row < nrow) {
                const long o = (long)(row0 + row) * M + col;
                dst[o] = (double)acc[s][0][r];
                dst[NM + o] = (double)acc[s][1][r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 propagation.  A_w is stored as hi/lo BF16 planes
// ([w][re, im][hi, lo][M][M]) and the state S as four BF16 planes (re hi,
// re lo, im hi, im lo); each real product is three BF16 MFMAs 16x16x32
// (hi hi + hi lo + lo hi) with FP32 accumulation.  The one-body halves are
// applied as P y = y + Q y with Q = P - I held as hi/lo BF16 planes
// ([hi, lo][M][M]): P is close to the identity, so splitting Q instead of P
// scales the rounding of the product down by |Q|, and the identity part is
// added exactly (in FP32) by starting the accumulators at y.

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf8 neg8(bf8 x) {
    return __builtin_bit_cast(bf8, __builtin_bit_cast(u4v, x) ^ 0x80008000u);
}
__device__ __forceinline__ bf8 bload8(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(bf8, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// CX (complex operand A_w, four planes): acc[s] = S x A_w^T from zero.
// !CX (real operand Q, two planes): acc[s] += S x Q^T, each part of S
// against Q.  This wave's column blocks; K in chunks of 32, lane group g
// supplying k = k0 + 8 g + e (e < 8) for both operands.
template <int MAXB, bool PF, int SPB, bool CX>
__device__ __forceinline__ void pass_split(__amdgpu_buffer_rsrc_t rb, int M, int Mp, int MB,
                                           const bf16_t* Sb, const int* cb,
                                           f4 (&acc)[MAXB][2]) {
    constexpr int NP = CX ? 4 : 2;  // operand planes: re hi, re lo (, im hi, im lo)
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, li = lane & 15;
    const int hl_b = (int)split_tile_elems(M) * 2;  // hi -> lo plane, bytes
    const int pl_b = 2 * hl_b;                        // re -> im plane
    const int kc = Mp / 32;
    const long spl = 16L * SPB;
    const bf16_t* s0 = Sb + li * SPB + 8 * g;
    int boff[MAXB];  // this lane's 16 bytes of chunk 0 of each column block
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        boff[s] = cb[s] < MB ? (cb[s] * kc * 64 + lane) * 16 : kOutOfRange;
        if constexpr (CX) acc[s][0] = acc[s][1] = f4{0, 0, 0, 0};
    }
    bf8 bc[MAXB][NP], bn[MAXB][NP];
    // unconditional loads and the PF choice as in pass()
    if constexpr (PF) {
#pragma unroll
        for (int s = 0; s < MAXB; ++s)
#pragma unroll
            for (int p = 0; p < NP; ++p)
                bc[s][p] = bload8(rb, boff[s] + (p & 1) * hl_b + (p >> 1) * pl_b);
    }
    for (int k0 = 0; k0 < Mp; k0 += 32) {
        const int kb = (k0 + (PF ? 32 : 0)) * 32;  // 1 KB per chunk
#pragma unroll
        for (int s = 0; s < MAXB; ++s) {
            bf8* d = PF ? bn[s] : bc[s];
#pragma unroll
            for (int p = 0; p < NP; ++p)
                d[p] = bload8(rb, boff[s] + kb + (p & 1) * hl_b + (p >> 1) * pl_b);
        }
        const bf8 rh = *reinterpret_cast<const bf8*>(s0 + k0);
        const bf8 rl = *reinterpret_cast<const bf8*>(s0 + spl + k0);
        const bf8 ih = *reinterpret_cast<const bf8*>(s0 + 2 * spl + k0);
        const bf8 il = *reinterpret_cast<const bf8*>(s0 + 3 * spl + k0);
        if constexpr (CX) {
            const bf8 nh = neg8(ih), nl = neg8(il);
#pragma unroll
            for (int s = 0; s < MAXB; ++s) {
                if (cb[s] >= MB) continue;  // wave-uniform
                f4 ar = acc[s][0], ai = acc[s][1];
                // re += Sr Ar - Si Ai
                ar = mma8(rl, bc[s][0], ar);
                ar = mma8(rh, bc[s][1], ar);
                ar = mma8(rh, bc[s][0], ar);
                ar = mma8(nl, bc[s][2], ar);
                ar = mma8(nh, bc[s][3], ar);
                ar = mma8(nh, bc[s][2], ar);
                // im += Sr Ai + Si Ar
                ai = mma8(rl, bc[s][2], ai);
                ai = mma8(rh, bc[s][3], ai);
                ai = mma8(rh, bc[s][2], ai);
                ai = mma8(il, bc[s][0], ai);
                ai = mma8(ih, bc[s][1], ai);
                ai = mma8(ih, bc[s][0], ai);
                acc[s][0] = ar;
                acc[s][1] = ai;
            }
        } else {
#pragma unroll
            for (int s = 0; s < MAXB; ++s) {
                if (cb[s] >= MB) continue;  // wave-uniform
                f4 ar = acc[s][0], ai = acc[s][1];
                ar = mma8(rl, bc[s][0], ar);
                ar = mma8(rh, bc[s][1], ar);
                ar = mma8(rh, bc[s][0], ar);
                ai = mma8(il, bc[s][0], ai);
                ai = mma8(ih, bc[s][1], ai);
                ai = mma8(ih, bc[s][0], ai);
                acc[s][0] = ar;
                acc[s][1] = ai;
            }
        }
        if constexpr (PF) {
#pragma unroll
            for (int s = 0; s < MAXB; ++s)
#pragma unroll
                for (int p = 0; p < NP; ++p) bc[s][p] = bn[s][p];
        }
    }
}

// As k_propagate (FP32 accumulation) with every product in split BF16: the
// four BF16 planes of the state are the only copy of it in LDS (Mp is M
// rounded up to 32; columns >= M stay zero), the identity parts of the
// one-body halves and the running Taylor sum are FP32 registers.
template <int NWAVE, int MAXB, bool PF>
__global__ __launch_bounds__(64 * NWAVE, 2) void k_propagate_split(
    const double* __restrict__ phi, double* __restrict__ phi_out, const bf16_t* __restrict__ Qs,
    const bf16_t* __restrict__ Af, const uint8_t* __restrict__ live, int nw, int M, int N, int K,
    int nrb) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    bf16_t* Sb = reinterpret_cast<bf16_t*>(smem_raw);
    constexpr int NT = 64 * NWAVE;
    const int Mp = (M + 31) / 32 * 32;
    const int MB = (M + 15) / 16;
    constexpr int SPB = kPitchB;  // fixed pitch (M <= 256)
    constexpr long bplane = 16L * SPB;
    const long nblk = (long)nw * nrb;
    const long per = (nblk + 7) / 8;
    const long L = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblk) return;
    const int w = (int)(L / nrb), row0 = (int)(L % nrb) * 16;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const long NM = (long)N * M;
    const double* src = phi + (long)w * 2 * NM;
    double* dst = phi_out + (long)w * 2 * NM;
    const int nrow = min(16, N - row0);
    if (nrow <= 0) return;
    if (!live[w]) {
        for (int e = tid; e < 2 * nrow * M; e += NT) {
            const int p = e / (nrow * M), rem = e % (nrow * M);
            const long o = p * NM + (long)(row0 + rem / M) * M + rem % M;
            dst[o] = src[o];
        }
        return;
    }
    const int vw = (wave + (int)(L % NWAVE)) % NWAVE;
    int cb[MAXB];
#pragma unroll
    for (int s = 0; s < MAXB; ++s) cb[s] = vw + s * NWAVE;
    const long Aplane = split_tile_elems(M);  // fragment-tiled operand planes
    const __amdgpu_buffer_rsrc_t rQ = make_rsrc(Qs, 2 * Aplane);
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(Af + (long)w * 4 * Aplane, 4 * Aplane);
    const int li = lane & 15;
    // the columns no block writes (MB * 16 .. Mp) stay zero throughout
    {
        const int pad = Mp - MB * 16;
        for (int e = tid; e < 4 * 16 * pad; e += NT) {
            const int q = e / (16 * pad), rem = e % (16 * pad);
            Sb[q * bplane + (rem / pad) * SPB + MB * 16 + rem % pad] = (bf16_t)0.0f;
        }
    }
    auto put_b = [&](int s, const f4& vr, const f4& vi) {
        const int col = cb[s] * 16 + li;
        const bool ok = col < M;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int off = acc_row<float>(lane, r) * SPB + col;
            const float xr = ok ? vr[r] : 0.0f, xi = ok ? vi[r] : 0.0f;
            const bf16_t hr = to_bf(xr), hi = to_bf(xi);
            Sb[off] = hr;
            Sb[bplane + off] = to_bf(xr - (float)hr);
            Sb[2 * bplane + off] = hi;
            Sb[3 * bplane + off] = to_bf(xi - (float)hi);
        }
    };
    // the walker's block in the accumulator layout (zero past the orbitals
    // and past column M), loaded unconditionally from clamped offsets
    f4 acc[MAXB][2], z[MAXB][2];
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        const int col = cb[s] * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = acc_row<float>(lane, r);
            const bool ok = cb[s] < MB && row < nrow && col < M;
            const long o = ok ? (long)(row0 + row) * M + col : 0;
            const double xr = src[o], xi = src[NM + o];
            acc[s][0][r] = ok ? (float)xr : 0.0f;
            acc[s][1][r] = ok ? (float)xi : 0.0f;
        }
        if (cb[s] < MB) put_b(s, acc[s][0], acc[s][1]);
    }
    __syncthreads();
    // first one-body half: y = x + Q x
    pass_split<MAXB, PF, SPB, false>(rQ, M, Mp, MB, Sb, cb, acc);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        z[s][0] = acc[s][0];
        z[s][1] = acc[s][1];
        if (cb[s] < MB) put_b(s, acc[s][0], acc[s][1]);
    }
    __syncthreads();
    for (int n = 1; n <= K; ++n) {
        pass_split<MAXB, PF, SPB, true>(rA, M, Mp, MB, Sb, cb, acc);
        __syncthreads();
        const float inv = inv_n_f(n);
#pragma unroll
        for (int s = 0; s < MAXB; ++s) {
            term_update(acc[s][0], z[s][0], inv);
            term_update(acc[s][1], z[s][1], inv);
            if (cb[s] < MB) {
                if (n == K)
                    put_b(s, z[s][0], z[s][1]);
                else
                    put_b(s, acc[s][0], acc[s][1]);
            }
        }
        __syncthreads();
    }
    // second one-body half on the Taylor sum (the BF16 view holds z)
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        acc[s][0] = z[s][0];
        acc[s][1] = z[s][1];
    }
    pass_split<MAXB, PF, SPB, false>(rQ, M, Mp, MB, Sb, cb, acc);
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        const int col = cb[s] * 16 + li;
        if (cb[s] >= MB || col >= M) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = acc_row<float>(lane, r);
            if (row < nrow) {
                const long o = (long)(row0 + row) * M + col;
                dst[o] = (double)acc[s][0][r];
                dst[NM + o] = (double)acc[s][1][r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// RB row blocks per workgroup (16 RB orbitals of one walker): every operand
// fragment of A_w or Q a wave loads serves RB row blocks, so the loads per
// matrix-core product drop by RB.  Operands are loaded chunk by chunk (no
// prefetch); row blocks past the walker's last orbital are skipped.  CX and
// the accumulation as in pass_split, with the same product order per
// accumulator.
template <int MAXB, int RB, bool CX>
__device__ __forceinline__ void pass_split_rb(__amdgpu_buffer_rsrc_t rb, int M, int Mp, int MB,
                                              int rlo, int rhi, const bf16_t* Sb, int SPB,
                                              const int* cb,
                                              f4 (&acc)[RB][MAXB][2]) {
    constexpr int NP = CX ? 4 : 2;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, li = lane & 15;
    const int hl_b = (int)split_tile_elems(M) * 2;
    const int pl_b = 2 * hl_b;
    const int kc = Mp / 32;
    const long spl = 16L * RB * SPB;
    int boff[MAXB];
#pragma unroll
    for (int s = 0; s < MAXB; ++s) {
        boff[s] = cb[s] < MB ? (cb[s] * kc * 64 + lane) * 16 : kOutOfRange;
        if constexpr (CX) {
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[r][s][0] = acc[r][s][1] = f4{0, 0, 0, 0};
        }
    }
    for (int k0 = 0; k0 < Mp; k0 += 32) {
        bf8 bc[MAXB][NP];  // re hi, re lo (, im hi, im lo)
#pragma unroll
        for (int s = 0; s < MAXB; ++s)
#pragma unroll
            for (int p = 0; p < NP; ++p)
                bc[s][p] = bload8(rb, boff[s] + k0 * 32 + (p & 1) * hl_b + (p >> 1) * pl_b);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (r < rlo || r >= rhi) continue;  // wave-uniform
            const bf16_t* s0 = Sb + (r * 16 + li) * SPB + 8 * g + k0;
            // real-part fragments first, then the imaginary ones (fewer live
            // registers; each accumulator sees the same product order)
            const bf8 rh = *reinterpret_cast<const bf8*>(s0);
            const bf8 rl = *reinterpret_cast<const bf8*>(s0 + spl);
#pragma unroll
            for (int s = 0; s < MAXB; ++s) {
                if (cb[s] >= MB) continue;  // wave-uniform
                f4 ar = acc[r][s][0];
                ar = mma8(rl, bc[s][0], ar);
                ar = mma8(rh, bc[s][1], ar);
                ar = mma8(rh, bc[s][0], ar);
                if constexpr (CX) {
                    f4 ai = acc[r][s][1];
                    ai = mma8(rl, bc[s][2], ai);
                    ai = mma8(rh, bc[s][3], ai);
                    ai = mma8(rh, bc[s][2], ai);
                    acc[r][s][1] = ai;
                }
                acc[r][s][0] = ar;
            }
            const bf8 ih = *reinterpret_cast<const bf8*>(s0 + 2 * spl);
            const bf8 il = *reinterpret_cast<const bf8*>(s0 + 3 * spl);
            if constexpr (CX) {
                // the imaginary products first: their fragments are then
                // dead, and the negated copies take their registers
#pragma unroll
                for (int s = 0; s < MAXB; ++s) {
                    if (cb[s] >= MB) continue;  // wave-uniform
                    f4 ai = acc[r][s][1];
                    ai = mma8(il, bc[s][0], ai);
                    ai = mma8(ih, bc[s][1], ai);
                    ai = mma8(ih, bc[s][0], ai);
                    acc[r][s][1] = ai;
                }
                const bf8 nh = neg8(ih), nl = neg8(il);
#pragma unroll
                for (int s = 0; s < MAXB; ++s) {
                    if (cb[s] >= MB) continue;  // wave-uniform
                    f4 ar = acc[r][s][0];
                    ar = mma8(nl, bc[s][2], ar);
                    ar = mma8(nh, bc[s][3], ar);
                    ar = mma8(nh, bc[s][2], ar);
                    acc[r][s][0] = ar;
                }
            } else {
#pragma unroll
                for (int s = 0; s < MAXB; ++s) {
                    if (cb[s] >= MB) continue;  // wave-uniform
                    f4 ai = acc[r][s][1];
                    ai = mma8(il, bc[s][0], ai);
                    ai = mma8(ih, bc[s][1], ai);
                    ai = mma8(ih, bc[s][0], ai);
                    acc[r][s][1] = ai;
                }
            }
            // keep each row block's operand fragments from being hoisted
            // together (register budget of the 16-wave shape)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}


// ZREG: the running Taylor sum in registers (else in LDS beside the state).
template <int NWAVE, int MAXB, int RB, bool ZREG>
__global__ __launch_bounds__(64 * NWAVE, 1) void k_propagate_split_rb(
    const double* __restrict__ phi, double* __restrict__ phi_out, const bf16_t* __restrict__ Qs,
    const bf16_t* __restrict__ Af, const uint8_t* __restrict__ live, int nw, int M, int N, int K,
    int nrb) {
    extern __shared__ __attribute__((aligned(16))) char smem_raw[];
    constexpr int NT = 64 * NWAVE;
    constexpr int ROWS = 16 * RB;
    const int Mp = (M + 31) / 32 * 32;
    const int MB = (M + 15) / 16;
    // fixed row pitches (M <= 256): LDS offsets become instruction immediates
    constexpr int SPT = kPitchF, SPB = rb_pitch(RB);
    constexpr long splane = (long)ROWS * SPT, bplane = (long)ROWS * SPB;
    bf16_t* Sb = reinterpret_cast<bf16_t*>(smem_raw);
    // running Taylor sum, FP32, rows of pitch SPT (own elements only: no
    // barrier needed for its updates)
    float* Zs = reinterpret_cast<float*>(smem_raw + 4 * bplane * sizeof(bf16_t));
    const long nblk = (long)nw * nrb;
    const long per = (nblk + 7) / 8;
    const long L = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblk) return;
    const int w = (int)(L / nrb), row0 = (int)(L % nrb) * ROWS;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const long NM = (long)N * M;
    const double* src = phi + (long)w * 2 * NM;
    double* dst = phi_out + (long)w * 2 * NM;
    const int nrow = min(ROWS, N - row0);
    if (nrow <= 0) return;
    const int nrbv = (nrow + 15) / 16;  // row blocks holding orbitals
    if (!live[w]) {
        for (int e = tid; e < 2 * nrow * M; e += NT) {
            const int p = e / (nrow * M), rem = e % (nrow * M);
            const long o = p * NM + (long)(row0 + rem / M) * M + rem % M;
            dst[o] = src[o];
        }
        return;
    }
    const int vw = (wave + (int)(L % NWAVE)) % NWAVE;
    int cb[MAXB];
#pragma unroll
    for (int s = 0; s < MAXB; ++s) cb[s] = vw + s * NWAVE;
    // this wave's row blocks [rlo, rhi) of its column blocks
    int rlo = 0, rhi = nrbv;
    if constexpr (MAXB == 1 && NWAVE % 4 == 0) balance_roles(NWAVE, MB, nrbv, vw, cb[0], rlo, rhi);
    f4 acc[RB][MAXB][2];
    f4 zr[ZREG ? RB : 1][MAXB][2];
    const long Aplane = split_tile_elems(M);  // fragment-tiled operand planes
    const __amdgpu_buffer_rsrc_t rQ = make_rsrc(Qs, 2 * Aplane);
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(Af + (long)w * 4 * Aplane, 4 * Aplane);
    const int li = lane & 15;
    // the columns no block writes (MB * 16 .. Mp) stay zero throughout
    {
        const int pad = Mp - MB * 16;
        for (int e = tid; e < 4 * ROWS * pad; e += NT) {
            const int q = e / (ROWS * pad), rem = e % (ROWS * pad);
            Sb[q * bplane + (rem / pad) * SPB + MB * 16 + rem % pad] = (bf16_t)0.0f;
        }
    }
    auto put_b = [&](int r, int s, const f4& vr, const f4& vi) {
        const int col = cb[s] * 16 + li;
        const bool ok = col < M;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int off = (r * 16 + acc_row<float>(lane, q)) * SPB + col;
            const float xr = ok ? vr[q] : 0.0f, xi = ok ? vi[q] : 0.0f;
            const bf16_t hr = to_bf(xr), hi = to_bf(xi);
            Sb[off] = hr;
            Sb[bplane + off] = to_bf(xr - (float)hr);
            Sb[2 * bplane + off] = hi;
            Sb[3 * bplane + off] = to_bf(xi - (float)hi);
        }
    };
    // z (this thread's elements) <- v, or += v
    auto zacc = [&](int r, int s, f4& vr, f4& vi, bool first) {
        if constexpr (ZREG) {
            if (first) {
                zr[r][s][0] = vr;
                zr[r][s][1] = vi;
            } else {
                vr = zr[r][s][0] = zr[r][s][0] + vr;
                vi = zr[r][s][1] = zr[r][s][1] + vi;
            }
            return;
        }
        const int col = cb[s] * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int off = (r * 16 + acc_row<float>(lane, q)) * SPT + col;
            if (first) {
                Zs[off] = vr[q];
                Zs[splane + off] = vi[q];
            } else {
                vr[q] = Zs[off] = Zs[off] + vr[q];
                vi[q] = Zs[splane + off] = Zs[splane + off] + vi[q];
            }
        }
    };
    // the walker's rows in the accumulator layout (zero past the orbitals
    // and past column M); row blocks past the orbitals (r >= nrbv) are never
    // read or stored
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int s = 0; s < MAXB; ++s) {
            const int col = cb[s] * 16 + li;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = r * 16 + acc_row<float>(lane, q);
                const bool ok = cb[s] < MB && row < nrow && col < M;
                const long o = ok ? (long)(row0 + row) * M + col : 0;
                const double xr = src[o], xi = src[NM + o];
                acc[r][s][0][q] = ok ? (float)xr : 0.0f;
                acc[r][s][1][q] = ok ? (float)xi : 0.0f;
            }
            if (r >= rlo && r < rhi && cb[s] < MB) put_b(r, s, acc[r][s][0], acc[r][s][1]);
        }
    __syncthreads();
    // first one-body half: y = x + Q x
    pass_split_rb<MAXB, RB, false>(rQ, M, Mp, MB, rlo, rhi, Sb, SPB, cb, acc);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int s = 0; s < MAXB; ++s)
            if (r >= rlo && r < rhi && cb[s] < MB) {
                put_b(r, s, acc[r][s][0], acc[r][s][1]);
                zacc(r, s, acc[r][s][0], acc[r][s][1], true);
            }
    __syncthreads();
    for (int n = 1; n <= K; ++n) {
        pass_split_rb<MAXB, RB, true>(rA, M, Mp, MB, rlo, rhi, Sb, SPB, cb, acc);
        __syncthreads();
        const float inv = inv_n_f(n);
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int s = 0; s < MAXB; ++s) {
                if (r < rlo || r >= rhi || cb[s] >= MB) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    acc[r][s][0][q] = acc[r][s][0][q] * inv;
                    acc[r][s][1][q] = acc[r][s][1][q] * inv;
                }
                if (n == K) {
                    zacc(r, s, acc[r][s][0], acc[r][s][1], false);  // acc <- z
                    put_b(r, s, acc[r][s][0], acc[r][s][1]);
                } else {
                    put_b(r, s, acc[r][s][0], acc[r][s][1]);
                    f4 tr = acc[r][s][0], ti = acc[r][s][1];
                    zacc(r, s, tr, ti, false);
                }
            }
        __syncthreads();
    }
    // second one-body half on the Taylor sum: acc and the BF16 view hold z
    // (with K = 0 both still hold y)
    pass_split_rb<MAXB, RB, false>(rQ, M, Mp, MB, rlo, rhi, Sb, SPB, cb, acc);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int s = 0; s < MAXB; ++s) {
            const int col = cb[s] * 16 + li;
            if (r < rlo || r >= rhi || cb[s] >= MB || col >= M) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = r * 16 + acc_row<float>(lane, q);
                if (row < nrow) {
                    const long o = (long)(row0 + row) * M + col;
                    dst[o] = (double)acc[r][s][0][q];
                    dst[NM + o] = (double)acc[r][s][1][q];
                }
            }
        }
}

template <int NWAVE, int MAXB, int RB, bool ZREG>
hipError_t launch_prop_split_rb(const double* phi, double* phi_out, const void* Qs, const void* Af,
                                const uint8_t* live, int nw, int M, int N, int K, hipStream_t s) {
    // the BF16 state + the FP32 running sum when it is not in registers
    const size_t shm = 4 * 16 * RB * (size_t)rb_pitch(RB) * sizeof(bf16_t) +
                       (ZREG ? 0 : 2 * 16 * RB * (size_t)kPitchF * sizeof(float));
    const int nrb = (N + 16 * RB - 1) / (16 * RB);
    const long nblk = (long)nw * nrb;
    const long grid = ((nblk + 7) / 8) * 8;
    static std::atomic<bool> attr{false};  // per kernel; set before any capture
    if (!attr && shm > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_propagate_split_rb<NWAVE, MAXB, RB, ZREG>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_propagate_split_rb<NWAVE, MAXB, RB, ZREG>), dim3(grid), dim3(64 * NWAVE),
                       shm, s, phi, phi_out, (const bf16_t*)Qs, (const bf16_t*)Af, live, nw, M, N,
                       K, nrb);
    return hipGetLastError();
}

template <int NWAVE, int MAXB, bool PF>
hipError_t launch_prop_split(const double* phi, double* phi_out, const void* Qs, const void* Af,
                             const uint8_t* live, int nw, int M, int N, int K, hipStream_t s) {
    const size_t shm = 4 * 16 * (size_t)kPitchB * sizeof(bf16_t);
    const int nrb = (N + 15) / 16;
    const long nblk = (long)nw * nrb;
    const long grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_propagate_split<NWAVE, MAXB, PF>), dim3(grid), dim3(64 * NWAVE), shm, s,
                       phi, phi_out, (const bf16_t*)Qs, (const bf16_t*)Af, live, nw, M, N, K, nrb);
    return hipGetLastError();
}

// x -> (hi, lo) BF16 planes: out[plane][hi, lo][n]
__global__ void k_split_planes(const float* __restrict__ in, bf16_t* __restrict__ out, long n,
                               long planes) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * planes) return;
    const long pl = e / n, i = e % n;
    const float v = in[e];
    const bf16_t h = to_bf(v);
    out[pl * 2 * n + i] = h;
    out[pl * 2 * n + n + i] = to_bf(v - (float)h);
}

// One workgroup per walker plane: the packed upper triangle (FP32) is staged
// whole in LDS, then every thread writes one 8-element run of the
// fragment-tiled hi/lo BF16 planes of the full symmetric matrix (A_ij from
// the packed row min(i, j); zero past M) as one 16-byte hi store and one
// 16-byte lo store; consecutive threads write consecutive runs (any M: the
// runs past column M are zero).  Needs the triangle in LDS (M <= 256); 512
// threads (two workgroups per CU by LDS, eight waves each).
constexpr int kUnpackThreads = 512;
__global__ __launch_bounds__(kUnpackThreads) void k_unpack_split_plane(
    const float* __restrict__ pk, bf16_t* __restrict__ full, int M) {
    extern __shared__ float tri[];
    const long P = (long)M * (M + 1) / 2;
    const long plane = blockIdx.x;
    const float* src = pk + plane * P;
    // eight loads in flight per thread
    for (long e0 = threadIdx.x; e0 < P; e0 += 8 * kUnpackThreads) {
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const long e = e0 + q * kUnpackThreads;
            v[q] = src[e < P ? e : 0];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (e0 + q * kUnpackThreads < P) tri[e0 + q * kUnpackThreads] = v[q];
    }
    __syncthreads();
    const long TE = split_tile_elems(M);
    bf16_t* hi = full + plane * 2 * TE;
    bf16_t* lo = hi + TE;
    const int kc = (M + 31) / 32;
    const int nrun = (int)(TE / 8);
    for (int u = threadIdx.x; u < nrun; u += kUnpackThreads) {
        // run u: tile u / 64, lane slot u % 64 (row r % 16, column run)
        const int t = u >> 6, l = u & 63;
        const int i = (t / kc) * 16 + (l & 15);
        const int j0 = (t % kc) * 32 + (l >> 4) * 8;
        bf8 h, lw;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = j0 + e;
            const int a = i < j ? i : j, b = i < j ? j : i;
            const bool in = i < M && j < M;
            const float v = in ? tri[(long)a * (2 * M - a + 1) / 2 + (b - a)] : 0.0f;
            const bf16_t x = to_bf(v);
            h[e] = x;
            lw[e] = to_bf(v - (float)x);
        }
        *reinterpret_cast<bf8*>(hi + (long)u * 8) = h;
        *reinterpret_cast<bf8*>(lo + (long)u * 8) = lw;
    }
}

template <typename T, int NWAVE, int MAXB, bool PF>
hipError_t launch_prop(const double* phi, double* phi_out, const void* Pm, const void* Af,
                       const uint8_t* live, int nw, int M, int N, int K, const Record& rec,
                       hipStream_t s) {
    const size_t shm = 2 * 16 * (size_t)kPitchF * sizeof(T);
    const int nrb = (N + 15) / 16;
    const long nblk = (long)nw * nrb;
    const long grid = ((nblk + 7) / 8) * 8;
    if (rec.terms && rec.y)
        hipLaunchKernelGGL((k_propagate<T, NWAVE, MAXB, PF, true>), dim3(grid), dim3(64 * NWAVE),
                           shm, s, phi, phi_out, (const T*)Pm, (const T*)Af, live, nw, M, N, K, nrb,
                           rec);
    else
        hipLaunchKernelGGL((k_propagate<T, NWAVE, MAXB, PF, false>), dim3(grid), dim3(64 * NWAVE),
                           shm, s, phi, phi_out, (const T*)Pm, (const T*)Af, live, nw, M, N, K, nrb,
                           rec);
    return hipGetLastError();
}

}  // namespace

hipError_t split_planes(const float* in, void* out, long n, long planes, hipStream_t s) {
    if (n * planes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_planes, dim3((unsigned)((n * planes + 255) / 256)), dim3(256), 0, s,
                       in, (bf16_t*)out, n, planes);
    return hipGetLastError();
}

hipError_t unpack_prepare() {
    return hipFuncSetAttribute((const void*)k_unpack_split_plane,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kUnpackLds);
}

hipError_t unpack_sym(const void* pk, void* full, int M, int planes, DType t, hipStream_t s) {
    if (planes <= 0) return hipSuccess;
    dim3 grid(planes, (M + 31) / 32);
    if (t == DT_F64)
        hipLaunchKernelGGL(k_unpack<double>, grid, dim3(256), 0, s, (const double*)pk,
                           (double*)full, M);
    else if (t == DT_F32)
        hipLaunchKernelGGL(k_unpack<float>, grid, dim3(256), 0, s, (const float*)pk, (float*)full,
                           M);
    else if (t == DT_SPLIT && (size_t)M * (M + 1) / 2 * 4 <= kUnpackLds)
        hipLaunchKernelGGL(k_unpack_split_plane, dim3(planes), dim3(kUnpackThreads),
                           (size_t)M * (M + 1) / 2 * 4, s, (const float*)pk, (bf16_t*)full, M);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Workgroup shapes (waves, column blocks per wave, B prefetch, 16-orbital
// row blocks): a shape serves M up to 16 * waves * blocks.  Fewer waves per
// workgroup leave no idle waves at small M; more waves shorten each wave's
// share at large M; without the prefetch a wave holds fewer registers and
// more waves fit; more row blocks let each operand fragment a wave loads
// serve more orbitals (five, all 80 orbitals at N = 80, need M <= 224 for
// the state to fit LDS).
namespace {
struct PropShape {
    int waves, blocks;
    bool pf;
    int rows;  // row blocks per workgroup (split BF16 only when > 1)
};
constexpr PropShape kPropShapes[kPropVariants] = {
    {8, 2, true, 1},   {4, 2, true, 1},   {4, 1, true, 1}, {2, 2, true, 1},
    {8, 2, false, 1},  {4, 2, false, 1},  {4, 1, false, 1}, {2, 2, false, 1},
    {16, 1, false, 2}, {8, 1, false, 2},  {8, 2, false, 2}, {4, 2, false, 2},
    {8, 2, false, 5},  {16, 1, false, 5}};
}  // namespace

bool propagate_variant_ok(int v, int M, DType t, DType ta) {
    if (v < 0 || v >= kPropVariants || M <= 0) return false;
    if (t != DT_F64 && t != DT_F32) return false;
    if (ta != t && !(t == DT_F32 && ta == DT_SPLIT)) return false;
    const PropShape p = kPropShapes[v];
    if (t == DT_F64 && !p.pf) return false;  // the FP64 path keeps the prefetching shapes
    if (p.rows > 1 && ta != DT_SPLIT) return false;
    if (p.rows == 5 && (M + 31) / 32 * 32 > kPitchB5 - 8) return false;  // 80 rows in LDS
    return (M + 15) / 16 <= p.waves * p.blocks;
}

hipError_t propagate(const double* phi, double* phi_out, const void* Pm, const void* Af,
                     const uint8_t* live, int nw, int M, int N, int K, DType t, DType ta,
                     int variant, hipStream_t s, const Record& rec) {
    if (nw <= 0) return hipSuccess;
    if ((rec.terms || rec.y) && ta == DT_SPLIT) return hipErrorNotSupported;
    if (M > 256 || M <= 0 || N <= 0) return hipErrorInvalidValue;
    if (!propagate_variant_ok(variant, M, t, ta)) return hipErrorInvalidValue;
#define AFQ_P(V, T_, W_, B_, F_)                                                          \
    if (variant == V)                                                                      \
        return launch_prop<T_, W_, B_, F_>(phi, phi_out, Pm, Af, live, nw, M, N, K, rec, s);
#define AFQ_S(V, W_, B_, F_)                                                               \
    if (variant == V)                                                                      \
        return launch_prop_split<W_, B_, F_>(phi, phi_out, Pm, Af, live, nw, M, N, K, s);
    if (t == DT_F64) {
        AFQ_P(0, double, 8, 2, true)
        AFQ_P(1, double, 4, 2, true)
        AFQ_P(2, double, 4, 1, true)
        AFQ_P(3, double, 2, 2, true)
    } else if (ta == DT_SPLIT) {
        AFQ_S(0, 8, 2, true)
        AFQ_S(1, 4, 2, true)
        AFQ_S(2, 4, 1, true)
        AFQ_S(3, 2, 2, true)
        AFQ_S(4, 8, 2, false)
        AFQ_S(5, 4, 2, false)
        AFQ_S(6, 4, 1, false)
        AFQ_S(7, 2, 2, false)
        if (variant == 8)
            return launch_prop_split_rb<16, 1, 2, false>(phi, phi_out, Pm, Af, live, nw, M, N, K,
                                                         s);
        if (variant == 9)
            return launch_prop_split_rb<8, 1, 2, false>(phi, phi_out, Pm, Af, live, nw, M, N, K, s);
        if (variant == 10)
            return launch_prop_split_rb<8, 2, 2, true>(phi, phi_out, Pm, Af, live, nw, M, N, K, s);
        if (variant == 11)
            return launch_prop_split_rb<4, 2, 2, true>(phi, phi_out, Pm, Af, live, nw, M, N, K, s);
        if (variant == 12)
            return launch_prop_split_rb<8, 2, 5, true>(phi, phi_out, Pm, Af, live, nw, M, N, K, s);
        if (variant == 13)
            return launch_prop_split_rb<16, 1, 5, true>(phi, phi_out, Pm, Af, live, nw, M, N, K,
                                                        s);
    } else {
        AFQ_P(0, float, 8, 2, true)
        AFQ_P(1, float, 4, 2, true)
        AFQ_P(2, float, 4, 1, true)
        AFQ_P(3, float, 2, 2, true)
        AFQ_P(4, float, 8, 2, false)
        AFQ_P(5, float, 4, 2, false)
        AFQ_P(6, float, 4, 1, false)
        AFQ_P(7, float, 2, 2, false)
    }
#undef AFQ_P
#undef AFQ_S
    return hipErrorInvalidValue;
}

}  // namespace afq
