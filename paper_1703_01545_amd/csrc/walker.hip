// Walker-wise FP64 kernels of the ph-AFQMC step (gfx950, wave64):
// auxiliary fields and force bias, per-spin determinants and Theta,
// hybrid/phaseless weights, modified Gram-Schmidt, local and mixed energy.
// Reductions use fixed-order wavefront butterflies and fixed-order LDS
// sums, so every run is bitwise reproducible.
#include <math.h>

#include <atomic>

#include "internal.h"
#include "mfma.h"

namespace afq {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Philox4x32-10 (Salmon et al., SC'11): multipliers 0xD2511F53 / 0xCD9E8D57,
// Weyl key increments 0x9E3779B9 / 0xBB67AE85, 10 rounds.
__device__ __forceinline__ void philox(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
}

// Four N(0,1) draws for Cholesky indices 4b..4b+3 of walker k at step t:
// counter (b, k, t, stream), key (seed lo, seed hi); Box-Muller on
// u = (r0 + 1) 2^-32, v = r1 2^-32 (and r2, r3).
__device__ __forceinline__ void normals4(uint64_t seed, uint64_t stream, int64_t t, uint32_t k,
                                         uint32_t b, double z[4]) {
    uint32_t c0 = b, c1 = k, c2 = (uint32_t)t, c3 = (uint32_t)stream;
    philox(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double sc = 2.3283064365386963e-10;  // 2^-32
    const uint32_t r[4] = {c0, c1, c2, c3};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double u = ((double)r[2 * p] + 1.0) * sc;
        const double v = (double)r[2 * p + 1] * sc;
        const double rad = sqrt(-2.0 * log(u));
        const double ang = (2.0 * M_PI) * v;
        z[2 * p] = rad * cos(ang);
        z[2 * p + 1] = rad * sin(ang);
    }
}

template <typename T>
__device__ __forceinline__ void put(void* p, long i, double v) {
    ((T*)p)[i] = (T)v;
}
__device__ __forceinline__ void put_dt(void* p, DType t, long i, double v) {
    if (t == DT_F64)
        put<double>(p, i, v);
    else if (t == DT_F32)
        put<float>(p, i, v);
    else
        ((bf16_t*)p)[i] = (bf16_t)(float)v;
}

// One wavefront per walker.  Force bias (Eq. 9): xbar = -sqrt(dt)(i f - i a);
// c = x - xbar; field-sum coefficients of A = i sqrt(dt) sum c_g L_g:
// Re A <- -sqrt(dt) Im c, Im A <- sqrt(dt) Re c; c-number
// s = -i sqrt(dt) sum c_g a_g; importance exponent sum (x xbar - xbar^2/2).
__global__ __launch_bounds__(256) void k_fields(FieldArgs f) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= f.nw) return;
    const bool live = f.alive[w] != 0;
    const double* Fr = f.F + (long)w * 2 * f.ldf;
    const double* Fi = Fr + f.ldf;
    const long xr = (long)w * 2 * f.ldx, xi = xr + f.ldx;
    double cia = 0.0, cra = 0.0, ir = 0.0, ii = 0.0;
    int capped = 0;
    const double sq = f.sqdt;
    const int64_t tstep = f.t_dev ? *f.t_dev + f.t : f.t;
    for (int b = lane; 4 * b < f.n_chol; b += 64) {
        double z[4];
        if (f.ext) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int g = 4 * b + e;
                z[e] = g < f.n_chol ? f.ext[(long)w * f.n_chol + g] : 0.0;
            }
        } else {
            normals4(f.seed, f.stream, tstep, (uint32_t)w, (uint32_t)b, z);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int g = 4 * b + e;
            if (g >= f.n_chol) break;
            const double x = z[e];
            double xbr = f.free_proj ? 0.0 : sq * Fi[g];
            double xbi = f.free_proj ? 0.0 : -sq * (Fr[g] - f.a[g]);
            if (f.fb_cap > 0.0) {
                const double mag = sqrt(xbr * xbr + xbi * xbi);
                if (mag > f.fb_cap) {
                    capped += 1;
                    if (f.cap_apply) {
                        const double sc = f.fb_cap / mag;
                        xbr = xbr * sc;
                        xbi = xbi * sc;
                    }
                }
            }
            const double cr = x - xbr, ci = -xbi;
            put_dt(f.X, f.tx, xr + g, live ? -sq * ci : 0.0);
            put_dt(f.X, f.tx, xi + g, live ? sq * cr : 0.0);
            cia += ci * f.a[g];
            cra += cr * f.a[g];
            ir += x * xbr - 0.5 * (xbr * xbr - xbi * xbi);
            ii += x * xbi - xbr * xbi;
        }
    }
    cia = wave_sum(cia);
    cra = wave_sum(cra);
    ir = wave_sum(ir);
    ii = wave_sum(ii);
    if (f.fb_cap > 0.0) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) capped += __shfl_xor(capped, o, 64);
        if (lane == 0 && live && f.cap_count) f.cap_count[w] += capped;
    }
    if (lane == 0) {
        double* o = f.s_imp + (long)w * 4;
        o[0] = sq * cia;
        o[1] = -sq * cra;
        o[2] = ir;
        o[3] = ii;
    }
}

__global__ void k_philox_normals(uint64_t seed, uint64_t stream, int64_t t, int nw, int n_chol,
                                 double* out) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = (n_chol + 3) / 4;
    if (idx >= (long)nw * nb) return;
    const int w = idx / nb, b = idx % nb;
    double z[4];
    normals4(seed, stream, t, (uint32_t)w, (uint32_t)b, z);
    for (int e = 0; e < 4; ++e) {
        const int g = 4 * b + e;
        if (g < n_chol) out[(long)w * n_chol + g] = z[e];
    }
}

// Per (walker, spin block), one workgroup, three phases:
// (1) the transposed overlap B = O^T, B[i][j] = sum_m Phi[i][m] Phi_T[j][m]
//     (i the walker orbital, j the trial orbital), on the FP64 matrix cores
//     straight into LDS (each lane reads 4 consecutive basis elements per
//     16-wide chunk: k = k0 + 4 g + s at sub-step s);
// (2) in-place Gauss-Jordan inversion of B with partial pivoting (rows are
//     swapped as the elimination goes; rho records which row of B sits at
//     each position, so B^{-1}[r][rho(i)] = R[r][i] for the result R), and
//     ln det B = sum_k ln pivot_k + i pi (number of swaps mod 2);
// (3) Theta^T = B^{-1} Phi^T, i.e. Theta rows c = sum_i R[c][i] Phi rows
//     rho(i), on the FP64 matrix cores: per 16-wide block of the basis index
//     a wave first loads the gathered Phi operand for every k, then runs the
//     orbital blocks against it.
typedef double d4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4v mma64(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// EPT: matrix elements per thread in the elimination (n * n <= 256 EPT);
// KS: k steps of 4 in phase (3) (n <= 4 KS); the LDS row pitch 4 KS + 1 is
// a compile-time constant (odd, so column walks cross the banks).
template <int EPT, int KS>
__global__ __launch_bounds__(256) void k_lu_theta(const double* __restrict__ phi,
                                                  const double* __restrict__ trialT,
                                                  double* __restrict__ theta, void* theta_lp,
                                                  DType tlp, double* __restrict__ lnd,
                                                  const uint8_t* __restrict__ live, int M, int N,
                                                  int na, int nb) {
    extern __shared__ double sh[];
    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? na : 0, n = spin ? nb : na;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, g = lane >> 4;
    double* out_lnd = lnd + ((long)w * 2 + spin) * 2;
    if (n == 0) {
        if (tid == 0) out_lnd[0] = out_lnd[1] = 0.0;
        return;
    }
    if (!live[w]) return;
    constexpr int LP = 4 * KS + 1;
    double* ar = sh;
    double* ai = sh + 4 * KS * LP;
    __shared__ int rho[64];
    __shared__ double piv_r[64], piv_i[64];
    __shared__ int s_swaps;
    const long NM = (long)N * M;
    const double* phr = phi + (long)w * 2 * NM;
    const double* phi_i = phr + NM;
    // (1) overlap
    const int nbk = (n + 15) / 16;
    for (int t = wave; t < nbk * nbk; t += 4) {
        const int ib = t / nbk, jb = t % nbk;
        const int i = ib * 16 + li, j = jb * 16 + li;
        const double* pr_row = phr + (long)(off + (i < n ? i : 0)) * M;
        const double* pi_row = phi_i + (long)(off + (i < n ? i : 0)) * M;
        const double* t_row = trialT + (long)(off + (j < n ? j : 0)) * M;
        d4v accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
        for (int k0 = 0; k0 < M; k0 += 16) {
            double xr[4], xi[4], tv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = k0 + 4 * g + q;
                const bool okm = m < M;
                xr[q] = (okm && i < n) ? pr_row[m] : 0.0;
                xi[q] = (okm && i < n) ? pi_row[m] : 0.0;
                tv[q] = (okm && j < n) ? t_row[m] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                accr = mma64(xr[q], tv[q], accr);
                acci = mma64(xi[q], tv[q], acci);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = ib * 16 + g + 4 * r, col = jb * 16 + li;
            if (row < n && col < n) {
                ar[row * LP + col] = accr[r];
                ai[row * LP + col] = acci[r];
            }
        }
    }
    if (tid < 64) rho[tid] = tid;
    if (tid == 0) s_swaps = 0;
    // element (r, c) of this thread's slots in the elimination
    int er[EPT], ec[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = tid + 256 * q;
        er[q] = e < n * n ? e / n : -1;
        ec[q] = e < n * n ? e % n : 0;
    }
    __syncthreads();
    // (2) Gauss-Jordan.  Every wave finds the pivot row itself (no broadcast
    // and no extra barrier); two barriers per column.
    for (int k = 0; k < n; ++k) {
        int p;
        {
            const int r = k + lane;
            double v = -1.0;
            if (r < n) v = fabs(ar[r * LP + k]) + fabs(ai[r * LP + k]);
            int best = r;
            // argmax, ties to the smaller row index
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double v2 = __shfl_xor(v, o, 64);
                const int b2 = __shfl_xor(best, o, 64);
                if (v2 > v || (v2 == v && b2 < best)) {
                    v = v2;
                    best = b2;
                }
            }
            p = __builtin_amdgcn_readfirstlane(best);
        }
        const double pr = ar[p * LP + k], pi = ai[p * LP + k];
        const double den = pr * pr + pi * pi;
        const double qr = pr / den, qi = -pi / den;  // 1 / pivot
        double nr[EPT], ni[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int r = er[q], c = ec[q];
            if (r < 0) continue;
            // pivot row element (column k replaced by 1), scaled by 1 / pivot
            const double br = c == k ? 1.0 : ar[p * LP + c];
            const double bi = c == k ? 0.0 : ai[p * LP + c];
            const double sr = br * qr - bi * qi, si = br * qi + bi * qr;
            if (r == k) {
                nr[q] = sr;
                ni[q] = si;
            } else {
                const int pr_ = r == p ? k : r;  // row r of the swapped matrix
                const double fr = ar[pr_ * LP + k], fi = ai[pr_ * LP + k];
                const double xr = c == k ? 0.0 : ar[pr_ * LP + c];
                const double xi = c == k ? 0.0 : ai[pr_ * LP + c];
                nr[q] = xr - (fr * sr - fi * si);
                ni[q] = xi - (fr * si + fi * sr);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            if (er[q] < 0) continue;
            ar[er[q] * LP + ec[q]] = nr[q];
            ai[er[q] * LP + ec[q]] = ni[q];
        }
        if (tid == 0) {
            piv_r[k] = pr;
            piv_i[k] = pi;
            if (p != k) {
                const int t = rho[k];
                rho[k] = rho[p];
                rho[p] = t;
                ++s_swaps;
            }
        }
        __syncthreads();
    }
    // ln det = sum_k ln(pivot_k) + i pi (swaps mod 2), summed in index order
    if (wave == 0) {
        double lr = 0.0, la = 0.0;
        bool sing = false;
        if (lane < n) {
            const double a = piv_r[lane], b = piv_i[lane];
            sing = (a == 0.0 && b == 0.0);
            lr = log(hypot(a, b));
            la = atan2(b, a);
        }
        lr = wave_sum(lr);
        la = wave_sum(la);
        const bool any_sing = __any(sing);
        if (lane == 0) {
            if (any_sing) {
                out_lnd[0] = -INFINITY;
                out_lnd[1] = 0.0;
            } else {
                out_lnd[0] = lr;
                out_lnd[1] = la + ((s_swaps & 1) ? M_PI : 0.0);
            }
        }
    }
    // (3) Theta rows c = sum_i R[c][i] Phi rows rho(i)
    double* tr_ = theta + (long)w * 2 * NM;
    double* ti_ = tr_ + NM;
    const int nmb = (M + 15) / 16;
    const int nks = (n + 3) / 4;
    for (int mb = wave; mb < nmb; mb += 4) {
        const int m = mb * 16 + li;
        double br[KS], bi[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + g;
            br[s] = bi[s] = 0.0;
            if (s < nks && k < n && m < M) {
                const long o = (long)(off + rho[k]) * M + m;
                br[s] = phr[o];
                bi[s] = phi_i[o];
            }
        }
        for (int cb = 0; cb < nbk; ++cb) {
            const int c = cb * 16 + li;
            d4v accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s >= nks) continue;
                const int k = 4 * s + g;
                const bool ok = k < n && c < n;
                const double a_r = ok ? ar[c * LP + k] : 0.0;
                const double a_i = ok ? ai[c * LP + k] : 0.0;
                accr = mma64(a_r, br[s], accr);
                accr = mma64(-a_i, bi[s], accr);
                acci = mma64(a_r, bi[s], acci);
                acci = mma64(a_i, br[s], acci);
            }
            if (m < M) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = cb * 16 + g + 4 * r;
                    if (row >= n) continue;
                    const long o = (long)(off + row) * M + m;
                    tr_[o] = accr[r];
                    ti_[o] = acci[r];
                    if (theta_lp) {
                        const long base = (long)w * 2 * NM;
                        put_dt(theta_lp, tlp, base + o, accr[r]);
                        put_dt(theta_lp, tlp, base + NM + o, acci[r]);
                    }
                }
            }
        }
    }
}

// Overlap, determinant and Theta for spin blocks of up to 48 orbitals, in two
// kernels per (walker, spin block):
// k_overlap: the transposed overlap B = O^T, B[j][i] = sum_m Phi[j][m]
//   Phi_T[i][m] (j the walker orbital, i the trial orbital), on the FP64
//   matrix cores, into a complex workspace [w][spin][j][i] (row pitch nmax);
// k_det_theta, one wavefront each:
//   (1) lane j loads row j of B into registers (NC complex entries);
//   (2) Gauss-Jordan inversion in registers with partial pivoting and no row
//       exchange.  At step k the column being eliminated is register column
//       0.  The pivot lane p_k (largest |Re| + |Im| among rows not yet used)
//       publishes its row through LDS; every lane forms row - mu prow with
//       mu = row[0] / pivot, shifted one column to the left, and appends -mu
//       as the new last column (the pivot lane itself: prow / pivot and
//       1 / pivot, i.e. mu = -1 / pivot and its row zeroed).  After n steps
//       lane p_c holds (O^{-1})[p_k][c] in register column NC - n + k, and
//       ln det O = sum_k ln pivot_k + i pi (parity of k -> p_k);
//   (3) Theta[m][c] = sum_k Phi[m][p_k] (O^{-1})[p_k][c] on the matrix cores:
//       FP64 into the FP64 Theta (TO = double), or FP32 products of the FP64
//       operands rounded to FP32 into the lower-precision copy (TO = float or
//       bf16_t) that the force-bias and exchange contractions read.
using dev::acc_row;
using dev::d2;
using dev::d4;
using dev::f4;
using dev::mma1;

template <typename TO>
struct ThetaMode {
    typedef float T;  // MFMA operand / accumulator element
    typedef f4 V;
};
template <>
struct ThetaMode<double> {
    typedef double T;
    typedef d4 V;
};

using dev::rdlane;
using dev::wave_max_u64;

// Four consecutive elements m .. m+3 of a row (zeros past M or for an
// absent row): loads from clamped, valid addresses, masked afterwards.
__device__ __forceinline__ void row4(const double* __restrict__ row, int m, int M, bool ok,
                                     double* v) {
    if ((M & 3) == 0) {
        const int mc = m < M ? m : M - 4;
        const d2 a = *(const d2*)(row + mc), b = *(const d2*)(row + mc + 2);
        const bool t = ok && m < M;
        v[0] = t ? a[0] : 0.0;
        v[1] = t ? a[1] : 0.0;
        v[2] = t ? b[0] : 0.0;
        v[3] = t ? b[1] : 0.0;
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double x = row[m + q < M ? m + q : M - 1];
            v[q] = (ok && m + q < M) ? x : 0.0;
        }
    }
}

template <typename TO>
__device__ __forceinline__ void store_theta(TO* p, double v);
template <>
__device__ __forceinline__ void store_theta<double>(double* p, double v) {
    *p = v;
}
template <>
__device__ __forceinline__ void store_theta<float>(float* p, double v) {
    *p = (float)v;
}
template <>
__device__ __forceinline__ void store_theta<bf16_t>(bf16_t* p, double v) {
    *p = (bf16_t)(float)v;
}

// One wavefront per (walker, spin block); NB 16-wide blocks of orbitals.
// Each lane reads 4 consecutive basis elements per 16-wide chunk of a row
// (k = k0 + 4 g + q at sub-step q), so the 16 x 16 tiles take whole row runs.
template <int NB>
__global__ __launch_bounds__(64) void k_overlap(const double* __restrict__ phi,
                                                const double* __restrict__ trialT,
                                                d2* __restrict__ ovl,
                                                const uint8_t* __restrict__ live, int M, int N,
                                                int na, int nb, int nmax) {
    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? na : 0, n = spin ? nb : na;
    if (n == 0 || !live[w]) return;
    const int lane = threadIdx.x, li = lane & 15, g = lane >> 4;
    const long NM = (long)N * M;
    const double* phr = phi + (long)w * 2 * NM;
    const int nbn = (n + 15) >> 4;
    d2* out = ovl + ((long)w * 2 + spin) * nmax * nmax;
    for (int ib = 0; ib < nbn; ++ib) {
        const int j = ib * 16 + li;
        const bool okj = j < n;
        const double* xr_row = phr + (long)(off + (okj ? j : 0)) * M;
        const double* xi_row = xr_row + NM;
        d4 accr[NB], acci[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) accr[b] = acci[b] = (d4){0, 0, 0, 0};
        for (int k0 = 0; k0 < M; k0 += 16) {
            const int m = k0 + 4 * g;
            double xr[4], xi[4];
            row4(xr_row, m, M, okj, xr);
            row4(xi_row, m, M, okj, xi);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b >= nbn) break;
                const int i = b * 16 + li;
                double tv[4];
                row4(trialT + (long)(off + (i < n ? i : 0)) * M, m, M, i < n, tv);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    accr[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[q], tv[q], accr[b], 0, 0, 0);
                    acci[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[q], tv[q], acci[b], 0, 0, 0);
                }
            }
        }
        // element (row j = ib 16 + g + 4 r, column i = b 16 + li)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = b * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jr = ib * 16 + g + 4 * r;
                if (b < nbn && jr < n && i < n) out[(long)jr * nmax + i] = (d2){accr[b][r], acci[b][r]};
            }
        }
    }
}

// Output rows c = sum_k S[c][k] Phi rows rowk[k] (c, k < n; S complex in LDS
// with pitch NC + 1) on the matrix cores: FP64 for TO = double, FP32 products
// of the rounded operands otherwise.  Every load is issued unconditionally
// from a valid address and masked afterwards, so the loops unroll and the
// loads of one column block go out together; the Phi operand of the next
// column block is loaded while the current one is on the matrix cores, and
// a column block is read in full before its output is stored (the output may
// be Phi itself).  One wavefront.
template <int NC, typename TO>
__device__ __forceinline__ void rows_times_phi(
    const typename ThetaMode<TO>::T __attribute__((ext_vector_type(2)))* S, const int* rowk,
    int n, const double* phr, const double* phm, int M, int off, TO* tr_, TO* ti_) {
    typedef typename ThetaMode<TO>::T ET;
    typedef typename ThetaMode<TO>::V EV;
    typedef ET __attribute__((ext_vector_type(2))) E2;
    constexpr int NB = (NC + 15) / 16;
    constexpr int KS = NC / 4;
    constexpr int SP = NC + 1;
    const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
    const int nbn = (n + 15) >> 4;
    long roff[KS];
    bool kok[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int k = 4 * s + g;
        kok[s] = k < n;
        roff[s] = (long)(off + rowk[kok[s] ? k : 0]) * M;
    }
    // the inverse operand: element (c, k) of S, zero outside n x n (held in
    // registers for FP32; re-read from LDS for FP64, which has no room)
    auto a_op = [&](int cb, int s) -> E2 {
        const int c = cb * 16 + li, k = 4 * s + g;
        const E2 v = S[(c < n ? c : 0) * SP + (kok[s] ? k : 0)];
        const bool ok = c < n && kok[s];
        return (E2){ok ? v[0] : (ET)0, ok ? v[1] : (ET)0};
    };
    constexpr bool HOLD = sizeof(ET) == 4;
    E2 a_h[HOLD ? NB : 1][HOLD ? KS : 1];
    if constexpr (HOLD) {
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int s = 0; s < KS; ++s) a_h[cb][s] = a_op(cb, s);
    }
    const int nmb = (M + 15) >> 4;
    // the Phi operand of the next column block is loaded while the current
    // one is on the matrix cores
    double xr[KS], xi[KS];
    auto load_b = [&](int mb_) {
        const int mm = mb_ * 16 + li;
        const int mc = mm < M ? mm : M - 1;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            xr[s] = phr[roff[s] + mc];
            xi[s] = phm[roff[s] + mc];
        }
    };
    load_b(0);
    for (int mb = 0; mb < nmb; ++mb) {
        const int m = mb * 16 + li;
        const bool mok = m < M;
        ET br[KS], bi[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            br[s] = (kok[s] && mok) ? (ET)xr[s] : (ET)0;
            bi[s] = (kok[s] && mok) ? (ET)xi[s] : (ET)0;
        }
        load_b(mb + 1 < nmb ? mb + 1 : mb);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            if (cb < nbn) {
                EV cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    E2 a;
                    if constexpr (HOLD)
                        a = a_h[cb][s];
                    else
                        a = a_op(cb, s);
                    cr = mma1(a[0], br[s], cr);
                    cr = mma1(-a[1], bi[s], cr);
                    ci = mma1(a[0], bi[s], ci);
                    ci = mma1(a[1], br[s], ci);
                }
                if (mok) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = cb * 16 + acc_row<ET>(lane, r);
                        if (row < n) {
                            const long o = (long)(off + row) * M + m;
                            store_theta<TO>(tr_ + o, cr[r]);
                            store_theta<TO>(ti_ + o, ci[r]);
                        }
                    }
                }
            }
        }
    }
}

template <int NC, typename TO>
__global__ __launch_bounds__(64, NC <= 40 ? 2 : 1) void k_det_theta(
    const double* __restrict__ phi, const d2* __restrict__ ovl, TO* __restrict__ theta,
    double* __restrict__ lnd, const uint8_t* __restrict__ live, int M, int N, int na, int nb,
    int nmax) {
    typedef typename ThetaMode<TO>::T ET;
    constexpr int SP = NC + 1;  // pitch (complex) of the inverse
    __shared__ __align__(16) unsigned char buf[NC * SP * 2 * sizeof(ET)];
    __shared__ double pv[2 * NC];
    __shared__ int ptab[NC];

    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? na : 0, n = spin ? nb : na;
    const int lane = threadIdx.x;
    double* out_lnd = lnd + ((long)w * 2 + spin) * 2;
    if (n == 0) {
        if (lane == 0) out_lnd[0] = out_lnd[1] = 0.0;
        return;
    }
    if (!live[w]) return;
    const long NM = (long)N * M;
    const double* phr = phi + (long)w * 2 * NM;
    const double* phm = phr + NM;

    // (1) row j of B into lane j (unconditional loads from valid addresses,
    // masked afterwards)
    double ar[NC], ai[NC];
    {
        const d2* row = ovl + ((long)w * 2 + spin) * nmax * nmax + (long)(lane < n ? lane : 0) * nmax;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const d2 v = row[c < n ? c : 0];
            const bool ok = lane < n && c < n;
            ar[c] = ok ? v[0] : 0.0;
            ai[c] = ok ? v[1] : 0.0;
        }
    }

    // (2) Gauss-Jordan; the pivot row goes from the pivot lane to the others
    // by lane reads into scalar registers (no LDS traffic in the loop)
    bool used = lane >= n;
    int mystep = 0;
    for (int k = 0; k < n; ++k) {
        // pivot: the largest |Re| + |Im| among unused rows; key = its bit
        // pattern (non-negative doubles order as integers) with the low six
        // bits replaced by 63 - lane, so ties and near-ties (2^-46 relative)
        // go to the smaller lane; NaN rows are never chosen
        const double v = fabs(ar[0]) + fabs(ai[0]);
        const bool sel = !used && v >= 0.0;
        const unsigned long long key =
            sel ? ((__builtin_bit_cast(unsigned long long, v) & ~63ull) | (unsigned)(63 - lane))
                : 0ull;
        const unsigned long long kmax = wave_max_u64(key);
        const int p = kmax ? 63 - (int)(kmax & 63) : __ffsll((long long)__ballot(!used)) - 1;
        const double pr = rdlane(ar[0], p), pi = rdlane(ai[0], p);
        const double rden = 1.0 / (pr * pr + pi * pi);
        const double qr = pr * rden, qi = -pi * rden;  // 1 / pivot
        const bool me = lane == p;
        if (me) {
            used = true;
            mystep = k;
            pv[2 * k] = pr;
            pv[2 * k + 1] = pi;
            ptab[k] = p;
        }
        const double mr = me ? -qr : ar[0] * qr - ai[0] * qi;
        const double mi = me ? -qi : ar[0] * qi + ai[0] * qr;
        const double al = me ? 0.0 : 1.0;
#pragma unroll
        for (int c = 1; c < NC; ++c) {
            const double sr = rdlane(ar[c], p), si = rdlane(ai[c], p);
            ar[c - 1] = al * ar[c] - (mr * sr - mi * si);
            ai[c - 1] = al * ai[c] - (mr * si + mi * sr);
            // bounded look-ahead of the lane reads (scalar register pressure)
            if ((c & 7) == 0) __builtin_amdgcn_sched_barrier(0);
        }
        ar[NC - 1] = -mr;
        ai[NC - 1] = -mi;
    }
    __syncthreads();
    // ln det = sum_k ln pivot_k + i pi (inversions of k -> p_k mod 2)
    {
        double lr = 0.0, la = 0.0;
        int inv = 0;
        bool sing = false;
        if (lane < n) {
            const double a = pv[2 * lane], b = pv[2 * lane + 1];
            sing = (a == 0.0 && b == 0.0);
            lr = log(hypot(a, b));
            la = atan2(b, a);
            const int pk = ptab[lane];
            for (int k2 = lane + 1; k2 < n; ++k2) inv += ptab[k2] < pk;
        }
        lr = wave_sum(lr);
        la = wave_sum(la);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) inv += __shfl_xor(inv, o, 64);
        const bool any_sing = __any(sing);
        if (lane == 0) {
            if (any_sing) {
                out_lnd[0] = -INFINITY;
                out_lnd[1] = 0.0;
            } else {
                out_lnd[0] = lr;
                out_lnd[1] = la + ((inv & 1) ? M_PI : 0.0);
            }
        }
    }
    // the inverse into LDS: row c = the step of this lane, column k
    typedef ET __attribute__((ext_vector_type(2))) E2;
    E2* S = (E2*)buf;
    if (lane < n) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c >= NC - n) S[mystep * SP + c - (NC - n)] = (E2){(ET)ar[c], (ET)ai[c]};
    }
    __syncthreads();

    // (3) Theta rows c = sum_k S[c][k] Phi rows p_k
    rows_times_phi<NC, TO>(S, ptab, n, phr, phm, M, off, theta + (long)w * 2 * NM,
                           theta + (long)w * 2 * NM + NM);
}

// Orthonormalization of a spin block (Sec. II.D): the modified Gram-Schmidt
// result Phi = Q R (R upper triangular with positive diagonal, Q^H Q = 1)
// is the unique QR factorization, obtained here from the Gram matrix
// S = Phi^H Phi = R^H R, in two kernels per (walker, spin block):
// k_gram: S on the FP64 matrix cores into the complex workspace [w][spin][i][j]
//   (row pitch nmax; real part sum (Re_i Re_j + Im_i Im_j), imaginary part
//   sum (Re_i Im_j - Im_i Re_j));
// k_cholqr, one wavefront: lane i loads row i of S; forward elimination in
//   order (pivot k at step k, no exchange) with the register rotation of
//   k_det_theta turns the identity into L^{-1} of S = L D L^H, so
//   R^{-1} = L^{-H} D^{-1/2}; Q row i = D_i^{-1/2} sum_{k <= i}
//   conj(L^{-1}[i][k]) Phi row k, on the FP64 matrix cores, in place.
template <int NB>
__global__ __launch_bounds__(64) void k_gram(const double* __restrict__ phi, d2* __restrict__ ovl,
                                             const uint8_t* __restrict__ live, int M, int N,
                                             int na, int nb, int nmax) {
    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? na : 0, n = spin ? nb : na;
    if (n == 0 || !live[w]) return;
    const int lane = threadIdx.x, li = lane & 15, g = lane >> 4;
    const long NM = (long)N * M;
    const double* phr = phi + (long)w * 2 * NM;
    const int nbn = (n + 15) >> 4;
    d2* out = ovl + ((long)w * 2 + spin) * nmax * nmax;
    for (int ib = 0; ib < nbn; ++ib) {
        const int i = ib * 16 + li;
        const bool oki = i < n;
        const double* xr_row = phr + (long)(off + (oki ? i : 0)) * M;
        const double* xi_row = xr_row + NM;
        d4 accr[NB], acci[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) accr[b] = acci[b] = (d4){0, 0, 0, 0};
        for (int k0 = 0; k0 < M; k0 += 16) {
            const int m = k0 + 4 * g;
            double xr[4], xi[4];
            row4(xr_row, m, M, oki, xr);
            row4(xi_row, m, M, oki, xi);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b >= nbn) break;
                const int j = b * 16 + li;
                const double* yr_row = phr + (long)(off + (j < n ? j : 0)) * M;
                double yr[4], yi[4];
                row4(yr_row, m, M, j < n, yr);
                row4(yr_row + NM, m, M, j < n, yi);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    accr[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[q], yr[q], accr[b], 0, 0, 0);
                    accr[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[q], yi[q], accr[b], 0, 0, 0);
                    acci[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[q], yi[q], acci[b], 0, 0, 0);
                    acci[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xi[q], yr[q], acci[b], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = b * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ir = ib * 16 + g + 4 * r;
                if (b < nbn && ir < n && j < n) out[(long)ir * nmax + j] = (d2){accr[b][r], acci[b][r]};
            }
        }
    }
}

// Loss-of-orthogonality record of one spin block at a Gram-Schmidt step
// (Sec. II.D): the lanes below n hold ell_k = 1/2 ln(S_kk / D_k), with S =
// Phi^H Phi = L D L^H (zero for orthogonal columns; the Gram-matrix QR loses
// about 2 ell / ln 10 decimal digits), and ln R_kk = 1/2 ln D_k.  mon[0]
// keeps the largest ell and mon[1] the largest |ln |det R|| since the record
// was cleared; anything non-finite counts as infinite.  One wavefront.
__device__ __forceinline__ void gs_record(double* mon, double ell, double lnr) {
    if (!(ell == ell)) ell = INFINITY;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        ell = fmax(ell, __shfl_xor(ell, o, 64));
        lnr += __shfl_xor(lnr, o, 64);
    }
    const double ld = (lnr == lnr) ? fabs(lnr) : INFINITY;
    if ((threadIdx.x & 63) == 0) {
        mon[0] = fmax(mon[0], ell);
        mon[1] = fmax(mon[1], ld);
    }
}

template <int NC>
__global__ __launch_bounds__(64, NC <= 40 ? 2 : 1) void k_cholqr(double* phi,
                                                                 const d2* __restrict__ ovl,
                                                                 const uint8_t* __restrict__ live,
                                                                 int M, int N, int na, int nb,
                                                                 int nmax,
                                                                 double* __restrict__ mon) {
    constexpr int SP = NC + 1;
    typedef double __attribute__((ext_vector_type(2))) E2;
    __shared__ __align__(16) E2 S[NC * SP];
    __shared__ double dv[NC];
    __shared__ int ident[NC];
    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? na : 0, n = spin ? nb : na;
    if (n == 0 || !live[w]) return;
    const int lane = threadIdx.x;
    const long NM = (long)N * M;
    double* phr = phi + (long)w * 2 * NM;
    double* phm = phr + NM;
    double ar[NC], ai[NC];
    {
        const d2* row = ovl + ((long)w * 2 + spin) * nmax * nmax + (long)(lane < n ? lane : 0) * nmax;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const d2 v = row[c < n ? c : 0];
            const bool ok = lane < n && c < n;
            ar[c] = ok ? v[0] : 0.0;
            ai[c] = ok ? v[1] : 0.0;
        }
    }
    if (lane < NC) ident[lane] = lane;
    for (int k = 0; k < n; ++k) {
        const double pr = rdlane(ar[0], k), pi = rdlane(ai[0], k);
        const double rden = 1.0 / (pr * pr + pi * pi);
        const double qr = pr * rden, qi = -pi * rden;  // 1 / pivot
        const bool below = lane > k;
        const double mr = below ? ar[0] * qr - ai[0] * qi : 0.0;
        const double mi = below ? ar[0] * qi + ai[0] * qr : 0.0;
        if (lane == k) dv[k] = pr;
#pragma unroll
        for (int c = 1; c < NC; ++c) {
            const double sr = rdlane(ar[c], k), si = rdlane(ai[c], k);
            ar[c - 1] = ar[c] - (mr * sr - mi * si);
            ai[c - 1] = ai[c] - (mr * si + mi * sr);
            if ((c & 7) == 0) __builtin_amdgcn_sched_barrier(0);
        }
        ar[NC - 1] = lane == k ? 1.0 : -mr;
        ai[NC - 1] = -mi;
    }
    __syncthreads();
    if (mon) {
        double ell = 0.0, lnr = 0.0;
        if (lane < n) {
            const d2 skk = ovl[((long)w * 2 + spin) * nmax * nmax + (long)lane * nmax + lane];
            ell = 0.5 * log(skk[0] / dv[lane]);
            lnr = 0.5 * log(dv[lane]);
        }
        gs_record(mon + ((long)w * 2 + spin) * 2, ell, lnr);
    }
    // S[i][k] = D_i^{-1/2} conj(L^{-1}[i][k]): R^{-1} transposed, by rows i
    if (lane < n) {
        const double sc = 1.0 / sqrt(dv[lane]);
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c >= NC - n) S[lane * SP + c - (NC - n)] = (E2){sc * ar[c], -sc * ai[c]};
    }
    __syncthreads();
    rows_times_phi<NC, double>(S, ident, n, phr, phm, M, off, phr, phm);
}

__global__ void k_weights(const double* __restrict__ lnd, const double* __restrict__ s_imp,
                          double* __restrict__ lnov, double* __restrict__ w,
                          uint8_t* __restrict__ alive, int nw, int mode, int commit,
                          double shift) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nw || !alive[k]) return;
    const double nr = lnd[4 * k + 0] + lnd[4 * k + 2];
    const double ni = lnd[4 * k + 1] + lnd[4 * k + 3];
    if (commit) {
        const double Rr = (nr - lnov[2 * k]) + s_imp[4 * k + 0];
        const double Ri = (ni - lnov[2 * k + 1]) + s_imp[4 * k + 1];
        if (mode == 0) {
            const double Ir = Rr + s_imp[4 * k + 2];
            const double fac = exp(Ir + shift) * fmax(0.0, cos(Ri));
            const double wn = w[k] * fac;
            const bool ok = isfinite(wn) && wn > 0.0;
            w[k] = ok ? wn : 0.0;
            if (!ok) alive[k] = 0;
        } else {
            const double er = exp(Rr + shift);
            const double fr = er * cos(Ri), fi = er * sin(Ri);
            const double wr = w[2 * k], wi = w[2 * k + 1];
            w[2 * k] = wr * fr - wi * fi;
            w[2 * k + 1] = wr * fi + wi * fr;
        }
    }
    lnov[2 * k] = nr;
    lnov[2 * k + 1] = ni;
}

// Modified Gram-Schmidt of one spin block per workgroup: for each column j
// in order, normalise it, then remove its projection q_j^H v_l from every
// later column l.  The block is staged in LDS when it fits (STAGE), else it
// is updated in place in global memory.
template <bool STAGE>
__global__ __launch_bounds__(256) void k_mgs(double* __restrict__ phi,
                                             const uint8_t* __restrict__ live, int M, int N,
                                             int na, int nb, double* __restrict__ mon) {
    extern __shared__ double stage_buf[];
    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? na : 0, n = spin ? nb : na;
    if (n == 0 || !live[w]) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long NM = (long)N * M;
    double* gr = phi + (long)w * 2 * NM + (long)off * M;
    double* gi = gr + NM;
    double* pr = gr;
    double* pi = gi;
    long ldp = M;
    if (STAGE) {
        pr = stage_buf;
        pi = stage_buf + (long)n * M;
        for (int e = tid; e < n * M; e += 256) {
            pr[e] = gr[e];
            pi[e] = gi[e];
        }
        __syncthreads();
    }
    __shared__ double red[4];
    __shared__ double proj[2 * 64];
    __shared__ double s0[256];  // column norms before the sweep (monitor)
    if (mon) {
        for (int j = wave; j < n; j += 4) {
            const double* qr = pr + (long)j * ldp;
            const double* qi = pi + (long)j * ldp;
            double a = 0.0;
            for (int m = lane; m < M; m += 64) a += qr[m] * qr[m] + qi[m] * qi[m];
            a = wave_sum(a);
            if (lane == 0) s0[j] = a;
        }
        __syncthreads();
    }
    double ell = 0.0, lnr = 0.0;  // monitor record, the same in every thread
    for (int j = 0; j < n; ++j) {
        double* qr = pr + (long)j * ldp;
        double* qi = pi + (long)j * ldp;
        double s = 0.0;
        for (int m = tid; m < M; m += 256) s += qr[m] * qr[m] + qi[m] * qi[m];
        s = wave_sum(s);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        const double dj = ((red[0] + red[1]) + red[2]) + red[3];
        const double nrm = sqrt(dj);
        if (mon) {
            ell = fmax(ell, 0.5 * log(s0[j] / dj));
            lnr += 0.5 * log(dj);
        }
        for (int m = tid; m < M; m += 256) {
            qr[m] = qr[m] / nrm;
            qi[m] = qi[m] / nrm;
        }
        __syncthreads();
        for (int l = j + 1 + wave; l < n; l += 4) {
            const double* vr = pr + (long)l * ldp;
            const double* vi = pi + (long)l * ldp;
            double a = 0.0, b = 0.0;
            for (int m = lane; m < M; m += 64) {
                a += qr[m] * vr[m] + qi[m] * vi[m];
                b += qr[m] * vi[m] - qi[m] * vr[m];
            }
            a = wave_sum(a);
            b = wave_sum(b);
            if (lane == 0) {
                proj[2 * (l - j - 1)] = a;
                proj[2 * (l - j - 1) + 1] = b;
            }
        }
        __syncthreads();
        const int rest = n - j - 1;
        for (int l = j + 1 + (tid >> 6); l < n; l += 4) {
            const double cr = proj[2 * (l - j - 1)], ci = proj[2 * (l - j - 1) + 1];
            for (int m = lane; m < M; m += 64) {
                const double xr = qr[m], xi = qi[m];
                pr[(long)l * ldp + m] -= cr * xr - ci * xi;
                pi[(long)l * ldp + m] -= cr * xi + ci * xr;
            }
        }
        (void)rest;
        __syncthreads();
    }
    if (STAGE) {
        for (int e = tid; e < n * M; e += 256) {
            gr[e] = pr[e];
            gi[e] = pi[e];
        }
    }
    if (mon && tid < 64) gs_record(mon + ((long)w * 2 + spin) * 2, lane == 0 ? ell : 0.0,
                                   lane == 0 ? lnr : 0.0);
}

__global__ void k_local_energy(const double* __restrict__ F, int ldf,
                               const double* __restrict__ exch, int n_gt, int n_gt_a, int n_gt_b,
                               int nw, int n_chol, double e_core, double* __restrict__ el) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= nw) return;
    const double* Fr = F + (long)w * 2 * ldf;
    const double* Fi = Fr + ldf;
    double cr = 0.0, ci = 0.0;
    for (int g = lane; g < n_chol; g += 64) {
        cr += Fr[g] * Fr[g] - Fi[g] * Fi[g];
        ci += 2.0 * Fr[g] * Fi[g];
    }
    cr = wave_sum(cr);
    ci = wave_sum(ci);
    if (lane == 0) {
        double xr = 0.0, xi = 0.0;
        for (int s = 0; s < 2; ++s) {
            const int nt = s ? n_gt_b : n_gt_a;
            const double* e = exch + ((long)w * 2 + s) * n_gt * 2;
            for (int t = 0; t < nt; ++t) {
                xr += e[2 * t];
                xi += e[2 * t + 1];
            }
        }
        el[2 * w] = e_core + Fr[n_chol] + 0.5 * (cr - xr);
        el[2 * w + 1] = Fi[n_chol] + 0.5 * (ci - xi);
    }
}

__global__ __launch_bounds__(256) void k_mixed(const double* __restrict__ el,
                                               const double* __restrict__ w,
                                               const uint8_t* __restrict__ alive, int nw, int mode,
                                               double* __restrict__ out) {
    __shared__ double red[4][256];
    const int tid = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int k = tid; k < nw; k += 256) {
        if (mode == 0) {
            if (alive[k]) {
                a0 += w[k] * el[2 * k];
                a1 += w[k];
            }
        } else {
            const double wr = w[2 * k], wi = w[2 * k + 1];
            a0 += wr * el[2 * k] - wi * el[2 * k + 1];
            a1 += wr * el[2 * k + 1] + wi * el[2 * k];
            a2 += wr;
            a3 += wi;
        }
    }
    red[0][tid] = a0;
    red[1][tid] = a1;
    red[2][tid] = a2;
    red[3][tid] = a3;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (tid < s)
            for (int q = 0; q < 4; ++q) red[q][tid] += red[q][tid + s];
        __syncthreads();
    }
    if (tid < 4) out[tid] = red[tid][0];
}

__global__ void k_set4(int64_t* ctr, int64_t c0, int64_t c1, int64_t c2, int64_t c3) {
    if (threadIdx.x == 0) {
        ctr[0] = c0;
        ctr[1] = c1;
        ctr[2] = c2;
        ctr[3] = c3;
    }
}

__global__ void k_advance(int64_t* ctr, int64_t d0, int64_t d1) {
    if (threadIdx.x == 0) {
        ctr[0] += d0;
        ctr[1] += d1;
    }
}

__global__ void k_trace(const double* sa, const double* sb, double* trace, long slot,
                        const int64_t* ctr, int pair, int mode) {
    if (threadIdx.x != 0) return;
    if (ctr) {
        trace = reinterpret_cast<double*>(static_cast<uintptr_t>(ctr[2]));
        slot += (long)pair * ctr[3] + ctr[1];
    }
    double ea, eb;
    if (mode == 0) {
        ea = sa[0] / sa[1];
        eb = sb[0] / sb[1];
    } else {
        // Re(num / den), num = sa[0] + i sa[1], den = sa[2] + i sa[3]
        ea = (sa[0] * sa[2] + sa[1] * sa[3]) / (sa[2] * sa[2] + sa[3] * sa[3]);
        eb = (sb[0] * sb[2] + sb[1] * sb[3]) / (sb[2] * sb[2] + sb[3] * sb[3]);
    }
    trace[3 * slot] = ea;
    trace[3 * slot + 1] = eb;
    trace[3 * slot + 2] = eb - ea;
}

template <typename T>
__global__ void k_convert(const double* __restrict__ s, T* __restrict__ d, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (T)s[i];
}
__global__ void k_convert_bf(const double* __restrict__ s, bf16_t* __restrict__ d, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (bf16_t)(float)s[i];
}

// Lp[q][g] = L[g][r][c], q = r (2M - r + 1) / 2 + (c - r), r <= c.
__global__ void k_pack(const double* __restrict__ L, void* Lp, DType t, int M, int n_chol) {
    const long P = (long)M * (M + 1) / 2;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * n_chol) return;
    const long q = idx / n_chol;
    const int g = idx % n_chol;
    // invert q -> (r, c)
    int r = (int)((2.0 * M + 1.0 - sqrt((2.0 * M + 1.0) * (2.0 * M + 1.0) - 8.0 * q)) / 2.0);
    if (r < 0) r = 0;
    while (r > 0 && (long)r * (2 * M - r + 1) / 2 > q) --r;
    while ((long)(r + 1) * (2 * M - r) / 2 <= q) ++r;
    const int c = r + (int)(q - (long)r * (2 * M - r + 1) / 2);
    put_dt(Lp, t, idx, L[(long)g * M * M + (long)r * M + c]);
}

__global__ void k_permute(const double* __restrict__ L, double* __restrict__ LT, int M, int n_chol) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)n_chol * M * M;
    if (idx >= tot) return;
    const int k = idx % M;
    const int g = (idx / M) % n_chol;
    const int i = idx / ((long)M * n_chol);
    LT[idx] = L[(long)g * M * M + (long)i * M + k];
}

__global__ void k_wsum(const double* __restrict__ L, const double* __restrict__ a,
                       double* __restrict__ out, int M, int n_chol) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)M * M) return;
    double s = 0.0;
    for (int g = 0; g < n_chol; ++g) s += a[g] * L[(long)g * M * M + idx];
    out[idx] = s;
}

// dst[k * n + e] = src[e] for k < copies (initial walker replicated).
__global__ void k_bcast(const double* __restrict__ src, double* __restrict__ dst, long n,
                        int copies) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * copies) return;
    dst[i] = src[i % n];
}

inline unsigned nblk(long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t fields(const FieldArgs& f, hipStream_t s) {
    if (f.nw <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fields, dim3(nblk(f.nw, 4)), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t philox_normals(uint64_t seed, uint64_t stream, int64_t t, int nw, int n_chol,
                          double* out, hipStream_t s) {
    const long n = (long)nw * ((n_chol + 3) / 4);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_normals, dim3(nblk(n, 256)), dim3(256), 0, s, seed, stream, t, nw,
                       n_chol, out);
    return hipGetLastError();
}

template <int NC>
hipError_t det_theta_nc(const double* phi, const double* trialT, double* theta, void* theta_lp,
                        DType tlp, double* lnd, const uint8_t* live, int nw, int M, int N, int na,
                        int nb, void* ws, hipStream_t s) {
    const dim3 grid(nw, 2), blk(64);
    const int nmax = na > nb ? na : nb;
    d2* ovl = (d2*)ws;
    hipLaunchKernelGGL((k_overlap<(NC + 15) / 16>), grid, blk, 0, s, phi, trialT, ovl, live, M, N,
                       na, nb, nmax);
    if (!theta_lp)
        hipLaunchKernelGGL((k_det_theta<NC, double>), grid, blk, 0, s, phi, ovl, theta, lnd, live,
                           M, N, na, nb, nmax);
    else if (tlp == DT_F32)
        hipLaunchKernelGGL((k_det_theta<NC, float>), grid, blk, 0, s, phi, ovl, (float*)theta_lp,
                           lnd, live, M, N, na, nb, nmax);
    else
        hipLaunchKernelGGL((k_det_theta<NC, bf16_t>), grid, blk, 0, s, phi, ovl,
                           (bf16_t*)theta_lp, lnd, live, M, N, na, nb, nmax);
    return hipGetLastError();
}

size_t lu_theta_ws_bytes(int nw, int na, int nb) {
    const int nmax = na > nb ? na : nb;
    return nmax <= 48 ? (size_t)nw * 2 * nmax * nmax * 16 : 0;
}

hipError_t lu_theta(const double* phi, const double* trialT, double* theta, void* theta_lp,
                    DType tlp, double* lnd, const uint8_t* live, int nw, int M, int N, int na,
                    int nb, void* ws, hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    const int nmax = na > nb ? na : nb;
    if (nmax > 64 || (theta_lp && tlp == DT_F64)) return hipErrorInvalidValue;
    // one wavefront per block, the rows in registers, up to 48 orbitals
#define AFQ_DET(NC) \
    if (nmax <= NC) \
        return det_theta_nc<NC>(phi, trialT, theta, theta_lp, tlp, lnd, live, nw, M, N, na, nb, \
                                ws, s);
    AFQ_DET(8)
    AFQ_DET(16)
    AFQ_DET(24)
    AFQ_DET(32)
    AFQ_DET(40)
    AFQ_DET(48)
#undef AFQ_DET
    // larger blocks: one workgroup of four wavefronts per block, the matrix in
    // LDS (writes the FP64 Theta and, if requested, the copy)
    const size_t shm = (size_t)2 * 64 * 65 * sizeof(double);
    static std::atomic<bool> attr{false};  // set once, outside graph capture
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_lu_theta<16, 16>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_lu_theta<16, 16>), dim3(nw, 2), dim3(256), shm, s, phi, trialT, theta,
                       theta_lp, tlp, lnd, live, M, N, na, nb);
    return hipGetLastError();
}

hipError_t weights(const double* lnd, const double* s_imp, double* lnov, double* w, uint8_t* alive,
                   int nw, int mode, int commit, double shift, hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_weights, dim3(nblk(nw, 256)), dim3(256), 0, s, lnd, s_imp, lnov, w, alive,
                       nw, mode, commit, shift);
    return hipGetLastError();
}

template <int NC>
hipError_t cholqr_nc(double* phi, const uint8_t* live, int nw, int M, int N, int na, int nb,
                     void* ws, double* mon, hipStream_t s) {
    const dim3 grid(nw, 2), blk(64);
    const int nmax = na > nb ? na : nb;
    hipLaunchKernelGGL((k_gram<(NC + 15) / 16>), grid, blk, 0, s, phi, (d2*)ws, live, M, N, na,
                       nb, nmax);
    hipLaunchKernelGGL((k_cholqr<NC>), grid, blk, 0, s, phi, (const d2*)ws, live, M, N, na, nb,
                       nmax, mon);
    return hipGetLastError();
}

hipError_t mgs(double* phi, const uint8_t* live, int nw, int M, int N, int na, int nb, void* ws,
               double* mon, hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    const int nmax = na > nb ? na : nb;
#define AFQ_QR(NC) \
    if (nmax <= NC) return cholqr_nc<NC>(phi, live, nw, M, N, na, nb, ws, mon, s);
    AFQ_QR(8)
    AFQ_QR(16)
    AFQ_QR(24)
    AFQ_QR(32)
    AFQ_QR(40)
    AFQ_QR(48)
#undef AFQ_QR
    // larger blocks: Gram-Schmidt column by column in one workgroup
    const size_t shm = (size_t)2 * nmax * M * sizeof(double);
    if (shm <= 128 * 1024) {
        static bool attr = false;
        if (!attr) {
            hipError_t e = hipFuncSetAttribute((const void*)k_mgs<true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               128 * 1024);
            if (e != hipSuccess) return e;
            attr = true;
        }
        hipLaunchKernelGGL(k_mgs<true>, dim3(nw, 2), dim3(256), shm, s, phi, live, M, N, na, nb,
                           mon);
    } else {
        hipLaunchKernelGGL(k_mgs<false>, dim3(nw, 2), dim3(256), 0, s, phi, live, M, N, na, nb,
                           mon);
    }
    return hipGetLastError();
}

hipError_t local_energy(const double* F, int ldf, const double* exch, int n_gt_a, int n_gt_b,
                        int nw, int n_chol, double e_core, double* el, hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    const int n_gt = n_gt_a > n_gt_b ? n_gt_a : n_gt_b;
    hipLaunchKernelGGL(k_local_energy, dim3(nblk(nw, 4)), dim3(256), 0, s, F, ldf, exch, n_gt,
                       n_gt_a, n_gt_b, nw, n_chol, e_core, el);
    return hipGetLastError();
}

hipError_t mixed_sums(const double* el, const double* w, const uint8_t* alive, int nw, int mode,
                      double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_mixed, dim3(1), dim3(256), 0, s, el, w, alive, nw, mode, out);
    return hipGetLastError();
}

hipError_t trace_record(const double* sa, const double* sb, double* trace, int slot,
                        const int64_t* ctr, int pair, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_trace, dim3(1), dim3(64), 0, s, sa, sb, trace, (long)slot, ctr, pair,
                       mode);
    return hipGetLastError();
}

hipError_t set_counters(int64_t* ctr, int64_t c0, int64_t c1, int64_t c2, int64_t c3,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_set4, dim3(1), dim3(64), 0, s, ctr, c0, c1, c2, c3);
    return hipGetLastError();
}

hipError_t advance_counters(int64_t* ctr, int64_t d0, int64_t d1, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctr, d0, d1);
    return hipGetLastError();
}

hipError_t broadcast(const double* src, double* dst, long n, int copies, hipStream_t s) {
    if (n <= 0 || copies <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bcast, dim3(nblk(n * copies, 256)), dim3(256), 0, s, src, dst, n, copies);
    return hipGetLastError();
}

hipError_t convert(const double* src, void* dst, DType t, long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (t == DT_F64)
        return hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (t == DT_F32)
        hipLaunchKernelGGL(k_convert<float>, dim3(nblk(n, 256)), dim3(256), 0, s, src, (float*)dst,
                           n);
    else
        hipLaunchKernelGGL(k_convert_bf, dim3(nblk(n, 256)), dim3(256), 0, s, src, (bf16_t*)dst, n);
    return hipGetLastError();
}

hipError_t pack_chol(const double* L, void* Lp, DType t, int M, int n_chol, hipStream_t s) {
    const long n = (long)M * (M + 1) / 2 * n_chol;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(nblk(n, 256)), dim3(256), 0, s, L, Lp, t, M, n_chol);
    return hipGetLastError();
}

hipError_t permute_chol(const double* L, double* LT, int M, int n_chol, hipStream_t s) {
    const long n = (long)n_chol * M * M;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute, dim3(nblk(n, 256)), dim3(256), 0, s, L, LT, M, n_chol);
    return hipGetLastError();
}

hipError_t chol_weighted_sum(const double* L, const double* a, double* out, int M, int n_chol,
                             hipStream_t s) {
    const long n = (long)M * M;
    hipLaunchKernelGGL(k_wsum, dim3(nblk(n, 256)), dim3(256), 0, s, L, a, out, M, n_chol);
    return hipGetLastError();
}

}  // namespace afq
