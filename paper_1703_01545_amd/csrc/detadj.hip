// Dense per-(walker, spin) kernels of the reverse pass: the adjoint of the
// overlap O = Phi_T^T Phi, its log-determinant and Theta = Phi O^{-1} (the
// force bias and local energy of Eq. 10 read Theta; the phaseless weight of
// Sec. II.A reads ln <Phi_T|Phi>), and the adjoint of the Gram-Schmidt of
// Sec. II.D.  Spin blocks of up to 64 orbitals.
//
// With Y = Theta_bar O^{-H}, the adjoint of Theta needs Theta^H Y, which is
// O^{-H} (Phi^H Theta_bar) O^{-H}: so one pass over the basis accumulates the
// two n x n contractions O and C = Phi^H Theta_bar on the FP64 matrix cores,
// the n x n algebra (an in-place Gauss-Jordan inverse, two products) stays in
// LDS, and a second pass adds Y + Phi_T Z to Phi_bar.  Neither Theta nor Y is
// formed.  Both passes stream the basis through LDS 16 (or 16 CT) columns at
// a time.
#include "mfma.h"

namespace afq {
namespace dev {
namespace {

constexpr int kMaxBlock = 64;  // orbitals per spin block
constexpr int W1 = 16;         // basis columns per chunk of the overlap pass

// basis columns per chunk of the update pass: 32 for blocks of up to 32
// orbitals (four 16 x 16 tiles per chunk, one per wave), 16 above
__host__ __device__ constexpr int update_width(int npmax) { return npmax <= 32 ? 32 : 16; }

struct Lay {
    int NP, LP, W2;  // padded order, matrix pitch, update chunk width
    long mat;        // doubles per complex matrix ([2][NP][LP])
    long c1, c2;     // doubles of the overlap-pass and update-pass chunks
    long total;      // doubles of dynamic LDS
};

// npmax: the kernel's largest padded order (32 or 64; it fixes W2)
__host__ __device__ inline Lay layout(int n, int npmax) {
    Lay l;
    l.NP = n <= 16 ? 16 : (n + 15) / 16 * 16;
    l.LP = l.NP + 1;
    l.W2 = update_width(npmax);
    l.mat = 2L * l.NP * l.LP;
    l.c1 = 5L * l.NP * (W1 + 1);
    l.c2 = 3L * l.NP * (l.W2 + 1);
    const long a = 2 * l.mat + l.c2;
    l.total = a > l.c1 ? a : l.c1;
    return l;
}

// element (i, j) of a complex matrix in planes [2][NP][LP]
#define MRE(X, i, j) (X)[(i) * L.LP + (j)]
#define MIM(X, i, j) (X)[L.NP * L.LP + (i) * L.LP + (j)]

// One plane of a chunk: rows r < n (zero up to NP), basis columns m0 .. m0 +
// W - 1 (zero past M), held by the workgroup's threads as elements
// e = tid + 256 u (row e / W, column e % W) between the global load and the
// LDS store ([NP][W + 1]), so that the next chunk loads during the products.
template <int W>
struct Rows {
    static constexpr int UMAX = kMaxBlock * W / 256;
    double v[UMAX];
    __device__ __forceinline__ void load(const double* __restrict__ src, int M, int n, int NP,
                                         int m0) {
        const int cnt = NP * W / 256;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < cnt) {
                const int e = threadIdx.x + 256 * u, r = e / W, m = m0 + e % W;
                v[u] = (r < n && m < M) ? src[(long)r * M + m] : 0.0;
            }
    }
    __device__ __forceinline__ void store(double* dst, int NP) const {
        const int cnt = NP * W / 256;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            if (u < cnt) {
                const int e = threadIdx.x + 256 * u;
                dst[(e / W) * (W + 1) + e % W] = v[u];
            }
    }
};

// In-place inverse of the leading n x n block of X by sweeps (Gauss-Jordan
// exchange steps, no row movement): step k pivots on (p_k, k), p_k the row not
// yet used with the largest |Re| + |Im| in column k (near-ties, 2^-46
// relative, to the lower row), and afterwards A^{-1}(i, j) = X(p_i, q_j) with
// q the inverse of k -> p_k.  The n^2 entries are dealt to the threads as
// e = tid + 256 u (row e / n, column e % n, worked out once); every wave
// finds the pivot itself, so a step takes two barriers.  EPT >= n^2 / 256.
// Returns false (for every thread) on a zero pivot.
template <int EPT>
__device__ bool sweep_inverse(double* X, const Lay& L, int n, int* perm, int* pinv) {
    const int tid = threadIdx.x, lane = tid & 63;
    int er[EPT], ec[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + 256 * u;
        const bool ok = e < n * n;
        er[u] = ok ? e / n : L.NP - 1;  // out-of-range entries read a padding row
        ec[u] = ok ? e % n : -1;
    }
    bool used = false;  // row `lane` has been a pivot row (the same in every wave)
    double nr[EPT], ni[EPT];
    for (int k = 0; k < n; ++k) {
        const bool cand = lane < n && !used;
        const double v = cand ? fabs(MRE(X, lane, k)) + fabs(MIM(X, lane, k)) : 0.0;
        const unsigned long long key =
            cand && v >= 0.0
                ? ((__builtin_bit_cast(unsigned long long, v) & ~63ull) | (unsigned)(63 - lane))
                : 0ull;
        const unsigned long long kmax = wave_max_u64(key);
        if ((kmax >> 6) == 0) return false;
        const int p = 63 - (int)(kmax & 63);
        if (lane == p) used = true;
        if (tid == 0) {
            perm[k] = p;
            pinv[p] = k;
        }
        const double pr = MRE(X, p, k), pi = MIM(X, p, k);
        const double den = pr * pr + pi * pi;
        const double ir = pr / den, ii = -pi / den;
        // every read first, then the arithmetic, so the reads overlap:
        //   pivot row p: X(p, j) / piv (j != k), 1 / piv (j == k)
        //   other rows:  X(r, j) - X(r, k) X(p, j) / piv (j != k), -X(r, k) / piv (j == k)
        double fr[EPT], fi[EPT], br[EPT], bi[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int c = ec[u] < 0 ? 0 : ec[u];
            fr[u] = MRE(X, er[u], k);
            fi[u] = MIM(X, er[u], k);
            nr[u] = MRE(X, er[u], c);
            ni[u] = MIM(X, er[u], c);
            br[u] = MRE(X, p, c);
            bi[u] = MIM(X, p, c);
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const bool col_k = ec[u] == k, row_p = er[u] == p;
            const double bq_r = col_k ? 1.0 : br[u], bq_i = col_k ? 0.0 : bi[u];
            const double qr = bq_r * ir - bq_i * ii, qi = bq_r * ii + bq_i * ir;  // new pivot-row entry
            const double gr = col_k ? 0.0 : nr[u], gi = col_k ? 0.0 : ni[u];
            nr[u] = row_p ? qr : gr - (fr[u] * qr - fi[u] * qi);
            ni[u] = row_p ? qi : gi - (fr[u] * qi + fi[u] * qr);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u)
            if (ec[u] >= 0) {
                MRE(X, er[u], ec[u]) = nr[u];
                MIM(X, er[u], ec[u]) = ni[u];
            }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int c = ec[u] < 0 ? 0 : ec[u];
        nr[u] = MRE(X, perm[er[u] < n ? er[u] : 0], pinv[c]);
        ni[u] = MIM(X, perm[er[u] < n ? er[u] : 0], pinv[c]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u)
        if (ec[u] >= 0) {
            MRE(X, er[u], ec[u]) = nr[u];
            MIM(X, er[u], ec[u]) = ni[u];
        }
    __syncthreads();
    return true;
}

// Complex 16 x 16 tile product on the FP64 matrix cores:
//   D(i, j) += sum_{k < K} A(i, k) B(k, j)
// fa(k, re, im) supplies A(i0 + lane % 16, k), fb(k, re, im) B(k, j0 + lane % 16),
// K a multiple of 4 (operands zero past the true length).
template <class FA, class FB>
__device__ __forceinline__ void cmm(FA fa, FB fb, int K, d4& dr, d4& di) {
    const int lane = threadIdx.x & 63;
    for (int kb = 0; kb < K; kb += 4) {
        const int k = kb + (lane >> 4);
        double ar, ai, br, bi;
        fa(k, ar, ai);
        fb(k, br, bi);
        dr = mma1(ar, br, dr);
        dr = mma1(-ai, bi, dr);
        di = mma1(ar, bi, di);
        di = mma1(ai, br, di);
    }
}

// Overlap pass: accumulators (tile t = wave + 4 u of the NP x NP block) over
// the basis of o(a, b) = sum_m T(a, m) X(b, m) (T real rows, X complex rows)
// and, with Y given, c(a, b) = sum_m conj(X(a, m)) Y(b, m), or with TY
// c(a, b) = sum_m T(a, m) Y(b, m).  Chunks at `buf`.
template <bool TY, int TPW>
__device__ void overlap_pass(const double* __restrict__ T, const double* __restrict__ X,
                             const double* __restrict__ Y, long NM, int M, int n, const Lay& L,
                             double* buf, d4 (&o)[TPW][2], d4 (&c)[TPW][2]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15;
    const int NT1 = L.NP / 16, NT = NT1 * NT1, P1 = W1 + 1;
    const long PX = (long)L.NP * P1;
    double* sT = buf;
    double* sX = sT + PX;
    double* sY = sX + 2 * PX;
#pragma unroll
    for (int u = 0; u < TPW; ++u)
        for (int h = 0; h < 2; ++h) o[u][h] = c[u][h] = d4{0, 0, 0, 0};
    Rows<W1> rt, rx0, rx1, ry0, ry1;
    auto fetch = [&](int m0) {
        rt.load(T, M, n, L.NP, m0);
        rx0.load(X, M, n, L.NP, m0);
        rx1.load(X + NM, M, n, L.NP, m0);
        if (Y) {
            ry0.load(Y, M, n, L.NP, m0);
            ry1.load(Y + NM, M, n, L.NP, m0);
        }
    };
    fetch(0);
    for (int m0 = 0; m0 < M; m0 += W1) {
        rt.store(sT, L.NP);
        rx0.store(sX, L.NP);
        rx1.store(sX + PX, L.NP);
        if (Y) {
            ry0.store(sY, L.NP);
            ry1.store(sY + PX, L.NP);
        }
        __syncthreads();
        if (m0 + W1 < M) fetch(m0 + W1);
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int t = wv + 4 * u;
            if (t >= NT) break;
            const int a0 = (t / NT1) * 16, b0 = (t % NT1) * 16;
#pragma unroll
            for (int kb = 0; kb < W1; kb += 4) {
                const int k = kb + (lane >> 4);
                const double ta = sT[(a0 + lr) * P1 + k];
                const double xr = sX[(b0 + lr) * P1 + k], xi = sX[PX + (b0 + lr) * P1 + k];
                o[u][0] = mma1(ta, xr, o[u][0]);
                o[u][1] = mma1(ta, xi, o[u][1]);
                if (Y && TY) {
                    const double yr = sY[(b0 + lr) * P1 + k], yi = sY[PX + (b0 + lr) * P1 + k];
                    c[u][0] = mma1(ta, yr, c[u][0]);
                    c[u][1] = mma1(ta, yi, c[u][1]);
                } else if (Y) {
                    const double ar = sX[(a0 + lr) * P1 + k], ai = sX[PX + (a0 + lr) * P1 + k];
                    const double yr = sY[(b0 + lr) * P1 + k], yi = sY[PX + (b0 + lr) * P1 + k];
                    // conj(X) Y: (ar - i ai)(yr + i yi)
                    c[u][0] = mma1(ar, yr, c[u][0]);
                    c[u][0] = mma1(ai, yi, c[u][0]);
                    c[u][1] = mma1(ar, yi, c[u][1]);
                    c[u][1] = mma1(-ai, yr, c[u][1]);
                }
            }
        }
        __syncthreads();  // the chunk has been read (and the chunks alias the matrices)
    }
}

// accumulator tiles -> complex matrix X
template <int TPW>
__device__ __forceinline__ void put_tiles(const d4 (&v)[TPW][2], double* X, const Lay& L) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int NT1 = L.NP / 16, NT = NT1 * NT1;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = wv + 4 * u;
        if (t >= NT) break;
        const int a0 = (t / NT1) * 16, b0 = (t % NT1) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = a0 + acc_row<double>(lane, r), j = b0 + (lane & 15);
            MRE(X, i, j) = v[u][0][r];
            MIM(X, i, j) = v[u][1][r];
        }
    }
}

// Update pass: D(c, m) = sum_{k < NP} A(c, k) B(k, m) for rows c < n of the
// walker block at gb (planes NM apart), chunk by chunk of W2 basis columns:
// the chunk's planes (T real at sT, G complex at sG) are staged, then wave v
// takes the 16 x 16 tiles v, v + 4, ... of the chunk and calls
// tile(c0, mc, dr, di) for its products; ADD: gb += D, else gb = D.
template <bool ADD, int W2, class TILE>
__device__ void update_pass(const double* __restrict__ T, const double* __restrict__ G,
                            double* gb, long NM, int M, int n, const Lay& L, double* sT,
                            double* sG, TILE tile) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15;
    constexpr int CT = W2 / 16;
    const int NTU = L.NP / 16 * CT;
    const long PG = (long)L.NP * (W2 + 1);
    Rows<W2> st, sg0, sg1;
    auto fetch = [&](int m0) {
        if (T) st.load(T, M, n, L.NP, m0);
        if (G) {
            sg0.load(G, M, n, L.NP, m0);
            sg1.load(G + NM, M, n, L.NP, m0);
        }
    };
    fetch(0);
    for (int m0 = 0; m0 < M; m0 += W2) {
        if (T) st.store(sT, L.NP);
        if (G) {
            sg0.store(sG, L.NP);
            sg1.store(sG + PG, L.NP);
        }
        __syncthreads();
        if (m0 + W2 < M) fetch(m0 + W2);
        for (int t = wv; t < NTU; t += 4) {
            const int c0 = (t / CT) * 16, mc = (t % CT) * 16;
            const int m = m0 + mc + lr;
            // the accumulated values are read before the products, so that
            // their latency overlaps the matrix cores
            double pr[4], pi[4];
            bool ok[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = c0 + acc_row<double>(lane, r);
                ok[r] = m < M && row < n;
                pr[r] = pi[r] = 0.0;
                if (ADD && ok[r]) {
                    pr[r] = gb[(long)row * M + m];
                    pi[r] = gb[NM + (long)row * M + m];
                }
            }
            d4 dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
            tile(c0, mc, dr, di);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (ok[r]) {
                    double* q = gb + (long)(c0 + acc_row<double>(lane, r)) * M + m;
                    q[0] = pr[r] + dr[r];
                    q[NM] = pi[r] + di[r];
                }
        }
        __syncthreads();
    }
}

// Per (walker, spin) block of n orbitals, walkers with mode[w] == active:
//   Phi_bar += Y + Phi_T Z,  Z = coef O^{-H} - O^{-H} (Phi^H Theta_bar) O^{-H},
//   Y = Theta_bar O^{-H},  O = Phi_T^T Phi,  coef = cscale coef[w]
// (Theta_bar NULL: Y = 0 and no C term; coef NULL: 0).  NPMAX: 32 or 64 (the
// largest padded order served; tiles per wave and rows per thread follow).
template <int NPMAX>
__global__ __launch_bounds__(256, NPMAX <= 32 ? 3 : 1) void k_det_adj(DetAdj a) {
    constexpr int TPW = (NPMAX / 16) * (NPMAX / 16) / 4, EPT = NPMAX * NPMAX / 256;
    extern __shared__ double sm[];
    __shared__ int perm[kMaxBlock], pinv[kMaxBlock];
    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? a.na : 0, n = spin ? a.nb : a.na;
    if (n == 0 || a.mode[w] != a.active) return;
    const Lay L = layout(n, NPMAX);
    const int M = a.M, lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15;
    const long NM = (long)a.N * M;
    const double* phi = a.phi + (long)w * 2 * NM + (long)off * M;
    const double* tb = a.thbar ? a.thbar + (long)w * 2 * NM + (long)off * M : nullptr;
    const double* tr = a.trialT + (long)off * M;
    double* Oi = sm;          // O, then O^{-1}
    double* Cm = sm + L.mat;  // C, then O^{-H} C, then Z
    d4 o[TPW][2], c[TPW][2];
    overlap_pass<false, TPW>(tr, phi, tb, NM, M, n, L, sm, o, c);
    put_tiles<TPW>(o, Oi, L);
    if (tb) put_tiles<TPW>(c, Cm, L);
    __syncthreads();
    if (!sweep_inverse<EPT>(Oi, L, n, perm, pinv)) return;  // singular: a frozen walker
    const int NT1 = L.NP / 16, NT = NT1 * NT1;
    double cr = 0.0, ci = 0.0;
    if (a.coef) {
        cr = a.cscale * a.coef[2 * w];
        ci = a.cscale * a.coef[2 * w + 1];
    }
    if (tb) {
        // T1 = O^{-H} C: A(i, k) = conj(Oinv(k, i)), B(k, j) = C(k, j)
        d4 v[TPW][2];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            v[u][0] = v[u][1] = d4{0, 0, 0, 0};
            const int t = wv + 4 * u;
            if (t >= NT) continue;
            const int i0 = (t / NT1) * 16, j0 = (t % NT1) * 16;
            cmm([&](int k, double& re, double& im) {
                    re = MRE(Oi, k, i0 + lr);
                    im = -MIM(Oi, k, i0 + lr);
                },
                [&](int k, double& re, double& im) {
                    re = MRE(Cm, k, j0 + lr);
                    im = MIM(Cm, k, j0 + lr);
                },
                L.NP, v[u][0], v[u][1]);
        }
        __syncthreads();
        put_tiles<TPW>(v, Cm, L);
        __syncthreads();
        // W = T1 O^{-H}: A(i, k) = T1(i, k), B(k, j) = conj(Oinv(j, k)); Z = coef O^{-H} - W
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            v[u][0] = v[u][1] = d4{0, 0, 0, 0};
            const int t = wv + 4 * u;
            if (t >= NT) continue;
            const int i0 = (t / NT1) * 16, j0 = (t % NT1) * 16;
            cmm([&](int k, double& re, double& im) {
                    re = MRE(Cm, i0 + lr, k);
                    im = MIM(Cm, i0 + lr, k);
                },
                [&](int k, double& re, double& im) {
                    re = MRE(Oi, j0 + lr, k);
                    im = -MIM(Oi, j0 + lr, k);
                },
                L.NP, v[u][0], v[u][1]);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int t = wv + 4 * u;
            if (t >= NT) break;
            const int i0 = (t / NT1) * 16, j0 = (t % NT1) * 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + acc_row<double>(lane, r), j = j0 + lr;
                const double hr = MRE(Oi, j, i), hi = -MIM(Oi, j, i);  // (O^{-H})(i, j)
                MRE(Cm, i, j) = cr * hr - ci * hi - v[u][0][r];
                MIM(Cm, i, j) = cr * hi + ci * hr - v[u][1][r];
            }
        }
    } else {
        for (int e = threadIdx.x; e < L.NP * L.NP; e += blockDim.x) {
            const int i = e / L.NP, j = e % L.NP;
            const double hr = MRE(Oi, j, i), hi = -MIM(Oi, j, i);
            MRE(Cm, i, j) = cr * hr - ci * hi;
            MIM(Cm, i, j) = cr * hi + ci * hr;
        }
    }
    // update pass (the chunk loop's first barrier publishes Z):
    //   Phi_bar(c, m) += sum_b conj(Oinv(c, b)) Theta_bar(b, m) + sum_a Z(a, c) T(a, m)
    double* sT = sm + 2 * L.mat;
    double* sG = sT + L.NP * (L.W2 + 1);
    const int P2 = L.W2 + 1;
    const long PG = (long)L.NP * P2;
    double* gb = a.phibar + (long)w * 2 * NM + (long)off * M;
    update_pass<true, update_width(NPMAX)>(tr, tb, gb, NM, M, n, L, sT, sG,
                      [&](int c0, int mc, d4& dr, d4& di) {
                          if (tb)
                              cmm([&](int k, double& re, double& im) {
                                      re = MRE(Oi, c0 + lr, k);
                                      im = -MIM(Oi, c0 + lr, k);
                                  },
                                  [&](int k, double& re, double& im) {
                                      re = sG[k * P2 + mc + lr];
                                      im = sG[PG + k * P2 + mc + lr];
                                  },
                                  L.NP, dr, di);
                          for (int kb = 0; kb < L.NP; kb += 4) {
                              const int k = kb + (lane >> 4);
                              const double tv = sT[k * P2 + mc + lr];
                              dr = mma1(MRE(Cm, k, c0 + lr), tv, dr);
                              di = mma1(MIM(Cm, k, c0 + lr), tv, di);
                          }
                      });
}

// Gram-Schmidt adjoint per (walker, spin) block of walkers alive after it:
// Phi_bar <- Phi_bar S^H with S = O(pre)^{-1} O(Q), O(X) = Phi_T^T X.
template <int NPMAX>
__global__ __launch_bounds__(256) void k_mgs_adj(MgsAdj a) {
    constexpr int TPW = (NPMAX / 16) * (NPMAX / 16) / 4, EPT = NPMAX * NPMAX / 256;
    extern __shared__ double sm[];
    __shared__ int perm[kMaxBlock], pinv[kMaxBlock];
    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? a.na : 0, n = spin ? a.nb : a.na;
    if (n == 0 || !a.alive[w]) return;
    const Lay L = layout(n, NPMAX);
    const int M = a.M, lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lr = lane & 15;
    const long NM = (long)a.N * M;
    const double* pre = a.pre + (long)w * 2 * NM + (long)off * M;
    const double* q = a.q + (long)w * 2 * NM + (long)off * M;
    const double* tr = a.trialT + (long)off * M;
    double* Op = sm;          // O(pre), then its inverse
    double* Oq = sm + L.mat;  // O(Q), then S
    d4 o[TPW][2], c[TPW][2];
    overlap_pass<true, TPW>(tr, pre, q, NM, M, n, L, sm, o, c);
    put_tiles<TPW>(o, Op, L);
    put_tiles<TPW>(c, Oq, L);
    __syncthreads();
    if (!sweep_inverse<EPT>(Op, L, n, perm, pinv)) return;
    const int NT1 = L.NP / 16, NT = NT1 * NT1;
    // S = O(pre)^{-1} O(Q)
    d4 v[TPW][2];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        v[u][0] = v[u][1] = d4{0, 0, 0, 0};
        const int t = wv + 4 * u;
        if (t >= NT) continue;
        const int i0 = (t / NT1) * 16, j0 = (t % NT1) * 16;
        cmm([&](int k, double& re, double& im) {
                re = MRE(Op, i0 + lr, k);
                im = MIM(Op, i0 + lr, k);
            },
            [&](int k, double& re, double& im) {
                re = MRE(Oq, k, j0 + lr);
                im = MIM(Oq, k, j0 + lr);
            },
            L.NP, v[u][0], v[u][1]);
    }
    __syncthreads();
    put_tiles<TPW>(v, Oq, L);
    // Phi_bar(c, m) <- sum_b conj(S(c, b)) Phi_bar(b, m), chunk by chunk (the
    // chunk is staged whole before any of it is written back)
    double* sG = sm + 2 * L.mat;
    const int P2 = L.W2 + 1;
    const long PG = (long)L.NP * P2;
    double* gb = a.phibar + (long)w * 2 * NM + (long)off * M;
    update_pass<false, update_width(NPMAX)>(nullptr, gb, gb, NM, M, n, L, nullptr, sG,
                       [&](int c0, int mc, d4& dr, d4& di) {
                           cmm([&](int k, double& re, double& im) {
                                   re = MRE(Oq, c0 + lr, k);
                                   im = -MIM(Oq, c0 + lr, k);
                               },
                               [&](int k, double& re, double& im) {
                                   re = sG[k * P2 + mc + lr];
                                   im = sG[PG + k * P2 + mc + lr];
                               },
                               L.NP, dr, di);
                       });
}

#undef MRE
#undef MIM

}  // namespace
}  // namespace dev

// dynamic LDS of a launch whose largest spin block has n orbitals
size_t dense_adj_lds(int n) { return (size_t)dev::layout(n, n <= 32 ? 32 : 64).total * 8; }

hipError_t dense_adj_prepare() {
    const int shm = (int)dense_adj_lds(dev::kMaxBlock);
    const void* fns[] = {(const void*)dev::k_det_adj<32>, (const void*)dev::k_det_adj<64>,
                         (const void*)dev::k_mgs_adj<32>, (const void*)dev::k_mgs_adj<64>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, shm);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t det_adjoint(const DetAdj& a, hipStream_t s) {
    const int nmax = a.na > a.nb ? a.na : a.nb;
    if (nmax > dev::kMaxBlock) return hipErrorInvalidValue;
    if (a.nw <= 0 || nmax == 0) return hipSuccess;
    const dim3 grid(a.nw, 2);
    if (nmax <= 32)
        hipLaunchKernelGGL(dev::k_det_adj<32>, grid, dim3(256), dense_adj_lds(nmax), s, a);
    else
        hipLaunchKernelGGL(dev::k_det_adj<64>, grid, dim3(256), dense_adj_lds(nmax), s, a);
    return hipGetLastError();
}

hipError_t mgs_adjoint(const MgsAdj& a, hipStream_t s) {
    const int nmax = a.na > a.nb ? a.na : a.nb;
    if (nmax > dev::kMaxBlock) return hipErrorInvalidValue;
    if (a.nw <= 0 || nmax == 0) return hipSuccess;
    const dim3 grid(a.nw, 2);
    if (nmax <= 32)
        hipLaunchKernelGGL(dev::k_mgs_adj<32>, grid, dim3(256), dense_adj_lds(nmax), s, a);
    else
        hipLaunchKernelGGL(dev::k_mgs_adj<64>, grid, dim3(256), dense_adj_lds(nmax), s, a);
    return hipGetLastError();
}

}  // namespace afq
