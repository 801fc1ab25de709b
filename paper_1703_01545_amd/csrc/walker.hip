// Walker-wise FP64 kernels of the ph-AFQMC step (gfx950, wave64):
// auxiliary fields and force bias, per-spin determinants and Theta,
// hybrid/phaseless weights, modified Gram-Schmidt, local and mixed energy.
// Reductions use fixed-order wavefront butterflies and fixed-order LDS
// sums, so every run is bitwise reproducible.
#include <math.h>

#include "internal.h"

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
            const double xbr = f.free_proj ? 0.0 : sq * Fi[g];
            const double xbi = f.free_proj ? 0.0 : -sq * (Fr[g] - f.a[g]);
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

// Per (walker, spin) block: Gauss-Jordan with partial pivoting on [O | I],
// O[j][i] = sum_m PhiT[m][j] Phi[m][i] (j: trial orbital, i: walker
// orbital).  ln det O = sum_k ln(pivot_k) + i pi (row swaps mod 2).  The
// right block ends as O^{-1}; Theta = Phi O^{-1}.
__global__ __launch_bounds__(256) void k_lu_theta(const double* __restrict__ ov,
                                                  const double* __restrict__ phi,
                                                  double* __restrict__ theta, void* theta_lp,
                                                  DType tlp, double* __restrict__ lnd,
                                                  const uint8_t* __restrict__ live, int M, int N,
                                                  int na, int nb) {
    extern __shared__ double sh[];
    const int w = blockIdx.x, spin = blockIdx.y;
    const int off = spin ? na : 0, n = spin ? nb : na;
    const int tid = threadIdx.x;
    double* out_lnd = lnd + ((long)w * 2 + spin) * 2;
    if (n == 0) {
        if (tid == 0) out_lnd[0] = out_lnd[1] = 0.0;
        return;
    }
    if (!live[w]) return;
    const int ld = 2 * n + 1;
    double* Ar = sh;
    double* Ai = sh + n * ld;
    __shared__ int s_piv;
    const long NM = (long)N * M, NN = (long)N * N;
    const double* ovr = ov + (long)w * 2 * NN;
    const double* ovi = ovr + NN;
    for (int idx = tid; idx < n * n; idx += 256) {
        const int i = idx / n, j = idx % n;  // ov row = walker orbital i, col = trial j
        Ar[j * ld + i] = ovr[(long)(off + i) * N + off + j];
        Ai[j * ld + i] = ovi[(long)(off + i) * N + off + j];
    }
    for (int idx = tid; idx < n * n; idx += 256) {
        const int r = idx / n, c = idx % n;
        Ar[r * ld + n + c] = (r == c) ? 1.0 : 0.0;
        Ai[r * ld + n + c] = 0.0;
    }
    __syncthreads();
    __shared__ double piv_r[64], piv_i[64];
    int swaps = 0;
    const int tx = tid & 63, ty = tid >> 6;  // 64 columns x 4 row groups
    for (int k = 0; k < n; ++k) {
        if (tid < 64) {
            const int r = k + tid;
            double v = -1.0;
            if (r < n) v = fabs(Ar[r * ld + k]) + fabs(Ai[r * ld + k]);
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
            if (tid == 0) s_piv = best;
        }
        __syncthreads();
        const int p = s_piv;
        if (p != k) {
            for (int c = tid; c < 2 * n; c += 256) {
                double t0 = Ar[k * ld + c], t1 = Ai[k * ld + c];
                Ar[k * ld + c] = Ar[p * ld + c];
                Ai[k * ld + c] = Ai[p * ld + c];
                Ar[p * ld + c] = t0;
                Ai[p * ld + c] = t1;
            }
            ++swaps;
        }
        __syncthreads();
        const double pr = Ar[k * ld + k], pi = Ai[k * ld + k];
        if (tid == 0) {
            piv_r[k] = pr;
            piv_i[k] = pi;
        }
        // 1 / pivot
        const double den = pr * pr + pi * pi;
        const double qr = pr / den, qi = -pi / den;
        __syncthreads();
        for (int c = k + 1 + tid; c < 2 * n; c += 256) {
            const double xr = Ar[k * ld + c], xi = Ai[k * ld + c];
            Ar[k * ld + c] = xr * qr - xi * qi;
            Ai[k * ld + c] = xr * qi + xi * qr;
        }
        __syncthreads();
        for (int r = ty; r < n; r += 4) {
            if (r == k) continue;
            const double fr = Ar[r * ld + k], fi = Ai[r * ld + k];
            for (int c = k + 1 + tx; c < 2 * n; c += 64) {
                const double br = Ar[k * ld + c], bi = Ai[k * ld + c];
                Ar[r * ld + c] -= fr * br - fi * bi;
                Ai[r * ld + c] -= fr * bi + fi * br;
            }
        }
        __syncthreads();
    }
    // ln det = sum_k ln(pivot_k) + i pi (swaps mod 2), summed in index order
    if (tid < 64) {
        double lr = 0.0, la = 0.0;
        bool sing = false;
        if (tid < n) {
            const double pr = piv_r[tid], pi = piv_i[tid];
            sing = (pr == 0.0 && pi == 0.0);
            lr = log(hypot(pr, pi));
            la = atan2(pi, pr);
        }
        lr = wave_sum(lr);
        la = wave_sum(la);
        const bool any_sing = __any(sing);
        if (tid == 0) {
            if (any_sing) {
                out_lnd[0] = -INFINITY;
                out_lnd[1] = 0.0;
            } else {
                out_lnd[0] = lr;
                out_lnd[1] = la + ((swaps & 1) ? M_PI : 0.0);
            }
        }
    }
    // Theta[m][c] = sum_l Phi[m][l] Inv[l][c]; Inv[l][c] = A[l][n + c].
    // One basis row m per thread (coalesced Phi loads), CC output columns in
    // registers, the Inv row broadcast from LDS.
    const double* pr_ = phi + (long)w * 2 * NM;
    const double* pi_ = pr_ + NM;
    double* tr_ = theta + (long)w * 2 * NM;
    double* ti_ = tr_ + NM;
    constexpr int CC = 20;
    for (int c0 = 0; c0 < n; c0 += CC) {
        for (int m = tid; m < M; m += 256) {
            double accr[CC], acci[CC];
#pragma unroll
            for (int q = 0; q < CC; ++q) accr[q] = acci[q] = 0.0;
#pragma unroll 4
            for (int l = 0; l < n; ++l) {
                const double xr = pr_[(long)(off + l) * M + m];
                const double xi = pi_[(long)(off + l) * M + m];
                const double* vr_ = Ar + l * ld + n + c0;
                const double* vi_ = Ai + l * ld + n + c0;
#pragma unroll
                for (int q = 0; q < CC; ++q) {
                    if (c0 + q < n) {
                        const double vr = vr_[q], vi = vi_[q];
                        accr[q] += xr * vr - xi * vi;
                        acci[q] += xr * vi + xi * vr;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < CC; ++q) {
                if (c0 + q < n) {
                    const long o = (long)(off + c0 + q) * M + m;
                    tr_[o] = accr[q];
                    ti_[o] = acci[q];
                    if (theta_lp) {
                        const long base = (long)w * 2 * NM;
                        put_dt(theta_lp, tlp, base + o, accr[q]);
                        put_dt(theta_lp, tlp, base + NM + o, acci[q]);
                    }
                }
            }
        }
    }
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
                                             int na, int nb) {
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
    for (int j = 0; j < n; ++j) {
        double* qr = pr + (long)j * ldp;
        double* qi = pi + (long)j * ldp;
        double s = 0.0;
        for (int m = tid; m < M; m += 256) s += qr[m] * qr[m] + qi[m] * qi[m];
        s = wave_sum(s);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        const double nrm = sqrt(((red[0] + red[1]) + red[2]) + red[3]);
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

hipError_t lu_theta(const double* ov, const double* phi, double* theta, void* theta_lp, DType tlp,
                    double* lnd, const uint8_t* live, int nw, int M, int N, int na, int nb,
                    hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    const int nmax = na > nb ? na : nb;
    const size_t shm = (size_t)2 * nmax * (2 * nmax + 1) * sizeof(double);
    static size_t allowed = 65536;  // raised once per new size, outside graph capture
    if (shm > allowed) {
        hipError_t e = hipFuncSetAttribute((const void*)k_lu_theta,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        allowed = shm;
    }
    hipLaunchKernelGGL(k_lu_theta, dim3(nw, 2), dim3(256), shm, s, ov, phi, theta, theta_lp, tlp,
                       lnd, live, M, N, na, nb);
    return hipGetLastError();
}

hipError_t weights(const double* lnd, const double* s_imp, double* lnov, double* w, uint8_t* alive,
                   int nw, int mode, int commit, double shift, hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_weights, dim3(nblk(nw, 256)), dim3(256), 0, s, lnd, s_imp, lnov, w, alive,
                       nw, mode, commit, shift);
    return hipGetLastError();
}

hipError_t mgs(double* phi, const uint8_t* live, int nw, int M, int N, int na, int nb,
               hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    const int nmax = na > nb ? na : nb;
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
        hipLaunchKernelGGL(k_mgs<true>, dim3(nw, 2), dim3(256), shm, s, phi, live, M, N, na, nb);
    } else {
        hipLaunchKernelGGL(k_mgs<false>, dim3(nw, 2), dim3(256), 0, s, phi, live, M, N, na, nb);
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
