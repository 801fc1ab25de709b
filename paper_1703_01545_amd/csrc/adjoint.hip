// Reverse-mode derivative of the mixed energy (Eq. 7, Eq. 10) with respect
// to a one-body perturbation h -> h + lambda V, through a window of walker
// steps (Eq. 3, 4, 8-11, the phaseless weight of Sec. II.A/II.D and the
// Gram-Schmidt of Sec. II.D).
//
// lambda enters the one-body halves P = expm(-dt (h~ + lambda V) / 2) of every
// step and h^half = Phi_T^T (h + lambda V) in the final local energy.  The
// derivative is pathwise (fields held fixed).  The forward pass keeps a
// snapshot of the walkers every k steps; the reverse pass recomputes one
// segment at a time from its snapshot (the same kernels, so the same
// trajectory), records what the reverse step needs, and walks the segment
// backwards.  Complex adjoints use z_bar = dL/dRe z + i dL/dIm z, so that
// dL = Re(conj(z_bar) dz); for C = A B, A_bar = C_bar B^H and B_bar = A^H C_bar.
//
// Per step, given Phi_bar (of the state after the step) and w_bar:
//   ln I_bar = w_bar w',  ln R_bar = ln I_bar - i w_bar w g sin(Im ln R)
//   (w' = w g cos(Im ln R), g = e^{Re ln I + shift});
//   ln <phi_T|phi'> and ln <phi_T|phi> receive +- ln R_bar (through O^{-H});
//   y_bar = P Phi_bar, the Taylor terms backwards (t_bar_{n-1} = y_bar +
//   conj(A) t_bar_n / n), A_bar = sum_n t_bar_n t_{n-1}^H / n;
//   c_bar = -i sqrt(dt) <L, A_bar> + i sqrt(dt) a s_bar, xbar_bar =
//   conj(x - xbar) ln I_bar - c_bar, f_bar = i sqrt(dt) xbar_bar,
//   Theta_bar = sum_g L^half_g^T f_bar_g, and Theta = Phi O^{-1} gives
//   Phi_bar += Y - Phi_T (Theta^H Y), Y = Theta_bar O^{-H};
//   dE/dlambda += <Phi_bar', dP y> + <u_bar, dP Phi>.
// Gram-Schmidt Q = Phi R^{-1}: everything after it is unchanged by Q -> Q U,
// so Phi_bar = Q_bar S^H with S = R^{-1} = O(Phi)^{-1} O(Q).
#include <atomic>

#include "host.h"

using namespace afq;
using namespace afq::host;

namespace afq {
namespace host {
namespace {

constexpr int kMaxSpin = 64;  // largest spin block of the dense adjoint kernels
constexpr uint8_t ACTIVE = 1;

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

__device__ __forceinline__ double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// out[b][c][coff + r] = scale * in[b][r][c] for b < nb, r < R, c < C.
__global__ __launch_bounds__(256) void k_tr(const double* __restrict__ in, double* __restrict__ out,
                                            int R, int C, long ldo, long coff, double scale) {
    __shared__ double tile[32][33];
    const long b = blockIdx.z;
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const double* src = in + b * (long)R * C;
    double* dst = out + b * (long)C * ldo;
    for (int r = ty; r < 32; r += 8)
        if (r0 + r < R && c0 + tx < C) tile[r][tx] = src[(long)(r0 + r) * C + c0 + tx];
    __syncthreads();
    for (int c = ty; c < 32; c += 8)
        if (c0 + c < C && r0 + tx < R) dst[(long)(c0 + c) * ldo + coff + r0 + tx] = scale * tile[tx][c];
}

void transpose(const double* in, double* out, int nb, int R, int C, long ldo, long coff,
               double scale, hipStream_t st) {
    dim3 grid((C + 31) / 32, (R + 31) / 32, nb);
    hipLaunchKernelGGL(k_tr, grid, dim3(256), 0, st, in, out, R, C, ldo, coff, scale);
}

// Lq[g][q] = L_g[i][j], q = i (2M - i + 1) / 2 + (j - i), i <= j.
__global__ void k_lq(const double* __restrict__ chol, double* __restrict__ lq, int M, int nc) {
    const long P = (long)M * (M + 1) / 2;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * nc) return;
    const int g = (int)(e / P);
    long q = e % P;
    int i = 0;
    while (q >= M - i) {
        q -= M - i;
        ++i;
    }
    const int j = i + (int)q;
    lq[e] = chol[((long)g * M + i) * M + j];
}

// lht2[m][g * n + j] = lhx[g][off + j][m]   (one spin block)
__global__ void k_lht2(const double* __restrict__ lhx, double* __restrict__ out, int M, int N,
                       int nc, int off, int n) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long K = (long)nc * n;
    if (e >= (long)M * K) return;
    const int m = (int)(e / K);
    const long k = e % K;
    const int g = (int)(k / n), j = (int)(k % n);
    out[e] = lhx[((long)g * N + off + j) * M + m];
}

// Adjoint of the weight update of one step (per walker).
__global__ void k_adj_scalars(const double* __restrict__ w_in, const double* __restrict__ w_out,
                              const uint8_t* __restrict__ alive_in,
                              const uint8_t* __restrict__ alive_out,
                              const double* __restrict__ lnov_in, const double* __restrict__ lnd,
                              const double* __restrict__ simp, const double* __restrict__ wbar_out,
                              double shift, double* __restrict__ wbar_in, uint8_t* __restrict__ mode,
                              double* __restrict__ lnr_bar, double* __restrict__ lni_bar, int nw) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    const bool act = alive_in[w] && alive_out[w];
    mode[w] = act ? ACTIVE : 0;
    if (!act) {
        wbar_in[w] = 0.0;
        lnr_bar[2 * w] = lnr_bar[2 * w + 1] = 0.0;
        lni_bar[w] = 0.0;
        return;
    }
    const double lrr = lnd[4 * w] + lnd[4 * w + 2] - lnov_in[2 * w] + simp[4 * w];
    const double lri = lnd[4 * w + 1] + lnd[4 * w + 3] - lnov_in[2 * w + 1] + simp[4 * w + 1];
    const double lir = lrr + simp[4 * w + 2];
    const double g = exp(lir + shift);
    const double cs = cos(lri), sn = sin(lri);
    const double wb = wbar_out[w];
    wbar_in[w] = wb * g * cs;
    const double lib = wb * w_out[w];
    lni_bar[w] = lib;
    lnr_bar[2 * w] = lib;
    lnr_bar[2 * w + 1] = -wb * w_in[w] * g * sn;
}

// f_bar of one step: from the A-contraction G = <L, A_bar> (re, im per g),
// ln R_bar (s_bar) and ln I_bar.  Fbar rows [w][2][ldf], column n_chol zero.
__global__ __launch_bounds__(256) void k_adj_fbar(const double* __restrict__ F, int ldf,
                                                  const double* __restrict__ a,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ G,
                                                  const double* __restrict__ lnr_bar,
                                                  const double* __restrict__ lni_bar,
                                                  const uint8_t* __restrict__ mode, double sq,
                                                  double* __restrict__ Fbar, int nw, int nc) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)nw * ldf) return;
    const int w = (int)(e / ldf), g = (int)(e % ldf);
    double* fr = Fbar + (long)w * 2 * ldf;
    if (g >= nc || mode[w] != ACTIVE) {
        fr[g] = 0.0;
        fr[ldf + g] = 0.0;
        return;
    }
    const double* Fw = F + (long)w * 2 * ldf;
    const double xbr = sq * Fw[ldf + g], xbi = -sq * (Fw[g] - a[g]);
    const double gr = G[(long)w * 2 * nc + g], gi = G[(long)w * 2 * nc + nc + g];
    const double sbr = lnr_bar[2 * w], sbi = lnr_bar[2 * w + 1];
    const double cbr = sq * (gi - a[g] * sbi), cbi = sq * (-gr + a[g] * sbr);
    const double lib = lni_bar[w];
    const double xg = x[(long)w * nc + g];
    const double xbbr = (xg - xbr) * lib - cbr, xbbi = xbi * lib - cbi;
    fr[g] = -sq * xbbi;
    fr[ldf + g] = sq * xbbr;
}

// Packed symmetric contraction weights of A_bar: q(i <= j) -> A_ij + A_ji
// (i < j), A_ii.  [w][2][M][M] -> [w][2][P].  One workgroup per 32 x 32 tile
// (bi <= bj) of the upper triangle of one plane: the mirror tile (bj, bi)
// goes through LDS so that both reads and the packed writes are coalesced.
__global__ __launch_bounds__(256) void k_adj_pack(const double* __restrict__ Af,
                                                  double* __restrict__ Apk, int M, int nt) {
    __shared__ double tt[32][33];
    const long pl = blockIdx.x;  // planes on x (limit 2^31 - 1 blocks)
    const long P = (long)M * (M + 1) / 2;
    int t = blockIdx.y, bi = 0;
    while (t >= nt - bi) {  // nt <= 8
        t -= nt - bi;
        ++bi;
    }
    const int bj = bi + t;
    const double* A = Af + pl * (long)M * M;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int j = bj * 32 + r, i = bi * 32 + tx;
        tt[r][tx] = (j < M && i < M) ? A[(long)j * M + i] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bi * 32 + r, j = bj * 32 + tx;
        if (i < M && j < M && i <= j) {
            const double v = i == j ? A[(long)i * M + i] : A[(long)i * M + j] + tt[tx][r];
            Apk[pl * P + (long)i * M - (long)i * (i - 1) / 2 + (j - i)] = v;
        }
    }
}

// Up to eight device-to-device copies in one launch: blockIdx.y picks the
// copy, the x blocks stride over its 8-byte words; block 0 copies the tail
// bytes.  Buffers are hipMalloc allocations (8-byte aligned).
struct CopySet {
    const void* src[8];
    void* dst[8];
    long bytes[8];
};
__global__ __launch_bounds__(256) void k_copyset(CopySet c) {
    const int b = blockIdx.y;
    const long words = c.bytes[b] / 8;
    const unsigned long long* s8 = (const unsigned long long*)c.src[b];
    unsigned long long* d8 = (unsigned long long*)c.dst[b];
    const long stride = (long)gridDim.x * blockDim.x;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < words; e += stride) d8[e] = s8[e];
    const long tail = c.bytes[b] - words * 8;
    if (blockIdx.x == 0 && threadIdx.x < tail)
        ((uint8_t*)c.dst[b])[words * 8 + threadIdx.x] =
            ((const uint8_t*)c.src[b])[words * 8 + threadIdx.x];
}

hipError_t copyset(const CopySet& c, int n, hipStream_t st) {
    long most = 0;
    for (int i = 0; i < n; ++i) most = c.bytes[i] > most ? c.bytes[i] : most;
    const long blocks = std::min(2048L, std::max(1L, (most / 8 + 255) / 256));
    hipLaunchKernelGGL(k_copyset, dim3((unsigned)blocks, n), dim3(256), 0, st, c);
    return hipGetLastError();
}

// dst[w][r] = scale * src[w][r], r < per (walker strides sbs, dbs)
__global__ void k_scale_copy(const double* __restrict__ src, long sbs, double* __restrict__ dst,
                             long dbs, long per, int nw, double scale) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= per * nw) return;
    const long w = e / per, r = e % per;
    dst[w * dbs + r] = scale * src[w * sbs + r];
}

// Zero the walker blocks of walkers that are not ACTIVE.
__global__ void k_mask(double* __restrict__ v, const uint8_t* __restrict__ mode, long per, int nw) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < per * nw && mode[i / per] != ACTIVE) v[i] = 0.0;
}

// part[w] = sum_k a[w][k] b[w][k] for ACTIVE walkers, else 0 (one block per
// walker, fixed-order reduction).
__global__ __launch_bounds__(256) void k_dot_part(const double* __restrict__ a,
                                                  const double* __restrict__ b,
                                                  const uint8_t* __restrict__ mode, long per,
                                                  double* __restrict__ part) {
    __shared__ double red[4];
    const int w = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    if (mode[w] == ACTIVE) {
        const double* x = a + (long)w * per;
        const double* y = b + (long)w * per;
        for (long k = tid; k < per; k += 256) s += x[k] * y[k];
    }
    s = wsum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) part[w] = (red[0] + red[1]) + (red[2] + red[3]);
}

// acc[slot] += sum_w part[w]  (one block, fixed order)
__global__ __launch_bounds__(256) void k_dot_sum(const double* __restrict__ part, int nw,
                                                 double* acc, int slot) {
    __shared__ double red[4];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int w = tid; w < nw; w += 256) s += part[w];
    s = wsum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) acc[slot] += (red[0] + red[1]) + (red[2] + red[3]);
}

void dot_acc(const double* a, const double* b, const uint8_t* mode, long per, int nw,
             double* part, double* acc, int slot, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_part, dim3(nw), dim3(256), 0, st, a, b, mode, per, part);
    hipLaunchKernelGGL(k_dot_sum, dim3(1), dim3(256), 0, st, part, nw, acc, slot);
}

// Energy adjoint set-up at the end of the window (one block): W = sum w,
// E = sum w Re E_L / W over live walkers; w_bar = (Re E_L - E) / W,
// scale = w / W, F_bar rows: (w/W) conj(f_g) for g < n_chol, w/W for the
// h^half column.
__global__ __launch_bounds__(256) void k_energy_adj(const double* __restrict__ el,
                                                    const double* __restrict__ w,
                                                    const uint8_t* __restrict__ alive,
                                                    const double* __restrict__ F, int ldf, int nw,
                                                    double* wbar, double* scale, double* Fbar,
                                                    uint8_t* mode, double* out) {
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    double sw = 0.0, se = 0.0;
    for (int k = tid; k < nw; k += 256)
        if (alive[k]) {
            sw += w[k];
            se += w[k] * el[2 * k];
        }
    sw = wsum(sw);
    se = wsum(se);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = sw;
        red[1][tid >> 6] = se;
    }
    __syncthreads();
    const double W = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double E = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3])) / W;
    if (tid == 0) {
        out[0] = E;
        out[1] = W;
    }
    for (int k = tid; k < nw; k += 256) {
        const bool a = alive[k] != 0;
        mode[k] = a ? ACTIVE : 0;
        wbar[k] = a ? (el[2 * k] - E) / W : 0.0;
        scale[k] = a ? w[k] / W : 0.0;
    }
    for (long e = tid; e < (long)nw * ldf; e += 256) {
        const int k = (int)(e / ldf), g = (int)(e % ldf);
        const double sc = alive[k] ? w[k] / W : 0.0;
        const double* Fw = F + (long)k * 2 * ldf;
        double* o = Fbar + (long)k * 2 * ldf;
        if (g == ldf - 1) {
            o[g] = sc;
            o[ldf + g] = 0.0;
        } else {
            o[g] = sc * Fw[g];
            o[ldf + g] = -sc * Fw[ldf + g];
        }
    }
}

// Theta_bar -= scale conj(U) (exchange part), per walker block
__global__ void k_exch_combine(double* __restrict__ thbar, const double* __restrict__ U,
                               const double* __restrict__ scale, long NM, int nw) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * NM * nw) return;
    const long w = e / (2 * NM);
    const bool im = (e % (2 * NM)) >= NM;
    thbar[e] += (im ? 1.0 : -1.0) * scale[w] * U[e];
}

// out[slot] += sum_w scale[w] v[2 w]  (explicit h^half term)
__global__ void k_explicit(const double* __restrict__ v, const double* __restrict__ scale, int nw,
                           double* out, int slot) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += scale[k] * v[2 * k];
    out[slot] += s;
}

// ---------------------------------------------------------------- host side

struct Snap {
    DevBuf phi, w, lnov, alive;
    int64_t t = 0;
};

}  // namespace

struct AdjState {
    int n_steps = 0, every = 0, n_seg = 0;
    uint64_t seed = 0;
    DType prec = DT_F64;
    bool ready = false;  // a forward pass is on the tape
    bool taped = false;  // the forward pass recorded every step (one segment)
    double E = 0.0;
    std::vector<double> V;
    std::vector<double> trial_host;  // Phi_T^T rows (host copy, for V^half)
    // constants
    DevBuf dP, vhalf, lht, lht2[2], lq, lp64;
    // snapshots: segment starts and the end state
    std::vector<Snap> ck;
    Snap fin;
    // per-step tape of one segment
    std::vector<DevBuf> t_phi, t_pre, t_F, t_lnov, t_w, t_alive, t_simp, t_lnd, t_wout, t_aout;
    std::vector<bool> t_mgs;
    // Taylor terms t_0 .. t_{K-1} ([w][n][2][N][M]) and y = sum_n t_n of each
    // recorded step, written by the step's own propagation (FP64 / FP32
    // products) when device memory allows; t_rec[j]: slot j holds them
    std::vector<DevBuf> t_terms, t_y;
    std::vector<bool> t_rec;
    bool record = false;
    std::vector<int64_t> t_t;
    // scratch
    DevBuf xc, simp_s, apk, A, x, tA, y, tT, tbT, ybar, Abar, Abpk, G, Fbar, thbar, phibar,
        phibar2, wbar, wbar2, mode, lnrb, lnib, z, acc, ebuf, scale, Tb, U, vd, part;
    // K ranges of G = <L_g, A_bar> (K = M(M+1)/2 is long, the output small)
    int g_ks = 1;
    DevBuf gws;
};

namespace {

afqmc_status snap_take(afqmc_sys s, Snap& c, hipStream_t st) {
    const size_t nphi = (size_t)s->nw * 2 * s->NM() * 8;
    if (!c.phi.p) {
        HIPCHK(c.phi.alloc(nphi));
        HIPCHK(c.w.alloc((size_t)s->nw * 8));
        HIPCHK(c.lnov.alloc((size_t)s->nw * 16));
        HIPCHK(c.alive.alloc((size_t)s->nw));
    }
    HIPCHK(hipMemcpyAsync(c.phi.p, s->d_phi.p, nphi, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c.w.p, s->d_w.p, (size_t)s->nw * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c.lnov.p, s->d_lnov.p, (size_t)s->nw * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c.alive.p, s->d_alive.p, (size_t)s->nw, hipMemcpyDeviceToDevice, st));
    c.t = s->t;
    return AFQMC_OK;
}

// Restore walkers (and recompute Theta with the step's own kernels).
afqmc_status snap_restore(afqmc_sys s, const Snap& c, hipStream_t st) {
    const size_t nphi = (size_t)s->nw * 2 * s->NM() * 8;
    HIPCHK(hipMemcpyAsync(s->d_phi.p, c.phi.p, nphi, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_w.p, c.w.p, (size_t)s->nw * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_lnov.p, c.lnov.p, (size_t)s->nw * 16, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(s->d_alive.p, c.alive.p, (size_t)s->nw, hipMemcpyDeviceToDevice, st));
    s->t = c.t;
    afqmc_status r = overlap_theta(s, s->d_phi.as<double>(), st);
    if (r != AFQMC_OK) return r;
    // overlap_theta refreshes the per-spin determinants; ln overlap stays as restored
    return AFQMC_OK;
}

// rows (w, p, i) times a shared real symmetric M x M matrix (output rows at rc)
hipError_t rgemm(const double* R, const double* B, double* C, long rows, int M, DType prec,
                 hipStream_t st, RowMap rc);
hipError_t rgemm(const double* R, const double* B, double* C, long rows, int M, DType prec,
                 hipStream_t st) {
    return rgemm(R, B, C, rows, M, prec, st, rows_strided(M));
}
hipError_t rgemm(const double* R, const double* B, double* C, long rows, int M, DType prec,
                 hipStream_t st, RowMap rc) {
    Gemm g{};
    g.A = B;
    g.ta = DT_F64;
    g.ra = rows_strided(M);
    g.B = R;
    g.tb = DT_F64;
    g.rb = rows_strided(M);
    g.C = C;
    g.tc = DT_F64;
    g.rc = rc;
    g.alpha = 1.0;
    g.m = (int)rows;
    g.n = M;
    g.k = M;
    g.batch = 1;
    return gemm(g, prec, st);
}

// The window's constant operators, on the host: dP = d/dlambda
// expm(-dt (h~ + lambda V) / 2), the upper-right block of the exponential of
// [[X, E], [0, X]] (X = -dt h~ / 2, E = -dt V / 2), and V^half = Phi_T^T V
// (rows = trial orbitals).  Called after the forward steps are queued, so
// the host work overlaps them (the forward pass needs neither).
afqmc_status adj_operators(afqmc_sys s, AdjState* a) {
    const int M = s->M, N = s->N;
    const long NM = s->NM();
    std::vector<double> B((size_t)4 * M * M, 0.0), Eb;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            const double x = -0.5 * s->par.dt * s->htilde[(size_t)i * M + j];
            B[(size_t)i * 2 * M + j] = x;
            B[(size_t)(M + i) * 2 * M + M + j] = x;
            B[(size_t)i * 2 * M + M + j] = -0.5 * s->par.dt * a->V[(size_t)i * M + j];
        }
    expm_host(B, 2 * M, Eb);
    std::vector<double> dP((size_t)M * M);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) dP[(size_t)i * M + j] = Eb[(size_t)i * 2 * M + M + j];
    HIPCHK(hipMemcpy(a->dP.p, dP.data(), dP.size() * 8, hipMemcpyHostToDevice));
    std::vector<double> vh((size_t)NM, 0.0);
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < M; ++k) {
            const double t = a->trial_host[(size_t)i * M + k];
            if (t == 0.0) continue;
            for (int m = 0; m < M; ++m) vh[(size_t)i * M + m] += t * a->V[(size_t)k * M + m];
        }
    HIPCHK(hipMemcpy(a->vhalf.p, vh.data(), vh.size() * 8, hipMemcpyHostToDevice));
    return AFQMC_OK;
}

afqmc_status adj_setup(afqmc_sys s, AdjState* a, hipStream_t st) {
    const int M = s->M, N = s->N, nc = s->n_chol, nw = s->nw, K = s->par.taylor_order;
    const long NM = s->NM(), P = s->P();
    if (!a->dP.p) {
        HIPCHK(a->dP.alloc((size_t)M * M * 8));
        HIPCHK(a->vhalf.alloc((size_t)NM * 8));
        a->trial_host.resize((size_t)NM);
        HIPCHK(hipMemcpy(a->trial_host.data(), s->d_trialT.p, NM * 8, hipMemcpyDeviceToHost));
    }
    static std::atomic<bool> lds_ready{false};  // process-wide kernel attribute
    if (!lds_ready) {
        HIPCHK(dense_adj_prepare());
        lds_ready = true;
    }
    if (a->lht.p) return AFQMC_OK;  // shape-dependent buffers already there
    const size_t rowb = (size_t)nw * 2 * NM * 8;
    HIPCHK(a->lht.alloc((size_t)NM * (nc + 1) * 8));
    transpose(s->d_lhx.as<double>(), a->lht.as<double>(), 1, nc + 1, (int)NM, nc + 1, 0, 1.0, st);
    for (int sp = 0; sp < 2; ++sp) {
        const int off = sp ? s->na : 0, n = sp ? s->nb : s->na;
        if (n == 0 || nc == 0) continue;
        HIPCHK(a->lht2[sp].alloc((size_t)M * nc * n * 8));
        hipLaunchKernelGGL(k_lht2, dim3(nblk((long)M * nc * n, 256)), dim3(256), 0, st,
                           s->d_lhx.as<double>(), a->lht2[sp].as<double>(), M, N, nc, off, n);
    }
    HIPCHK(a->lq.alloc((size_t)std::max(nc, 1) * P * 8));
    HIPCHK(a->lp64.alloc((size_t)std::max(nc, 1) * P * 8));
    if (nc > 0) {
        hipLaunchKernelGGL(k_lq, dim3(nblk((long)nc * P, 256)), dim3(256), 0, st,
                           s->ham->d_chol.as<double>(), a->lq.as<double>(), M, nc);
        HIPCHK(pack_chol(s->ham->d_chol.as<double>(), a->lp64.p, DT_F64, M, nc, st));
    }
    struct B_ {
        DevBuf* b;
        size_t n;
    } bufs[] = {
        {&a->xc, (size_t)nw * 2 * std::max(nc, 1) * 8}, {&a->simp_s, (size_t)nw * 4 * 8},
        {&a->apk, (size_t)nw * 2 * P * 8},   {&a->A, (size_t)nw * 2 * M * M * 8},
        {&a->x, (size_t)nw * std::max(nc, 1) * 8}, {&a->tA, rowb}, {&a->y, rowb},
        {&a->tT, (size_t)nw * 2 * M * K * N * 8}, {&a->tbT, (size_t)nw * 2 * M * K * N * 8},
        {&a->ybar, rowb}, {&a->Abar, (size_t)nw * 2 * M * M * 8}, {&a->Abpk, (size_t)nw * 2 * P * 8},
        {&a->G, (size_t)nw * 2 * std::max(nc, 1) * 8}, {&a->Fbar, (size_t)nw * 2 * (nc + 1) * 8},
        {&a->thbar, rowb}, {&a->phibar, rowb}, {&a->phibar2, rowb}, {&a->wbar, (size_t)nw * 8},
        {&a->wbar2, (size_t)nw * 8}, {&a->mode, (size_t)nw}, {&a->lnrb, (size_t)nw * 16},
        {&a->lnib, (size_t)nw * 8}, {&a->z, rowb},
        {&a->acc, 64 * 8}, {&a->ebuf, 16}, {&a->scale, (size_t)nw * 8}, {&a->U, rowb},
        {&a->vd, (size_t)nw * 2 * 8}, {&a->part, (size_t)nw * 8},
    };
    for (auto& b : bufs) HIPCHK(b.b->alloc(b.n));
    a->g_ks = P >= 512 ? (int)std::min(8L, P / 256) : 1;
    if (a->g_ks > 1) HIPCHK(a->gws.alloc(gemm_ws_bytes(2 * nw, std::max(nc, 1), a->g_ks, a->prec)));
    const int nmax = std::max(s->na, s->nb);
    HIPCHK(a->Tb.alloc((size_t)nw * 2 * std::max(nc, 1) * nmax * nmax * 8));
    return AFQMC_OK;
}

// Record one step (and its Gram-Schmidt) of the system onto tape slot j.
afqmc_status taped_step(afqmc_sys s, AdjState* a, int j, hipStream_t st) {
    const int nw = s->nw;
    const size_t nphi = (size_t)nw * 2 * s->NM() * 8;
    auto ensure = [&](std::vector<DevBuf>& v, size_t bytes) -> hipError_t {
        if (!v[j].p) return v[j].alloc(bytes);
        return hipSuccess;
    };
    HIPCHK(ensure(a->t_phi, nphi));
    HIPCHK(ensure(a->t_F, (size_t)nw * 2 * (s->n_chol + 1) * 8));
    HIPCHK(ensure(a->t_lnov, (size_t)nw * 16));
    HIPCHK(ensure(a->t_w, (size_t)nw * 8));
    HIPCHK(ensure(a->t_alive, (size_t)nw));
    HIPCHK(ensure(a->t_simp, (size_t)nw * 32));
    HIPCHK(ensure(a->t_lnd, (size_t)nw * 32));
    HIPCHK(ensure(a->t_wout, (size_t)nw * 8));
    HIPCHK(ensure(a->t_aout, (size_t)nw));
    {
        // the state before the step
        CopySet c{};
        c.src[0] = s->d_phi.p, c.dst[0] = a->t_phi[j].p, c.bytes[0] = (long)nphi;
        c.src[1] = s->d_lnov.p, c.dst[1] = a->t_lnov[j].p, c.bytes[1] = (long)nw * 16;
        c.src[2] = s->d_w.p, c.dst[2] = a->t_w[j].p, c.bytes[2] = (long)nw * 8;
        c.src[3] = s->d_alive.p, c.dst[3] = a->t_alive[j].p, c.bytes[3] = nw;
        HIPCHK(copyset(c, 4, st));
    }
    a->t_t[j] = s->t;
    a->t_rec[j] = false;
    if (a->record) {
        const long TS = 2 * s->NM(), K = s->par.taylor_order;
        HIPCHK(ensure(a->t_terms, (size_t)nw * K * TS * 8));
        HIPCHK(ensure(a->t_y, (size_t)nw * TS * 8));
        s->rec.terms = a->t_terms[j].as<double>();
        s->rec.bs_walker = K * TS;
        s->rec.bs_slot = TS;
        s->rec.y = a->t_y[j].as<double>();
    }
    afqmc_status r = one_step(s, a->seed, 0, nullptr, st);
    s->rec = Record();
    if (r != AFQMC_OK) return r;
    a->t_rec[j] = a->record;
    {
        // what the step computed
        CopySet c{};
        c.src[0] = s->d_F.p, c.dst[0] = a->t_F[j].p, c.bytes[0] = (long)nw * 2 * (s->n_chol + 1) * 8;
        c.src[1] = s->d_simp.p, c.dst[1] = a->t_simp[j].p, c.bytes[1] = (long)nw * 32;
        c.src[2] = s->d_lnd.p, c.dst[2] = a->t_lnd[j].p, c.bytes[2] = (long)nw * 32;
        c.src[3] = s->d_w.p, c.dst[3] = a->t_wout[j].p, c.bytes[3] = (long)nw * 8;
        c.src[4] = s->d_alive.p, c.dst[4] = a->t_aout[j].p, c.bytes[4] = nw;
        HIPCHK(copyset(c, 5, st));
    }
    const int oe = s->par.ortho_every;
    a->t_mgs[j] = oe > 0 && s->t % oe == 0;
    if (a->t_mgs[j]) {
        HIPCHK(ensure(a->t_pre, nphi));
        HIPCHK(hipMemcpyAsync(a->t_pre[j].p, s->d_phi.p, nphi, hipMemcpyDeviceToDevice, st));
        if ((r = ortho(s, st)) != AFQMC_OK) return r;
    }
    return AFQMC_OK;
}

// Tape slots 0..n (n steps and the state after them).
void tape_resize(AdjState* a, int n) {
    for (auto* v : {&a->t_phi, &a->t_pre, &a->t_F, &a->t_lnov, &a->t_w, &a->t_alive, &a->t_simp,
                    &a->t_lnd, &a->t_wout, &a->t_aout, &a->t_terms, &a->t_y})
        if ((int)v->size() < n + 1) v->resize(n + 1);
    a->t_mgs.assign(n + 1, false);
    a->t_rec.assign(n + 1, false);
    a->t_t.assign(n + 1, 0);
}

// Record the Taylor terms of the next n taped steps when the propagation
// computes them in FP64 / FP32 (not split BF16) and the slots still to be
// allocated fit in 3/4 of the free device memory; otherwise the reverse pass
// recomputes them.
void plan_record(afqmc_sys s, AdjState* a, int n) {
    a->record = false;
    if (s->ta == DT_SPLIT) return;
    const size_t slot = (size_t)s->nw * 2 * s->NM() * 8 * (s->par.taylor_order + 1);
    size_t need = 0;
    for (int j = 0; j < n; ++j)
        if (!a->t_terms[j].p) need += slot;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return;
    a->record = need <= free_b / 4 * 3;
}

// The state after the last of n recorded steps into tape slot n.
afqmc_status tape_end(afqmc_sys s, AdjState* a, int n, hipStream_t st) {
    const size_t nphi = (size_t)s->nw * 2 * s->NM() * 8;
    if (!a->t_phi[n].p) HIPCHK(a->t_phi[n].alloc(nphi));
    HIPCHK(hipMemcpyAsync(a->t_phi[n].p, s->d_phi.p, nphi, hipMemcpyDeviceToDevice, st));
    return AFQMC_OK;
}

afqmc_status det_adj(afqmc_sys s, const double* phi, const double* thbar, const double* coef,
                     double cscale, const uint8_t* mode, double* phibar, hipStream_t st) {
    DetAdj d{};
    d.phi = phi;
    d.trialT = s->d_trialT.as<double>();
    d.thbar = thbar;
    d.coef = coef;
    d.cscale = cscale;
    d.mode = mode;
    d.active = ACTIVE;
    d.phibar = phibar;
    d.nw = s->nw;
    d.M = s->M;
    d.N = s->N;
    d.na = s->na;
    d.nb = s->nb;
    HIPCHK(det_adjoint(d, st));
    return AFQMC_OK;
}

// Theta_bar (rows [w][2][N][M]) = sum_g Fbar[(w,p), g] L^half rows g (incl. h^half)
hipError_t fbar_to_thbar(afqmc_sys s, AdjState* a, hipStream_t st) {
    Gemm g{};
    g.A = a->Fbar.p;
    g.ta = DT_F64;
    g.ra = rows_strided(s->n_chol + 1);
    g.B = a->lht.p;
    g.tb = DT_F64;
    g.rb = rows_strided(s->n_chol + 1);
    g.C = a->thbar.p;
    g.tc = DT_F64;
    g.rc = rows_strided(s->NM());
    g.alpha = 1.0;
    g.m = 2 * s->nw;
    g.n = (int)s->NM();
    g.k = s->n_chol + 1;
    g.batch = 1;
    return gemm(g, a->prec, st);
}

// Reverse of step j of the current segment: phibar / wbar hold the adjoint of
// the state after the step (after its Gram-Schmidt) and receive the adjoint
// of the state before it.
afqmc_status reverse_step(afqmc_sys s, AdjState* a, int j, const double* phi_next,
                          hipStream_t st) {
    const int M = s->M, N = s->N, nw = s->nw, nc = s->n_chol, K = s->par.taylor_order;
    const long NM = s->NM(), rows = 2L * N * nw, nel = rows * M;
    const double sq = sqrt(s->par.dt);
    const DType pr = a->prec;
    double* pb = a->phibar.as<double>();
    const double* phi_in = a->t_phi[j].as<double>();
    const double* phi_out = a->t_mgs[j] ? a->t_pre[j].as<double>() : phi_next;
    uint8_t* mode = a->mode.as<uint8_t>();
    // Gram-Schmidt after the step
    if (a->t_mgs[j]) {
        MgsAdj g{};
        g.pre = phi_out;
        g.q = phi_next;
        g.trialT = s->d_trialT.as<double>();
        g.alive = a->t_aout[j].as<uint8_t>();
        g.phibar = pb;
        g.nw = nw;
        g.M = M;
        g.N = N;
        g.na = s->na;
        g.nb = s->nb;
        HIPCHK(mgs_adjoint(g, st));
    }
    // weight update
    hipLaunchKernelGGL(k_adj_scalars, dim3(nblk(nw, 256)), dim3(256), 0, st,
                       a->t_w[j].as<double>(), a->t_wout[j].as<double>(),
                       a->t_alive[j].as<uint8_t>(), a->t_aout[j].as<uint8_t>(),
                       a->t_lnov[j].as<double>(), a->t_lnd[j].as<double>(),
                       a->t_simp[j].as<double>(), a->wbar.as<double>(), s->par.dt * s->e_shift,
                       a->wbar2.as<double>(), mode, a->lnrb.as<double>(), a->lnib.as<double>(), nw);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_mask, dim3(nblk(nel, 256)), dim3(256), 0, st, pb, mode, 2 * NM, nw);
    // ln <phi_T|phi'> receives ln R_bar
    afqmc_status r = det_adj(s, phi_out, nullptr, a->lnrb.as<double>(), 1.0, mode, pb, st);
    if (r != AFQMC_OK) return r;
    // A of the step (FP64), from the recorded force bias and the regenerated fields
    {
        FieldArgs f{};
        f.F = a->t_F[j].as<double>();
        f.ldf = nc + 1;
        f.a = s->d_a.as<double>();
        f.ext = nullptr;
        f.seed = a->seed;
        f.stream = 0;
        f.t = a->t_t[j];
        f.t_dev = nullptr;
        f.alive = a->t_alive[j].as<uint8_t>();
        f.X = a->xc.p;
        f.tx = DT_F64;
        f.ldx = nc;
        f.s_imp = a->simp_s.as<double>();
        f.nw = nw;
        f.n_chol = nc;
        f.sqdt = sq;
        f.free_proj = 0;
        HIPCHK(fields(f, st));
        HIPCHK(philox_normals(a->seed, 0, a->t_t[j], nw, nc, a->x.as<double>(), st));
        Gemm g{};
        g.A = a->xc.p;
        g.ta = DT_F64;
        g.ra = rows_strided(nc);
        g.B = a->lp64.p;
        g.tb = DT_F64;
        g.rb = rows_strided(nc);
        g.C = a->apk.p;
        g.tc = DT_F64;
        g.rc = rows_strided(s->P());
        g.alpha = 1.0;
        g.m = 2 * nw;
        g.n = (int)s->P();
        g.k = nc;
        g.batch = 1;
        if (nc > 0) HIPCHK(gemm(g, pr, st));
        else HIPCHK(hipMemsetAsync(a->apk.p, 0, a->apk.n, st));
        HIPCHK(unpack_sym(a->apk.p, a->A.p, M, 2 * nw, DT_F64, st));
    }
    const double* A = a->A.as<double>();
    // Taylor tapes, one walker's K terms contiguous: [w][n][2][N][M]
    const long TS = 2 * NM, KTS = (long)K * TS;
    const bool rec = a->t_rec[j];  // the step's propagation recorded them
    double* tt = rec ? a->t_terms[j].as<double>() : a->tT.as<double>();  // t_n, n < K
    double* tb = a->tbT.as<double>();  // t_bar_{n+1} / (n + 1), n < K
    double* y = rec ? a->t_y[j].as<double>() : a->y.as<double>();
    // forward terms: t_0 = P phi_in; t_n = A t_{n-1} / n; y = sum_{n <= K} t_n
    if (!rec)
        HIPCHK(rgemm(s->d_P.as<double>(), phi_in, tt, rows, M, pr, st, rows_2level(2 * N, M, KTS)));
    for (int n = 1; n <= K && !rec; ++n) {
        CTerm c{};
        c.in = tt + (long)(n - 1) * TS;
        c.in_bs = KTS;
        c.A = A;
        c.out = n < K ? tt + (long)n * TS : nullptr;
        c.out_bs = KTS;
        c.acc_in = n == 1 ? tt : y;
        c.acc_in_bs = n == 1 ? KTS : TS;
        c.acc_out = y;
        c.acc_out_bs = TS;
        c.alpha = 1.0 / n;
        c.oscale = 1.0;
        c.nw = nw;
        c.M = M;
        c.N = N;
        HIPCHK(cterm(c, pr, st));
    }
    // dE/dlambda += <phi_bar', dP y>
    HIPCHK(rgemm(a->dP.as<double>(), y, a->z.as<double>(), rows, M, pr, st));
    dot_acc(pb, a->z.as<double>(), mode, 2 * NM, nw, a->part.as<double>(), a->acc.as<double>(),
            0, st);
    // y_bar = P phi_bar'; t_bar_K = y_bar; t_bar_{n-1} = y_bar + conj(A) t_bar_n / n, with
    // t_bar_n / n kept on the tape for A_bar and u_bar = t_bar_0
    double* yb = a->ybar.as<double>();
    double* ub = a->tA.as<double>();
    HIPCHK(rgemm(s->d_P.as<double>(), pb, yb, rows, M, pr, st));
    hipLaunchKernelGGL(k_scale_copy, dim3(nblk((long)nw * TS, 256)), dim3(256), 0, st, yb, TS,
                       tb + (long)(K - 1) * TS, KTS, TS, nw, 1.0 / K);
    HIPCHK(hipGetLastError());
    for (int n = K; n >= 1; --n) {
        CTerm c{};
        c.in = tb + (long)(n - 1) * TS;
        c.in_bs = KTS;
        c.A = A;
        c.conj = 1;
        c.base = yb;
        c.base_bs = TS;
        c.out = n >= 2 ? tb + (long)(n - 2) * TS : ub;
        c.out_bs = n >= 2 ? KTS : TS;
        c.alpha = 1.0;
        c.oscale = n >= 2 ? 1.0 / (n - 1) : 1.0;
        c.nw = nw;
        c.M = M;
        c.N = N;
        HIPCHK(cterm(c, pr, st));
    }
    // A_bar = sum_n (t_bar_n / n) t_{n-1}^H
    {
        CAbar c{};
        c.S = tb;
        c.T = tt;
        c.bs = KTS;
        c.nq = K;
        c.Abar = a->Abar.as<double>();
        c.nw = nw;
        c.M = M;
        c.N = N;
        HIPCHK(cabar(c, pr, st));
    }
    // G = <L_g, A_bar> through the packed upper triangle
    {
        const long P = s->P();
        const int nt = (M + 31) / 32;
        hipLaunchKernelGGL(k_adj_pack, dim3(2 * nw, nt * (nt + 1) / 2), dim3(256), 0, st,
                           a->Abar.as<double>(), a->Abpk.as<double>(), M, nt);
        Gemm g{};
        g.A = a->Abpk.p;
        g.ta = DT_F64;
        g.ra = rows_strided(P);
        g.B = a->lq.p;
        g.tb = DT_F64;
        g.rb = rows_strided(P);
        g.C = a->G.p;
        g.tc = DT_F64;
        g.rc = rows_strided(nc);
        g.alpha = 1.0;
        g.m = 2 * nw;
        g.n = nc;
        g.k = (int)P;
        g.batch = 1;
        if (a->g_ks > 1) {
            g.ksplit = a->g_ks;
            g.ws = a->gws.p;
        }
        if (nc > 0) HIPCHK(gemm(g, pr, st));
    }
    hipLaunchKernelGGL(k_adj_fbar, dim3(nblk((long)nw * (nc + 1), 256)), dim3(256), 0, st,
                       a->t_F[j].as<double>(), nc + 1, s->d_a.as<double>(), a->x.as<double>(),
                       a->G.as<double>(), a->lnrb.as<double>(), a->lnib.as<double>(), mode, sq,
                       a->Fbar.as<double>(), nw, nc);
    HIPCHK(hipGetLastError());
    HIPCHK(fbar_to_thbar(s, a, st));
    // phi_bar (before the step) = P u_bar + Theta / ln-overlap terms
    double* pn = a->phibar2.as<double>();
    HIPCHK(rgemm(s->d_P.as<double>(), ub, pn, rows, M, pr, st));
    HIPCHK(rgemm(a->dP.as<double>(), phi_in, a->z.as<double>(), rows, M, pr, st));
    dot_acc(ub, a->z.as<double>(), mode, 2 * NM, nw, a->part.as<double>(), a->acc.as<double>(),
            0, st);
    r = det_adj(s, phi_in, a->thbar.as<double>(), a->lnrb.as<double>(), -1.0, mode, pn, st);
    if (r != AFQMC_OK) return r;
    hipLaunchKernelGGL(k_mask, dim3(nblk(nel, 256)), dim3(256), 0, st, pn, mode, 2 * NM, nw);
    std::swap(a->phibar.p, a->phibar2.p);
    std::swap(a->wbar.p, a->wbar2.p);
    return AFQMC_OK;
}

// Adjoint of the final mixed energy: phibar / wbar of the end state and the
// explicit h^half term (acc[1]); energy into ebuf[0].
afqmc_status energy_adjoint(afqmc_sys s, AdjState* a, hipStream_t st) {
    const int M = s->M, nw = s->nw, nc = s->n_chol;
    const long NM = s->NM();
    afqmc_status r = measure(s, st);
    if (r != AFQMC_OK) return r;
    hipLaunchKernelGGL(k_energy_adj, dim3(1), dim3(256), 0, st, s->d_el.as<double>(),
                       s->d_w.as<double>(), s->d_alive.as<uint8_t>(), s->d_F.as<double>(), nc + 1,
                       nw, a->wbar.as<double>(), a->scale.as<double>(), a->Fbar.as<double>(),
                       a->mode.as<uint8_t>(), a->ebuf.as<double>());
    HIPCHK(hipGetLastError());
    HIPCHK(fbar_to_thbar(s, a, st));
    // exchange: U = sum_g L^half_g^T T_g^T per spin, T_g = L^half_g Theta, with
    // the FP64 Theta (the lower-precision plans keep only their copy in the step)
    if (s->ts != DT_F64)
        HIPCHK(lu_theta(s->d_phi.as<double>(), s->d_trialT.as<double>(), s->d_theta.as<double>(),
                        nullptr, DT_F64, s->d_lnd.as<double>(), s->d_alive.as<uint8_t>(), nw, M,
                        s->N, s->na, s->nb, s->d_ovl.p, st));
    const double* th = s->d_theta.as<double>();
    for (int sp = 0; sp < 2 && nc > 0; ++sp) {
        const int off = sp ? s->na : 0, n = sp ? s->nb : s->na;
        if (n == 0) continue;
        const long TS = (long)nc * n * n;  // one plane of T for one walker
        for (int p = 0; p < 2; ++p) {
            Gemm g{};
            g.A = s->d_lhx.p;
            g.ta = DT_F64;
            g.ra = rows_2level(n, M, NM, (long)off * M);
            g.B = th + p * NM;
            g.tb = DT_F64;
            g.rb = rows_strided(M, (long)off * M);
            g.b_bs = 2 * NM;
            g.C = a->Tb.as<double>() + p * TS;
            g.tc = DT_F64;
            g.rc = rows_2level(n, (long)nc * n, n);
            g.c_bs = 2 * TS;
            g.alpha = 1.0;
            g.m = nc * n;
            g.n = n;
            g.k = M;
            g.batch = nw;
            HIPCHK(gemm(g, a->prec, st));
            Gemm u{};
            u.A = a->Tb.as<double>() + p * TS;
            u.ta = DT_F64;
            u.ra = rows_strided((long)nc * n);
            u.a_bs = 2 * TS;
            u.B = a->lht2[sp].p;
            u.tb = DT_F64;
            u.rb = rows_strided((long)nc * n);
            u.C = a->U.as<double>() + p * NM;
            u.tc = DT_F64;
            u.rc = rows_strided(M, (long)off * M);
            u.c_bs = 2 * NM;
            u.alpha = 1.0;
            u.m = n;
            u.n = M;
            u.k = nc * n;
            u.batch = nw;
            HIPCHK(gemm(u, a->prec, st));
        }
    }
    if (nc > 0)
        hipLaunchKernelGGL(k_exch_combine, dim3(nblk(2 * NM * nw, 256)), dim3(256), 0, st,
                           a->thbar.as<double>(), a->U.as<double>(), a->scale.as<double>(), NM, nw);
    HIPCHK(hipMemsetAsync(a->phibar.p, 0, a->phibar.n, st));
    r = det_adj(s, s->d_phi.as<double>(), a->thbar.as<double>(), nullptr, 0.0,
                a->mode.as<uint8_t>(), a->phibar.as<double>(), st);
    if (r != AFQMC_OK) return r;
    // explicit term: sum_w (w/W) Re sum_s Tr(V^half_s Theta_s)
    Gemm g{};
    g.A = th;
    g.ta = DT_F64;
    g.ra = rows_strided(NM);
    g.B = a->vhalf.p;
    g.tb = DT_F64;
    g.rb = rows_strided(NM);
    g.C = a->vd.p;
    g.tc = DT_F64;
    g.rc = rows_strided(1);
    g.alpha = 1.0;
    g.m = 2 * nw;
    g.n = 1;
    g.k = (int)NM;
    g.batch = 1;
    HIPCHK(gemm(g, DT_F64, st));
    hipLaunchKernelGGL(k_explicit, dim3(1), dim3(64), 0, st, a->vd.as<double>(),
                       a->scale.as<double>(), nw, a->acc.as<double>(), 1);
    (void)M;
    return AFQMC_OK;
}

}  // namespace

void free_adjoint(afqmc_sys s) {
    delete s->adj;
    s->adj = nullptr;
}

}  // namespace host
}  // namespace afq

extern "C" {

afqmc_status afqmc_adjoint_forward(afqmc_sys s, const double* V, uint64_t seed, int n_steps,
                                   int checkpoint_every, afqmc_prec prec, double* energy) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (!V || n_steps <= 0 || checkpoint_every <= 0)
        return fail(AFQMC_E_INVALID, "need V, n_steps > 0 and checkpoint_every > 0");
    if (prec != AFQMC_FP64 && prec != AFQMC_FP32)
        return fail(AFQMC_E_INVALID, "adjoint precision is AFQMC_FP64 or AFQMC_FP32");
    if (s->par.mode != AFQMC_PHASELESS) return fail(AFQMC_E_STATE, "adjoint needs phaseless mode");
    if (s->n_det > 1) return fail(AFQMC_E_STATE, "adjoint with a multi-determinant trial");
    if (s->par.fb_cap > 0.0 && s->par.caps_enabled)
        return fail(AFQMC_E_STATE, "adjoint of a step with an applied force-bias cap");
    if (std::max(s->na, s->nb) > kMaxSpin) return fail(AFQMC_E_SHAPE, "spin block above 64");
    hipStream_t st = s->ham->stream;
    if (!s->adj) s->adj = new AdjState();
    AdjState* a = s->adj;
    a->ready = false;
    a->n_steps = n_steps;
    a->every = checkpoint_every;
    a->n_seg = (n_steps + checkpoint_every - 1) / checkpoint_every;
    a->seed = seed;
    a->prec = prec == AFQMC_FP64 ? DT_F64 : DT_F32;
    a->V.assign(V, V + (size_t)s->M * s->M);
    if ((r = adj_setup(s, a, st)) != AFQMC_OK) return r;
    if ((int)a->ck.size() < a->n_seg) a->ck.resize(a->n_seg);
    // one segment: the window is recorded now and the reverse pass recomputes
    // nothing; otherwise snapshots only, each segment recorded again in reverse
    a->taped = a->n_seg == 1;
    if (a->taped) {
        tape_resize(a, n_steps);
        plan_record(s, a, n_steps);
    }
    for (int sg = 0; sg < a->n_seg; ++sg) {
        if ((r = snap_take(s, a->ck[sg], st)) != AFQMC_OK) return r;
        const int n = std::min(checkpoint_every, n_steps - sg * checkpoint_every);
        for (int i = 0; i < n; ++i) {
            if (a->taped) {
                if ((r = taped_step(s, a, i, st)) != AFQMC_OK) return r;
                continue;
            }
            if ((r = one_step(s, seed, 0, nullptr, st)) != AFQMC_OK) return r;
            if (s->par.ortho_every > 0 && s->t % s->par.ortho_every == 0)
                if ((r = ortho(s, st)) != AFQMC_OK) return r;
        }
        if (a->taped && (r = tape_end(s, a, n, st)) != AFQMC_OK) return r;
    }
    if ((r = adj_operators(s, a)) != AFQMC_OK) return r;
    if ((r = snap_take(s, a->fin, st)) != AFQMC_OK) return r;
    if ((r = measure(s, st)) != AFQMC_OK) return r;
    double sums[4];
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(sums, s->d_sums.p, sizeof(sums), hipMemcpyDeviceToHost));
    a->E = sums[0] / sums[1];
    if (energy) *energy = a->E;
    a->ready = true;
    return AFQMC_OK;
}

afqmc_status afqmc_adjoint_backward(afqmc_sys s, double* dE) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    AdjState* a = s->adj;
    if (!a || !a->ready) return fail(AFQMC_E_STATE, "no adjoint forward pass on this system");
    if (!dE) return fail(AFQMC_E_INVALID, "dE is null");
    hipStream_t st = s->ham->stream;
    const int k = a->every;
    if (!a->taped) tape_resize(a, k);
    HIPCHK(hipMemsetAsync(a->acc.p, 0, a->acc.n, st));
    // the end state: restore and take the energy adjoint
    if ((r = snap_restore(s, a->fin, st)) != AFQMC_OK) return r;
    if ((r = energy_adjoint(s, a, st)) != AFQMC_OK) return r;
    for (int sg = a->n_seg - 1; sg >= 0; --sg) {
        const int n = std::min(k, a->n_steps - sg * k);
        if (!a->taped) {
            plan_record(s, a, n);
            if ((r = snap_restore(s, a->ck[sg], st)) != AFQMC_OK) return r;
            for (int j = 0; j < n; ++j)
                if ((r = taped_step(s, a, j, st)) != AFQMC_OK) return r;
            if ((r = tape_end(s, a, n, st)) != AFQMC_OK) return r;
        }
        for (int j = n - 1; j >= 0; --j)
            if ((r = reverse_step(s, a, j, a->t_phi[j + 1].as<double>(), st)) != AFQMC_OK)
                return r;
    }
    // leave the system at the end of the window
    if ((r = snap_restore(s, a->fin, st)) != AFQMC_OK) return r;
    double acc[2];
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(acc, a->acc.p, sizeof(acc), hipMemcpyDeviceToHost));
    *dE = acc[0] + acc[1];
    return AFQMC_OK;
}

}  // extern "C"
