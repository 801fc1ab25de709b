// Internal launch interface between the C-ABI host code and the gfx950
// kernels.  Nothing here is part of the public ABI (include/afqmc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace afq {

typedef __bf16 bf16_t;

// Row r of a K-contiguous operand starts at element
//   base + (r / n_in) * s_out + (r % n_in) * s_in
// (a two-level row index: e.g. (walker*2 + plane, orbital) rows of a walker
// block, or (gamma, orbital) rows of the half-rotated Cholesky tensor).
struct RowMap {
    long base;
    int n_in;
    long s_in;
    long s_out;
};

inline RowMap rows_strided(long stride, long base = 0) { return RowMap{base, 1, 0, stride}; }
inline RowMap rows_2level(int n_in, long s_in, long s_out, long base = 0) {
    return RowMap{base, n_in, s_in, s_out};
}

// Storage / compute types.  DT_SPLIT is a compute type only: FP32 operands
// carried as hi + lo BF16 pairs on the BF16 matrix cores.
enum DType { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_SPLIT = 3 };

// C[b][i, j] = alpha * sum_k A[b](i, k) * B[b](j, k) + beta * C[b][i, j]
// A(i, k) = A[b * a_bs + rowA(i) + k], B(j, k) = B[b * b_bs + rowB(j) + k],
// C element (i, j) at c_base + b * c_bs + rowC(i) + j.
// An optional second output C2 (same layout) receives the same values
// (alpha * acc) without the beta term.
struct Gemm {
    const void* A;
    DType ta;
    RowMap ra;
    long a_bs;
    const void* B;
    DType tb;
    RowMap rb;
    long b_bs;
    void* C;
    DType tc;
    RowMap rc;
    long c_bs;
    void* C2;
    double alpha;
    double beta;
    int m, n, k, batch;
    int tile;  // 0: size heuristic; 1: 64 x 64 tiles; 2: 128 x 128; 3: 256 x 128;
               // 4: 256 x 128 over 16 wavefronts (split BF16; else as 3)
    // ksplit > 1: K cut into ksplit ranges of gemm_kchunk(k, ksplit) (the same
    // for every tile shape), partial sums (FP32; FP64 for FP64 compute) into
    // ws[ksplit][m][n] (batch 1), then summed in range order into C
    int ksplit;
    void* ws;
};

// Compute precision of a GEMM (the MFMA input type; accumulation is FP64 for
// DT_F64 and FP32 otherwise).
hipError_t gemm(const Gemm& g, DType compute, hipStream_t s);
int gemm_kchunk(int k, int ksplit);
size_t gemm_ws_bytes(int m, int n, int ksplit, DType compute);

// One complex Taylor term per walker on walker rows (planes [2][N][M], FP64
// storage): C = in op(A)^T, op(A) = A or conj(A) (A complex symmetric,
// [w][2][M][M]), o = (base + alpha C) oscale written to out, and
// acc_out = acc_in + o (acc_in may equal acc_out).  base, out and acc_* are
// optional (NULL; acc_in is required with acc_out); *_bs are walker strides in
// doubles.
struct CTerm {
    const double* in;
    long in_bs;
    const double* A;
    const double* base;
    long base_bs;
    double* out;
    long out_bs;
    const double* acc_in;
    long acc_in_bs;
    double* acc_out;
    long acc_out_bs;
    double alpha, oscale;
    int conj;
    int nw, M, N;
};
hipError_t cterm(const CTerm& c, DType compute, hipStream_t s);

// A_bar[w] = sum_{q < nq} S_q^T conj(T_q): S, T tapes [w][q][2][N][M] (walker
// stride bs), A_bar [w][2][M][M], overwritten.
struct CAbar {
    const double* S;
    const double* T;
    long bs;
    int nq;
    double* Abar;
    int nw, M, N;
};
hipError_t cabar(const CAbar& c, DType compute, hipStream_t s);

// Dense per-(walker, spin) adjoint kernels of spin blocks of up to 64
// orbitals (walker rows [w][2][N][M], trialT [N][M]).
// det_adjoint, for walkers with mode[w] == active:
//   phibar += Y + Phi_T Z,  Z = coef O^{-H} - O^{-H} (Phi^H Theta_bar) O^{-H},
//   Y = Theta_bar O^{-H},  O = Phi_T^T Phi,  coef = cscale coef[w] (complex)
// (thbar NULL: Y = 0, no Theta_bar term; coef NULL: 0).  A walker whose
// overlap has a zero pivot is left unchanged.
struct DetAdj {
    const double* phi;
    const double* trialT;
    const double* thbar;
    const double* coef;
    double cscale;
    const uint8_t* mode;
    uint8_t active;
    double* phibar;
    int nw, M, N, na, nb;
};
hipError_t det_adjoint(const DetAdj& a, hipStream_t s);
// mgs_adjoint, for walkers with alive[w]: phibar <- phibar S^H,
// S = O(pre)^{-1} O(q), O(X) = Phi_T^T X.
struct MgsAdj {
    const double* pre;
    const double* q;
    const double* trialT;
    const uint8_t* alive;
    double* phibar;
    int nw, M, N, na, nb;
};
hipError_t mgs_adjoint(const MgsAdj& a, hipStream_t s);
// Raise both kernels' LDS limit to what 64-orbital blocks need (once, outside
// graph capture).
hipError_t dense_adj_prepare();

// Fragment-tiled layout of an M x M operand of the split-BF16 propagation:
// rows padded to 16 (MT), columns to 32 (MP), stored as 1 KB tiles of 16 rows
// x 32 columns ordered [row block][column chunk], inside a tile element
// (16 rows, 8 column runs) at ((c % 32) / 8 * 16 + r % 16) * 8 + c % 8, so
// that lane l of a wave reads row l % 16, columns 8 (l / 16) .. + 7 of a
// chunk with one 16-byte load and a wave's load is 1 KB contiguous.
// Padding elements are zero.
__host__ __device__ inline long split_tile_elems(int M) {
    return (long)((M + 15) / 16 * 16) * ((M + 31) / 32 * 32);
}
__host__ __device__ inline long split_tile_index(int M, int r, int c) {
    const long kc = (M + 31) / 32;
    return ((r / 16 * kc + c / 32) * 64 + (c % 32) / 8 * 16 + r % 16) * 8 + c % 8;
}

// Packed upper triangle (P = M(M+1)/2 per plane) -> full symmetric M x M,
// for `planes` consecutive planes (types DT_F64 / DT_F32 row-major;
// DT_SPLIT: FP32 input, hi/lo BF16 output planes [plane][hi, lo][tiles] in
// the fragment-tiled layout, M <= 256).
hipError_t unpack_sym(const void* pk, void* full, int M, int planes, DType t, hipStream_t s);
// LDS limit of the one-plane split unpack (the packed triangle of M = 256);
// unpack_prepare raises the kernel's dynamic LDS limit to it (call once,
// outside graph capture).
constexpr size_t kUnpackLds = 160 * 1024;
hipError_t unpack_prepare();
// FP32 planes of n elements -> hi/lo BF16 planes [plane][hi, lo][n].
hipError_t split_planes(const float* in, void* out, long n, long planes, hipStream_t s);

// Fused propagation of every walker (Eq. 3 and Eq. 11):
//   Phi_out[w] = P T_K(A_w) P Phi[w],  T_K(A) = sum_{n <= K} A^n / n!
// phi, phi_out: FP64 walker blocks [w][plane][N][M]; Pm: M x M real
// symmetric, Af: [w][plane][M][M] complex symmetric, both in type t
// (DT_F64 or DT_F32, the product precision).  ta: type of Af, equal to t,
// or DT_SPLIT with t == DT_F32: every product in split BF16, Af as hi/lo
// planes [w][plane][hi, lo][tiles] and Pm holding Q = P - I as hi/lo planes
// [hi, lo][tiles], both in the fragment-tiled layout (P y computed as
// y + Q y).  Frozen walkers (live == 0)
// are copied unchanged.  M <= 256.  `variant` selects the workgroup shape
// (waves per workgroup x column blocks per wave, with or without B prefetch,
// one, two or five row blocks per workgroup; see kPropShapes); every variant gives
// bitwise the same result, 0 is the default.
constexpr int kPropVariants = 14;
bool propagate_variant_ok(int variant, int M, DType t, DType ta);
// Optional record of the Taylor series (the FP64 / FP32 products only; the
// split-BF16 propagation refuses it): terms t_0 = P Phi, t_n = A t_{n-1} / n
// for n < K at terms + w bs_walker + n bs_slot, and y = sum_{n <= K} t_n at
// y + w 2 N M, all in the walker row layout [2][N][M] (FP64); frozen walkers
// record zeros.  NULL pointers: nothing recorded.
struct Record {
    double* terms = nullptr;
    long bs_walker = 0, bs_slot = 0;
    double* y = nullptr;
};
hipError_t propagate(const double* phi, double* phi_out, const void* Pm, const void* Af,
                     const uint8_t* live, int nw, int M, int N, int K, DType t, DType ta,
                     int variant, hipStream_t s, const Record& rec = Record());

// Exchange partial sums of the mixed local energy:
//   out[(w * 2 + spin) * n_gtiles + gt] = sum over gamma in tile gt of
//   sum_ij T_ij T_ji,  T = L^half_{gamma, spin} Theta^spin_w   (complex, 2 doubles)
// lhalf: [(n_chol + 1)][N][M] in type t (last row unused here);
// theta: [w][plane][N][M] in type t.  exchange_gtiles: the slot count of a
// spin block for the kernel exchange() launches (depends on nsig, M and t).
hipError_t exchange(const void* lhalf, const void* theta, double* out, int nw, int M, int N,
                    int n_chol, int off, int nsig, int spin, int n_gtiles_alloc, DType t,
                    hipStream_t s);
int exchange_gtiles(int n_chol, int nsig, int M, DType t);

// ---------------------------------------------------------------- walker-wise
struct FieldArgs {
    const double* F;      // [w][2][ldf]  force-bias traces f_g (re, im), gamma < n_chol
    int ldf;
    const double* a;      // [n_chol] mean-field shift a_g
    const double* ext;    // NULL or external fields for this step: [nw][n_chol]
    uint64_t seed, stream;
    int64_t t;            // absolute step (Philox counter word), or an offset
    const int64_t* t_dev; // non-NULL: step = *t_dev + t (device-side step counter)
    const uint8_t* alive;
    void* X;              // [w][2][ldx] field-sum coefficients, type tx
    DType tx;
    int ldx;
    double* s_imp;        // [w][4]: s (re, im), importance exponent (re, im)
    int nw, n_chol;
    double sqdt;
    int free_proj;        // 1: xbar = 0 (free projection)
    // optional force-bias cap: with fb_cap > 0 every live walker's xbar_g
    // with |xbar_g| > fb_cap adds one to cap_count[w] (one entry per walker,
    // owned by its wavefront), and with cap_apply it is scaled to modulus
    // fb_cap (same phase)
    double fb_cap;
    int cap_apply;
    int64_t* cap_count;
};
hipError_t fields(const FieldArgs& f, hipStream_t s);

hipError_t philox_normals(uint64_t seed, uint64_t stream, int64_t t, int nw, int n_chol,
                          double* out, hipStream_t s);

// Per walker and spin block: the overlap O = Phi_T^T Phi (trialT: [N][M],
// rows = trial orbitals), ln det O (lnd[w][spin] complex) and
// Theta = Phi O^{-1}, [w][2][N][M]: with theta_lp NULL the FP64 Theta into
// theta (FP64 matrix-core products); otherwise Theta in type tlp (DT_F32 or
// DT_BF16) into theta_lp from FP32 matrix-core products of the rounded FP64
// operands, theta untouched for spin blocks of at most 48 orbitals (49..64:
// both written).  Spin blocks of at most 64 orbitals.
// ws: workspace of lu_theta_ws_bytes(nw, na, nb) bytes (the overlap matrices).
hipError_t lu_theta(const double* phi, const double* trialT, double* theta, void* theta_lp,
                    DType tlp, double* lnd, const uint8_t* live, int nw, int M, int N, int na,
                    int nb, void* ws, hipStream_t s);
size_t lu_theta_ws_bytes(int nw, int na, int nb);

// Weight update: lnR = sum_s lnd - lnov + s; lnI = lnR + imp;
// phaseless: w *= exp(Re lnI + shift) max(0, cos Im lnR), frozen when not
// > 0; free: complex W *= exp(lnR + shift).  shift = dt * e_shift is the
// constant energy shift of the system.  lnov <- sum_s lnd for live walkers.
// commit == 0 (after Gram-Schmidt): only lnov is refreshed.
hipError_t weights(const double* lnd, const double* s_imp, double* lnov, double* w, uint8_t* alive,
                   int nw, int mode, int commit, double shift, hipStream_t s);

// Orthonormalize every spin block of every live walker in place (the QR
// factor Q with positive diagonal R, as modified Gram-Schmidt gives it):
// blocks of at most 48 orbitals through the Gram matrix and its Cholesky
// factor (ws: lu_theta_ws_bytes bytes), larger ones column by column.  mon
// (or NULL): [w][spin][2] record of the largest loss of orthogonality
// max_k 1/2 ln(S_kk / D_k) and the largest |ln |det R|| seen by each block.
hipError_t mgs(double* phi, const uint8_t* live, int nw, int M, int N, int na, int nb, void* ws,
               double* mon, hipStream_t s);

// E_L[w] (complex) from F (f_g and the one-body trace at column n_chol) and
// the exchange partials.
hipError_t local_energy(const double* F, int ldf, const double* exch, int n_gt_a, int n_gt_b,
                        int nw, int n_chol, double e_core, double* el, hipStream_t s);

// out[0] = sum_w alive w Re E_L, out[1] = sum_w alive w (phaseless); free
// mode: out[0..3] = sum W E_L (re, im), sum W (re, im).
hipError_t mixed_sums(const double* el, const double* w, const uint8_t* alive, int nw, int mode,
                      double* out, hipStream_t s);

// Population control by the comb (one workgroup): csum (nw doubles) and sel
// (nw ints) are workspaces; w and alive become the new population's weights
// (W / nw) and flags; sel[j] = walker copied into slot j.  status[0] = 1 when
// no walker has positive weight (then nothing is changed).
hipError_t comb_select(double* w, uint8_t* alive, int nw, double xi, double* csum, int* sel,
                       int* status, hipStream_t s);
// dst walker j <- src walker sel[j], `per` doubles per walker.
hipError_t gather_walkers(const double* src, double* dst, const int* sel, int nw, long per,
                          hipStream_t s);
// Secondary walkers from primary ones: per walker and plane, rows
// 0..na_sec-1 from the primary's alpha rows, the rest from its beta rows.
hipError_t take_columns(const double* pri, double* sec, int nw, int M, int n_pri, int na_pri,
                        int n_sec, int na_sec, hipStream_t s);
// w_sec = w_pri |r| max(0, cos arg r), r = exp(lnov_sec - lnov_pri); alive
// cleared where the result is not positive.
hipError_t secondary_weights(const double* w_pri, const double* lnov_pri, const double* lnov_sec,
                             double* w_sec, uint8_t* alive, int nw, hipStream_t s);

// Multi-determinant trial: per walker, the combined ln <phi_T|phi> =
// ln sum_i c_i exp(ln det_i) into lnd_out[w][0..1] (zeros in [2..3]) and the
// weights r_i = c_i <D_i|phi> / <phi_T|phi> into rw[w][i][re, im], from the
// per-determinant, per-spin ln dets lnd_all[i][w][4] (frozen walkers skipped).
hipError_t msd_overlap(const double* lnd_all, const double* coef, int n_det, const uint8_t* alive,
                       int nw, double* lnd_out, double* rw, hipStream_t s);
// out[w][re, im][j] = sum_i r_i in_i[w][re, im][j], in_i = in_all + i det_stride.
hipError_t msd_combine(const double* in_all, long det_stride, const double* rw, int n_det,
                       const uint8_t* alive, int nw, int ld, double* out, hipStream_t s);

// Small helpers.
hipError_t broadcast(const double* src, double* dst, long n, int copies, hipStream_t s);
hipError_t convert(const double* src, void* dst, DType t, long n, hipStream_t s);
hipError_t pack_chol(const double* L, void* Lp, DType t, int M, int n_chol, hipStream_t s);
hipError_t permute_chol(const double* L, double* LT, int M, int n_chol, hipStream_t s);
hipError_t chol_weighted_sum(const double* L, const double* a, double* out, int M, int n_chol,
                             hipStream_t s);
// trace[slot] = (E_a, E_b, E_b - E_a).  With device counters ctr (non-NULL)
// the row is written at ((double*)ctr[2])[3 * (pair * ctr[3] + ctr[1] + slot)]
// instead (trace ignored).
hipError_t trace_record(const double* sums_a, const double* sums_b, double* trace, int slot,
                        const int64_t* ctr, int pair, int mode, hipStream_t s);
// Device counters of a replayed graph: ctr[0] step, ctr[1] measurement slot,
// ctr[2] trace address, ctr[3] trace rows per pair.
hipError_t set_counters(int64_t* ctr, int64_t c0, int64_t c1, int64_t c2, int64_t c3,
                        hipStream_t s);
// ctr[0] += d0; ctr[1] += d1.
hipError_t advance_counters(int64_t* ctr, int64_t d0, int64_t d1, hipStream_t s);

}  // namespace afq
