// Population control by the comb and the start of the secondary system in
// the preliminary equilibration scheme (Sec. II.B).
//
// Comb: with C the running sum of the live weights in walker order and
// W = C[nw - 1], new walker j copies the first walker k with
// C[k] > (j + xi) W / nw, and every new walker is live with weight W / nw.
// The running sum is taken by one thread in walker order, so the selection is
// a pure function of the weights and xi (no dependence on a reduction tree).
//
// Secondary start: the secondary system's walkers take the primary's
// determinants (the first n_alpha and n_beta columns of each spin block),
// and their weights become w_pri |r| max(0, cos arg r) with
// r = <phi_T^sec|phi> / <phi_T^pri|phi>.
#include <math.h>

#include "internal.h"

namespace afq {
namespace {

// One workgroup.  Thread 0 forms the running sum (csum) and the last walker
// of positive weight; then every thread places its share of the nw comb
// points by bisection.  w and alive are overwritten with the new population's
// weights (W / nw) and flags only after the barrier that ends the reads.
// status[0] = 1 when no walker has positive weight (nothing changed).
__global__ __launch_bounds__(256) void k_comb_select(double* __restrict__ w,
                                                     uint8_t* __restrict__ alive, int nw, double xi,
                                                     double* __restrict__ csum,
                                                     int* __restrict__ sel,
                                                     int* __restrict__ status) {
    __shared__ double W_s;
    __shared__ int last_s;
    if (threadIdx.x == 0) {
        double c = 0.0;
        int last = -1;
        for (int k = 0; k < nw; ++k) {
            const double v = alive[k] ? w[k] : 0.0;
            c = c + v;
            csum[k] = c;
            if (v > 0.0) last = k;
        }
        W_s = c;
        last_s = last;
        status[0] = (last < 0 || !(c > 0.0)) ? 1 : 0;
    }
    __threadfence_block();
    __syncthreads();
    const double W = W_s;
    const int last = last_s;
    if (last < 0 || !(W > 0.0)) return;
    const double wn = W / (double)nw;
    for (int j = threadIdx.x; j < nw; j += blockDim.x) {
        const double z = ((double)j + xi) * W / (double)nw;
        int lo = 0, hi = nw;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (csum[mid] > z)
                hi = mid;
            else
                lo = mid + 1;
        }
        sel[j] = lo < nw ? lo : last;
        w[j] = wn;
        alive[j] = 1;
    }
}

// dst walker j <- src walker sel[j] (`per` doubles per walker); one
// workgroup per walker.
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ src,
                                                double* __restrict__ dst,
                                                const int* __restrict__ sel, long per) {
    const long j = blockIdx.x;
    const double* s = src + (long)sel[j] * per;
    double* d = dst + j * per;
    for (long e = threadIdx.x; e < per; e += blockDim.x) d[e] = s[e];
}

// Secondary walker k, plane p, orbital row i <- primary row i (alpha block)
// or n_alpha_pri + (i - n_alpha_sec) (beta block).  grid (rows, walkers).
__global__ __launch_bounds__(256) void k_take_columns(const double* __restrict__ pri,
                                                      double* __restrict__ sec, int M, int n_pri,
                                                      int na_pri, int n_sec, int na_sec) {
    const int i = blockIdx.x, k = blockIdx.y;
    const int ip = i < na_sec ? i : na_pri + (i - na_sec);
    for (int p = 0; p < 2; ++p) {
        const double* s = pri + ((long)k * 2 + p) * n_pri * M + (long)ip * M;
        double* d = sec + ((long)k * 2 + p) * n_sec * M + (long)i * M;
        for (int m = threadIdx.x; m < M; m += blockDim.x) d[m] = s[m];
    }
}

__global__ void k_secondary_weights(const double* __restrict__ w_pri,
                                    const double* __restrict__ lnov_pri,
                                    const double* __restrict__ lnov_sec,
                                    double* __restrict__ w_sec, uint8_t* __restrict__ alive,
                                    int nw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nw) return;
    if (!alive[k]) {
        w_sec[k] = 0.0;
        return;
    }
    const double lr = lnov_sec[2 * k] - lnov_pri[2 * k];
    const double li = lnov_sec[2 * k + 1] - lnov_pri[2 * k + 1];
    const double v = w_pri[k] * exp(lr) * fmax(0.0, cos(li));
    const bool ok = isfinite(v) && v > 0.0;
    w_sec[k] = ok ? v : 0.0;
    if (!ok) alive[k] = 0;
}

}  // namespace

hipError_t comb_select(double* w, uint8_t* alive, int nw, double xi, double* csum, int* sel,
                       int* status, hipStream_t s) {
    hipLaunchKernelGGL(k_comb_select, dim3(1), dim3(256), 0, s, w, alive, nw, xi, csum, sel,
                       status);
    return hipGetLastError();
}

hipError_t gather_walkers(const double* src, double* dst, const int* sel, int nw, long per,
                          hipStream_t s) {
    if (nw <= 0 || per <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(nw), dim3(256), 0, s, src, dst, sel, per);
    return hipGetLastError();
}

hipError_t take_columns(const double* pri, double* sec, int nw, int M, int n_pri, int na_pri,
                        int n_sec, int na_sec, hipStream_t s) {
    if (nw <= 0 || n_sec <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_take_columns, dim3(n_sec, nw), dim3(256), 0, s, pri, sec, M, n_pri,
                       na_pri, n_sec, na_sec);
    return hipGetLastError();
}

hipError_t secondary_weights(const double* w_pri, const double* lnov_pri, const double* lnov_sec,
                             double* w_sec, uint8_t* alive, int nw, hipStream_t s) {
    hipLaunchKernelGGL(k_secondary_weights, dim3((nw + 255) / 256), dim3(256), 0, s, w_pri,
                       lnov_pri, lnov_sec, w_sec, alive, nw);
    return hipGetLastError();
}

}  // namespace afq
