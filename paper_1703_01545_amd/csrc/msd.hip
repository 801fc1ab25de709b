// Multi-determinant trial (Sec. II.D, the CASSCF trial): the per-walker
// combination of quantities computed against each determinant D_i of
// phi_T = sum_i c_i D_i.
//
//   <phi_T|phi> = sum_i c_i <D_i|phi>,     r_i = c_i <D_i|phi> / <phi_T|phi>,
//   f_g = sum_i r_i f_g^(i),               E_L = sum_i r_i E_L^(i),
//
// with f^(i) and E_L^(i) the single-determinant force-bias traces and local
// energy against D_i.  The sums run over i in order.
#include <math.h>

#include "internal.h"

namespace afq {
namespace {

// One thread per walker.  lnd_all[i][w][4]: ln det of determinant i per spin
// (re, im, re, im).  Writes the combined ln <phi_T|phi> to lnd_out[w][0..1]
// (zeros in [2..3], so the weight kernel's spin sum reads it unchanged) and
// r_i to rw[w][i][2].  Frozen walkers are skipped.
__global__ void k_msd_overlap(const double* __restrict__ lnd_all, const double* __restrict__ coef,
                              int n_det, const uint8_t* __restrict__ alive, int nw,
                              double* __restrict__ lnd_out, double* __restrict__ rw) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw || !alive[w]) return;
    const long stride = (long)nw * 4;
    double top = -INFINITY;
    for (int i = 0; i < n_det; ++i) {
        const double* l = lnd_all + i * stride + (long)w * 4;
        top = fmax(top, l[0] + l[2]);
    }
    double tr = 0.0, ti = 0.0;
    for (int i = 0; i < n_det; ++i) {
        const double* l = lnd_all + i * stride + (long)w * 4;
        const double e = exp((l[0] + l[2]) - top), ph = l[1] + l[3];
        const double xr = coef[i] * (e * cos(ph)), xi = coef[i] * (e * sin(ph));
        rw[((long)w * n_det + i) * 2] = xr;
        rw[((long)w * n_det + i) * 2 + 1] = xi;
        tr += xr;
        ti += xi;
    }
    const double den = tr * tr + ti * ti;
    for (int i = 0; i < n_det; ++i) {
        double* r = rw + ((long)w * n_det + i) * 2;
        const double xr = r[0], xi = r[1];
        r[0] = (xr * tr + xi * ti) / den;
        r[1] = (xi * tr - xr * ti) / den;
    }
    double* o = lnd_out + (long)w * 4;
    o[0] = log(hypot(tr, ti)) + top;
    o[1] = atan2(ti, tr);
    o[2] = 0.0;
    o[3] = 0.0;
}

// out[w][re, im][j] = sum_i r_i in_i[w][re, im][j] for j < ld (complex
// products); grid (columns, walkers).
__global__ void k_msd_combine(const double* __restrict__ in_all, long det_stride,
                              const double* __restrict__ rw, int n_det,
                              const uint8_t* __restrict__ alive, int nw, int ld,
                              double* __restrict__ out) {
    const int w = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw || j >= ld || !alive[w]) return;
    double re = 0.0, im = 0.0;
    for (int i = 0; i < n_det; ++i) {
        const double* x = in_all + i * det_stride + (long)w * 2 * ld;
        const double rr = rw[((long)w * n_det + i) * 2], ri = rw[((long)w * n_det + i) * 2 + 1];
        const double fr = x[j], fi = x[ld + j];
        re += rr * fr - ri * fi;
        im += rr * fi + ri * fr;
    }
    out[(long)w * 2 * ld + j] = re;
    out[(long)w * 2 * ld + ld + j] = im;
}

}  // namespace

hipError_t msd_overlap(const double* lnd_all, const double* coef, int n_det, const uint8_t* alive,
                       int nw, double* lnd_out, double* rw, hipStream_t s) {
    hipLaunchKernelGGL(k_msd_overlap, dim3((nw + 255) / 256), dim3(256), 0, s, lnd_all, coef,
                       n_det, alive, nw, lnd_out, rw);
    return hipGetLastError();
}

hipError_t msd_combine(const double* in_all, long det_stride, const double* rw, int n_det,
                       const uint8_t* alive, int nw, int ld, double* out, hipStream_t s) {
    if (nw <= 0 || ld <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_msd_combine, dim3((ld + 255) / 256, nw), dim3(256), 0, s, in_all,
                       det_stride, rw, n_det, alive, nw, ld, out);
    return hipGetLastError();
}

}  // namespace afq
