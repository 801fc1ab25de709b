// Allocation-free variant of the correlated pair step, for callers that
// cannot allocate device memory during a call (HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).  The only memory afqmc_pair_step
// allocates per call is the device staging of the energy-trace rows; here
// those rows live in a file-scope device array.
#include <mutex>
#include <string>

#include "host.h"

using namespace afq;
using namespace afq::host;

namespace {

// Staging rows of the energy trace: each GPU holds its own copy for the life
// of the process.  In host code this name is not a device address; the
// address comes from hipGetSymbolAddress on that device.
__device__ __align__(256) double scratch[AFQMC_NOALLOC_MAX_MEASUREMENTS * 3];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
afqmc_status trace_scratch(double** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(AFQMC_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(AFQMC_E_DEVICE, "hipGetSymbolAddress returned null for the scratch array");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return AFQMC_OK;
}

}  // namespace

extern "C" {

afqmc_status afqmc_pair_step_noalloc(afqmc_sys a, afqmc_sys b, uint64_t seed, int n_steps,
                                     const double* fields_dev, double* e_trace) {
    int n_meas = 0;
    afqmc_status r = pair_check(a, b, n_steps, &n_meas);
    if (r != AFQMC_OK) return r;
    if (n_meas > AFQMC_NOALLOC_MAX_MEASUREMENTS)
        return fail(AFQMC_E_INVALID, "afqmc_pair_step_noalloc: " + std::to_string(n_meas) +
                                         " measurements exceed the staging limit of " +
                                         std::to_string(AFQMC_NOALLOC_MAX_MEASUREMENTS) +
                                         " per call");
    if (a->prof.on || b->prof.on)
        return fail(AFQMC_E_STATE, "afqmc_pair_step_noalloc: profiling creates events; disable it");
    double* staging = nullptr;
    if ((r = trace_scratch(&staging)) != AFQMC_OK) return r;
    return pair_run(a, b, seed, n_steps, fields_dev, e_trace, staging, n_meas);
}

}  // extern "C"
