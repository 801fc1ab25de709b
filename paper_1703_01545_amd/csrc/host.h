// Host-side state shared by the C-ABI translation units: handles, device
// buffers, the phase profiler and the device phases of one step.  Private to
// the library (the public interface is include/afqmc.h).
#pragma once

#include <math.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "../../include/afqmc.h"
#include "internal.h"

namespace afq {
namespace host {

// Message of the last non-OK status of this thread (afqmc_last_error).
extern thread_local std::string g_err;

inline afqmc_status fail(afqmc_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(AFQMC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline size_t dt_size(DType t) { return t == DT_F64 ? 8 : (t == DT_F32 ? 4 : 2); }

// Owning device allocation: move-only, so that containers that grow (the
// tape and snapshot vectors) move buffers instead of freeing copies of them.
struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) {
        o.p = nullptr;
        o.n = 0;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t bytes) {
        release();
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) n = bytes;
        return e;
    }
    template <typename T>
    T* as() const { return (T*)p; }
};

// profiling is enabled.
enum Phase {
    PH_FORCE_BIAS = 0,
    PH_FIELDS,
    PH_FIELD_SUM,
    PH_UNPACK,
    PH_PROPAGATE,
    PH_DET_THETA,
    PH_WEIGHTS,
    PH_MGS,
    PH_EXCHANGE,
    PH_ENERGY,
    PH_COUNT
};
extern const char* const kPhaseNames[PH_COUNT];
struct Profiler {
    bool on = false;
    struct Pend {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Pend> pend;
    std::vector<hipEvent_t> pool;
    double total_ms[PH_COUNT] = {};
    int64_t launches[PH_COUNT] = {};
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipError_t resolve(hipStream_t st) {
        if (pend.empty()) return hipSuccess;
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        for (auto& p : pend) {
            float ms = 0.f;
            if (p.a && p.b && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                total_ms[p.phase] += ms;
                launches[p.phase] += 1;
            }
            if (p.a) pool.push_back(p.a);
            if (p.b) pool.push_back(p.b);
        }
        pend.clear();
        return hipSuccess;
    }
    void reset() {
        for (int i = 0; i < PH_COUNT; ++i) {
            total_ms[i] = 0.0;
            launches[i] = 0;
        }
    }
    ~Profiler() {
        for (auto& p : pend) {
            if (p.a) (void)hipEventDestroy(p.a);
            if (p.b) (void)hipEventDestroy(p.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
struct AdjState;

}  // namespace host
}  // namespace afq

struct afqmc_ham_s {
    int M = 0, n_chol = 0;
    double e_core = 0.0;
    hipStream_t stream = nullptr;
    uint64_t chol_hash = 0;
    std::vector<double> h;
    afq::host::DevBuf d_h, d_chol;
    afq::host::DevBuf d_lp[4];  // packed L^T per storage type: [P][n_chol]
    int refs = 1;
    bool released = false;
};

struct afqmc_sys_s {
    afqmc_ham ham = nullptr;
    int M = 0, n_chol = 0, na = 0, nb = 0, N = 0, nw = 0;
    afqmc_params par{};
    afq::DType ts = afq::DT_F64;  // storage type of the contraction operands (L^half, Theta, X, L)
    afq::DType tc = afq::DT_F64;  // compute type of the contractions (DT_SPLIT: split BF16)
    afq::DType tp = afq::DT_F64;  // propagator product type (FP64 or FP32)
    afq::DType ta = afq::DT_F64;  // Taylor operand A_w: tp, or DT_SPLIT (hi/lo BF16 planes)
    int64_t t = 0;
    double e_shift = 0.0;  // constant energy shift of the weight factor
    bool dead = false;
    std::vector<double> a_host;
    std::vector<double> htilde;  // one-body part after the mean-field subtraction (host copy)
    afq::host::AdjState* adj = nullptr;  // reverse-mode tape (adjoint.hip)
    afq::Record rec;  // Taylor terms the next propagation records (set only by the adjoint)
    // constant per-system data
    // d_Plp: P in FP32, or with ta == DT_SPLIT Q = P - I as hi/lo BF16 planes
    // in the fragment-tiled layout (split_tile_elems(M) * 4 bytes)
    afq::host::DevBuf d_trialT, d_P, d_Plp, d_a, d_lhx, d_lhx_lp;
    // walker state
    afq::host::DevBuf d_phi, d_phinew, d_theta, d_theta_lp, d_w, d_lnov, d_alive;
    // step scratch
    afq::host::DevBuf d_F, d_X, d_simp, d_Apk, d_Af, d_lnd, d_exch, d_el, d_sums;
    afq::host::DevBuf d_ovl;  // overlap matrices of the determinant kernels
    afq::host::DevBuf d_kws;  // split-K partial sums of the force-bias GEMM
    afq::host::DevBuf d_pc;   // comb workspace: running sums, selection, status
    afq::host::DevBuf d_capcount;  // force-bias cap events per walker (int64)
    afq::host::DevBuf d_gsmon;     // Gram-Schmidt monitor [w][spin][ell, |ln det R|]
    // Multi-determinant trial (Sec. II.D): determinant 0 uses d_trialT, d_lhx,
    // d_lhx_lp, d_theta, d_theta_lp and d_exch; determinants 1.. their own
    // buffers in xdet.  With n_det > 1 the per-determinant ln dets, force-bias
    // traces and local energies go to d_lnd_all, d_F_all and d_el_all, and
    // d_lnd, d_F, d_el hold the combined values the step reads; d_rw holds
    // r_i = c_i <D_i|phi> / <phi_T|phi> per walker.
    int n_det = 1;
    struct DetBufs {
        afq::host::DevBuf trialT, lhx, lhx_lp, theta, theta_lp, exch;
    };
    std::vector<std::unique_ptr<DetBufs>> xdet;
    afq::host::DevBuf d_coef, d_lnd_all, d_F_all, d_el_all, d_rw;
    int n_gt_a = 0, n_gt_b = 0, n_gt = 0;
    // launch shapes (autotuned; 0 = size heuristic): GEMM tiles of the force
    // bias and the field sum, and the propagation workgroup shape
    int tile_fb = 0, tile_fs = 0, prop_var = 0;
    int fb_ks = 1;  // K ranges of the force-bias GEMM (fb_ksplit at creation)
    // graph capture: the Philox step word is read from *t_dev (plus the
    // step's offset t - t_base) instead of being baked into the launch
    const int64_t* t_dev = nullptr;
    int64_t t_base = 0;
    uint64_t id = 0;  // unique per handle (keys of cached batch graphs)
    afq::host::Profiler prof;
    long P() const { return (long)M * (M + 1) / 2; }
    long NM() const { return (long)N * M; }
};

namespace afq {
namespace host {

inline afqmc_status check_sys(afqmc_sys s) {
    if (!s) return fail(AFQMC_E_INVALID, "null system handle");
    if (s->dead) return fail(AFQMC_E_STATE, "system handle already freed");
    return AFQMC_OK;
}

inline void ham_unref(afqmc_ham h) {
    if (--h->refs == 0) delete h;
}

inline const void* lp_or(const DevBuf& lp, const DevBuf& hi, DType t) { return t == DT_F64 ? hi.p : lp.p; }  // by storage type

// Per-determinant buffers of the trial expansion (determinant 0: the
// system's own).
inline const DevBuf& det_trialT(afqmc_sys s, int i) { return i ? s->xdet[i - 1]->trialT : s->d_trialT; }
inline const DevBuf& det_lhx(afqmc_sys s, int i) { return i ? s->xdet[i - 1]->lhx : s->d_lhx; }
inline const DevBuf& det_lhx_lp(afqmc_sys s, int i) { return i ? s->xdet[i - 1]->lhx_lp : s->d_lhx_lp; }
inline const DevBuf& det_theta(afqmc_sys s, int i) { return i ? s->xdet[i - 1]->theta : s->d_theta; }
inline const DevBuf& det_theta_lp(afqmc_sys s, int i) { return i ? s->xdet[i - 1]->theta_lp : s->d_theta_lp; }
inline const DevBuf& det_exch(afqmc_sys s, int i) { return i ? s->xdet[i - 1]->exch : s->d_exch; }
// where determinant i's ln dets, force-bias traces and local energies go
inline double* det_lnd(afqmc_sys s, int i) {
    return s->n_det > 1 ? s->d_lnd_all.as<double>() + (size_t)i * s->nw * 4 : s->d_lnd.as<double>();
}
inline double* det_F(afqmc_sys s, int i) {
    return s->n_det > 1 ? s->d_F_all.as<double>() + (size_t)i * s->nw * 2 * (s->n_chol + 1)
                        : s->d_F.as<double>();
}
inline double* det_el(afqmc_sys s, int i) {
    return s->n_det > 1 ? s->d_el_all.as<double>() + (size_t)i * s->nw * 2 : s->d_el.as<double>();
}

// Brackets one phase with a pair of HIP events when profiling is on.
struct PhaseTimer {
    Profiler* p;
    hipStream_t st;
    int phase;
    hipEvent_t a = nullptr;
    PhaseTimer(afqmc_sys s, int ph, hipStream_t stream) : p(&s->prof), st(stream), phase(ph) {
        if (p->on) {
            a = p->get();
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~PhaseTimer() {
        if (p->on && a) {
            hipEvent_t b = p->get();
            if (b) (void)hipEventRecord(b, st);
            p->pend.push_back({phase, a, b});
        }
    }
};

// ---- device phases of one step -------------------------------------------

// GEMM descriptors of the contraction phases (their tile from the system's
// tuned shapes).
// K ranges of the force-bias GEMM for K = k: 1 below K = 8000 (K / 4000 up to
// 8 between), else about one per 1800 K, 4..12.  It depends on K alone, so a
// walker's force bias has the same bits whatever the walker count, the batch
// or the device, and it does not depend on the tile the autotuner picks.
int fb_ksplit(int k);
Gemm force_bias_gemm(afqmc_sys s, int det = 0);
Gemm field_sum_gemm(afqmc_sys s);

// Device phases of one step of one system on stream st (Sec. II.A, II.D).
afqmc_status force_bias(afqmc_sys s, hipStream_t st);
afqmc_status overlap_theta(afqmc_sys s, double* phi, hipStream_t st);
afqmc_status one_step(afqmc_sys s, uint64_t seed, uint64_t stream_id, const double* ext,
                      hipStream_t st);
afqmc_status ortho(afqmc_sys s, hipStream_t st);
afqmc_status measure(afqmc_sys s, hipStream_t st);
// Validation shared by the pair entry points (*n_meas: measurements among
// the n_steps), and the steps of a correlated pair with the measurement rows
// staged in the device array `trace` (n_meas x 3), then copied to e_trace.
afqmc_status pair_check(afqmc_sys a, afqmc_sys b, int n_steps, int* n_meas);
afqmc_status pair_run(afqmc_sys a, afqmc_sys b, uint64_t seed, int n_steps,
                      const double* fields_dev, double* e_trace, double* trace, int n_meas);

// Autotuner: fills the system's launch shapes (tile_fb, tile_fs, prop_var) from the process-wide table, timing the candidates of shapes not
// seen before.  Synchronises st.
afqmc_status autotune(afqmc_sys s, hipStream_t st);
// Drops every cached batch graph that references system `id`.
void drop_batch_plans(uint64_t id);
// Releases the reverse-mode tape of a system.
void free_adjoint(afqmc_sys s);
// exp(X) of a small dense real matrix (host).
void expm_host(const std::vector<double>& X, int n, std::vector<double>& out);

}  // namespace host
}  // namespace afq
