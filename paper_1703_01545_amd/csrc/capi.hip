// C ABI of the correlated-sampling ph-AFQMC walker step (see include/afqmc.h).
// Host code: handle management, validation, the per-system precompute, and
// the ordering of the device phases of one step.
#include <atomic>
#include <string>
#include <vector>

#include "host.h"

using namespace afq;
using namespace afq::host;

namespace afq {
namespace host {

thread_local std::string g_err;

// exp(X) for a small dense real matrix: scaling and squaring with a
// degree-13 Taylor polynomial; with ||X / 2^s||_1 <= 1/4 the truncation is
// below (1/4)^14 / 14! e^(1/4) < 1e-19 relative.
void expm_host(const std::vector<double>& X, int n, std::vector<double>& out) {
    double nrm = 0.0;
    for (int j = 0; j < n; ++j) {
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += fabs(X[(size_t)i * n + j]);
        nrm = std::max(nrm, c);
    }
    int s = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        ++s;
    }
    const double sc = ldexp(1.0, -s);
    std::vector<double> A(X.size()), term((size_t)n * n, 0.0), tmp((size_t)n * n);
    for (size_t i = 0; i < A.size(); ++i) A[i] = X[i] * sc;
    out.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) out[(size_t)i * n + i] = term[(size_t)i * n + i] = 1.0;
    auto mul = [&](const std::vector<double>& a, const std::vector<double>& b,
                   std::vector<double>& c) {
        std::fill(c.begin(), c.end(), 0.0);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                const double v = a[(size_t)i * n + k];
                if (v == 0.0) continue;
                for (int j = 0; j < n; ++j) c[(size_t)i * n + j] += v * b[(size_t)k * n + j];
            }
    };
    for (int k = 1; k <= 13; ++k) {
        mul(term, A, tmp);
        for (size_t i = 0; i < tmp.size(); ++i) term[i] = tmp[i] / k;
        for (size_t i = 0; i < tmp.size(); ++i) out[i] += term[i];
    }
    for (int q = 0; q < s; ++q) {
        mul(out, out, tmp);
        out.swap(tmp);
    }
}


const char* const kPhaseNames[PH_COUNT] = {
    "force_bias_gemm", "fields", "field_sum_gemm", "unpack_a", "propagate",
    "det_theta",       "weights", "mgs",            "exchange", "energy"};


int fb_ksplit(int k) {
    // a function of K = N M alone: the same K ranges, and so the same bits for
    // every walker, whatever the walker count, the batch a walker runs in or
    // the device; about 1000 K per range below K = 8000 (where the output is
    // small and takes 64 x 64 tiles: 4 ranges at K = 4000 give 448 workgroups
    // for 512 walkers and 401 columns, not 112), about 1800 K per range above
    // (9 ranges at K = 16000, which with 256 x 128 tiles fill 1008 workgroups
    // for 2048 walkers and 801 columns on 256 CUs)
    if (k < 8000) return std::max(1, std::min(7, k / 1000));
    return std::max(4, std::min(12, (k + 900) / 1800));
}

Gemm force_bias_gemm(afqmc_sys s, int det) {
    // F[(w,p), g] = sum_(i,m) Theta[(w,p),(i,m)] L^half[g,(i,m)], g <= n_chol
    Gemm g{};
    g.A = lp_or(det_theta_lp(s, det), det_theta(s, det), s->ts);
    g.ta = s->ts;
    g.ra = rows_strided(s->NM());
    g.B = lp_or(det_lhx_lp(s, det), det_lhx(s, det), s->ts);
    g.tb = s->ts;
    g.rb = rows_strided(s->NM());
    g.C = det_F(s, det);
    g.tc = DT_F64;
    g.rc = rows_strided(s->n_chol + 1);
    g.alpha = 1.0;
    g.m = 2 * s->nw;
    g.n = s->n_chol + 1;
    g.k = (int)s->NM();
    g.batch = 1;
    g.tile = s->tile_fb;
    // long K (= N M): fixed K ranges so that large tiles still fill the chip
    g.ksplit = s->fb_ks;
    g.ws = s->d_kws.p;
    return g;
}

afqmc_status force_bias(afqmc_sys s, hipStream_t st) {
    PhaseTimer pt(s, PH_FORCE_BIAS, st);
    for (int i = 0; i < s->n_det; ++i) HIPCHK(gemm(force_bias_gemm(s, i), s->tc, st));
    if (s->n_det > 1)
        HIPCHK(msd_combine(s->d_F_all.as<double>(), (long)s->nw * 2 * (s->n_chol + 1),
                           s->d_rw.as<double>(), s->n_det, s->d_alive.as<uint8_t>(), s->nw,
                           s->n_chol + 1, s->d_F.as<double>(), st));
    return AFQMC_OK;
}

afqmc_status overlap_theta(afqmc_sys s, double* phi, hipStream_t st) {
    // overlap, ln det and Theta in one launch per (walker, spin), per
    // determinant of the trial; then the expansion's combination
    PhaseTimer pt(s, PH_DET_THETA, st);
    for (int i = 0; i < s->n_det; ++i)
        HIPCHK(lu_theta(phi, det_trialT(s, i).as<double>(), det_theta(s, i).as<double>(),
                        s->ts == DT_F64 ? nullptr : det_theta_lp(s, i).p, s->ts, det_lnd(s, i),
                        s->d_alive.as<uint8_t>(), s->nw, s->M, s->N, s->na, s->nb, s->d_ovl.p,
                        st));
    if (s->n_det > 1)
        HIPCHK(msd_overlap(s->d_lnd_all.as<double>(), s->d_coef.as<double>(), s->n_det,
                           s->d_alive.as<uint8_t>(), s->nw, s->d_lnd.as<double>(),
                           s->d_rw.as<double>(), st));
    return AFQMC_OK;
}

Gemm field_sum_gemm(afqmc_sys s) {
    // A[(w,p), q] = sum_g X[(w,p), g] Lpacked[q, g]
    Gemm g{};
    g.A = s->d_X.p;
    g.ta = s->ts;
    g.ra = rows_strided(s->n_chol);
    g.B = s->ham->d_lp[s->ts].p;
    g.tb = s->ts;
    g.rb = rows_strided(s->n_chol);
    g.C = s->d_Apk.p;
    g.tc = s->tp;
    g.rc = rows_strided(s->P());
    g.alpha = 1.0;
    g.m = 2 * s->nw;
    g.n = (int)s->P();
    g.k = s->n_chol;
    g.batch = 1;
    g.tile = s->tile_fs;
    return g;
}

afqmc_status one_step(afqmc_sys s, uint64_t seed, uint64_t stream_id, const double* ext,
                      hipStream_t st) {
    afqmc_status r;
    if ((r = force_bias(s, st)) != AFQMC_OK) return r;
    FieldArgs f{};
    f.F = s->d_F.as<double>();
    f.ldf = s->n_chol + 1;
    f.a = s->d_a.as<double>();
    f.ext = ext;
    f.seed = seed;
    f.stream = stream_id;
    f.t = s->t_dev ? s->t - s->t_base : s->t;
    f.t_dev = s->t_dev;
    f.alive = s->d_alive.as<uint8_t>();
    f.X = s->d_X.p;
    f.tx = s->ts;
    f.ldx = s->n_chol;
    f.s_imp = s->d_simp.as<double>();
    f.nw = s->nw;
    f.n_chol = s->n_chol;
    f.sqdt = sqrt(s->par.dt);
    f.free_proj = s->par.mode == AFQMC_FREE;
    f.fb_cap = s->par.mode == AFQMC_FREE ? 0.0 : s->par.fb_cap;
    f.cap_apply = s->par.caps_enabled;
    f.cap_count = s->d_capcount.as<int64_t>();
    {
        PhaseTimer pt(s, PH_FIELDS, st);
        HIPCHK(fields(f, st));
    }
    {
        const Gemm g = field_sum_gemm(s);
        PhaseTimer pt(s, PH_FIELD_SUM, st);
        HIPCHK(gemm(g, s->tc, st));
    }
    {
        PhaseTimer pt(s, PH_UNPACK, st);
        HIPCHK(unpack_sym(s->d_Apk.p, s->d_Af.p, s->M, 2 * s->nw, s->ta, st));
    }
    // Phi' = P T_K(A) P Phi, fused per walker
    {
        const void* Pm = s->tp == DT_F64 ? s->d_P.p : s->d_Plp.p;
        PhaseTimer pt(s, PH_PROPAGATE, st);
        HIPCHK(propagate(s->d_phi.as<double>(), s->d_phinew.as<double>(), Pm, s->d_Af.p,
                         s->d_alive.as<uint8_t>(), s->nw, s->M, s->N, s->par.taylor_order, s->tp,
                         s->ta, s->prop_var, st, s->rec));
    }
    if ((r = overlap_theta(s, s->d_phinew.as<double>(), st)) != AFQMC_OK) return r;
    PhaseTimer pt(s, PH_WEIGHTS, st);
    HIPCHK(weights(s->d_lnd.as<double>(), s->d_simp.as<double>(), s->d_lnov.as<double>(),
                   s->d_w.as<double>(), s->d_alive.as<uint8_t>(), s->nw, (int)s->par.mode, 1,
                   s->par.dt * s->e_shift, st));
    std::swap(s->d_phi.p, s->d_phinew.p);
    s->t += 1;
    return AFQMC_OK;
}

afqmc_status ortho(afqmc_sys s, hipStream_t st) {
    {
        PhaseTimer pt(s, PH_MGS, st);
        HIPCHK(mgs(s->d_phi.as<double>(), s->d_alive.as<uint8_t>(), s->nw, s->M, s->N, s->na, s->nb,
                   s->d_ovl.p, s->d_gsmon.as<double>(), st));
    }
    afqmc_status r = overlap_theta(s, s->d_phi.as<double>(), st);
    if (r != AFQMC_OK) return r;
    PhaseTimer pt(s, PH_WEIGHTS, st);
    HIPCHK(weights(s->d_lnd.as<double>(), s->d_simp.as<double>(), s->d_lnov.as<double>(),
                   s->d_w.as<double>(), s->d_alive.as<uint8_t>(), s->nw, (int)s->par.mode, 0, 0.0,
                   st));
    return AFQMC_OK;
}

afqmc_status measure(afqmc_sys s, hipStream_t st) {
    afqmc_status r = force_bias(s, st);
    if (r != AFQMC_OK) return r;
    for (int i = 0; i < s->n_det; ++i) {
        const void* lh = lp_or(det_lhx_lp(s, i), det_lhx(s, i), s->ts);
        const void* th = lp_or(det_theta_lp(s, i), det_theta(s, i), s->ts);
        for (int spin = 0; spin < 2; ++spin) {
            const int off = spin ? s->na : 0, n = spin ? s->nb : s->na;
            if (n == 0) continue;
            PhaseTimer pt(s, PH_EXCHANGE, st);
            HIPCHK(exchange(lh, th, det_exch(s, i).as<double>(), s->nw, s->M, s->N, s->n_chol,
                            off, n, spin, s->n_gt, s->tc, st));
        }
        PhaseTimer pt(s, PH_ENERGY, st);
        HIPCHK(local_energy(det_F(s, i), s->n_chol + 1, det_exch(s, i).as<double>(), s->n_gt_a,
                            s->n_gt_b, s->nw, s->n_chol, s->ham->e_core, det_el(s, i), st));
    }
    PhaseTimer pt(s, PH_ENERGY, st);
    if (s->n_det > 1)
        HIPCHK(msd_combine(s->d_el_all.as<double>(), (long)s->nw * 2, s->d_rw.as<double>(),
                           s->n_det, s->d_alive.as<uint8_t>(), s->nw, 1, s->d_el.as<double>(),
                           st));
    HIPCHK(mixed_sums(s->d_el.as<double>(), s->d_w.as<double>(), s->d_alive.as<uint8_t>(), s->nw,
                      (int)s->par.mode, s->d_sums.as<double>(), st));
    return AFQMC_OK;
}

// Validation shared by the pair entry points; *n_meas = measurements among
// the n_steps.
afqmc_status pair_check(afqmc_sys a, afqmc_sys b, int n_steps, int* n_meas) {
    afqmc_status r;
    if ((r = check_sys(a)) != AFQMC_OK || (r = check_sys(b)) != AFQMC_OK) return r;
    if (n_steps < 0) return fail(AFQMC_E_INVALID, "n_steps < 0");
    if (a == b) return fail(AFQMC_E_INVALID, "a pair needs two distinct systems");
    if (a->M != b->M || a->n_chol != b->n_chol || a->nw != b->nw ||
        a->ham->chol_hash != b->ham->chol_hash)
        return fail(AFQMC_E_SHAPE, "pair systems must share M, n_chol, walker count and L");
    if (a->par.dt != b->par.dt || a->par.ortho_every != b->par.ortho_every ||
        a->par.measure_every != b->par.measure_every || a->par.mode != b->par.mode)
        return fail(AFQMC_E_SHAPE, "pair systems must share dt, periods and mode");
    if (a->t != b->t) return fail(AFQMC_E_STATE, "pair systems are at different steps");
    if (a->ham->stream != b->ham->stream) return fail(AFQMC_E_SHAPE, "pair systems need one stream");
    const int me = a->par.measure_every;
    int n = 0;
    for (int i = 0; i < n_steps; ++i)
        if (me > 0 && (a->t + i + 1) % me == 0) ++n;
    *n_meas = n;
    return AFQMC_OK;
}

// The steps of a correlated pair (Sec. II.B); measurement rows go to the
// device array `trace` (n_meas x 3), then to e_trace on the host.
afqmc_status pair_run(afqmc_sys a, afqmc_sys b, uint64_t seed, int n_steps,
                      const double* fields_dev, double* e_trace, double* trace, int n_meas) {
    afqmc_status r;
    hipStream_t st = a->ham->stream;
    const int me = a->par.measure_every, oe = a->par.ortho_every;
    int slot = 0;
    for (int i = 0; i < n_steps; ++i) {
        const double* ext = fields_dev ? fields_dev + (size_t)i * a->nw * a->n_chol : nullptr;
        if ((r = one_step(a, seed, 0, ext, st)) != AFQMC_OK) return r;
        if ((r = one_step(b, seed, 0, ext, st)) != AFQMC_OK) return r;
        if (oe > 0 && a->t % oe == 0) {
            if ((r = ortho(a, st)) != AFQMC_OK) return r;
            if ((r = ortho(b, st)) != AFQMC_OK) return r;
        }
        if (me > 0 && a->t % me == 0) {
            if ((r = measure(a, st)) != AFQMC_OK) return r;
            if ((r = measure(b, st)) != AFQMC_OK) return r;
            HIPCHK(trace_record(a->d_sums.as<double>(), b->d_sums.as<double>(), trace, slot++,
                                nullptr, 0, (int)a->par.mode, st));
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    if (e_trace && n_meas > 0)
        HIPCHK(hipMemcpy(e_trace, trace, (size_t)n_meas * 3 * 8, hipMemcpyDeviceToHost));
    return AFQMC_OK;
}

}  // namespace host
}  // namespace afq

namespace {

// FNV-1a over 64-bit words (identity check of Cholesky tensors, not a
// cryptographic hash).
uint64_t fnv1a(const void* data, size_t n) {
    const unsigned char* b = (const unsigned char*)data;
    uint64_t h = 1469598103934665603ull;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        memcpy(&w, b + i, 8);
        h ^= w;
        h *= 1099511628211ull;
    }
    for (; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Solve for Theta_T = Phi_T (Phi_T^T Phi_T)^{-1} of one spin block (host,
// small): Gauss-Jordan with partial pivoting.
bool theta_trial(const double* trial, int M, int N, int off, int n, double* out /* n x M rows */) {
    std::vector<double> O((size_t)n * n), inv((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int m = 0; m < M; ++m)
                s += trial[(size_t)m * N + off + a] * trial[(size_t)m * N + off + b];
            O[(size_t)a * n + b] = s;
        }
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(O[(size_t)r * n + k]) > fabs(O[(size_t)p * n + k])) p = r;
        if (O[(size_t)p * n + k] == 0.0) return false;
        for (int c = 0; c < n; ++c) {
            std::swap(O[(size_t)k * n + c], O[(size_t)p * n + c]);
            std::swap(inv[(size_t)k * n + c], inv[(size_t)p * n + c]);
        }
        const double d = O[(size_t)k * n + k];
        for (int c = 0; c < n; ++c) {
            O[(size_t)k * n + c] /= d;
            inv[(size_t)k * n + c] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == k) continue;
            const double f = O[(size_t)r * n + k];
            if (f == 0.0) continue;
            for (int c = 0; c < n; ++c) {
                O[(size_t)r * n + c] -= f * O[(size_t)k * n + c];
                inv[(size_t)r * n + c] -= f * inv[(size_t)k * n + c];
            }
        }
    }
    // Theta[m][c] = sum_l trial[m][off + l] inv[l][c]; stored as out[c][m]
    for (int c = 0; c < n; ++c)
        for (int m = 0; m < M; ++m) {
            double s = 0.0;
            for (int l = 0; l < n; ++l) s += trial[(size_t)m * N + off + l] * inv[(size_t)l * n + c];
            out[(size_t)c * M + m] = s;
        }
    return true;
}

// Theta_ij = D_j (D_i^T D_j)^{-1} of one spin block (rows: out[c][m]) and
// ln |det(D_i^T D_j)| with its sign, by Gauss-Jordan with partial pivoting on
// the host (determinants i, j: M x N row-major, columns off .. off + n - 1).
// Returns false when a pivot is exactly zero.
bool theta_pair(const double* Di, const double* Dj, int M, int N, int off, int n, double* out,
                double* logabs, int* sign) {
    std::vector<double> O((size_t)n * n), inv((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double v = 0.0;
            for (int m = 0; m < M; ++m) v += Di[(size_t)m * N + off + a] * Dj[(size_t)m * N + off + b];
            O[(size_t)a * n + b] = v;
        }
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    double la = 0.0;
    int sg = 1;
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(O[(size_t)r * n + k]) > fabs(O[(size_t)p * n + k])) p = r;
        if (O[(size_t)p * n + k] == 0.0) return false;
        if (p != k) {
            sg = -sg;
            for (int c = 0; c < n; ++c) {
                std::swap(O[(size_t)k * n + c], O[(size_t)p * n + c]);
                std::swap(inv[(size_t)k * n + c], inv[(size_t)p * n + c]);
            }
        }
        const double d = O[(size_t)k * n + k];
        la += log(fabs(d));
        if (d < 0) sg = -sg;
        for (int c = 0; c < n; ++c) {
            O[(size_t)k * n + c] /= d;
            inv[(size_t)k * n + c] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == k) continue;
            const double f = O[(size_t)r * n + k];
            if (f == 0.0) continue;
            for (int c = 0; c < n; ++c) {
                O[(size_t)r * n + c] -= f * O[(size_t)k * n + c];
                inv[(size_t)r * n + c] -= f * inv[(size_t)k * n + c];
            }
        }
    }
    for (int c = 0; c < n; ++c)
        for (int m = 0; m < M; ++m) {
            double v = 0.0;
            for (int l = 0; l < n; ++l) v += Dj[(size_t)m * N + off + l] * inv[(size_t)l * n + c];
            out[(size_t)c * M + m] = v;
        }
    *logabs = la;
    *sign = sg;
    return true;
}

// Phases of the step, each one kernel launch (the Taylor phase is one
// launch per term).  Timed with HIP events on the system's stream when

}  // namespace

extern "C" {

const char* afqmc_last_error(void) { return g_err.c_str(); }

afqmc_status afqmc_load_hamiltonian(int M, int n_chol, const double* h1, const double* chol,
                                    double e_core, void* hip_stream, afqmc_ham* out) {
    if (!out) return fail(AFQMC_E_INVALID, "out is null");
    *out = nullptr;
    if (M <= 0 || n_chol < 0) return fail(AFQMC_E_INVALID, "M must be > 0 and n_chol >= 0");
    if (!h1 || (n_chol > 0 && !chol)) return fail(AFQMC_E_INVALID, "null h1 or chol");
    afqmc_ham h = new afqmc_ham_s();
    h->M = M;
    h->n_chol = n_chol;
    h->e_core = e_core;
    h->stream = (hipStream_t)hip_stream;
    h->h.assign(h1, h1 + (size_t)M * M);
    const size_t nL = (size_t)n_chol * M * M;
    h->chol_hash = fnv1a(chol, nL * sizeof(double));
    hipError_t e;
    if ((e = h->d_h.alloc((size_t)M * M * 8)) != hipSuccess ||
        (e = h->d_chol.alloc(nL * 8)) != hipSuccess) {
        delete h;
        return fail(AFQMC_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    if ((e = hipMemcpy(h->d_h.p, h1, (size_t)M * M * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (nL && (e = hipMemcpy(h->d_chol.p, chol, nL * 8, hipMemcpyHostToDevice)) != hipSuccess)) {
        delete h;
        return fail(AFQMC_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    *out = h;
    return AFQMC_OK;
}

void afqmc_free_ham(afqmc_ham h) {
    if (!h || h->released) return;
    h->released = true;
    ham_unref(h);
}

}  // extern "C"

namespace {

// One system on `ham` with the trial sum_i coeffs[i] D_i (n_det determinants
// of shape M x N in `dets`; one determinant: the single-determinant trial).
afqmc_status init_system(afqmc_ham ham, int n_alpha, int n_beta, int n_det, const double* coeffs,
                         const double* dets, const double* init_phi, int n_walkers,
                         const afqmc_params* par, afqmc_sys* out) {
    if (!out) return fail(AFQMC_E_INVALID, "out is null");
    *out = nullptr;
    if (!ham || ham->released) return fail(AFQMC_E_INVALID, "null or freed Hamiltonian");
    if (!dets || !par || (n_det > 1 && !coeffs)) return fail(AFQMC_E_INVALID, "null trial or params");
    if (n_det < 1 || n_det > 256) return fail(AFQMC_E_INVALID, "n_det must lie in 1 .. 256");
    const double* trial = dets;
    const int M = ham->M;
    if (n_alpha < 0 || n_beta < 0 || n_alpha > M || n_beta > M || n_alpha + n_beta == 0)
        return fail(AFQMC_E_SHAPE, "need 0 <= n_alpha, n_beta <= M and n_alpha + n_beta > 0");
    if (n_alpha > 64 || n_beta > 64) return fail(AFQMC_E_SHAPE, "at most 64 electrons per spin");
    if (M > 256) return fail(AFQMC_E_SHAPE, "the fused propagation supports M <= 256");
    if (n_walkers <= 0) return fail(AFQMC_E_INVALID, "n_walkers must be > 0");
    if (!(par->dt > 0.0) || par->taylor_order < 1 || par->ortho_every < 0 || par->measure_every < 0)
        return fail(AFQMC_E_INVALID, "bad params (dt > 0, taylor_order >= 1, periods >= 0)");
    if (!(par->fb_cap >= 0.0)) return fail(AFQMC_E_INVALID, "fb_cap must be >= 0");
    static std::atomic<bool> unpack_ready{false};  // kernel attribute, set outside any capture
    if (!unpack_ready) {
        if (unpack_prepare() != hipSuccess) return fail(AFQMC_E_DEVICE, "unpack kernel attribute");
        unpack_ready = true;
    }
    if (par->contract_prec < AFQMC_FP64 || par->contract_prec > AFQMC_BF16X3)
        return fail(AFQMC_E_INVALID, "bad contract_prec");
    if (par->mode != AFQMC_PHASELESS && par->mode != AFQMC_FREE)
        return fail(AFQMC_E_INVALID, "bad mode");
    hipStream_t st = ham->stream;
    afqmc_sys s = new afqmc_sys_s();
    static std::atomic<uint64_t> next_id{0};
    s->id = ++next_id;
    s->ham = ham;
    ham->refs++;
    s->M = M;
    s->n_chol = ham->n_chol;
    s->na = n_alpha;
    s->nb = n_beta;
    s->N = n_alpha + n_beta;
    s->nw = n_walkers;
    s->par = *par;
    s->ta = DT_F64;
    switch (par->contract_prec) {
        case AFQMC_FP64: s->ts = DT_F64; s->tc = DT_F64; s->tp = DT_F64; break;
        case AFQMC_FP32: s->ts = DT_F32; s->tc = DT_F32; s->tp = DT_F32; break;
        case AFQMC_BF16: s->ts = DT_F32; s->tc = DT_SPLIT; s->tp = DT_F32; break;
        case AFQMC_BF16X3: s->ts = DT_F32; s->tc = DT_SPLIT; s->tp = DT_F32; break;
        default: s->ts = DT_BF16; s->tc = DT_BF16; s->tp = DT_F32; break;
    }
    s->ta = par->contract_prec == AFQMC_BF16X3 ? DT_SPLIT : s->tp;
    auto bail = [&](afqmc_status r) {
        afqmc_free_sys(s);
        return r;
    };
    const int N = s->N, nc = s->n_chol, nw = n_walkers;
    const long NM = s->NM(), P = s->P();
    s->n_gt_a = exchange_gtiles(nc, s->na, M, s->tc);
    s->n_gt_b = exchange_gtiles(nc, s->nb, M, s->tc);  // tiles depend on the compute type
    s->n_gt = std::max(1, std::max(s->n_gt_a, s->n_gt_b));
    s->fb_ks = fb_ksplit((int)NM);
    struct A_ {
        DevBuf* b;
        size_t bytes;
    } allocs[] = {
        {&s->d_trialT, (size_t)NM * 8},
        {&s->d_P, (size_t)M * M * 8},
        {&s->d_Plp, s->ta == DT_SPLIT ? (size_t)split_tile_elems(M) * 2 * 2 : (size_t)M * M * 4},
        {&s->d_a, (size_t)std::max(nc, 1) * 8},
        {&s->d_lhx, (size_t)(nc + 1) * NM * 8},
        {&s->d_lhx_lp, s->ts == DT_F64 ? 0 : (size_t)(nc + 1) * NM * dt_size(s->ts)},
        {&s->d_phi, (size_t)nw * 2 * NM * 8},
        {&s->d_phinew, (size_t)nw * 2 * NM * 8},
        {&s->d_theta, (size_t)nw * 2 * NM * 8},
        {&s->d_theta_lp, s->ts == DT_F64 ? 0 : (size_t)nw * 2 * NM * dt_size(s->ts)},
        {&s->d_w, (size_t)nw * 2 * 8},
        {&s->d_lnov, (size_t)nw * 2 * 8},
        {&s->d_alive, (size_t)nw},
        {&s->d_F, (size_t)nw * 2 * (nc + 1) * 8},
        {&s->d_X, (size_t)nw * 2 * std::max(nc, 1) * dt_size(s->ts)},
        {&s->d_simp, (size_t)nw * 4 * 8},
        {&s->d_Apk, (size_t)nw * 2 * P * dt_size(s->tp)},
        {&s->d_Af, s->ta == DT_SPLIT ? (size_t)nw * 4 * split_tile_elems(M) * 2
                                     : (size_t)nw * 2 * M * M * dt_size(s->tp)},
        {&s->d_lnd, (size_t)nw * 4 * 8},
        {&s->d_ovl, lu_theta_ws_bytes(nw, n_alpha, n_beta)},
        {&s->d_kws, gemm_ws_bytes(2 * nw, nc + 1, s->fb_ks, s->tc)},
        {&s->d_exch, (size_t)nw * 2 * s->n_gt * 2 * 8},
        {&s->d_el, (size_t)nw * 2 * 8},
        {&s->d_sums, 8 * 8},
        {&s->d_pc, (size_t)nw * 12 + 16},
        {&s->d_capcount, (size_t)nw * 8},
        {&s->d_gsmon, (size_t)nw * 4 * 8},
    };
    for (auto& a : allocs) {
        hipError_t e = a.b->alloc(a.bytes);
        if (e != hipSuccess)
            return bail(fail(AFQMC_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)));
    }
    s->n_det = n_det;
    if (n_det > 1) {
        std::vector<std::pair<DevBuf*, size_t>> more = {
            {&s->d_coef, (size_t)n_det * 8},
            {&s->d_lnd_all, (size_t)n_det * nw * 4 * 8},
            {&s->d_F_all, (size_t)n_det * nw * 2 * (nc + 1) * 8},
            {&s->d_el_all, (size_t)n_det * nw * 2 * 8},
            {&s->d_rw, (size_t)n_det * nw * 2 * 8}};
        for (int i = 1; i < n_det; ++i) {
            s->xdet.push_back(std::make_unique<afqmc_sys_s::DetBufs>());
            afqmc_sys_s::DetBufs& d = *s->xdet.back();
            more.push_back({&d.trialT, (size_t)NM * 8});
            more.push_back({&d.lhx, (size_t)(nc + 1) * NM * 8});
            more.push_back({&d.lhx_lp, s->ts == DT_F64 ? 0 : (size_t)(nc + 1) * NM * dt_size(s->ts)});
            more.push_back({&d.theta, (size_t)nw * 2 * NM * 8});
            more.push_back({&d.theta_lp, s->ts == DT_F64 ? 0 : (size_t)nw * 2 * NM * dt_size(s->ts)});
            more.push_back({&d.exch, (size_t)nw * 2 * s->n_gt * 2 * 8});
        }
        for (auto& m : more) {
            hipError_t e = m.first->alloc(m.second);
            if (e != hipSuccess)
                return bail(fail(AFQMC_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)));
        }
        for (auto& d : s->xdet)
            for (DevBuf* b : {&d->theta, &d->theta_lp, &d->lhx, &d->exch}) {
                hipError_t e = hipMemsetAsync(b->p, 0, b->n, st);
                if (e != hipSuccess) return bail(fail(AFQMC_E_DEVICE, hipGetErrorString(e)));
            }
        if (hipMemcpy(s->d_coef.p, coeffs, (size_t)n_det * 8, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "upload coefficients"));
    }
    // zero buffers read before first written (theta padding, F one-body row)
    for (DevBuf* b : {&s->d_theta, &s->d_theta_lp, &s->d_lhx, &s->d_exch, &s->d_simp,
                      &s->d_capcount, &s->d_gsmon}) {
        hipError_t e = hipMemsetAsync(b->p, 0, b->n, st);
        if (e != hipSuccess) return bail(fail(AFQMC_E_DEVICE, hipGetErrorString(e)));
    }
    for (int di = 0; di < n_det; ++di) {
        const double* D = dets + (size_t)di * M * N;
        // D^T (rows = orbitals)
        std::vector<double> trialT((size_t)NM);
        for (int i = 0; i < N; ++i)
            for (int m = 0; m < M; ++m) trialT[(size_t)i * M + m] = D[(size_t)m * N + i];
        if (hipMemcpy(det_trialT(s, di).p, trialT.data(), NM * 8, hipMemcpyHostToDevice) !=
            hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "upload trial"));
        // L^half_g[i][n] = sum_m D[m][i] L_g[n][m]; row n_chol holds h^half.
        Gemm g{};
        g.A = det_trialT(s, di).p;
        g.ta = DT_F64;
        g.ra = rows_strided(M);
        g.a_bs = 0;
        g.B = ham->d_chol.p;
        g.tb = DT_F64;
        g.rb = rows_strided(M);
        g.b_bs = (long)M * M;
        g.C = det_lhx(s, di).p;
        g.tc = DT_F64;
        g.rc = rows_strided(M);
        g.c_bs = NM;
        g.alpha = 1.0;
        g.m = N;
        g.n = M;
        g.k = M;
        g.batch = nc;
        if (nc > 0 && gemm(g, DT_F64, st) != hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "L^half GEMM"));
        g.B = ham->d_h.p;
        g.b_bs = 0;
        g.C = det_lhx(s, di).as<double>() + (size_t)nc * NM;
        g.batch = 1;
        if (gemm(g, DT_F64, st) != hipSuccess) return bail(fail(AFQMC_E_DEVICE, "h^half GEMM"));
    }
    // a_g = <phi_T|rho_g|phi_T> / <phi_T|phi_T> (Eq. 2, 9).  With the determinant
    // pairs (i, j): sum_ij c_i c_j <D_i|D_j> f^(i)_g(D_j) / sum_ij c_i c_j <D_i|D_j>,
    // f^(i)_g(D_j) = sum_s Tr(L^half_{i,gs} Theta_ij^s), Theta_ij = D_j (D_i^T D_j)^{-1};
    // one determinant: the force-bias trace of the trial.
    std::vector<double> Ftrial((size_t)2 * (nc + 1), 0.0);
    {
        const int nd = n_det;
        std::vector<double> thT((size_t)nd * 2 * NM, 0.0), lw((size_t)nd * nd);
        std::vector<int> sgn((size_t)nd * nd);
        DevBuf dth, dF;
        if (dth.alloc((size_t)nd * 2 * NM * 8) != hipSuccess ||
            dF.alloc((size_t)nd * 2 * (nc + 1) * 8) != hipSuccess)
            return bail(fail(AFQMC_E_NOMEM, "scratch"));
        std::vector<double> Fij((size_t)nd * nd * (nc + 1));
        for (int i = 0; i < nd; ++i) {
            const double* Di = dets + (size_t)i * M * N;
            for (int j = 0; j < nd; ++j) {
                const double* Dj = dets + (size_t)j * M * N;
                double la = 0.0, l1 = 0.0;
                int sg = 1, s1 = 1;
                double* th = thT.data() + (size_t)j * 2 * NM;
                if (s->na && !theta_pair(Di, Dj, M, N, 0, s->na, th, &l1, &s1))
                    return bail(fail(AFQMC_E_SINGULAR, "alpha blocks of trial determinants " +
                                                           std::to_string(i) + " and " +
                                                           std::to_string(j) + " are orthogonal"));
                la += l1;
                sg *= s1;
                if (s->nb && !theta_pair(Di, Dj, M, N, s->na, s->nb, th + (size_t)s->na * M, &l1,
                                         &s1))
                    return bail(fail(AFQMC_E_SINGULAR, "beta blocks of trial determinants " +
                                                           std::to_string(i) + " and " +
                                                           std::to_string(j) + " are orthogonal"));
                la += l1;
                sg *= s1;
                lw[(size_t)i * nd + j] = la;
                sgn[(size_t)i * nd + j] = sg;
            }
            if (hipMemcpy(dth.p, thT.data(), (size_t)nd * 2 * NM * 8, hipMemcpyHostToDevice) !=
                hipSuccess)
                return bail(fail(AFQMC_E_DEVICE, "upload"));
            Gemm g{};
            g.A = dth.p;
            g.ta = DT_F64;
            g.ra = rows_strided(NM);
            g.B = det_lhx(s, i).p;
            g.tb = DT_F64;
            g.rb = rows_strided(NM);
            g.C = dF.p;
            g.tc = DT_F64;
            g.rc = rows_strided(nc + 1);
            g.alpha = 1.0;
            g.m = 2 * nd;
            g.n = nc + 1;
            g.k = (int)NM;
            g.batch = 1;
            if (gemm(g, DT_F64, st) != hipSuccess) return bail(fail(AFQMC_E_DEVICE, "a GEMM"));
            std::vector<double> Fd((size_t)nd * 2 * (nc + 1));
            if (hipStreamSynchronize(st) != hipSuccess ||
                hipMemcpy(Fd.data(), dF.p, Fd.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
                return bail(fail(AFQMC_E_DEVICE, "a download"));
            for (int j = 0; j < nd; ++j)  // real part: row 2 j of the GEMM
                std::copy(Fd.begin() + (size_t)j * 2 * (nc + 1),
                          Fd.begin() + (size_t)j * 2 * (nc + 1) + nc + 1,
                          Fij.begin() + ((size_t)i * nd + j) * (nc + 1));
        }
        if (nd == 1) {
            std::copy(Fij.begin(), Fij.end(), Ftrial.begin());
        } else {
            double top = -INFINITY;
            for (double v : lw) top = std::max(top, v);
            double den = 0.0;
            std::vector<double> num((size_t)nc + 1, 0.0);
            for (int i = 0; i < nd; ++i)
                for (int j = 0; j < nd; ++j) {
                    const double wt = coeffs[i] * coeffs[j] * sgn[(size_t)i * nd + j] *
                                      exp(lw[(size_t)i * nd + j] - top);
                    den += wt;
                    for (int g = 0; g <= nc; ++g) num[g] += wt * Fij[((size_t)i * nd + j) * (nc + 1) + g];
                }
            if (!(den != 0.0)) return bail(fail(AFQMC_E_SINGULAR, "the trial expansion has zero norm"));
            for (int g = 0; g <= nc; ++g) Ftrial[g] = num[g] / den;
        }
    }
    s->a_host.assign(Ftrial.begin(), Ftrial.begin() + nc);
    if (nc > 0 && hipMemcpy(s->d_a.p, s->a_host.data(), nc * 8, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(AFQMC_E_DEVICE, "upload a"));
    // h~ = h - 1/2 sum_g L_g L_g + sum_g a_g L_g  (Eq. 2 remainder), P = exp(-dt h~ / 2)
    std::vector<double> ht(ham->h);
    if (nc > 0) {
        DevBuf dLT, dL2, daL;
        if (dLT.alloc((size_t)nc * M * M * 8) != hipSuccess || dL2.alloc((size_t)M * M * 8) ||
            daL.alloc((size_t)M * M * 8))
            return bail(fail(AFQMC_E_NOMEM, "scratch"));
        Gemm g{};
        g.A = dLT.p;
        g.ta = DT_F64;
        g.ra = rows_strided((long)nc * M);
        g.B = dLT.p;
        g.tb = DT_F64;
        g.rb = rows_strided((long)nc * M);
        g.C = dL2.p;
        g.tc = DT_F64;
        g.rc = rows_strided(M);
        g.alpha = 1.0;
        g.m = M;
        g.n = M;
        g.k = nc * M;
        g.batch = 1;
        if (permute_chol(ham->d_chol.as<double>(), dLT.as<double>(), M, nc, st) != hipSuccess ||
            gemm(g, DT_F64, st) != hipSuccess ||
            chol_weighted_sum(ham->d_chol.as<double>(), s->d_a.as<double>(), daL.as<double>(), M,
                              nc, st) != hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "h~ kernels"));
        std::vector<double> l2((size_t)M * M), al((size_t)M * M);
        if (hipStreamSynchronize(st) != hipSuccess ||
            hipMemcpy(l2.data(), dL2.p, l2.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(al.data(), daL.p, al.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "h~ download"));
        for (size_t i = 0; i < ht.size(); ++i) ht[i] = ht[i] - 0.5 * l2[i] + al[i];
    }
    s->htilde = ht;
    {
        std::vector<double> X(ht.size()), Pm;
        for (size_t i = 0; i < X.size(); ++i) X[i] = -0.5 * par->dt * ht[i];
        expm_host(X, M, Pm);
        // split products carry Q = P - I (formed in FP64) as hi/lo BF16 planes
        // in the fragment-tiled layout
        std::vector<float> Pf(Pm.begin(), Pm.end());
        if (s->ta == DT_SPLIT) {
            Pf.assign((size_t)split_tile_elems(M), 0.0f);
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j)
                    Pf[split_tile_index(M, i, j)] =
                        (float)(Pm[(size_t)i * M + j] - (i == j ? 1.0 : 0.0));
        }
        if (hipMemcpy(s->d_P.p, Pm.data(), Pm.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "upload P"));
        if (s->ta == DT_SPLIT) {
            DevBuf q32;
            if (q32.alloc(Pf.size() * 4) != hipSuccess)
                return bail(fail(AFQMC_E_NOMEM, "Q staging"));
            if (hipMemcpy(q32.p, Pf.data(), Pf.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                split_planes(q32.as<float>(), s->d_Plp.p, (long)Pf.size(), 1, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return bail(fail(AFQMC_E_DEVICE, "upload Q"));
        } else if (hipMemcpy(s->d_Plp.p, Pf.data(), Pf.size() * 4, hipMemcpyHostToDevice) !=
                   hipSuccess) {
            return bail(fail(AFQMC_E_DEVICE, "upload P"));
        }
    }
    // low-precision copies of the contraction operands
    for (int di = 0; di < n_det; ++di)
        if (s->ts != DT_F64 &&
            convert(det_lhx(s, di).as<double>(), (void*)det_lhx_lp(s, di).p, s->ts,
                    (long)(nc + 1) * NM, st) != hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "convert L^half"));
    if (!ham->d_lp[s->ts].p) {
        if (ham->d_lp[s->ts].alloc((size_t)P * std::max(nc, 1) * dt_size(s->ts)) != hipSuccess)
            return bail(fail(AFQMC_E_NOMEM, "packed L"));
        if (pack_chol(ham->d_chol.as<double>(), ham->d_lp[s->ts].p, s->ts, M, nc, st) != hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "pack L"));
    }
    // walkers: Phi = init (real), w = 1, alive = 1
    {
        const double* src = init_phi ? init_phi : trial;
        std::vector<double> one((size_t)2 * NM, 0.0);
        for (int i = 0; i < N; ++i)
            for (int m = 0; m < M; ++m) one[(size_t)i * M + m] = src[(size_t)m * N + i];
        // one walker up, replicated on the device (phinew serves as staging)
        if (hipMemcpyAsync(s->d_phinew.p, one.data(), 2 * NM * 8, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            broadcast(s->d_phinew.as<double>(), s->d_phi.as<double>(), 2 * NM, nw, st) !=
                hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "upload walkers"));
        std::vector<double> w((size_t)2 * nw, 0.0);
        for (int k = 0; k < nw; ++k) w[par->mode == AFQMC_FREE ? 2 * k : k] = 1.0;
        std::vector<uint8_t> al((size_t)nw, 1);
        if (hipMemcpyAsync(s->d_w.p, w.data(), w.size() * 8, hipMemcpyHostToDevice, st) ||
            hipMemcpyAsync(s->d_alive.p, al.data(), nw, hipMemcpyHostToDevice, st))
            return bail(fail(AFQMC_E_DEVICE, "upload weights"));
        if (hipStreamSynchronize(st) != hipSuccess) return bail(fail(AFQMC_E_DEVICE, "sync"));
    }
    afqmc_status r = overlap_theta(s, s->d_phi.as<double>(), st);
    if (r != AFQMC_OK) return bail(r);
    if (weights(s->d_lnd.as<double>(), s->d_simp.as<double>(), s->d_lnov.as<double>(),
                s->d_w.as<double>(), s->d_alive.as<uint8_t>(), nw, (int)par->mode, 0, 0.0,
                st) != hipSuccess)
        return bail(fail(AFQMC_E_DEVICE, "lnov"));
    std::vector<double> lnov((size_t)2 * nw);
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(lnov.data(), s->d_lnov.p, lnov.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return bail(fail(AFQMC_E_DEVICE, "init overlap"));
    for (int k = 0; k < nw; ++k)
        if (!std::isfinite(lnov[2 * k]))
            return bail(fail(AFQMC_E_SINGULAR, "initial determinant has zero overlap with the trial"));
    // Energy shift: e_shift = Re E_L(initial walker) - c0, c0 = e_core - 1/2 sum a_g^2
    // (the constant of H_1).  A uniform factor e^{dt e_shift} per step on every
    // weight of the system: it cancels in the mixed estimator and keeps the
    // weights O(1) over long runs.
    {
        r = measure(s, st);
        if (r != AFQMC_OK) return bail(r);
        double el0[2];
        if (hipStreamSynchronize(st) != hipSuccess ||
            hipMemcpy(el0, s->d_el.p, sizeof(el0), hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(AFQMC_E_DEVICE, "initial energy"));
        double c0 = ham->e_core;
        for (int g = 0; g < nc; ++g) c0 -= 0.5 * s->a_host[g] * s->a_host[g];
        s->e_shift = el0[0] - c0;
    }
    *out = s;
    return AFQMC_OK;
}

}  // namespace

extern "C" {

afqmc_status afqmc_init_walkers(afqmc_ham ham, int n_alpha, int n_beta, const double* trial,
                                const double* init_phi, int n_walkers, const afqmc_params* par,
                                afqmc_sys* out) {
    const double one = 1.0;
    return init_system(ham, n_alpha, n_beta, 1, &one, trial, init_phi, n_walkers, par, out);
}

afqmc_status afqmc_init_walkers_msd(afqmc_ham ham, int n_alpha, int n_beta, int n_det,
                                    const double* coeffs, const double* dets,
                                    const double* init_phi, int n_walkers,
                                    const afqmc_params* par, afqmc_sys* out) {
    if (!coeffs) return fail(AFQMC_E_INVALID, "null coefficients");
    return init_system(ham, n_alpha, n_beta, n_det, coeffs, dets, init_phi, n_walkers, par, out);
}

void afqmc_free_sys(afqmc_sys s) {
    if (!s || s->dead) return;
    s->dead = true;
    afqmc_ham h = s->ham;
    // release device memory now; the (dead) handle itself stays valid so that
    // later calls on it report E_STATE instead of touching freed memory
    for (DevBuf* b : {&s->d_trialT, &s->d_P, &s->d_Plp, &s->d_a, &s->d_lhx, &s->d_lhx_lp,
                      &s->d_phi, &s->d_phinew, &s->d_theta, &s->d_theta_lp, &s->d_w, &s->d_lnov,
                      &s->d_alive, &s->d_F, &s->d_X, &s->d_simp, &s->d_Apk, &s->d_Af,
                      &s->d_lnd, &s->d_ovl, &s->d_kws, &s->d_exch, &s->d_el, &s->d_sums,
                      &s->d_pc, &s->d_capcount, &s->d_gsmon, &s->d_coef, &s->d_lnd_all, &s->d_F_all,
                      &s->d_el_all, &s->d_rw})
        b->release();
    s->xdet.clear();
    drop_batch_plans(s->id);
    free_adjoint(s);
    s->ham = nullptr;
    if (h) ham_unref(h);
}

afqmc_status afqmc_step(afqmc_sys s, uint64_t seed, uint64_t stream_id, int n_steps,
                        const double* fields_dev) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (n_steps < 0) return fail(AFQMC_E_INVALID, "n_steps < 0");
    hipStream_t st = s->ham->stream;
    for (int i = 0; i < n_steps; ++i) {
        const double* ext = fields_dev ? fields_dev + (size_t)i * s->nw * s->n_chol : nullptr;
        if ((r = one_step(s, seed, stream_id, ext, st)) != AFQMC_OK) return r;
        if (s->par.ortho_every > 0 && s->t % s->par.ortho_every == 0)
            if ((r = ortho(s, st)) != AFQMC_OK) return r;
    }
    return AFQMC_OK;
}

afqmc_status afqmc_orthonormalize(afqmc_sys s) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    return ortho(s, s->ham->stream);
}

afqmc_status afqmc_local_energy(afqmc_sys s, double* e_local, double* weights_out, double* e_mixed) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    hipStream_t st = s->ham->stream;
    if ((r = measure(s, st)) != AFQMC_OK) return r;
    HIPCHK(hipStreamSynchronize(st));
    if (e_local) HIPCHK(hipMemcpy(e_local, s->d_el.p, (size_t)s->nw * 16, hipMemcpyDeviceToHost));
    if (weights_out)
        HIPCHK(hipMemcpy(weights_out, s->d_w.p,
                         (size_t)s->nw * 8 * (s->par.mode == AFQMC_FREE ? 2 : 1),
                         hipMemcpyDeviceToHost));
    if (e_mixed) {
        double sums[4];
        HIPCHK(hipMemcpy(sums, s->d_sums.p, sizeof(sums), hipMemcpyDeviceToHost));
        if (s->par.mode == AFQMC_PHASELESS)
            *e_mixed = sums[0] / sums[1];
        else
            *e_mixed = (sums[0] * sums[2] + sums[1] * sums[3]) / (sums[2] * sums[2] + sums[3] * sums[3]);
    }
    return AFQMC_OK;
}

afqmc_status afqmc_pair_step(afqmc_sys a, afqmc_sys b, uint64_t seed, int n_steps,
                             const double* fields_dev, double* e_trace) {
    int n_meas = 0;
    afqmc_status r = pair_check(a, b, n_steps, &n_meas);
    if (r != AFQMC_OK) return r;
    DevBuf trace;
    HIPCHK(trace.alloc((size_t)std::max(1, n_meas) * 3 * 8));
    return pair_run(a, b, seed, n_steps, fields_dev, e_trace, trace.as<double>(), n_meas);
}

afqmc_status afqmc_cap_events(afqmc_sys s, int64_t* count) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (!count) return fail(AFQMC_E_INVALID, "count is null");
    std::vector<int64_t> c((size_t)s->nw);
    HIPCHK(hipStreamSynchronize(s->ham->stream));
    HIPCHK(hipMemcpy(c.data(), s->d_capcount.p, c.size() * 8, hipMemcpyDeviceToHost));
    int64_t n = 0;
    for (int64_t v : c) n += v;
    *count = n;
    return AFQMC_OK;
}

afqmc_status afqmc_gs_monitor(afqmc_sys s, double threshold, double* max_ell,
                              double* max_lndet, int64_t* trips) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (!(threshold >= 0.0)) return fail(AFQMC_E_INVALID, "threshold must be >= 0");
    hipStream_t st = s->ham->stream;
    std::vector<double> m((size_t)s->nw * 4);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(m.data(), s->d_gsmon.p, m.size() * 8, hipMemcpyDeviceToHost));
    double me = 0.0, ml = 0.0;
    int64_t n = 0;
    for (size_t b = 0; b < m.size(); b += 2) {
        me = std::max(me, m[b]);
        ml = std::max(ml, m[b + 1]);
        n += m[b] > threshold;
    }
    if (max_ell) *max_ell = me;
    if (max_lndet) *max_lndet = ml;
    if (trips) *trips = n;
    HIPCHK(hipMemsetAsync(s->d_gsmon.p, 0, s->d_gsmon.n, st));
    HIPCHK(hipStreamSynchronize(st));
    return AFQMC_OK;
}

afqmc_status afqmc_population_control(afqmc_sys s, double xi) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (s->par.mode != AFQMC_PHASELESS)
        return fail(AFQMC_E_STATE, "population control needs real weights (phaseless mode)");
    if (!(xi >= 0.0 && xi < 1.0)) return fail(AFQMC_E_INVALID, "xi must lie in [0, 1)");
    hipStream_t st = s->ham->stream;
    double* csum = s->d_pc.as<double>();
    int* sel = (int*)(csum + s->nw);
    int* status = sel + s->nw;
    HIPCHK(comb_select(s->d_w.as<double>(), s->d_alive.as<uint8_t>(), s->nw, xi, csum, sel, status,
                       st));
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flag) return fail(AFQMC_E_STATE, "population control: no walker has positive weight");
    HIPCHK(gather_walkers(s->d_phi.as<double>(), s->d_phinew.as<double>(), sel, s->nw,
                          2 * s->NM(), st));
    std::swap(s->d_phi.p, s->d_phinew.p);
    // overlaps and Theta of the copied determinants (the same kernels, so the
    // same values as the originals')
    if ((r = overlap_theta(s, s->d_phi.as<double>(), st)) != AFQMC_OK) return r;
    HIPCHK(weights(s->d_lnd.as<double>(), s->d_simp.as<double>(), s->d_lnov.as<double>(),
                   s->d_w.as<double>(), s->d_alive.as<uint8_t>(), s->nw, (int)s->par.mode, 0, 0.0,
                   st));
    return AFQMC_OK;
}

afqmc_status afqmc_init_from_primary(afqmc_sys sec, afqmc_sys pri) {
    afqmc_status r;
    if ((r = check_sys(sec)) != AFQMC_OK || (r = check_sys(pri)) != AFQMC_OK) return r;
    if (sec == pri) return fail(AFQMC_E_INVALID, "secondary and primary must differ");
    if (sec->M != pri->M || sec->nw != pri->nw)
        return fail(AFQMC_E_SHAPE, "secondary and primary must share M and the walker count");
    if (sec->na > pri->na || sec->nb > pri->nb)
        return fail(AFQMC_E_SHAPE, "the secondary may not have more electrons of a spin");
    if (sec->par.mode != AFQMC_PHASELESS || pri->par.mode != AFQMC_PHASELESS)
        return fail(AFQMC_E_STATE, "the secondary start needs phaseless systems");
    if (sec->ham->stream != pri->ham->stream)
        return fail(AFQMC_E_SHAPE, "secondary and primary need one stream");
    hipStream_t st = pri->ham->stream;
    HIPCHK(take_columns(pri->d_phi.as<double>(), sec->d_phi.as<double>(), sec->nw, sec->M, pri->N,
                        pri->na, sec->N, sec->na, st));
    HIPCHK(hipMemcpyAsync(sec->d_alive.p, pri->d_alive.p, sec->nw, hipMemcpyDeviceToDevice, st));
    if ((r = overlap_theta(sec, sec->d_phi.as<double>(), st)) != AFQMC_OK) return r;
    HIPCHK(weights(sec->d_lnd.as<double>(), sec->d_simp.as<double>(), sec->d_lnov.as<double>(),
                   sec->d_w.as<double>(), sec->d_alive.as<uint8_t>(), sec->nw, 0, 0, 0.0, st));
    HIPCHK(secondary_weights(pri->d_w.as<double>(), pri->d_lnov.as<double>(),
                             sec->d_lnov.as<double>(), sec->d_w.as<double>(),
                             sec->d_alive.as<uint8_t>(), sec->nw, st));
    HIPCHK(hipStreamSynchronize(st));
    sec->t = pri->t;
    return AFQMC_OK;
}

afqmc_status afqmc_get_walkers(afqmc_sys s, double* phi, double* w, double* log_ovlp,
                               unsigned char* alive) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    HIPCHK(hipStreamSynchronize(s->ham->stream));
    if (phi) HIPCHK(hipMemcpy(phi, s->d_phi.p, (size_t)s->nw * 2 * s->NM() * 8, hipMemcpyDeviceToHost));
    if (w)
        HIPCHK(hipMemcpy(w, s->d_w.p, (size_t)s->nw * 8 * (s->par.mode == AFQMC_FREE ? 2 : 1),
                         hipMemcpyDeviceToHost));
    if (log_ovlp) HIPCHK(hipMemcpy(log_ovlp, s->d_lnov.p, (size_t)s->nw * 16, hipMemcpyDeviceToHost));
    if (alive) HIPCHK(hipMemcpy(alive, s->d_alive.p, (size_t)s->nw, hipMemcpyDeviceToHost));
    return AFQMC_OK;
}

afqmc_status afqmc_sys_info(afqmc_sys s, int* M, int* n_chol, int* n_alpha, int* n_beta,
                            int* n_walkers, int64_t* step) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (M) *M = s->M;
    if (n_chol) *n_chol = s->n_chol;
    if (n_alpha) *n_alpha = s->na;
    if (n_beta) *n_beta = s->nb;
    if (n_walkers) *n_walkers = s->nw;
    if (step) *step = s->t;
    return AFQMC_OK;
}

afqmc_status afqmc_checkpoint(afqmc_sys s, void* dst, size_t* bytes) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (!bytes) return fail(AFQMC_E_INVALID, "bytes is null");
    const size_t nphi = (size_t)s->nw * 2 * s->NM() * 8;
    // Theta as the step stores it: FP64, or the copy in the storage type
    const DevBuf& th = s->ts == DT_F64 ? s->d_theta : s->d_theta_lp;
    const size_t nth = (size_t)s->nw * 2 * s->NM() * dt_size(s->ts);
    const size_t need = 64 + nphi + nth + s->d_w.n + s->d_lnov.n + s->nw;
    if (!dst) {
        *bytes = need;
        return AFQMC_OK;
    }
    if (*bytes < need) return fail(AFQMC_E_INVALID, "checkpoint buffer too small");
    HIPCHK(hipStreamSynchronize(s->ham->stream));
    char* p = (char*)dst;
    int64_t hdr[8] = {0x41465143, s->t, s->M, s->N, s->nw, s->n_chol, (int64_t)need, 0};
    memcpy(p, hdr, 64);
    p += 64;
    HIPCHK(hipMemcpy(p, s->d_phi.p, nphi, hipMemcpyDeviceToHost));
    p += nphi;
    HIPCHK(hipMemcpy(p, th.p, nth, hipMemcpyDeviceToHost));
    p += nth;
    HIPCHK(hipMemcpy(p, s->d_w.p, s->d_w.n, hipMemcpyDeviceToHost));
    p += s->d_w.n;
    HIPCHK(hipMemcpy(p, s->d_lnov.p, s->d_lnov.n, hipMemcpyDeviceToHost));
    p += s->d_lnov.n;
    HIPCHK(hipMemcpy(p, s->d_alive.p, s->nw, hipMemcpyDeviceToHost));
    *bytes = need;
    return AFQMC_OK;
}

afqmc_status afqmc_restore(afqmc_sys s, const void* src, size_t bytes) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (!src) return fail(AFQMC_E_INVALID, "src is null");
    const size_t nphi = (size_t)s->nw * 2 * s->NM() * 8;
    const DevBuf& th = s->ts == DT_F64 ? s->d_theta : s->d_theta_lp;
    const size_t nth = (size_t)s->nw * 2 * s->NM() * dt_size(s->ts);
    const size_t need = 64 + nphi + nth + s->d_w.n + s->d_lnov.n + s->nw;
    int64_t hdr[8];
    if (bytes < need) return fail(AFQMC_E_SHAPE, "checkpoint too small for this system");
    memcpy(hdr, src, 64);
    if (hdr[0] != 0x41465143 || hdr[2] != s->M || hdr[3] != s->N || hdr[4] != s->nw ||
        hdr[5] != s->n_chol || hdr[6] != (int64_t)need)
        return fail(AFQMC_E_SHAPE, "checkpoint does not match this system");
    hipStream_t st = s->ham->stream;
    const char* p = (const char*)src + 64;
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(s->d_phi.p, p, nphi, hipMemcpyHostToDevice));
    p += nphi;
    HIPCHK(hipMemcpy(th.p, p, nth, hipMemcpyHostToDevice));
    p += nth;
    HIPCHK(hipMemcpy(s->d_w.p, p, s->d_w.n, hipMemcpyHostToDevice));
    p += s->d_w.n;
    HIPCHK(hipMemcpy(s->d_lnov.p, p, s->d_lnov.n, hipMemcpyHostToDevice));
    p += s->d_lnov.n;
    HIPCHK(hipMemcpy(s->d_alive.p, p, s->nw, hipMemcpyHostToDevice));
    if (s->n_det > 1) {
        // Theta and ln det against every determinant of the expansion, and the
        // weights r_i, from the restored determinants (the same kernels, so
        // the same values as before the snapshot)
        if ((r = overlap_theta(s, s->d_phi.as<double>(), st)) != AFQMC_OK) return r;
        HIPCHK(hipStreamSynchronize(st));
    }
    s->t = hdr[1];
    return AFQMC_OK;
}

afqmc_status afqmc_profile_enable(afqmc_sys s, int enable) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    HIPCHK(s->prof.resolve(s->ham->stream));
    s->prof.reset();
    s->prof.on = enable != 0;
    return AFQMC_OK;
}

afqmc_status afqmc_profile_read(afqmc_sys s, int phase, double* total_ms, int64_t* launches) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if (phase < 0 || phase >= PH_COUNT) return fail(AFQMC_E_INVALID, "phase out of range");
    HIPCHK(s->prof.resolve(s->ham->stream));
    if (total_ms) *total_ms = s->prof.total_ms[phase];
    if (launches) *launches = s->prof.launches[phase];
    return AFQMC_OK;
}

const char* afqmc_phase_name(int phase) {
    return (phase >= 0 && phase < PH_COUNT) ? kPhaseNames[phase] : nullptr;
}

afqmc_status afqmc_selftest_gemm(afqmc_prec prec, int m, int n, int k, const double* A,
                                 const double* B, double* C) {
    if (!A || !B || !C || m <= 0 || n <= 0 || k <= 0) return fail(AFQMC_E_INVALID, "bad args");
    DevBuf dA, dB, dC;
    HIPCHK(dA.alloc((size_t)m * k * 8));
    HIPCHK(dB.alloc((size_t)n * k * 8));
    HIPCHK(dC.alloc((size_t)m * n * 8));
    HIPCHK(hipMemcpy(dA.p, A, (size_t)m * k * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dB.p, B, (size_t)n * k * 8, hipMemcpyHostToDevice));
    Gemm g{};
    g.A = dA.p;
    g.ta = DT_F64;
    g.ra = rows_strided(k);
    g.B = dB.p;
    g.tb = DT_F64;
    g.rb = rows_strided(k);
    g.C = dC.p;
    g.tc = DT_F64;
    g.rc = rows_strided(n);
    g.alpha = 1.0;
    g.m = m;
    g.n = n;
    g.k = k;
    g.batch = 1;
    const DType c = prec == AFQMC_FP64   ? DT_F64
                    : prec == AFQMC_FP32 ? DT_F32
                    : prec == AFQMC_BF16 ? DT_SPLIT
                                         : DT_BF16;
    HIPCHK(gemm(g, c, nullptr));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(C, dC.p, (size_t)m * n * 8, hipMemcpyDeviceToHost));
    return AFQMC_OK;
}

afqmc_status afqmc_selftest_gemm_shape(afqmc_prec prec, int tile, int ksplit, int m, int n, int k,
                                       const double* A, const double* B, double* C) {
    if (!A || !B || !C || m <= 0 || n <= 0 || k <= 0 || tile < 0 || tile > 4 || ksplit < 1)
        return fail(AFQMC_E_INVALID, "bad args");
    if (prec != AFQMC_FP64 && prec != AFQMC_FP32 && prec != AFQMC_BF16)
        return fail(AFQMC_E_INVALID, "precision: fp64, fp32 or split bf16");
    const DType st = prec == AFQMC_FP64 ? DT_F64 : DT_F32;  // operand storage
    const DType c = prec == AFQMC_FP64 ? DT_F64 : prec == AFQMC_FP32 ? DT_F32 : DT_SPLIT;
    const size_t es = dt_size(st);
    std::vector<float> a32, b32;
    const void* ha = A;
    const void* hb = B;
    if (st == DT_F32) {
        a32.assign(A, A + (size_t)m * k);
        b32.assign(B, B + (size_t)n * k);
        ha = a32.data();
        hb = b32.data();
    }
    DevBuf dA, dB, dC, dW;
    HIPCHK(dA.alloc((size_t)m * k * es));
    HIPCHK(dB.alloc((size_t)n * k * es));
    HIPCHK(dC.alloc((size_t)m * n * 8));
    HIPCHK(hipMemcpy(dA.p, ha, (size_t)m * k * es, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dB.p, hb, (size_t)n * k * es, hipMemcpyHostToDevice));
    Gemm g{};
    g.A = dA.p;
    g.ta = st;
    g.ra = rows_strided(k);
    g.B = dB.p;
    g.tb = st;
    g.rb = rows_strided(k);
    g.C = dC.p;
    g.tc = DT_F64;
    g.rc = rows_strided(n);
    g.alpha = 1.0;
    g.m = m;
    g.n = n;
    g.k = k;
    g.batch = 1;
    g.tile = tile;
    if (ksplit > 1) {
        g.ksplit = ksplit;
        HIPCHK(dW.alloc(gemm_ws_bytes(m, n, ksplit, c)));
        g.ws = dW.p;
    }
    HIPCHK(gemm(g, c, nullptr));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(C, dC.p, (size_t)m * n * 8, hipMemcpyDeviceToHost));
    return AFQMC_OK;
}

afqmc_status afqmc_selftest_propagate(afqmc_prec prec, int M, int N, int nw, int K, int variant,
                                      const double* phi, const double* P, const double* A,
                                      double* out) {
    if (!phi || !P || !A || !out || M <= 0 || N <= 0 || nw <= 0 || K < 0)
        return fail(AFQMC_E_INVALID, "bad args");
    if (M > 256) return fail(AFQMC_E_SHAPE, "M <= 256");
    const DType t = prec == AFQMC_FP64 ? DT_F64 : DT_F32;
    const DType ta = prec == AFQMC_BF16X3 ? DT_SPLIT : t;
    if (!propagate_variant_ok(variant, M, t, ta))
        return fail(AFQMC_E_SHAPE, "workgroup shape or precision does not serve this M");
    const size_t nphi = (size_t)nw * 2 * N * M, nA = (size_t)nw * 2 * M * M, nP = (size_t)M * M;
    const size_t nT = ta == DT_SPLIT ? (size_t)split_tile_elems(M) : nP;  // one operand plane
    DevBuf dphi, dout, dP, dA, dA32, dP64, dA64, dlive;
    HIPCHK(dphi.alloc(nphi * 8));
    HIPCHK(dout.alloc(nphi * 8));
    HIPCHK(dP64.alloc(nP * 8));
    HIPCHK(dA64.alloc(nA * 8));
    HIPCHK(dP.alloc(nT * dt_size(t)));
    HIPCHK(dA.alloc((size_t)nw * 2 * nT * dt_size(t)));
    HIPCHK(dlive.alloc(nw));
    HIPCHK(hipMemcpy(dphi.p, phi, nphi * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dP64.p, P, nP * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dA64.p, A, nA * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(dlive.p, 1, nw));
    if (ta == DT_SPLIT) {  // Q = P - I as fragment-tiled hi/lo BF16 planes
        std::vector<float> q(nT, 0.0f);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j)
                q[split_tile_index(M, i, j)] =
                    (float)(P[(size_t)i * M + j] - (i == j ? 1.0 : 0.0));
        DevBuf dq;
        HIPCHK(dq.alloc(nT * 4));
        HIPCHK(hipMemcpy(dq.p, q.data(), nT * 4, hipMemcpyHostToDevice));
        HIPCHK(split_planes(dq.as<float>(), dP.p, (long)nT, 1, nullptr));
        HIPCHK(hipDeviceSynchronize());
    } else {
        HIPCHK(convert(dP64.as<double>(), dP.p, t, (long)nP, nullptr));
    }
    if (ta == DT_SPLIT) {  // each walker plane fragment-tiled, then split
        std::vector<float> at((size_t)nw * 2 * nT, 0.0f);
        for (size_t pl = 0; pl < (size_t)nw * 2; ++pl)
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j)
                    at[pl * nT + split_tile_index(M, i, j)] = (float)A[pl * nP + (size_t)i * M + j];
        HIPCHK(dA32.alloc(at.size() * 4));
        HIPCHK(hipMemcpy(dA32.p, at.data(), at.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(split_planes(dA32.as<float>(), dA.p, (long)nT, 2L * nw, nullptr));
    } else {
        HIPCHK(convert(dA64.as<double>(), dA.p, t, (long)nA, nullptr));
    }
    HIPCHK(propagate(dphi.as<double>(), dout.as<double>(), dP.p, dA.p, dlive.as<uint8_t>(), nw, M,
                     N, K, t, ta, variant, nullptr));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(out, dout.p, nphi * 8, hipMemcpyDeviceToHost));
    return AFQMC_OK;
}

afqmc_status afqmc_selftest_fields(uint64_t seed, uint64_t stream_id, int64_t t, int nw, int n_chol,
                                   double* out) {
    if (!out || nw <= 0 || n_chol <= 0) return fail(AFQMC_E_INVALID, "bad args");
    DevBuf d;
    HIPCHK(d.alloc((size_t)nw * n_chol * 8));
    HIPCHK(philox_normals(seed, stream_id, t, nw, n_chol, d.as<double>(), nullptr));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(out, d.p, (size_t)nw * n_chol * 8, hipMemcpyDeviceToHost));
    return AFQMC_OK;
}

}  // extern "C"
