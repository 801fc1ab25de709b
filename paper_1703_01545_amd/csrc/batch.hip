// Many correlated pairs in one replayed HIP graph, and the launch-shape
// autotuner that picks each system's tiles before capture.
//
// Correlated pairs carry no population control (Sec. II.B), so every pair is
// an independent chain of launches.  The pairs are spread over a few streams
// ("lanes", largest first onto the least-loaded lane) so that small systems
// overlap on the chip, and one period of lcm(ortho_every, measure_every)
// steps of every pair is captured once, with fork/join event edges between
// the lanes, and replayed.  The only values that change between periods are
// the Philox step word and the measurement slot; both are read by the
// kernels from a small device counter block that a node at the end of the
// graph advances.
#include <algorithm>
#include <array>
#include <cstdio>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>

#include "host.h"

using namespace afq;
using namespace afq::host;

namespace afq {
namespace host {
namespace {

// ---------------------------------------------------------------- autotuner

typedef std::array<long, 8> ShapeKey;
std::map<ShapeKey, int> g_tuned;  // problem shape -> fastest candidate
// Guards the process-wide caches (g_tuned, g_plans): calls on unrelated
// handles may come from different host threads.
std::mutex g_cache_mu;

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Average milliseconds of `reps` back-to-back launches after one warm-up.
template <typename F>
hipError_t time_launches(F run, hipStream_t st, int reps, float* ms) {
    hipError_t e = run();
    if (e != hipSuccess) return e;
    EventPair ev;
    if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess)
        return e;
    if ((e = hipEventRecord(ev.a, st)) != hipSuccess) return e;
    for (int r = 0; r < reps; ++r)
        if ((e = run()) != hipSuccess) return e;
    if ((e = hipEventRecord(ev.b, st)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(ev.b)) != hipSuccess) return e;
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, ev.a, ev.b)) != hipSuccess) return e;
    *ms = t / reps;
    return hipSuccess;
}

// Fastest of `cands` for `key` (cached), timing run(candidate) on st.
template <typename F>
hipError_t pick(const ShapeKey& key, const std::vector<int>& cands, F run, hipStream_t st,
                int* out) {
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            *out = it->second;
            return hipSuccess;
        }
    }
    int best = cands.front();
    float best_ms = 1e30f;
    for (int c : cands) {
        float ms = 0.f;
        hipError_t e = time_launches([&] { return run(c); }, st, 3, &ms);
        if (e != hipSuccess) return e;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_tuned[key] = best;
    }
    *out = best;
    return hipSuccess;
}

hipError_t tune_gemm(int role, Gemm g, DType compute, hipStream_t st, int* out) {
    const ShapeKey key{role, g.m, g.n, g.k, g.ta, g.tb, g.tc, compute};
    std::vector<int> cands{1, 2, 3};
    if (compute == DT_SPLIT) cands.push_back(4);
    return pick(key, cands,
                [&](int c) {
                    g.tile = c;
                    return gemm(g, compute, st);
                },
                st, out);
}

// ------------------------------------------------------------- batch graphs

struct Lanes {
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> ev;  // [0]: fork; [1 + j]: join of lane j
    ~Lanes() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto s : st)
            if (s) (void)hipStreamDestroy(s);
    }
    hipError_t create(int n) {
        hipError_t e;
        st.assign(n, nullptr);
        ev.assign(n + 1, nullptr);
        for (int j = 0; j < n; ++j)
            if ((e = hipStreamCreateWithFlags(&st[j], hipStreamNonBlocking)) != hipSuccess) return e;
        for (auto& x : ev)
            if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming)) != hipSuccess) return e;
        return hipSuccess;
    }
};

struct BatchPlan {
    std::vector<uint64_t> ids, seeds;
    int lanes = 0;
    std::vector<void*> phi0;  // d_phi of every system when captured
    int period = 0, meas_per_period = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Lanes ln;
    DevBuf ctr;
    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Never destroyed: graphs and streams must not be released from static
// destructors after the HIP runtime has shut down.
std::vector<std::unique_ptr<BatchPlan>>& g_plans = *new std::vector<std::unique_ptr<BatchPlan>>();

struct Pair {
    afqmc_sys a, b;
    uint64_t seed;
    int index;
    double cost;
};

// Issue `n` steps of every pair on the lanes (fork from lane 0, join back to
// it).  Eager mode records trace rows at trace + 3 (index * rows + slot);
// under capture (ctr != NULL) the slot is relative to the device counters.
afqmc_status issue_steps(const std::vector<std::vector<Pair>>& lanes, Lanes& ln, int n,
                         double* trace, long rows, const std::vector<long>& slot0,
                         const int64_t* ctr) {
    const int L = (int)lanes.size();
    HIPCHK(hipEventRecord(ln.ev[0], ln.st[0]));
    for (int j = 1; j < L; ++j) HIPCHK(hipStreamWaitEvent(ln.st[j], ln.ev[0], 0));
    for (int j = 0; j < L; ++j) {
        hipStream_t st = ln.st[j];
        for (const Pair& p : lanes[j]) {
            const int oe = p.a->par.ortho_every, me = p.a->par.measure_every;
            long slot = ctr ? 0 : slot0[p.index];
            for (int i = 0; i < n; ++i) {
                afqmc_status r;
                if ((r = one_step(p.a, p.seed, 0, nullptr, st)) != AFQMC_OK) return r;
                if ((r = one_step(p.b, p.seed, 0, nullptr, st)) != AFQMC_OK) return r;
                if (oe > 0 && p.a->t % oe == 0) {
                    if ((r = ortho(p.a, st)) != AFQMC_OK) return r;
                    if ((r = ortho(p.b, st)) != AFQMC_OK) return r;
                }
                if (me > 0 && p.a->t % me == 0) {
                    if ((r = measure(p.a, st)) != AFQMC_OK) return r;
                    if ((r = measure(p.b, st)) != AFQMC_OK) return r;
                    double* row = ctr ? nullptr : trace + 3 * (p.index * rows);
                    HIPCHK(trace_record(p.a->d_sums.as<double>(), p.b->d_sums.as<double>(), row,
                                        (int)slot, ctr, p.index, (int)p.a->par.mode, st));
                    ++slot;
                }
            }
        }
    }
    for (int j = 1; j < L; ++j) {
        HIPCHK(hipEventRecord(ln.ev[1 + j], ln.st[j]));
        HIPCHK(hipStreamWaitEvent(ln.st[0], ln.ev[1 + j], 0));
    }
    return AFQMC_OK;
}

// Capture one period of every pair into plan->graph / plan->exec.
afqmc_status capture(BatchPlan* plan, const std::vector<std::vector<Pair>>& lanes,
                     const std::vector<afqmc_sys>& all) {
    int64_t* ctr = plan->ctr.as<int64_t>();
    std::vector<bool> prof(all.size());
    for (size_t i = 0; i < all.size(); ++i) {
        prof[i] = all[i]->prof.on;
        all[i]->prof.on = false;
        all[i]->t_dev = ctr;
        all[i]->t_base = all[i]->t;
    }
    auto restore = [&] {
        for (size_t i = 0; i < all.size(); ++i) {
            all[i]->t = all[i]->t_base;
            all[i]->t_dev = nullptr;
            all[i]->t_base = 0;
            all[i]->prof.on = prof[i];
        }
    };
    hipStream_t s0 = plan->ln.st[0];
    hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        restore();
        return fail(AFQMC_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    afqmc_status r = issue_steps(lanes, plan->ln, plan->period, nullptr, 0, {}, ctr);
    if (r == AFQMC_OK && advance_counters(ctr, plan->period, plan->meas_per_period, s0) != hipSuccess)
        r = fail(AFQMC_E_DEVICE, "advance_counters");
    const std::string msg = g_err;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s0, &g);
    restore();
    if (r != AFQMC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return fail(r, "while capturing: " + msg);
    }
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(AFQMC_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    plan->graph = g;
    e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess)
        return fail(AFQMC_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    for (size_t i = 0; i < all.size(); ++i) plan->phi0[i] = all[i]->d_phi.p;
    return AFQMC_OK;
}

long gcd_l(long x, long y) { return y ? gcd_l(y, x % y) : x; }

constexpr const char* kTuneCacheTag = "afqmc-tune-cache 1";

// The device the tuned shapes belong to: architecture and compute units.
hipError_t device_tag(std::string* tag) {
    int dev = 0;
    hipDeviceProp_t p;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return e;
    *tag = std::string(p.gcnArchName) + " cu=" + std::to_string(p.multiProcessorCount);
    return hipSuccess;
}

// A cached choice a tuner could have made for its key.
bool valid_choice(const ShapeKey& k, int v) {
    if (k[0] == 0 || k[0] == 1) return v >= 1 && v <= (k[7] == DT_SPLIT ? 4 : 3);
    if (k[0] == 3)
        return k[1] > 0 && k[1] <= 256 && propagate_variant_ok(v, (int)k[1], (DType)k[5],
                                                                (DType)k[6]);
    return false;
}

}  // namespace

afqmc_status autotune(afqmc_sys s, hipStream_t st) {
    HIPCHK(tune_gemm(0, force_bias_gemm(s), s->tc, st, &s->tile_fb));
    HIPCHK(tune_gemm(1, field_sum_gemm(s), s->tc, st, &s->tile_fs));
    std::vector<int> cands;
    for (int v = 0; v < kPropVariants; ++v)
        if (propagate_variant_ok(v, s->M, s->tp, s->ta)) cands.push_back(v);
    if (cands.empty()) return fail(AFQMC_E_SHAPE, "no propagation shape serves this M");
    const void* Pm = s->tp == DT_F64 ? s->d_P.p : s->d_Plp.p;
    // the candidates write the step's scratch output (phinew) only
    const ShapeKey key{3, s->M, s->N, s->nw, s->par.taylor_order, s->tp, s->ta, 0};
    HIPCHK(pick(key, cands,
                [&](int v) {
                    return propagate(s->d_phi.as<double>(), s->d_phinew.as<double>(), Pm,
                                     s->d_Af.p, s->d_alive.as<uint8_t>(), s->nw, s->M, s->N,
                                     s->par.taylor_order, s->tp, s->ta, v, st);
                },
                st, &s->prop_var));
    HIPCHK(hipStreamSynchronize(st));
    return AFQMC_OK;
}

void drop_batch_plans(uint64_t id) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (size_t i = 0; i < g_plans.size();) {
        const auto& ids = g_plans[i]->ids;
        if (std::find(ids.begin(), ids.end(), id) != ids.end())
            g_plans.erase(g_plans.begin() + i);
        else
            ++i;
    }
}

}  // namespace host
}  // namespace afq

extern "C" {

afqmc_status afqmc_autotune(afqmc_sys s, int* choice) {
    afqmc_status r = check_sys(s);
    if (r != AFQMC_OK) return r;
    if ((r = autotune(s, s->ham->stream)) != AFQMC_OK) return r;
    if (choice) {
        choice[0] = s->tile_fb;
        choice[1] = s->tile_fs;
        choice[2] = s->prop_var;
    }
    return AFQMC_OK;
}

afqmc_status afqmc_tune_cache_save(const char* path) {
    if (!path) return fail(AFQMC_E_INVALID, "path is null");
    std::string tag;
    if (device_tag(&tag) != hipSuccess) return fail(AFQMC_E_DEVICE, "no device to tag the cache");
    std::map<ShapeKey, int> copy;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        copy = g_tuned;
    }
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(AFQMC_E_INVALID, std::string("cannot write ") + path);
    bool ok = std::fprintf(f, "%s\n%s\n", kTuneCacheTag, tag.c_str()) > 0;
    for (const auto& kv : copy) {
        for (long x : kv.first) ok = ok && std::fprintf(f, "%ld ", x) > 0;
        ok = ok && std::fprintf(f, "%d\n", kv.second) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(AFQMC_E_INVALID, std::string("write failed: ") + path);
    return AFQMC_OK;
}

afqmc_status afqmc_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_tuned.clear();
    return AFQMC_OK;
}

afqmc_status afqmc_tune_cache_load(const char* path) {
    if (!path) return fail(AFQMC_E_INVALID, "path is null");
    std::ifstream in(path);
    if (!in) return fail(AFQMC_E_INVALID, std::string("cannot read ") + path);
    std::string head, dev;
    if (!std::getline(in, head) || head != kTuneCacheTag || !std::getline(in, dev))
        return fail(AFQMC_E_INVALID, "not a tune cache of this library version");
    std::string tag;
    if (device_tag(&tag) != hipSuccess) return fail(AFQMC_E_DEVICE, "no device to check the cache");
    if (dev != tag) return fail(AFQMC_E_INVALID, "tune cache written on another device: " + dev);
    std::vector<std::pair<ShapeKey, int>> rows;
    std::string line;
    while (std::getline(in, line)) {
        if (line.empty()) continue;
        std::istringstream ls(line);
        ShapeKey k;
        int v;
        for (long& x : k)
            if (!(ls >> x)) return fail(AFQMC_E_INVALID, "malformed tune cache line: " + line);
        std::string rest;
        if (!(ls >> v) || (ls >> rest) || !valid_choice(k, v))
            return fail(AFQMC_E_INVALID, "malformed tune cache line: " + line);
        rows.emplace_back(k, v);
    }
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (const auto& kv : rows) g_tuned.emplace(kv.first, kv.second);  // tuned here wins
    return AFQMC_OK;
}

afqmc_status afqmc_pair_batch_step(int n_pairs, const afqmc_sys* a, const afqmc_sys* b,
                                   const uint64_t* seeds, int n_steps, int lanes, int flags,
                                   double* e_traces) {
    if (n_pairs <= 0 || !a || !b || !seeds) return fail(AFQMC_E_INVALID, "empty or null batch");
    if (n_steps < 0) return fail(AFQMC_E_INVALID, "n_steps < 0");
    afqmc_status r;
    std::vector<afqmc_sys> all;
    for (int p = 0; p < n_pairs; ++p) {
        if ((r = check_sys(a[p])) != AFQMC_OK || (r = check_sys(b[p])) != AFQMC_OK) return r;
        all.push_back(a[p]);
        all.push_back(b[p]);
    }
    {
        std::vector<afqmc_sys> sorted(all);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return fail(AFQMC_E_INVALID, "a system appears twice in the batch");
    }
    const afqmc_sys s0 = a[0];
    for (int p = 0; p < n_pairs; ++p) {
        const afqmc_sys x = a[p], y = b[p];
        if (x->M != y->M || x->n_chol != y->n_chol || x->nw != y->nw ||
            x->ham->chol_hash != y->ham->chol_hash)
            return fail(AFQMC_E_SHAPE, "pair " + std::to_string(p) +
                                           ": systems must share M, n_chol, walker count and L");
        for (afqmc_sys z : {x, y}) {
            if (z->par.dt != s0->par.dt || z->par.ortho_every != s0->par.ortho_every ||
                z->par.measure_every != s0->par.measure_every || z->par.mode != s0->par.mode)
                return fail(AFQMC_E_SHAPE, "batch systems must share dt, periods and mode");
            if (z->t != s0->t) return fail(AFQMC_E_STATE, "batch systems are at different steps");
            if (z->ham->stream != s0->ham->stream)
                return fail(AFQMC_E_SHAPE, "batch systems must share one stream");
        }
    }
    const hipStream_t user = s0->ham->stream;
    const int oe = s0->par.ortho_every, me = s0->par.measure_every;
    long period = 1;
    for (int q : {oe, me})
        if (q > 0) period = period / gcd_l(period, q) * q;
    if (period % 2) period *= 2;  // phi / phinew end where they started
    const int meas_pp = me > 0 ? (int)(period / me) : 0;
    int64_t n_meas = 0;
    for (int i = 1; i <= n_steps; ++i)
        if (me > 0 && (s0->t + i) % me == 0) ++n_meas;

    // lanes: largest pair first onto the least-loaded lane
    const int L = std::max(1, std::min(lanes > 0 ? lanes : 4, n_pairs));
    std::vector<Pair> pairs;
    for (int p = 0; p < n_pairs; ++p) {
        const afqmc_sys x = a[p];
        const double M = x->M, K = x->par.taylor_order, nc = x->n_chol;
        double cost = 0.0;
        for (afqmc_sys z : {a[p], b[p]})
            cost += z->nw * ((8.0 * K + 8.0) * z->N * M * M + 4.0 * nc * (z->N * M + z->P()));
        pairs.push_back({a[p], b[p], seeds[p], p, cost});
    }
    std::vector<Pair> order(pairs);
    std::stable_sort(order.begin(), order.end(),
                     [](const Pair& x, const Pair& y) { return x.cost > y.cost; });
    std::vector<std::vector<Pair>> lane_pairs(L);
    std::vector<double> load(L, 0.0);
    for (const Pair& p : order) {
        const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_pairs[j].push_back(p);
        load[j] += p.cost;
    }
    // each lane keeps its pairs in batch order
    for (auto& v : lane_pairs)
        std::sort(v.begin(), v.end(), [](const Pair& x, const Pair& y) { return x.index < y.index; });

    std::vector<uint64_t> ids, sds(seeds, seeds + n_pairs);
    for (afqmc_sys z : all) ids.push_back(z->id);
    const bool use_graph = !(flags & 1);
    BatchPlan* plan = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (auto& pl : g_plans)
            if (pl->ids == ids && pl->seeds == sds && pl->lanes == L) plan = pl.get();
        if (plan) {
            bool same = true;
            for (size_t i = 0; i < all.size(); ++i) same = same && plan->phi0[i] == all[i]->d_phi.p;
            if (!same) {  // odd number of direct steps since capture: capture again
                for (size_t i = 0; i < g_plans.size(); ++i)
                    if (g_plans[i].get() == plan) g_plans.erase(g_plans.begin() + i);
                plan = nullptr;
            }
        }
    }
    if (!plan) {
        auto pl = std::make_unique<BatchPlan>();
        pl->ids = ids;
        pl->seeds = sds;
        pl->lanes = L;
        pl->period = (int)period;
        pl->meas_per_period = meas_pp;
        pl->phi0.assign(all.size(), nullptr);
        HIPCHK(pl->ln.create(L));
        HIPCHK(pl->ctr.alloc(4 * sizeof(int64_t)));
        plan = pl.get();
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_plans.push_back(std::move(pl));
    }
    Lanes& ln = plan->ln;

    DevBuf trace;
    HIPCHK(trace.alloc((size_t)std::max<int64_t>(1, n_meas) * n_pairs * 3 * 8));
    std::vector<long> slot(n_pairs, 0);
    // lane 0 follows the caller's stream
    HIPCHK(hipEventRecord(ln.ev[0], user));
    HIPCHK(hipStreamWaitEvent(ln.st[0], ln.ev[0], 0));

    auto direct = [&](int n) -> afqmc_status {
        if (n <= 0) return AFQMC_OK;
        afqmc_status rr = issue_steps(lane_pairs, ln, n, trace.as<double>(), n_meas, slot, nullptr);
        if (rr != AFQMC_OK) return rr;
        for (int p = 0; p < n_pairs; ++p)
            for (int i = 1; i <= n; ++i)
                if (me > 0 && (a[p]->t - n + i) % me == 0) ++slot[p];
        return AFQMC_OK;
    };
    int left = n_steps;
    if (use_graph) {
        const int head = std::min<long>(left, (period - s0->t % period) % period);
        if ((r = direct(head)) != AFQMC_OK) return r;
        left -= head;
        const int reps = (int)(left / period);
        if (reps > 0) {
            for (afqmc_sys z : all)
                if ((r = autotune(z, ln.st[0])) != AFQMC_OK) return r;
            if (!plan->exec && (r = capture(plan, lane_pairs, all)) != AFQMC_OK) return r;
            HIPCHK(set_counters(plan->ctr.as<int64_t>(), s0->t, slot[0],
                                (int64_t)(uintptr_t)trace.p, n_meas, ln.st[0]));
            for (int k = 0; k < reps; ++k) HIPCHK(hipGraphLaunch(plan->exec, ln.st[0]));
            for (afqmc_sys z : all) z->t += (int64_t)reps * period;
            for (int p = 0; p < n_pairs; ++p) slot[p] += (long)reps * meas_pp;
            left -= reps * (int)period;
        }
    }
    if ((r = direct(left)) != AFQMC_OK) return r;
    HIPCHK(hipEventRecord(ln.ev[0], ln.st[0]));
    HIPCHK(hipStreamWaitEvent(user, ln.ev[0], 0));
    HIPCHK(hipStreamSynchronize(ln.st[0]));
    if (e_traces && n_meas > 0)
        HIPCHK(hipMemcpy(e_traces, trace.p, (size_t)n_meas * n_pairs * 3 * 8,
                         hipMemcpyDeviceToHost));
    return AFQMC_OK;
}

}  // extern "C"
