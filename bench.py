#!/usr/bin/env python3
"""Throughput benchmark of the correlated-pair ph-AFQMC walker step.

Default workload: the M = 200 pair (n_chol = 800, neutral 40/40 vs ion
40/39 electrons, 2048 walkers per system, dt = 0.005, Taylor order 6,
modified Gram-Schmidt every 10 steps, mixed energy every 20 steps), Cholesky
contractions in split BF16 (hi + lo products) with FP32 accumulation,
propagator products (Taylor terms and one-body halves) in split BF16,
determinants / Gram-Schmidt / weights in FP64.  One "step" is one pair-step:
both systems advanced one dt, with the periodic Gram-Schmidt and energy
measurement in it where the cadence puts them.  The warm-up is rounded up to
whole periods of that cadence (20 steps) so the timed window starts on a
period boundary; exactly --steps steps are timed, replayed from a HIP graph;
a following profiled pass of direct launches (whole periods) gives the
per-kernel times.

--workload batch: 64 uneven pairs (M in 40..240, FP32 contractions unless
--precision says otherwise) stepped together from one graph, against the
same pairs stepped one at a time.
--workload adjoint: dE/dlambda through the last 100 of 500 steps at M = 100
against correlated finite differences.
--workload se_study: standard error of the energy difference over 11 repeats,
correlated against uncorrelated fields, versus basis size and walker count
(FP64 unless --precision says otherwise).

Prints one JSON line.  value = walker-steps/s (2 systems x walkers x steps /
wall time of the timed steps, inputs resident in HBM).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "walker-steps/s at M=200, Nw=2048 (pair); ΔE error vs FP64 oracle (kcal/mol)"
EH_TO_KCAL = 627.5095
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}


def phase_flops(name, M, nc, na, nb, nw, taylor_order=6):
    """Algorithmic FLOPs of one launch of a phase for one system (real FLOPs;
    a complex multiply-add is 8, real x complex 4)."""
    N = na + nb
    P = M * (M + 1) // 2
    nsq = na * na + nb * nb
    return {
        "force_bias_gemm": 4.0 * nw * nc * N * M,
        "field_sum_gemm": 4.0 * nw * nc * P,
        # P T_K(A) P: two real x complex and K complex x complex products
        "propagate": nw * (2 * 4.0 * N * M * M + taylor_order * 8.0 * N * M * M),
        # one launch per spin; the average over the two spin launches
        "exchange": 0.5 * nw * (4.0 * nc * M * nsq + 8.0 * nc * nsq),
    }.get(name)


def phase_dtype(name, prec, M):
    """Matrix-core input type of a phase under a precision plan."""
    contract = {"fp64": "fp64", "fp32": "fp32", "bf16": "bf16", "bf16_plain": "bf16",
                "bf16x3": "bf16"}[prec]
    prop = "fp64" if prec == "fp64" else ("bf16" if prec == "bf16x3" else "fp32")
    return {"force_bias_gemm": contract, "field_sum_gemm": contract, "exchange": contract,
            "propagate": prop}.get(name)


def round_up(n: int, period: int) -> int:
    return -(-n // period) * period if period > 0 else n


def plan_counts(steps: int, warmup: int, profile_steps: int, period: int):
    """Step counts actually run.  The timed steps are exactly the requested
    number; the warm-up is rounded up to a whole number of periods of the
    Gram-Schmidt / measurement cadence so that the timed window starts where
    a period starts (its first measurement and orthonormalisation fall at
    the same offsets as in a long run), and the profiled pass is rounded up
    to whole periods so its per-step phase times carry the amortised
    measurement."""
    if steps <= 0 or warmup < 0 or profile_steps < 0:
        raise ValueError("--steps must be positive; --warmup and --profile-steps non-negative")
    return steps, round_up(warmup, period), round_up(profile_steps, period)


def _cpu_model() -> str:
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def _oracle_rate(cfg, n_walkers, n_steps, threads):
    """Walker-steps/s of the FP64 oracle on n_walkers walkers per system of the
    pair cfg over n_steps pair-steps, BLAS limited to `threads` threads."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import afqmc as O
    ham = cfg.hamiltonian()
    sa = O.System(ham.h, ham.chol, ham.e_core, cfg.trial_a(), cfg.na_a, cfg.nb_a, cfg.dt)
    sb = O.System(ham.h, ham.chol, ham.e_core, cfg.trial_b(), cfg.na_b, cfg.nb_b, cfg.dt)
    wa, wb = O.init_walkers(sa, n_walkers), O.init_walkers(sb, n_walkers)
    with threadpool_limits(limits=threads):
        used = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        t0 = time.perf_counter()
        out = O.run_pair(sa, sb, wa, wb, O.PhiloxFields(cfg.seed, 0, cfg.n_chol), n_steps,
                         cfg.ortho_every, cfg.measure_every)
        el = time.perf_counter() - t0
    assert np.all(np.isfinite(out["dE"]))
    return 2 * n_walkers * n_steps / el, int(used), el


def cpu_baseline(cfg, cfg_small, n_walkers, n_steps):
    """The FP64 oracle, as it stands, on bounded samples: the benchmark pair on
    all host threads (the reported value) and on one thread, and the M = 100
    pair on all threads.  Walkers are independent without population
    control, so a walker subset runs at the full batch's per-walker rate."""
    import numpy as np  # noqa: F401
    host = os.cpu_count() or 1
    v_all, used_all, el_all = _oracle_rate(cfg, n_walkers, n_steps, host)
    v_one, used_one, el_one = _oracle_rate(cfg, n_walkers, n_steps, 1)
    v_s, used_s, el_s = _oracle_rate(cfg_small, 8 * n_walkers, n_steps, host)
    return {"value": v_all, "unit": "walker-steps/s", "cores": used_all, "kind": "oracle",
            "sample": f"{n_walkers} walkers per system x {n_steps} pair-steps of the same "
                      f"M={cfg.M} pair (MGS every {cfg.ortho_every}, energy every "
                      f"{cfg.measure_every}), FP64 numpy/scipy, {used_all} BLAS threads, "
                      f"{el_all:.1f} s",
            "single_thread": {"value": v_one, "cores": used_one,
                              "sample": f"same sample on 1 thread, {el_one:.1f} s"},
            "M100_pair": {"value": v_s, "cores": used_s,
                          "sample": f"{8 * n_walkers} walkers per system x {n_steps} pair-steps "
                                    f"of the M={cfg_small.M} pair, {el_s:.1f} s"},
            "host_cpus": host, "cpu_model": _cpu_model()}


def _traffic(roof, cfg, prec, shapes):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by a copy kernel of known size),
    only while the kernel source, shape and workload are the ones profiled."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))):
        with open(path) as f:
            t = json.load(f)
        h = hashlib.sha256()
        for rel in t.get("sources", [t.get("source")]):
            with open(os.path.join(ROOT, rel), "rb") as f:
                h.update(f.read())
        sha = h.hexdigest()
        if (roof["kernel"] == "propagate" and sha == t["source_sha256"] and prec == t["precision"]
                and cfg.M == t["M"] and cfg.n_walkers == t["n_walkers"]
                and all(s[2] == t["prop_shape"] for s in shapes)):
            rd, wr = t["read_bytes_per_launch"], t["write_bytes_per_launch"]
            roof["traffic"] = rd + wr
            roof["traffic_detail"] = {"read_bytes": rd, "write_bytes": wr,
                                      "kernel": t["kernel"],
                                      "source": "profiles/" + os.path.basename(path)}
            return


def _roofline(prof_a, prof_b, steps, cfg, prec):
    phases = {}
    for name in prof_a:
        ms = prof_a[name][0] + prof_b[name][0]
        n = prof_a[name][1] + prof_b[name][1]
        phases[name] = {"ms_per_step": ms / steps, "launches": n,
                        "avg_launch_ms": ms / n if n else 0.0}
    gemm_phases = [p for p in phases if phase_flops(p, 1, 1, 1, 1, 1) is not None]
    dom = max(gemm_phases, key=lambda p: phases[p]["ms_per_step"])
    fl_a = phase_flops(dom, cfg.M, cfg.n_chol, cfg.na_a, cfg.nb_a, cfg.n_walkers)
    fl_b = phase_flops(dom, cfg.M, cfg.n_chol, cfg.na_b, cfg.nb_b, cfg.n_walkers)
    n_a, n_b = prof_a[dom][1], prof_b[dom][1]
    tot_s = (prof_a[dom][0] + prof_b[dom][0]) * 1e-3
    achieved = (fl_a * n_a + fl_b * n_b) / tot_s / 1e12
    dtype = phase_dtype(dom, prec, cfg.M)
    # split BF16 issues three BF16 products per algorithmic product
    split = prec in ("bf16", "bf16x3") and dtype == "bf16"
    peak = PEAK_TFLOPS[dtype]
    peak_issued = peak / 3 if split else peak
    roof = {"bound": "mfma", "kernel": dom, "kernel_dtype": dtype,
            "flops_per_launch": (fl_a * n_a + fl_b * n_b) / max(n_a + n_b, 1),
            "avg_launch_ms": tot_s * 1e3 / max(n_a + n_b, 1),
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "frac_of_issue_peak": achieved / peak_issued, "traffic": None}
    return phases, roof


def bench_pair(args):
    import numpy as np
    import torch

    from paper_1703_01545_amd import afqmc as lib
    from synth import config

    cfg = config(2)
    if args.walkers:
        cfg = cfg.with_(n_walkers=args.walkers)
    prec = args.precision
    me = cfg.measure_every
    period = math.lcm(cfg.ortho_every, me)
    steps, warmup, profile_steps = plan_counts(args.steps, args.warmup, args.profile_steps, period)
    if profile_steps == 0:
        # the phase times and the roofline come from the profiled pass
        profile_steps = period
        print(f"[bench] --profile-steps 0: {period} steps profiled (the roofline needs them)",
              file=sys.stderr, flush=True)
    ham = cfg.hamiltonian()
    ta, tb = cfg.trial_a(), cfg.trial_b()
    print(f"[bench] M={cfg.M} n_chol={cfg.n_chol} Nw={cfg.n_walkers} precision={prec}",
          file=sys.stderr, flush=True)

    def make(precision):
        H = lib.Hamiltonian(ham.h, ham.chol, ham.e_core)
        kw = dict(taylor_order=cfg.taylor_order, ortho_every=cfg.ortho_every,
                  measure_every=me, precision=precision)
        a = lib.System(H, cfg.na_a, cfg.nb_a, ta, cfg.n_walkers, cfg.dt, **kw)
        b = lib.System(H, cfg.na_b, cfg.nb_b, tb, cfg.n_walkers, cfg.dt, **kw)
        return H, a, b

    def run(a, b, n):
        # one pair through the graph-replayed batch path (captured on first use)
        return lib.pair_batch_step([(a, b)], [args.seed], n, lanes=1)[0]

    H, ga, gb = make(prec)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()
    tr_w = run(ga, gb, warmup)
    print(f"[bench] warmup done ({warmup} steps)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr_t = run(ga, gb, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] timed {steps} graph-replayed steps in {elapsed:.3f} s", file=sys.stderr,
          flush=True)
    # per-kernel HIP events on the launch stream over a profiled pass of the
    # same trajectory (direct launches)
    ga.profile(True)
    gb.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tr_p = lib.pair_step(ga, gb, profile_steps, seed=args.seed)
    torch.cuda.synchronize()
    el_prof = time.perf_counter() - t1
    prof_a, prof_b = ga.profile_read(), gb.profile_read()
    ga.profile(False)
    gb.profile(False)
    alive = (ga.walkers()["alive"].mean(), gb.walkers()["alive"].mean())
    trace = np.concatenate([x for x in (tr_w, tr_t, tr_p) if len(x)])
    if args.metrics_jsonl:
        from paper_1703_01545_amd import metrics

        alive_n = (int(ga.walkers()["alive"].sum()), int(gb.walkers()["alive"].sum()))
        recs = []
        t = 0
        for name, tr, n in (("warmup", tr_w, warmup), ("timed", tr_t, steps),
                            ("profiled", tr_p, profile_steps)):
            recs += list(metrics.trace_records(tr, t, me, **{"pass": name}))
            t += n
        recs.append({"step": t, "alive_A": alive_n[0], "alive_B": alive_n[1],
                     "n_walkers": cfg.n_walkers,
                     "walker_steps_per_s": 2 * cfg.n_walkers * steps / elapsed})
        metrics.write_jsonl(args.metrics_jsonl, recs)
    tuned = [list(lib.autotune(x)) for x in (ga, gb)]  # cached: the shapes the graph used
    phases, roofline = _roofline(prof_a, prof_b, profile_steps, cfg, prec)
    _traffic(roofline, cfg, prec, tuned)
    roofline["measured_over"] = (f"{profile_steps} pair-steps of the same run, direct "
                                 "launches, HIP events around every launch on its stream")

    ws = 2 * cfg.n_walkers * steps / elapsed
    out = {
        "metric": METRIC, "value": ws, "unit": "walker-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "warmup_requested": args.warmup,
        "ms_per_step": elapsed * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"correlated pair M={cfg.M} n_chol={cfg.n_chol} "
                               f"{cfg.na_a}/{cfg.nb_a} vs {cfg.na_b}/{cfg.nb_b} electrons, "
                               f"{cfg.n_walkers} walkers per system",
                   "M": cfg.M, "n_chol": cfg.n_chol, "n_walkers": cfg.n_walkers, "dt": cfg.dt,
                   "taylor_order": cfg.taylor_order, "ortho_every": cfg.ortho_every,
                   "measure_every": me, "contractions": prec,
                   "walker_arithmetic": "fp64", "launch": "HIP graph replay",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "profiled_ms_per_step": el_prof * 1e3 / profile_steps,
        "tuned_shapes": {"fb_tile/fs_tile/prop_shape": tuned},
        "phases_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in phases.items()},
        "alive_fraction": [float(alive[0]), float(alive[1])],
        "dE_trace_Eh": [float(x) for x in trace[:, 2]],
    }

    n_all = warmup + steps + profile_steps
    if prec != "fp64" and not args.no_fp64_check:
        del ga, gb, H
        H64, fa, fb = make("fp64")
        tr64 = run(fa, fb, n_all)
        err = np.abs(trace[:, 2] - tr64[:, 2])
        # statistical scale: spread of the measured dE over the run
        sd = float(np.std(tr64[:, 2])) if len(tr64) > 1 else None
        out["dE_err_vs_fp64_kcal_per_mol"] = {
            "max": float(err.max() * EH_TO_KCAL), "last": float(err[-1] * EH_TO_KCAL),
            "mean_dE_err": float(abs(trace[:, 2].mean() - tr64[:, 2].mean()) * EH_TO_KCAL),
            "steps": n_all,
            "dE_spread_fp64_kcal_per_mol": None if sd is None else sd * EH_TO_KCAL,
            "note": "same fields, GPU FP64 path (itself matched to the FP64 oracle at 1e-10)"}
        out["dE_fp64_trace_Eh"] = [float(x) for x in tr64[:, 2]]
        print("[bench] fp64 check done", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, config(1), args.cpu_walkers, args.cpu_steps)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """64 uneven correlated pairs in one graph-replayed launch sequence vs the
    same pairs stepped one pair at a time."""
    import numpy as np
    import torch

    from paper_1703_01545_amd import afqmc as lib
    from synth import pair_batch_configs

    cfgs = pair_batch_configs(n_pairs=args.pairs)
    prec = args.precision
    me = cfgs[0].measure_every
    steps, warmup, _ = plan_counts(args.steps, args.warmup, 0,
                                   math.lcm(cfgs[0].ortho_every, me))
    pairs, hams, seeds = [], [], []
    t_gen = time.perf_counter()
    for p, c in enumerate(cfgs):
        ham = c.hamiltonian()
        H = lib.Hamiltonian(ham.h, ham.chol, ham.e_core)
        kw = dict(taylor_order=c.taylor_order, ortho_every=c.ortho_every, measure_every=me,
                  precision=prec)
        a = lib.System(H, c.na_a, c.nb_a, c.trial_a(), c.n_walkers, c.dt, **kw)
        b = lib.System(H, c.na_b, c.nb_b, c.trial_b(), c.n_walkers, c.dt, **kw)
        del ham
        hams.append(H)
        pairs.append((a, b))
        seeds.append(args.seed + p)
        if p % 8 == 7:
            print(f"[bench] {p + 1} pairs set up ({time.perf_counter() - t_gen:.0f} s)",
                  file=sys.stderr, flush=True)
    walkers = sum(c.n_walkers for c in cfgs)
    # standalone: one pair at a time, direct launches
    torch.cuda.synchronize()
    solo = []
    for (a, b), sd in zip(pairs, seeds):
        t0 = time.perf_counter()
        lib.pair_step(a, b, steps, seed=sd)
        torch.cuda.synchronize()
        solo.append(time.perf_counter() - t0)
    print(f"[bench] standalone pairs: {sum(solo):.2f} s", file=sys.stderr, flush=True)
    # batch: warm-up (autotune + capture), then timed graph replays
    lib.pair_batch_step(pairs, seeds, warmup, lanes=args.lanes)
    torch.cuda.synchronize()
    print("[bench] batch warmup done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tr = lib.pair_batch_step(pairs, seeds, steps, lanes=args.lanes)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(f"[bench] batch: {el:.2f} s", file=sys.stderr, flush=True)
    choices = {}
    for a, b in pairs:
        for s in (a, b):
            ch = lib.autotune(s)  # cached: returns the shapes the graph uses
            key = f"prop{ch[2]}/fb{ch[0]}/fs{ch[1]}"
            choices[key] = choices.get(key, 0) + 1
    ws = 2 * walkers * steps / el
    fl = 0.0
    for c in cfgs:
        P = c.M * (c.M + 1) // 2
        for na, nb in ((c.na_a, c.nb_a), (c.na_b, c.nb_b)):
            N = na + nb
            fl += c.n_walkers * (4.0 * c.n_chol * N * c.M + 4.0 * c.n_chol * P
                                 + (2 * 4.0 + c.taylor_order * 8.0) * N * c.M * c.M)
    out = {
        "metric": "aggregate walker-steps/s, 64 uneven correlated pairs (batched)",
        "value": ws, "unit": "walker-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": el * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": f"{len(cfgs)} pairs, M in [{min(c.M for c in cfgs)}, "
                               f"{max(c.M for c in cfgs)}], n_chol = 4M, N_sigma = M//5, "
                               f"{walkers} walkers per system in total",
                   "lanes": args.lanes, "launch": "HIP graph replay, autotuned shapes"},
        "standalone_sum_s": sum(solo), "batch_s": el,
        "batch_over_standalone": el / sum(solo),
        "contraction_tflops_per_s": fl * steps / el / 1e12,
        "tuned_shapes": choices,
        "dE_finite": bool(np.all(np.isfinite(tr[:, :, 2]))),
    }
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """dE/dlambda for h -> h + lambda V at M = 100 (512 walkers): 400 steps at
    lambda = 0, then the reverse pass through the last 100 steps, FP64 and
    FP32, against correlated finite differences at lambda = +-1e-3 on the same
    fields (the last 100 steps, and the whole 500-step run for the truncation
    bias of the window).  Timed two ways, each after one untimed pass:
    snapshots every 10 steps (each segment recorded again in reverse), and the
    whole window recorded in the forward pass (3.6 GB here; nothing
    recomputed); both give bitwise the same derivative."""
    import torch

    from paper_1703_01545_amd import afqmc as lib
    from synth import config, perturbation

    cfg = config(3)
    ham = cfg.hamiltonian()
    V = perturbation(cfg.M, seed=3, scale=0.1)
    trial = cfg.trial_a()
    burn, window, every, eps = 400, 100, 10, 1e-3
    kw = dict(taylor_order=cfg.taylor_order, ortho_every=cfg.ortho_every, measure_every=0)
    res = {}
    for prec in ("fp64", "fp32"):
        H = lib.Hamiltonian(ham.h, ham.chol, ham.e_core)
        s = lib.System(H, cfg.na_a, cfg.nb_a, trial, cfg.n_walkers, cfg.dt, precision=prec, **kw)
        s.step(burn, seed=args.seed)
        snap = s.checkpoint()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(window, seed=args.seed)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        # each mode once untimed (buffer and tape allocation), then timed:
        # snapshots every `every` steps (segments recorded again in reverse) and
        # the whole window recorded in the forward pass (nothing recomputed)
        modes = {}
        for name, ce in (("snapshots", every), ("tape", window)):
            for rep in range(2):
                s.restore(snap)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                E = s.adjoint_forward(V, window, seed=args.seed, checkpoint_every=ce,
                                      precision=prec)
                t_af = time.perf_counter() - t0
                t0 = time.perf_counter()
                dE = s.adjoint_backward()
                t_ab = time.perf_counter() - t0
            modes[name] = (E, dE, t_af, t_ab)
        assert modes["tape"][:2] == modes["snapshots"][:2], modes
        E, dE, t_af, t_ab = modes["snapshots"]
        _, _, t_af2, t_ab2 = modes["tape"]
        fd = {}
        for name, steps_pert in (("window", window), ("full", burn + window)):
            e = []
            for lam in (eps, -eps):
                Hl = lib.Hamiltonian(ham.h + lam * V, ham.chol, ham.e_core)
                sl = lib.System(Hl, cfg.na_a, cfg.nb_a, trial, cfg.n_walkers, cfg.dt,
                                precision=prec, **kw)
                if name == "window":
                    sl.restore(snap)
                    sl.step(window, seed=args.seed)
                else:
                    sl.step(burn + window, seed=args.seed)
                e.append(sl.local_energy()[2])
                del sl, Hl
            fd[name] = (e[0] - e[1]) / (2 * eps)
        res[prec] = {"E": E, "dE_dlambda": dE, "fd_window": fd["window"], "fd_full": fd["full"],
                     "rel_err_vs_fd_window": abs(dE - fd["window"]) / abs(fd["window"]),
                     "forward_window_s": t_fwd, "adjoint_forward_s": t_af,
                     "adjoint_backward_s": t_ab,
                     "adjoint_cost_over_forward": (t_af + t_ab) / t_fwd,
                     "tape_adjoint_forward_s": t_af2, "tape_adjoint_backward_s": t_ab2,
                     "tape_adjoint_cost_over_forward": (t_af2 + t_ab2) / t_fwd}
        print(f"[bench] adjoint {prec}: dE={dE:.10g} fd={fd['window']:.10g}", file=sys.stderr,
              flush=True)
    out = {"metric": "dE_mixed/dlambda through the last 100 steps (reverse mode) vs correlated FD",
           "value": res["fp64"]["dE_dlambda"], "unit": "Eh per unit lambda", "n_gpus": 1,
           "steps": window, "warmup": burn, "higher_is_better": None, "vs_baseline": None,
           "dtype": "fp64", "data": "synthetic",
           "config": {"workload": f"M={cfg.M} n_chol={cfg.n_chol} {cfg.na_a}/{cfg.nb_a} electrons, "
                                  f"{cfg.n_walkers} walkers, V = sym(N(0,1))/10, window {window} "
                                  f"of {burn + window} steps, snapshots every {every}",
                      "fd_step": eps},
           "results": res}
    print(json.dumps(out), flush=True)


def bench_se_study(args):
    """Synthetic analogue of the paper's efficiency study (Sec. II.B, III.C):
    11 repeats of neutral/ion pairs (n_chol = 4M, N_sigma = M/5, the ion one
    beta electron short) propagated to tau = 3 with dt = 0.01 (MGS every 0.05,
    energies every 0.1), fields correlated between the two systems or not.
    The standard error of the cumulative averages of dE after tau = 1, over
    the repeats, against the basis size M (at 32 walkers) and against the
    walker count (at M = 48).  Since the error falls as 1/sqrt(walkers), an
    uncorrelated run needs (SE_unc / SE_cor)^2 times the walkers, and so that
    much more time, to reach the correlated error at the same tau."""
    import numpy as np

    from paper_1703_01545_amd import afqmc as lib
    from paper_1703_01545_amd import repeats, stats
    from synth import make_hamiltonian, make_trial

    n_rep, dt, steps, me, oe, j_eq = 11, 0.01, 300, 10, 5, 10
    rows = []
    cases = [(24, 32), (48, 32), (96, 32), (48, 8), (48, 128)]
    t_all = time.perf_counter()
    for M, nw in cases:
        ham = make_hamiltonian(M, 4 * M, seed=50 + M)
        H = lib.Hamiltonian(ham.h, ham.chol, ham.e_core)
        n = M // 5
        sa = (n, n, make_trial(ham.h, n, n))
        sb = (n, n - 1, make_trial(ham.h, n, n - 1))
        kw = dict(ortho_every=oe, measure_every=me, precision=args.precision)
        t0 = time.perf_counter()
        cor = repeats.correlated_repeats(H, sa, sb, nw, n_rep, steps, dt, seed0=args.seed, **kw)
        unc = repeats.uncorrelated_repeats(H, sa, sb, nw, n_rep, steps, dt, seed0=args.seed,
                                           **kw)
        el = time.perf_counter() - t0
        ec = stats.final_estimate(cor[:, :, 2], j_eq)
        eu = stats.final_estimate(unc[:, :, 2], j_eq)
        se_c = stats.mean_and_se(stats.cumulative_averages(cor[:, :, 2], j_eq), axis=0)[1]
        se_u = stats.mean_and_se(stats.cumulative_averages(unc[:, :, 2], j_eq), axis=0)[1]
        rows.append({"M": M, "n_chol": 4 * M, "electrons": [n, n, n, n - 1], "walkers": nw,
                     "dE_correlated": ec.value, "se_correlated": ec.se,
                     "dE_uncorrelated": eu.value, "se_uncorrelated": eu.se,
                     "se_at_tau3_correlated": float(se_c[-1]),
                     "se_at_tau3_uncorrelated": float(se_u[-1]),
                     "walker_factor_for_equal_error": float((se_u[-1] / se_c[-1]) ** 2),
                     "seconds": el})
        print(f"[bench] M={M} Nw={nw}: SE cor {se_c[-1]:.2e} unc {se_u[-1]:.2e} ({el:.1f} s)",
              file=sys.stderr, flush=True)
        del H
    factors = [r["walker_factor_for_equal_error"] for r in rows]
    out = {"metric": "walker (CPU-time) factor for equal standard error of dE, uncorrelated "
                     "over correlated sampling, 11 repeats, tau = 3",
           "value": float(np.median(factors)), "unit": "x", "n_gpus": 1,
           "higher_is_better": True, "vs_baseline": None, "dtype": args.precision,
           "data": "synthetic",
           "config": {"workload": "neutral/ion pairs, n_chol = 4M, N_sigma = M/5, dt = 0.01, "
                                  "300 steps, 11 repeats, equilibration tau = 1",
                      "cases": [[M, nw] for M, nw in cases]},
           "rows": rows, "seconds": time.perf_counter() - t_all}
    print(json.dumps(out), flush=True)


def make_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="pair", choices=["pair", "batch", "adjoint", "se_study"])
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--precision", default=None,
                    choices=["bf16", "bf16x3", "fp32", "fp64", "bf16_plain"],
                    help="precision plan (default: bf16x3 for the pair, fp32 contractions for the "
                         "batch as its configuration states, fp64 for the SE study)")
    ap.add_argument("--walkers", type=int, default=None, help="override walkers per system")
    ap.add_argument("--pairs", type=int, default=64, help="batch workload: number of pairs")
    ap.add_argument("--lanes", type=int, default=4, help="batch workload: stream lanes")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walkers", type=int, default=4,
                    help="oracle sample: walkers per system (M = 200; eight times as many at M = 100)")
    ap.add_argument("--cpu-steps", type=int, default=40, help="oracle sample: pair-steps")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy a buffer of this size once (device to device) before the timed "
                         "steps: the reference kernel for scaling HBM traffic counters")
    ap.add_argument("--metrics-jsonl", default=None,
                    help="pair workload: write every measurement (step, E_A, E_B, dE, pass) and the "
                         "end-of-run alive counts to this file as JSON lines")
    ap.add_argument("--no-fp64-check", action="store_true",
                    help="skip the FP64 rerun that measures the energy-difference error")
    return ap


def main(argv=None):
    args = make_parser().parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (walkers and "
              "pairs are independent; sharding them across GPUs is described in the design "
              "notes).", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.precision is None:
        args.precision = {"batch": "fp32", "se_study": "fp64"}.get(args.workload, "bf16x3")
    if args.workload == "batch":
        bench_batch(args)
    elif args.workload == "adjoint":
        bench_adjoint(args)
    elif args.workload == "se_study":
        bench_se_study(args)
    else:
        bench_pair(args)


if __name__ == "__main__":
    main()
