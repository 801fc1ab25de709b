#!/usr/bin/env python3
"""Throughput benchmark of the correlated-pair ph-AFQMC walker step.

Workload: the M = 200 pair (n_chol = 800, neutral 40/40 vs ion 40/39
electrons, 2048 walkers per system, dt = 0.005, Taylor order 6, modified
Gram-Schmidt every 10 steps, mixed energy every 20 steps), Cholesky
contractions in BF16 with FP32 accumulation, propagator products in FP32,
determinants / Gram-Schmidt / weights in FP64.  One "step" is one pair-step:
both systems advanced one dt, with the periodic Gram-Schmidt and energy
measurement amortised in (steps are a multiple of the measurement period).

Prints one JSON line.  value = walker-steps/s (2 systems x walkers x steps /
wall time of the timed steps, inputs resident in HBM).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "walker-steps/s at M=200, Nw=2048 (pair); ΔE error vs FP64 oracle (kcal/mol)"
EH_TO_KCAL = 627.5095
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
# split-BF16 contractions issue three BF16 products per algorithmic product
ISSUE_FACTOR = {"bf16": 3.0}


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
        "overlap_gemm": 4.0 * M * nsq * nw,
        # one launch per spin; the average over the two spin launches
        "exchange": 0.5 * nw * (4.0 * nc * M * nsq + 8.0 * nc * nsq),
    }.get(name)


def phase_dtype(name, prec):
    """Matrix-core input type of a phase under a precision plan."""
    contract = {"fp64": "fp64", "fp32": "fp32", "bf16": "bf16", "bf16_plain": "bf16"}[prec]
    prop = "fp64" if prec == "fp64" else "fp32"
    return {"force_bias_gemm": contract, "field_sum_gemm": contract, "exchange": contract,
            "propagate": prop, "overlap_gemm": "fp64"}.get(name)


def cpu_baseline(cfg, n_walkers, n_steps):
    """The FP64 oracle, as it stands, on a bounded sample of the same pair."""
    import numpy as np
    from oracle import afqmc as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    ham = cfg.hamiltonian()
    sa = O.System(ham.h, ham.chol, ham.e_core, cfg.trial_a(), cfg.na_a, cfg.nb_a, cfg.dt)
    sb = O.System(ham.h, ham.chol, ham.e_core, cfg.trial_b(), cfg.na_b, cfg.nb_b, cfg.dt)
    wa, wb = O.init_walkers(sa, n_walkers), O.init_walkers(sb, n_walkers)
    t0 = time.perf_counter()
    out = O.run_pair(sa, sb, wa, wb, O.PhiloxFields(cfg.seed, 0, cfg.n_chol), n_steps,
                     cfg.ortho_every, cfg.measure_every)
    el = time.perf_counter() - t0
    assert np.all(np.isfinite(out["dE"]))
    return {"value": 2 * n_walkers * n_steps / el, "unit": "walker-steps/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{n_walkers} walkers per system x {n_steps} pair-steps of the same "
                      f"M={cfg.M} pair (MGS every {cfg.ortho_every}, energy every "
                      f"{cfg.measure_every}), FP64 numpy, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32", "fp64", "bf16_plain"])
    ap.add_argument("--walkers", type=int, default=None, help="override walkers per system")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walkers", type=int, default=4)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-fp64-check", action="store_true",
                    help="skip the FP64 rerun that measures the energy-difference error")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(walkers and pairs are independent, see the sharding notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1703_01545_amd import afqmc as lib
    from synth import config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = config(2)
    if args.walkers:
        cfg = cfg.with_(n_walkers=args.walkers)
    prec = args.precision
    me = cfg.measure_every
    if args.steps % me or args.warmup % me:
        print(f"--steps and --warmup must be multiples of the measurement period {me}",
              file=sys.stderr)
        sys.exit(2)
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

    H, ga, gb = make(prec)
    torch.cuda.synchronize()
    tr_w = lib.pair_step(ga, gb, args.warmup, seed=args.seed)
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
    ga.profile(True)
    gb.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr_t = lib.pair_step(ga, gb, args.steps, seed=args.seed)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof_a, prof_b = ga.profile_read(), gb.profile_read()
    ga.profile(False)
    gb.profile(False)
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
    alive = (ga.walkers()["alive"].mean(), gb.walkers()["alive"].mean())
    trace = np.concatenate([tr_w, tr_t]) if len(tr_w) else tr_t

    ws = 2 * cfg.n_walkers * args.steps / elapsed
    phases = {}
    for name in prof_a:
        ms = prof_a[name][0] + prof_b[name][0]
        n = prof_a[name][1] + prof_b[name][1]
        phases[name] = {"ms_per_step": ms / args.steps, "launches": n,
                        "avg_launch_ms": ms / n if n else 0.0}
    gemm_phases = [p for p in phases if phase_flops(p, 1, 1, 1, 1, 1) is not None]
    dom = max(gemm_phases, key=lambda p: phases[p]["ms_per_step"])
    fl_a = phase_flops(dom, cfg.M, cfg.n_chol, cfg.na_a, cfg.nb_a, cfg.n_walkers)
    fl_b = phase_flops(dom, cfg.M, cfg.n_chol, cfg.na_b, cfg.nb_b, cfg.n_walkers)
    n_a, n_b = prof_a[dom][1], prof_b[dom][1]
    tot_s = (prof_a[dom][0] + prof_b[dom][0]) * 1e-3
    achieved = (fl_a * n_a + fl_b * n_b) / tot_s / 1e12
    dtype = phase_dtype(dom, prec)
    peak = PEAK_TFLOPS[dtype]
    roofline = {"bound": "mfma", "kernel": dom, "kernel_dtype": dtype,
                "flops_per_launch": (fl_a * n_a + fl_b * n_b) / max(n_a + n_b, 1),
                "avg_launch_ms": tot_s * 1e3 / max(n_a + n_b, 1),
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None}

    out = {
        "metric": METRIC, "value": ws, "unit": "walker-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"correlated pair M={cfg.M} n_chol={cfg.n_chol} "
                               f"{cfg.na_a}/{cfg.nb_a} vs {cfg.na_b}/{cfg.nb_b} electrons, "
                               f"{cfg.n_walkers} walkers per system",
                   "M": cfg.M, "n_chol": cfg.n_chol, "n_walkers": cfg.n_walkers, "dt": cfg.dt,
                   "taylor_order": cfg.taylor_order, "ortho_every": cfg.ortho_every,
                   "measure_every": me, "contractions": prec,
                   "walker_arithmetic": "fp64", "parallelism": "single GPU"},
        "roofline": roofline,
        "phases_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in phases.items()},
        "alive_fraction": [float(alive[0]), float(alive[1])],
        "dE_trace_Eh": [float(x) for x in trace[:, 2]],
    }

    if prec != "fp64" and not args.no_fp64_check:
        del ga, gb, H
        H64, fa, fb = make("fp64")
        tr64 = lib.pair_step(fa, fb, args.warmup + args.steps, seed=args.seed)
        err = np.abs(trace[:, 2] - tr64[:, 2])
        out["dE_err_vs_fp64_kcal_per_mol"] = {
            "max": float(err.max() * EH_TO_KCAL), "last": float(err[-1] * EH_TO_KCAL),
            "steps": args.warmup + args.steps,
            "note": "same fields, GPU FP64 path (itself matched to the FP64 oracle at 1e-10)"}
        out["dE_fp64_trace_Eh"] = [float(x) for x in tr64[:, 2]]
        print("[bench] fp64 check done", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_walkers, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
