"""Writes the stored expected values of the GPU parity tests at the sizes of
the benchmark configurations.  Calls only the FP64 oracle (``oracle``) and the
seeded input generators (``synth``); nothing here touches the GPU library.

Walkers are independent under correlated sampling without population control
(Sec. II.B) and walker k's fields depend only on (seed, step, k), so a walker
subset of a large run is reproduced exactly by a small one.

Files (JSON; floats are written with full round-trip precision):

* m100_pair_subset16.json: the M = 100 pair (n_chol = 400, 20/20 vs 20/19
  electrons, dt = 0.005), walkers 0..15, 500 steps, Gram-Schmidt every 10,
  energies every 20, Philox seed 0: per-measurement E_A, E_B, dE of the
  16-walker estimator, and every walker's final weight, ln overlap and alive
  flag in both systems.
* m100_adjoint_subset16.json: the gradient workload (the M = 100 neutral
  system, V = sym(N(0,1))/10 from seed 3): walkers 0..15, 400 steps at
  lambda = 0, then the mixed energy after 100 more steps and its derivative
  dE/dlambda through those 100 steps by the oracle's tangent-linear pass.

Usage: python tests/golden/make_golden.py  (about three minutes on one core)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import afqmc as O  # noqa: E402
from oracle import tangent as T  # noqa: E402
from synth import config, perturbation  # noqa: E402

N_SUB = 16


def _walker_state(wk):
    return {"weight": [float(x) for x in wk.weight],
            "lnov_re": [float(x) for x in wk.lnov.real],
            "lnov_im": [float(x) for x in np.mod(wk.lnov.imag, 2 * np.pi)],
            "alive": [bool(x) for x in wk.alive]}


def pair_subset():
    c = config(1)
    ham = c.hamiltonian()
    sa = O.System(ham.h, ham.chol, ham.e_core, c.trial_a(), c.na_a, c.nb_a, c.dt)
    sb = O.System(ham.h, ham.chol, ham.e_core, c.trial_b(), c.na_b, c.nb_b, c.dt)
    wa, wb = O.init_walkers(sa, N_SUB), O.init_walkers(sb, N_SUB)
    out = O.run_pair(sa, sb, wa, wb, O.PhiloxFields(c.seed, 0, c.n_chol), c.n_steps,
                     c.ortho_every, c.measure_every)
    return {"workload": f"pair M={c.M} n_chol={c.n_chol} {c.na_a}/{c.nb_a} vs {c.na_b}/{c.nb_b}, "
                        f"walkers 0..{N_SUB - 1}, dt={c.dt}, {c.n_steps} steps, "
                        f"Gram-Schmidt every {c.ortho_every}, energies every {c.measure_every}, "
                        f"Philox seed {c.seed} stream 0",
            "seed": c.seed, "n_walkers": N_SUB, "n_steps": c.n_steps,
            "t": [int(x) for x in out["t"]], "EA": out["EA"], "EB": out["EB"], "dE": out["dE"],
            "A": _walker_state(wa), "B": _walker_state(wb)}


def adjoint_subset(seed=0, burn=400, window=100):
    c = config(3)
    ham = c.hamiltonian()
    V = perturbation(c.M, seed=3, scale=0.1)
    s = O.System(ham.h, ham.chol, ham.e_core, c.trial_a(), c.na_a, c.nb_a, c.dt)
    fields = O.PhiloxFields(seed, 0, c.n_chol)
    wk = O.init_walkers(s, N_SUB)
    for _ in range(burn):
        O.step(s, wk, fields(wk.t, N_SUB))
        if wk.t % c.ortho_every == 0:
            O.orthonormalize(s, wk)
    E, dE, _ = T.window_tangent(s, V, wk, fields, window, c.ortho_every)
    return {"workload": f"system M={c.M} n_chol={c.n_chol} {c.na_a}/{c.nb_a}, walkers 0..{N_SUB - 1}, "
                        f"dt={c.dt}, {burn} steps at lambda=0 then dE/dlambda through {window} "
                        f"steps, Gram-Schmidt every {c.ortho_every}, V = sym(N(0,1))/10 (seed 3), "
                        f"Philox seed {seed} stream 0",
            "seed": seed, "n_walkers": N_SUB, "burn": burn, "window": window,
            "E": float(E), "dE_dlambda": float(dE)}


def main():
    for name, fn in (("m100_pair_subset16.json", pair_subset),
                     ("m100_adjoint_subset16.json", adjoint_subset)):
        t0 = time.time()
        data = fn()
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(data, f, indent=1)
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
