"""Repeats of a correlated pair on the GPU, and their uncorrelated
counterparts, for the statistics of Sec. II.B (``stats.py``).

Correlated: repeat r is the pair (A_r, B_r) with Philox seed seed0 + r;
walker k of A_r and of B_r draw the same fields at every step, and all
repeats advance together through the batched pair step.  Uncorrelated: the
same systems, but B_r draws from an independent field stream (stream id 1;
A_r keeps stream 0, so A's energies are those of the correlated run).
Returns traces[r, j, :] = (E_A, E_B, E_B - E_A) at every measurement j.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import afqmc as lib


def _systems(ham: "lib.Hamiltonian", spec_a, spec_b, n_walkers: int, n_repeats: int, dt: float,
             **kw) -> List[Tuple["lib.System", "lib.System"]]:
    (na_a, nb_a, trial_a), (na_b, nb_b, trial_b) = spec_a, spec_b
    return [(lib.System(ham, na_a, nb_a, trial_a, n_walkers, dt, **kw),
             lib.System(ham, na_b, nb_b, trial_b, n_walkers, dt, **kw))
            for _ in range(n_repeats)]


def correlated_repeats(ham, spec_a, spec_b, n_walkers: int, n_repeats: int, n_steps: int,
                       dt: float, seed0: int = 0, lanes: int = 0, **kw) -> np.ndarray:
    """spec = (n_alpha, n_beta, trial) per system; kw: System options
    (taylor_order, ortho_every, measure_every, precision)."""
    pairs = _systems(ham, spec_a, spec_b, n_walkers, n_repeats, dt, **kw)
    try:
        return lib.pair_batch_step(pairs, [seed0 + r for r in range(n_repeats)], n_steps,
                                   lanes=lanes)
    finally:
        for a, b in pairs:
            a.free()
            b.free()


def uncorrelated_repeats(ham, spec_a, spec_b, n_walkers: int, n_repeats: int, n_steps: int,
                         dt: float, seed0: int = 0, **kw) -> np.ndarray:
    me = kw.get("measure_every", 20)
    if me <= 0:
        raise ValueError("uncorrelated repeats need a measurement period")
    pairs = _systems(ham, spec_a, spec_b, n_walkers, n_repeats, dt, **kw)
    n_meas = n_steps // me
    out = np.empty((n_repeats, n_meas, 3))
    try:
        for r, (a, b) in enumerate(pairs):
            for j in range(n_meas):
                a.step(me, seed=seed0 + r, stream_id=0)
                b.step(me, seed=seed0 + r, stream_id=1)
                ea, eb = a.local_energy()[2], b.local_energy()[2]
                out[r, j] = (ea, eb, eb - ea)
    finally:
        for a, b in pairs:
            a.free()
            b.free()
    return out
