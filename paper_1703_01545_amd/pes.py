"""Preliminary equilibration scheme (Sec. II.B) on the GPU: the primary
system is equilibrated alone with population control (the comb every
`pc_every` steps), the secondary system is then started from the primary's
walkers (afqmc_init_from_primary), and the two continue as a correlated pair
without population control."""
from __future__ import annotations

import numpy as np

from . import afqmc as lib


def preliminary_equilibration(primary: "lib.System", secondary: "lib.System", n_steps: int,
                              pc_every: int, seed: int = 0, xi_seed: int = 0) -> None:
    """Advance `primary` n_steps (Philox seed `seed`, stream 0) with the comb
    after every pc_every steps (one uniform xi per comb from
    numpy.random.default_rng(xi_seed)), then start `secondary` from it.
    Afterwards lib.pair_step(primary, secondary, ..., seed=seed) continues the
    pair on the same field counters."""
    if pc_every <= 0:
        raise ValueError("pc_every must be positive")
    rng = np.random.default_rng(xi_seed)
    done = 0
    while done < n_steps:
        n = min(pc_every, n_steps - done)
        primary.step(n, seed=seed)
        done += n
        if n == pc_every:
            primary.population_control(float(rng.random()))
    secondary.init_from_primary(primary)
