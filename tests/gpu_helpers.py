"""Shared helpers of the GPU parity tests: build the same workload for the
HIP path and the oracle from the seeded generators in ``synth``."""
from __future__ import annotations

import sys

import numpy as np

from oracle import afqmc as O
from synth import gaussian_fields, make_hamiltonian, make_trial


def banner(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b) -> float:
    a, b = np.asarray(a), np.asarray(b)
    den = np.max(np.abs(b)) if b.size else 1.0
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0)) if b.size else 0.0


def phase_diff(a, b):
    """|exp(i a) - exp(i b)| for imaginary parts of logs (defined mod 2 pi)."""
    return np.abs(np.exp(1j * np.asarray(a)) - np.exp(1j * np.asarray(b)))


class Workload:
    """A correlated pair on one seeded Hamiltonian."""

    def __init__(self, M, n_chol, na_a, nb_a, na_b, nb_b, nw, dt, ham_seed=0, e_core=0.0):
        self.ham = make_hamiltonian(M, n_chol, seed=ham_seed, e_core=e_core)
        self.M, self.n_chol, self.nw, self.dt = M, n_chol, nw, dt
        self.spins = ((na_a, nb_a), (na_b, nb_b))
        self.trials = [make_trial(self.ham.h, na, nb) for na, nb in self.spins]

    def oracle_systems(self, K=6):
        return [O.System(self.ham.h, self.ham.chol, self.ham.e_core, t, na, nb, self.dt,
                         taylor_order=K) for t, (na, nb) in zip(self.trials, self.spins)]

    def gpu_systems(self, lib, precision="fp64", K=6, ortho_every=10, measure_every=20, nw=None):
        H = lib.Hamiltonian(self.ham.h, self.ham.chol, self.ham.e_core)
        out = []
        for t, (na, nb) in zip(self.trials, self.spins):
            out.append(lib.System(H, na, nb, t, self.nw if nw is None else nw, self.dt,
                                  taylor_order=K, ortho_every=ortho_every,
                                  measure_every=measure_every, precision=precision))
        return H, out

    def fields(self, n_steps, seed=0):
        return gaussian_fields(seed, n_steps, self.nw, self.n_chol)
