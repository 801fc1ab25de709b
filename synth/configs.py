"""Synthetic Hamiltonians, trials, walkers and fields (seeded, numpy only).

The paper's molecular integrals are not available, so seeded random
Hamiltonians with the paper's structure stand in for them: a real one-body
matrix h and real symmetric Cholesky vectors L_gamma whose products give the
two-body matrix elements (Sec. II.A, Eq. 1).  The recipe:

* h = diag(linspace(-2, 1, M)) + sym(G)/sqrt(M), G_ij ~ N(0, 1);
* L_gamma = sym(G_gamma) * 0.3 * exp(-gamma/10) * sqrt(12/M), gamma = 0..n_chol-1
  (the M = 12 recipe with its random parts scaled by 1/sqrt(M), so the
  spectrum of every L_gamma stays that of the M = 12 case; without the
  factor the force bias diverges and every walker is frozen within ten steps
  at M = 200);
* sym(G) = (G + G^T)/2;
* draws come from numpy.random.default_rng(seed): h's random part first, then
  the L_gamma in gamma order;
* the trial determinant of a system with (n_alpha, n_beta) electrons holds the
  lowest n_alpha (resp. n_beta) eigenvectors of h, each with its
  largest-magnitude component made positive; alpha columns come first.

A correlated pair is a neutral system and its ion with one fewer beta electron
on the same h and L, the vertical-ionisation setting of Sec. II.C.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np


def _sym(g: np.ndarray) -> np.ndarray:
    return 0.5 * (g + np.swapaxes(g, -1, -2))


@dataclass
class Hamiltonian:
    """h (M x M), chol (n_chol x M x M), e_core; all float64, all symmetric."""

    h: np.ndarray
    chol: np.ndarray
    e_core: float = 0.0

    @property
    def M(self) -> int:
        return self.h.shape[0]

    @property
    def n_chol(self) -> int:
        return self.chol.shape[0]


def make_hamiltonian(M: int, n_chol: int, seed: int = 0, e_core: float = 0.0,
                     chol_scale: float = 0.3, chol_decay: float = 10.0,
                     ref_M: int = 12) -> Hamiltonian:
    rng = np.random.default_rng(seed)
    h = np.diag(np.linspace(-2.0, 1.0, M)) + _sym(rng.standard_normal((M, M))) / np.sqrt(M)
    chol = np.empty((n_chol, M, M))
    size_scale = np.sqrt(ref_M / M)
    for g in range(n_chol):
        chol[g] = (_sym(rng.standard_normal((M, M))) * chol_scale * np.exp(-g / chol_decay)
                   * size_scale)
    return Hamiltonian(h=np.ascontiguousarray(h), chol=chol, e_core=float(e_core))


def make_trial(h: np.ndarray, n_alpha: int, n_beta: int) -> np.ndarray:
    """M x (n_alpha + n_beta) real trial: lowest eigenvectors of h per spin."""
    _, vec = np.linalg.eigh(h)
    idx = np.argmax(np.abs(vec), axis=0)
    sgn = np.sign(vec[idx, np.arange(vec.shape[1])])
    sgn[sgn == 0] = 1.0
    vec = vec * sgn
    return np.ascontiguousarray(np.concatenate([vec[:, :n_alpha], vec[:, :n_beta]], axis=1))


def make_expansion(h: np.ndarray, n_alpha: int, n_beta: int, n_det: int, seed: int = 0,
                   n_act: int = 3, scale: float = 0.25):
    """Synthetic multi-determinant trial in the form of a truncated CASSCF
    expansion: the orbitals are the eigenvectors of h (signs as in
    make_trial); determinant 0 occupies the lowest n_alpha / n_beta of them;
    the others are distinct single and double excitations, per spin, from
    the highest n_act occupied into the lowest n_act virtual orbitals, with
    coefficients scale * N(0, 1) (determinant 0 has coefficient 1).  Returns
    (coeffs (n_det,), dets (n_det, M, n_alpha + n_beta)), alpha columns first."""
    M = h.shape[0]
    vec = make_trial(h, M, 0)  # all eigenvectors, ascending, sign-fixed
    rng = np.random.default_rng(seed)

    def excite(n):
        occ = list(range(n))
        holes = occ[max(0, n - n_act):]
        parts = list(range(n, min(M, n + n_act)))
        k = int(rng.integers(1, 3)) if holes and parts else 0
        k = min(k, len(holes), len(parts))
        h_ = sorted(rng.choice(holes, size=k, replace=False).tolist()) if k else []
        p_ = sorted(rng.choice(parts, size=k, replace=False).tolist()) if k else []
        return tuple(sorted([o for o in occ if o not in h_] + p_))

    seen = {(tuple(range(n_alpha)), tuple(range(n_beta)))}
    occs = [next(iter(seen))]
    tries = 0
    while len(occs) < n_det and tries < 10000:
        tries += 1
        cand = (excite(n_alpha), excite(n_beta))
        if cand not in seen:
            seen.add(cand)
            occs.append(cand)
    if len(occs) < n_det:
        raise ValueError("active space too small for the requested number of determinants")
    coeffs = np.concatenate([[1.0], scale * rng.standard_normal(n_det - 1)])
    dets = np.stack([np.concatenate([vec[:, list(a)], vec[:, list(b)]], axis=1) for a, b in occs])
    return coeffs, np.ascontiguousarray(dets)


def perturbation(M: int, seed: int = 3, scale: float = 0.1) -> np.ndarray:
    """Random symmetric one-body perturbation V with entries N(0,1)*scale."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_sym(rng.standard_normal((M, M))) * scale)


def gaussian_fields(seed: int, n_steps: int, n_walkers: int, n_chol: int) -> np.ndarray:
    """Explicit auxiliary fields x[t, k, gamma] ~ N(0, 1), float64, C order."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_steps, n_walkers, n_chol))


def random_walkers(M: int, n_orb: int, n_walkers: int, seed: int = 7,
                   complex_: bool = True) -> np.ndarray:
    """Random walker determinants, shape (n_walkers, M, n_orb)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n_walkers, M, n_orb))
    if complex_:
        w = w + 1j * rng.standard_normal((n_walkers, M, n_orb))
    return w


@dataclass
class PairConfig:
    """One correlated pair run: system A (primary) and B (secondary)."""

    name: str
    M: int
    n_chol: int
    na_a: int
    nb_a: int
    na_b: int
    nb_b: int
    n_walkers: int
    dt: float
    n_steps: int
    taylor_order: int = 6
    ortho_every: int = 10
    measure_every: int = 20
    seed: int = 0
    ham_seed: int = 0
    precision: str = "fp64"
    _ham: Optional[Hamiltonian] = field(default=None, repr=False, compare=False)

    def hamiltonian(self) -> Hamiltonian:
        if self._ham is None:
            self._ham = make_hamiltonian(self.M, self.n_chol, seed=self.ham_seed)
        return self._ham

    def trial_a(self) -> np.ndarray:
        return make_trial(self.hamiltonian().h, self.na_a, self.nb_a)

    def trial_b(self) -> np.ndarray:
        return make_trial(self.hamiltonian().h, self.na_b, self.nb_b)

    def with_(self, **kw) -> "PairConfig":
        c = replace(self, **kw)
        if any(k in kw for k in ("M", "n_chol", "ham_seed")):
            c._ham = None
        return c


def config(i: int) -> PairConfig:
    """The four single-pair workloads (M = 12, 100, 200, and the gradient case)."""
    if i == 0:
        return PairConfig("pair-M12-fp64", M=12, n_chol=36, na_a=3, nb_a=3, na_b=3, nb_b=2,
                          n_walkers=64, dt=0.01, n_steps=200, taylor_order=6,
                          ortho_every=5, measure_every=1)
    if i == 1:
        return PairConfig("pair-M100-fp64", M=100, n_chol=400, na_a=20, nb_a=20, na_b=20, nb_b=19,
                          n_walkers=1024, dt=0.005, n_steps=500, ortho_every=10,
                          measure_every=20)
    if i == 2:
        return PairConfig("pair-M200-mixed", M=200, n_chol=800, na_a=40, nb_a=40, na_b=40, nb_b=39,
                          n_walkers=2048, dt=0.005, n_steps=200, ortho_every=10,
                          measure_every=20, precision="bf16")
    if i == 3:
        return PairConfig("adjoint-M100", M=100, n_chol=400, na_a=20, nb_a=20, na_b=20, nb_b=19,
                          n_walkers=512, dt=0.005, n_steps=500, ortho_every=10,
                          measure_every=20)
    raise ValueError(f"no single-pair configuration {i}")


def pair_batch_configs(n_pairs: int = 64, seed: int = 0, m_lo: int = 40, m_hi: int = 240,
                       nw_lo: int = 128, nw_hi: int = 2048) -> List[PairConfig]:
    """Uneven batch of pairs: M ~ U{m_lo..m_hi}, n_chol = 4M, N_sigma = M // 5
    (ion lacks one beta electron), Nw ~ U{nw_lo..nw_hi}; M then Nw per pair
    from default_rng(seed); pair p's Hamiltonian uses seed 1000 + p."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(n_pairs):
        M = int(rng.integers(m_lo, m_hi + 1))
        nw = int(rng.integers(nw_lo, nw_hi + 1))
        n = M // 5
        out.append(PairConfig(f"batch-pair{p}-M{M}", M=M, n_chol=4 * M, na_a=n, nb_a=n,
                              na_b=n, nb_b=n - 1, n_walkers=nw, dt=0.005, n_steps=200,
                              ortho_every=10, measure_every=20, ham_seed=1000 + p,
                              precision="fp32"))
    return out
