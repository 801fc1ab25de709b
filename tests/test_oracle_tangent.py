"""Pins of the oracle's tangent-linear dE/dlambda (h -> h + lambda V).

* correlated finite differences: the same fields at lambda = +-eps through
  the oracle's own (separately pinned) forward step, central difference;
* V = c I: every one-body energy moves by c N while the propagator only
  rescales every walker alike, so dE/dlambda = c N exactly;
* one-body limit (no Cholesky vectors): the walkers are e^{-tau (h + lambda V)}
  Phi_0 in closed form; its derivative by a complex step (no cancellation)
  through scipy's expm.
"""
import numpy as np
import pytest

from oracle import afqmc as O
from oracle import tangent as T
from synth import make_hamiltonian, make_trial, perturbation, random_walkers


def _system(M, nc, na, nb, dt, seed=0, V=None, lam=0.0):
    ham = make_hamiltonian(M, nc, seed=seed, e_core=0.3)
    trial = make_trial(ham.h, na, nb)
    return O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt, h_pert=V, lam=lam)


def _burn_in(sys, nw, n, oe, fields):
    wk = O.init_walkers(sys, nw)
    for _ in range(n):
        O.step(sys, wk, fields(wk.t, nw))
        if wk.t % oe == 0:
            O.orthonormalize(sys, wk)
    return wk


@pytest.mark.parametrize("na,nb", [(3, 3), (3, 2)])
def test_tangent_matches_correlated_fd(na, nb):
    M, nc, dt, nw = 12, 36, 0.01, 12
    V = perturbation(M, seed=3, scale=0.1)
    fields = O.PhiloxFields(11, 0, nc)
    s0 = _system(M, nc, na, nb, dt)
    wk = _burn_in(s0, nw, 15, 5, fields)
    E, dE, _ = T.window_tangent(s0, V, wk, fields, 20, 5)
    eps = 1e-4
    ep = T.window_energy(_system(M, nc, na, nb, dt, V=V, lam=eps), wk, fields, 20, 5)
    em = T.window_energy(_system(M, nc, na, nb, dt, V=V, lam=-eps), wk, fields, 20, 5)
    e0 = T.window_energy(s0, wk, fields, 20, 5)
    assert abs(E - e0) <= 1e-12 * abs(e0)
    fd = (ep - em) / (2 * eps)
    assert abs(dE) > 1e-3
    assert abs(dE - fd) <= 1e-8 * abs(fd), (dE, fd)


def test_tangent_identity_perturbation_is_c_times_n():
    M, nc, na, nb, dt = 12, 36, 3, 2, 0.01
    c = 0.7
    s0 = _system(M, nc, na, nb, dt)
    fields = O.PhiloxFields(5, 0, nc)
    wk = _burn_in(s0, 8, 10, 5, fields)
    _, dE, _ = T.window_tangent(s0, c * np.eye(M), wk, fields, 10, 5)
    assert abs(dE - c * (na + nb)) <= 1e-10 * c * (na + nb)


def test_tangent_one_body_limit_complex_step():
    M, na, nb, dt, n = 10, 3, 2, 0.02, 15
    ham = make_hamiltonian(M, 0, seed=4, e_core=0.1)
    trial = make_trial(ham.h, na, nb)
    sys = O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt)
    phi0 = random_walkers(M, na + nb, 1, seed=9, complex_=False)[0]
    wk = O.init_walkers(sys, 2, init_phi=phi0)
    V = perturbation(M, seed=3, scale=0.1)
    E, dE, _ = T.window_tangent(sys, V, wk, O.ExplicitFields(np.zeros((n + 1, 2, 0))), n, 4)

    def energy(lam):
        prop = __import__("scipy").linalg.expm(-n * dt * (ham.h + lam * V))
        e = ham.e_core + 0j
        for off, k in ((0, na), (na, nb)):
            t = trial[:, off:off + k]
            ph = prop @ phi0[:, off:off + k]
            th = ph @ np.linalg.inv(t.T @ ph)
            e += np.trace(t.T @ (ham.h + lam * V) @ th)
        return e

    h = 1e-20
    assert abs(E - energy(0.0).real) <= 1e-11 * abs(E)
    assert abs(dE - energy(1j * h).imag / h) <= 1e-9 * abs(dE)
