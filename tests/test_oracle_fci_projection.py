"""Pins of the oracle's weights, estimator and multi-step projection against
dense determinant-space (FCI) quantities.

* The phaseless weight update (Sec. II.A, with the hybrid weight of
  Sec. II.D): the factor one step gives a walker equals |I| max(0, cos arg R)
  with R and I computed from the FCI propagator, for walkers on both sides
  of the projection, including ones where the phases of R and I disagree
  in sign.
* The mixed estimator with unequal complex weights (Eq. 7): a Gauss-Hermite
  population of one-step walkers, each carrying its quadrature weight times
  its free-projection weight, must give the FCI ratio
  <phi_T|H B|phi>/<phi_T|B|phi> of the Trotter propagator B (one Cholesky
  vector: the Hubbard-Stratonovich identity is exact).  The phaseless
  branch: splitting a walker into two of half the weight, and adding frozen
  walkers, leave the estimate unchanged.
* Free projection and importance-sampled free projection over many steps
  (Sec. II.A; the time-step extrapolation of Sec. II.D): E(tau) at three
  time steps, extrapolated linearly to dt -> 0, matches the exact
  <phi_T|H e^{-tau H}|phi_T>/<phi_T|e^{-tau H}|phi_T> within three standard
  errors over independent seeds.
"""
import numpy as np
import pytest

from oracle import afqmc as O
from oracle import fci
from synth import make_hamiltonian, make_trial, random_walkers


class FciStep:
    """Dense FCI-sector pieces of one walker step for a tiny Hamiltonian:
    rho_g, a_g = <rho_g>_T, H2 = 1/2 sum_g (rho_g - a_g)^2 (Eq. 2 with
    v = i rho), the one-body half e^{-dt H1/2} with H1 = H - H2, and the
    constant c0 of H1 that the walker step drops."""

    def __init__(self, ham, trial, na, nb, dt):
        M = ham.h.shape[0]
        self.sec = fci.Sector(M, na, nb)
        ops = self.sec.one_body_ops()
        self.H = fci.hamiltonian(self.sec, ham.h, ham.chol, ham.e_core, ops)
        self.rho = fci.rho_ops(ops, ham.chol)
        self.vt = self.sec.slater(trial)
        self.a = np.array([(self.vt @ r @ self.vt) / (self.vt @ self.vt) for r in self.rho]).real
        self.eye = np.eye(self.sec.dim)
        H2 = sum(0.5 * (r - ai * self.eye) @ (r - ai * self.eye) for r, ai in zip(self.rho, self.a))
        self.half = fci.expm(-0.5 * dt * (self.H - H2))
        self.c0 = ham.e_core - 0.5 * float(np.sum(self.a * self.a))
        self.dt = dt

    def xbar(self, v):
        """Eq. 9 from FCI expectations: xbar = -sqrt(dt)(vbar - <v>)."""
        ov = self.vt @ v
        vbar = np.array([1j * (self.vt @ r @ v) / ov for r in self.rho])
        return -np.sqrt(self.dt) * (vbar - 1j * self.a)

    def propagator(self, x, xbar):
        """B(x - xbar) = e^{-dt H1/2} e^{sqrt(dt) sum (x - xbar)(v - <v>)} e^{-dt H1/2}."""
        gen = sum(np.sqrt(self.dt) * (x[g] - xbar[g]) * 1j * (r - self.a[g] * self.eye)
                  for g, r in enumerate(self.rho))
        return self.half @ fci.expm(gen) @ self.half


# ------------------------------------------------------- phaseless weight rule

def test_phaseless_weight_factor_matches_fci_overlap_ratio():
    """w <- w |I| max(0, cos arg R): R = <phi_T|B(x - xbar)|phi>/<phi_T|phi> and
    I = R e^{sum(x xbar - xbar^2/2)} computed in the FCI sector.  The scan of
    field strengths crosses cos arg R = 0 several times and contains walkers
    where cos arg R and cos arg I have opposite signs, so using the phase of
    I, or Re I instead of |I|, fails here."""
    M, na, nb, nch, dt = 5, 2, 1, 3, 0.05
    ham = make_hamiltonian(M, nch, seed=4, e_core=0.2)
    ham.chol *= 3.0
    trial = make_trial(ham.h, na, nb)
    F = FciStep(ham, trial, na, nb, dt)
    sys_ = O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt, taylor_order=40)
    phi = random_walkers(M, na + nb, 1, seed=9)[0]
    v = F.sec.slater(phi)
    xbar = F.xbar(v)
    direction = np.random.default_rng(3).standard_normal(nch)
    signs = set()
    for s in np.linspace(0.5, 4.0, 15):
        x = s * direction
        R = (F.vt @ F.propagator(x, xbar) @ v) / (F.vt @ v)
        I = R * np.exp(np.sum(x * xbar - 0.5 * xbar ** 2))
        wk = O.init_walkers(sys_, 1, init_phi=phi)
        O.step(sys_, wk, x[None])
        # the walker step drops the constant of H1 (e^{-dt c0}) and applies
        # the uniform shift e^{dt e_shift}; neither changes the phase
        expect = abs(I) * np.exp(dt * (F.c0 + wk.e_shift)) * max(0.0, np.cos(np.angle(R)))
        # (order-40 Taylor series at |A| of a few: rounding ~1e-9 relative)
        assert abs(wk.weight[0] - expect) <= 1e-8 * max(expect, 1e-300)
        assert bool(wk.alive[0]) == (np.cos(np.angle(R)) > 0)
        signs.add((np.cos(np.angle(R)) > 0, np.cos(np.angle(I)) > 0))
    # both projections and both disagreements occur in the scan
    assert signs == {(True, True), (True, False), (False, True), (False, False)}


# ---------------------------------------------------- weighted mixed estimator

@pytest.mark.parametrize("mode", [O.FREE, O.IS_FREE])
def test_weighted_estimator_one_field_quadrature(mode):
    """Eq. 7 with unequal complex weights.  Each Gauss-Hermite node x_q gives
    one propagated walker with weight omega_q W(x_q) (W = R in free
    projection, I in importance-sampled free projection), and
    Re(sum W E_L / sum W) over that population must equal
    Re <phi_T|H B|phi>/<phi_T|B|phi> with B the dense Trotter product
    e^{-dt H1/2} e^{-dt H2} e^{-dt H1/2}."""
    M, na, nb, dt = 5, 2, 1, 0.05
    ham = make_hamiltonian(M, 1, seed=4, e_core=0.2)
    ham.chol *= 4.0
    trial = make_trial(ham.h, na, nb)
    F = FciStep(ham, trial, na, nb, dt)
    sys_ = O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt, taylor_order=40)
    nodes, wts = np.polynomial.hermite_e.hermegauss(80)
    wts = wts / np.sqrt(2 * np.pi)
    H2 = 0.5 * (F.rho[0] - F.a[0] * F.eye) @ (F.rho[0] - F.a[0] * F.eye)
    trotter = F.half @ fci.expm(-dt * H2) @ F.half
    for phi in random_walkers(M, na + nb, 2, seed=9):
        nq = len(nodes)
        wk = O.init_walkers(sys_, nq, init_phi=phi, complex_weights=True)
        O.step(sys_, wk, nodes[:, None], mode)
        pop = O.Walkers(wk.phi, wk.weight * wts, wk.lnov, wk.theta, wk.alive, wk.t, wk.e_shift)
        # the weights really are unequal (and complex)
        assert np.ptp(np.abs(pop.weight)) > 0.1 * np.max(np.abs(pop.weight))
        assert np.max(np.abs(np.angle(pop.weight))) > 0.1
        e = O.mixed_energy(pop, O.local_energy(sys_, wk.theta), mode)
        v = F.sec.slater(phi)
        e_fci = ((F.vt @ F.H @ trotter @ v) / (F.vt @ trotter @ v)).real
        assert abs(e - e_fci) < 1e-10 * abs(e_fci)


def test_phaseless_estimator_population_invariances():
    """The walker population represents sum_k w_k |phi_k> (Eq. 7): a walker of
    weight 2 and two copies of it with weight 1 give the same estimate, and
    frozen walkers (weight 0, alive = False) contribute nothing whatever their
    local energy.  An unweighted mean, or one that counts frozen walkers,
    fails here."""
    ham = make_hamiltonian(8, 10, seed=2)
    trial = make_trial(ham.h, 2, 2)
    sys_ = O.System(ham.h, ham.chol, 0.0, trial, 2, 2, 0.02)
    wk = O.init_walkers(sys_, 3)
    f = O.PhiloxFields(3, 0, 10)
    for _ in range(5):
        O.step(sys_, wk, f(wk.t, 3))
    el = O.local_energy(sys_, wk.theta)
    assert np.ptp(el.real) > 1e-3
    base = O.Walkers(wk.phi, np.array([2.0, 0.5, 1.0]), wk.lnov, wk.theta,
                     np.ones(3, dtype=bool))
    e1 = O.mixed_energy(base, el)
    split = [0, 0, 1, 2]
    dup = O.Walkers(wk.phi[split], np.array([1.0, 1.0, 0.5, 1.0]), wk.lnov[split],
                    wk.theta[split], np.ones(4, dtype=bool))
    e2 = O.mixed_energy(dup, el[split])
    assert abs(e1 - e2) < 1e-14 * abs(e1)
    dead = [0, 1, 2, 1]
    with_dead = O.Walkers(wk.phi[dead], np.array([2.0, 0.5, 1.0, 0.0]), wk.lnov[dead],
                          wk.theta[dead], np.array([True, True, True, False]))
    el_dead = el[dead].copy()
    el_dead[3] = 1e6
    assert O.mixed_energy(with_dead, el_dead) == e1
    # the estimate is not the unweighted mean
    assert abs(e1 - float(np.mean(el.real))) > 1e-4


# ------------------------------------- multi-step free projection vs exact FCI

def _projected_energy(mode, ham, trial, na, nb, tau, dt, nw, seeds):
    sys_ = O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt)
    n = int(round(tau / dt))
    es = []
    for seed in seeds:
        wk = O.init_walkers(sys_, nw, complex_weights=True)
        f = O.PhiloxFields(seed, 7, ham.chol.shape[0])
        for _ in range(n):
            O.step(sys_, wk, f(wk.t, nw), mode)
        es.append(O.mixed_energy(wk, O.local_energy(sys_, wk.theta), mode))
    es = np.array(es)
    return es.mean(), es.std(ddof=1) / np.sqrt(len(es))


@pytest.mark.slow
@pytest.mark.parametrize("mode", [O.FREE, O.IS_FREE])
def test_free_projection_extrapolates_to_fci(mode):
    """E(tau) by free projection (W <- W R) and importance-sampled free
    projection (force bias, W <- W I), both unbiased (Sec. II.A), at
    dt = 0.02, 0.01, 0.005, extrapolated linearly in dt (weighted by the
    standard errors over 8 seeds) must match the exact projection of the
    trial at tau = 0.5 within 3 standard errors.  The trial energy lies more
    than thirty standard errors away, so the run must have projected."""
    M, na, nb, nch, tau = 5, 2, 1, 5, 0.5
    ham = make_hamiltonian(M, nch, seed=5, e_core=0.0)
    ham.chol *= 0.8
    trial = make_trial(ham.h, na, nb)
    sec = fci.Sector(M, na, nb)
    H = fci.hamiltonian(sec, ham.h, ham.chol, ham.e_core)
    vt = sec.slater(trial)
    proj = fci.expm(-tau * H) @ vt
    e_tau = (vt @ H @ proj) / (vt @ proj)
    e_hf = (vt @ H @ vt) / (vt @ vt)
    dts = np.array([0.02, 0.01, 0.005])
    res = [_projected_energy(mode, ham, trial, na, nb, tau, dt, 1500, range(1000, 1008))
           for dt in dts]
    e = np.array([r[0] for r in res])
    se = np.array([r[1] for r in res])
    A = np.vstack([np.ones_like(dts), dts]).T
    Wm = np.diag(1.0 / se ** 2)
    cov = np.linalg.inv(A.T @ Wm @ A)
    e0, _slope = cov @ A.T @ Wm @ e
    se0 = np.sqrt(cov[0, 0])
    assert abs(e0 - e_tau) < 3.0 * se0, (e0, e_tau, se0)
    assert abs(e_hf - e_tau) > 30.0 * se0
