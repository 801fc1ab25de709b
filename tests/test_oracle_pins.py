"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check compares the oracle with something other than itself: dense
determinant-space (FCI) operators built from V_ijkl, closed forms, Gauss-
Hermite quadrature of the Hubbard-Stratonovich integral, invariants, and the
published known-answer vectors of the random generator.
"""
import os

import numpy as np
import pytest

from oracle import afqmc as O
from oracle import fci
from oracle import philox
from synth import make_hamiltonian, make_trial, random_walkers

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_system(M, n_chol, na, nb, dt=0.01, seed=0, e_core=0.37, K=6, trial=None, **kw):
    ham = make_hamiltonian(M, n_chol, seed=seed, e_core=e_core)
    if trial is None:
        trial = make_trial(ham.h, na, nb)
    return ham, O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt, taylor_order=K, **kw)


# ----------------------------------------------------------- Philox (K9 pin)

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r[:6]]
        expect = [int(x, 16) for x in r[7:11]] if r[6] == "->" else [int(x, 16) for x in r[6:10]]
        got = philox.philox4x32_10(*v)
        assert [int(g) for g in got] == expect


def test_normals_moments_and_layout():
    x = philox.normals(seed=12345, stream=3, t=7, walkers=np.arange(400), n_chol=250)
    assert x.shape == (400, 250)
    z = x.ravel()
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.02
    assert abs(np.mean(z ** 4) - 3.0) < 0.1
    # a walker subset sees exactly the draws it sees in the full batch
    sub = philox.normals(seed=12345, stream=3, t=7, walkers=np.array([5, 399]), n_chol=250)
    assert np.array_equal(sub, x[[5, 399]])
    # ragged n_chol is a prefix of the padded draw
    y = philox.normals(seed=12345, stream=3, t=7, walkers=np.arange(3), n_chol=252)
    assert np.array_equal(y[:, :250], x[:3])


def test_normals_joint_distribution():
    """Box-Muller must turn each pair of uniforms into two independent standard
    normals.  Over 4 x 25 600 draws: the covariance of the four draws of one
    generator call is the identity, each draw is N(0, 1) by a
    Kolmogorov-Smirnov test, the polar angle of each pair is uniform and its
    squared radius is exponential with mean 2 (chi-square, 2 degrees of
    freedom).  Swapping sin for cos, or reusing one uniform for both
    coordinates, fails here even though the moments of single draws survive."""
    from scipy import stats
    x = philox.normals(seed=2024, stream=1, t=3, walkers=np.arange(400), n_chol=256)
    q = x.reshape(-1, 4)
    cov = np.cov(q, rowvar=False)
    assert np.max(np.abs(cov - np.eye(4))) < 0.04
    for j in range(4):
        assert stats.kstest(q[:, j], "norm").pvalue > 1e-3
    for p in (0, 2):
        z0, z1 = q[:, p], q[:, p + 1]
        ang = np.mod(np.arctan2(z1, z0), 2 * np.pi) / (2 * np.pi)
        assert stats.kstest(ang, "uniform").pvalue > 1e-3
        assert stats.kstest(z0 ** 2 + z1 ** 2, "expon", args=(0, 2.0)).pvalue > 1e-3
        quad = np.bincount((z0 > 0) * 2 + (z1 > 0), minlength=4) / len(z0)
        assert np.max(np.abs(quad - 0.25)) < 0.01


# -------------------------------------------------- FCI-space pins (P1)

@pytest.fixture(scope="module", params=[(5, 2, 2, 4), (5, 2, 1, 3), (6, 3, 2, 5), (4, 1, 0, 3)])
def fci_case(request):
    M, na, nb, nch = request.param
    ham, sys = tiny_system(M, nch, na, nb, seed=11 + M + na + nb)
    sec = fci.Sector(M, na, nb)
    ops = sec.one_body_ops()
    H = fci.hamiltonian(sec, ham.h, ham.chol, ham.e_core, ops)
    return dict(ham=ham, sys=sys, sec=sec, ops=ops, H=H)


def test_fci_thouless(fci_case):
    """exp(sum_pq A_pq E_pq)|phi(Phi)> = |phi(e^A Phi)> (Thouless theorem, Sec. II.A)."""
    sec, ops, sys = fci_case["sec"], fci_case["ops"], fci_case["sys"]
    rng = np.random.default_rng(1)
    A = 0.3 * (rng.standard_normal((sec.M, sec.M)) + 1j * rng.standard_normal((sec.M, sec.M)))
    phi = random_walkers(sec.M, sys.N, 1, seed=3)[0]
    lhs = fci.expm(fci.one_body_operator(ops, A)) @ sec.slater(phi)
    rhs = sec.slater(fci.expm(A) @ phi)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12 * np.abs(rhs).max())


def test_fci_overlap_theta_energy(fci_case):
    """Overlap, force-bias density and mixed local energy vs FCI (Eq. 7, 9)."""
    sec, ops, sys, H, ham = (fci_case[k] for k in ("sec", "ops", "sys", "H", "ham"))
    vt = sec.slater(sys.trial)
    phis = random_walkers(sec.M, sys.N, 4, seed=5)
    lnov, theta = O.overlap(sys, phis)
    el = O.local_energy(sys, theta)
    f = O.force_bias_f(sys, theta)
    rho = fci.rho_ops(ops, ham.chol)
    for k in range(4):
        v = sec.slater(phis[k])
        ov = vt @ v
        assert abs(np.exp(lnov[k]) - ov) < 1e-12 * abs(ov)
        e_fci = (vt @ H @ v) / ov
        assert abs(el[k] - e_fci) < 1e-11 * max(1.0, abs(e_fci))
        f_fci = np.array([(vt @ r @ v) / ov for r in rho])
        assert np.allclose(f[k], f_fci, rtol=0, atol=1e-12 * max(1.0, np.abs(f_fci).max()))
    a_fci = np.array([(vt @ r @ vt) / (vt @ vt) for r in rho])
    assert np.allclose(sys.a, a_fci, atol=1e-12)


def test_fci_trial_energy(fci_case):
    sec, sys, H = fci_case["sec"], fci_case["sys"], fci_case["H"]
    vt = sec.slater(sys.trial)
    lnov, theta = O.overlap(sys, sys.trial[None].astype(complex))
    el = O.local_energy(sys, theta)[0]
    assert abs(el - (vt @ H @ vt) / (vt @ vt)) < 1e-11
    assert abs(el.imag) < 1e-12


def _fci_trotter_ratio(case, phi, dt, chol):
    """<phi_T| e^{-dt H1/2} e^{-dt H2} e^{-dt H1/2} |phi> / <phi_T|phi> with
    H2 = 1/2 sum_g (rho_g - a_g)^2 (Eq. 2, v = i rho) and H1 = H - H2, both
    built as dense matrices in the FCI sector."""
    sec, ops, ham = case["sec"], case["ops"], case["ham"]
    H = fci.hamiltonian(sec, ham.h, chol, ham.e_core, ops)
    vt = sec.slater(case["trial"])
    rho = fci.rho_ops(ops, chol)
    a = np.array([(vt @ r @ vt) / (vt @ vt) for r in rho])
    eye = np.eye(sec.dim)
    H2 = sum(0.5 * (r - ai * eye) @ (r - ai * eye) for r, ai in zip(rho, a))
    H1 = H - H2
    half = fci.expm(-0.5 * dt * H1)
    v = sec.slater(phi)
    val = vt @ half @ fci.expm(-dt * H2) @ half @ v / (vt @ v)
    c0 = ham.e_core - 0.5 * np.sum(a * a)
    return val, c0


@pytest.mark.parametrize("mode", [O.PHASELESS, O.FREE])
def test_hs_quadrature_single_field(mode):
    """P9: with one Cholesky vector the HS identity (Eq. 4) is exact, so the
    Gauss-Hermite average of the hybrid weight I(x) (force-biased) or of the
    overlap ratio R(x) (free projection) equals the dense Trotter product of
    Eq. 3 / Eq. 11 divided by the trial overlap, up to the dropped constant
    e^{dt c0}.  Pins h~ (Eq. 2 remainder), P, the c-number s, the Taylor
    propagator, xbar's use and the importance factor."""
    M, na, nb, dt = 5, 2, 1, 0.05
    ham = make_hamiltonian(M, 1, seed=4, e_core=0.2)
    ham.chol *= 4.0
    trial = make_trial(ham.h, na, nb)
    sys = O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt, taylor_order=40)
    sec = fci.Sector(M, na, nb)
    case = dict(sec=sec, ops=sec.one_body_ops(), ham=ham, trial=trial)
    nodes, wts = np.polynomial.hermite_e.hermegauss(80)
    wts = wts / np.sqrt(2 * np.pi)
    phis = random_walkers(M, na + nb, 2, seed=9)
    ratios = []
    for phi in phis:
        lnov, theta = O.overlap(sys, phi[None])
        acc = 0.0
        for xq, wq in zip(nodes, wts):
            _, _, _, lnR, lnI, _ = O.propagate(sys, phi[None], lnov, theta,
                                               np.array([[xq]]), mode=mode)
            acc += wq * np.exp(lnI[0] if mode == O.PHASELESS else lnR[0])
        exact, c0 = _fci_trotter_ratio(case, phi, dt, ham.chol)
        ratios.append(acc / exact)
        assert abs(acc / exact - np.exp(dt * c0)) < 1e-11
    assert abs(ratios[0] - ratios[1]) < 1e-11


def test_hs_two_fields_trotter_order():
    """P9 with two non-commuting fields: the single-exponential propagator
    averages to the Trotter product up to O(dt^2) per step."""
    M, na, nb = 4, 1, 1
    ham = make_hamiltonian(M, 2, seed=5, e_core=0.0)
    ham.chol *= 3.0
    trial = make_trial(ham.h, na, nb)
    sec = fci.Sector(M, na, nb)
    case = dict(sec=sec, ops=sec.one_body_ops(), ham=ham, trial=trial)
    phi = random_walkers(M, 2, 1, seed=2)[0]
    nodes, wts = np.polynomial.hermite_e.hermegauss(30)
    wts = wts / np.sqrt(2 * np.pi)
    errs = []
    for dt in (0.04, 0.02):
        sys = O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt, taylor_order=40)
        lnov, theta = O.overlap(sys, phi[None])
        acc = 0.0
        for x1, w1 in zip(nodes, wts):
            for x2, w2 in zip(nodes, wts):
                _, _, _, lnR, _, _ = O.propagate(sys, phi[None], lnov, theta,
                                                 np.array([[x1, x2]]), mode=O.FREE)
                acc += w1 * w2 * np.exp(lnR[0])
        exact, c0 = _fci_trotter_ratio(case, phi, dt, ham.chol)
        errs.append(abs(acc * np.exp(-dt * c0) - exact))
    assert errs[0] > 0
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_force_bias_stationarity():
    """Eq. 8: with the optimal xbar of Eq. 9 the x-derivative at x = 0 of the
    biased weight vanishes at leading order; with xbar = 0 (or the opposite
    sign) it does not."""
    M, na, nb = 5, 2, 2
    ham = make_hamiltonian(M, 1, seed=8)
    ham.chol *= 3.0
    trial = make_trial(ham.h, na, nb)
    sec = fci.Sector(M, na, nb)
    ops = sec.one_body_ops()
    rho = fci.rho_ops(ops, ham.chol)[0]
    vt = sec.slater(trial)
    a = (vt @ rho @ vt) / (vt @ vt)
    o = 1j * (rho - a * np.eye(sec.dim))
    phi = random_walkers(M, na + nb, 1, seed=4)[0]
    v = sec.slater(phi)
    ov = vt @ v

    def dF(dt, xbar):
        e = fci.expm(-np.sqrt(dt) * xbar * o)
        return (np.sqrt(dt) * (vt @ o @ e @ v) + xbar * (vt @ e @ v)) / ov * np.exp(-0.5 * xbar ** 2)

    rel = []
    for dt in (1e-3, 2.5e-4):
        sys = O.System(ham.h, ham.chol, 0.0, trial, na, nb, dt)
        _, theta = O.overlap(sys, phi[None])
        xb = O.xbar_of(sys, O.force_bias_f(sys, theta))[0, 0]
        d_opt, d_zero, d_flip = abs(dF(dt, xb)), abs(dF(dt, 0.0)), abs(dF(dt, -xb))
        assert d_opt < 0.1 * d_zero
        assert d_flip > 1.5 * d_zero
        rel.append(d_opt / d_zero)
    assert 2.5 < rel[0] / rel[1] < 6.0


# ------------------------------------------------------------- closed forms

def test_single_electron_two_body_vanishes():
    """P2: one electron has no two-body energy; with the trial the lowest
    eigenvector of h every walker's E_L equals that eigenvalue (Sec. II.A)."""
    M = 9
    ham = make_hamiltonian(M, 7, seed=3, e_core=0.0)
    trial = make_trial(ham.h, 1, 0)
    sys = O.System(ham.h, ham.chol, 0.0, trial, 1, 0, 0.01)
    phis = random_walkers(M, 1, 6, seed=1)
    _, theta = O.overlap(sys, phis)
    el = O.local_energy(sys, theta)
    eps0 = np.linalg.eigvalsh(ham.h)[0]
    assert np.allclose(el, eps0, rtol=0, atol=1e-12)
    # propagate a few steps with random fields: still exactly eps0
    wk = O.init_walkers(sys, 6, init_phi=phis[0])
    rng = np.random.default_rng(0)
    for _ in range(5):
        O.step(sys, wk, rng.standard_normal((6, 7)))
        assert np.allclose(O.local_energy(sys, wk.theta), eps0, rtol=0, atol=1e-12)


def test_hartree_fock_energy_closed_form():
    """P3: at tau = 0 every walker is the trial and E_L = E_HF, computed here
    from the brute-force four-index V in the orbital basis."""
    for (M, nch, na, nb) in ((12, 36, 3, 3), (12, 36, 3, 2), (10, 20, 4, 1)):
        ham, sys = tiny_system(M, nch, na, nb, seed=0, e_core=0.5)
        _, vec = np.linalg.eigh(ham.h)
        V = np.einsum("gik,gjl->ijkl", ham.chol, ham.chol)
        C = vec
        Vmo = np.einsum("ai,bj,ck,dl,abcd->ijkl", C, C, C, C, V, optimize=True)
        hmo = C.T @ ham.h @ C
        occ = [list(range(na)), list(range(nb))]
        e = ham.e_core + sum(hmo[i, i] for o in occ for i in o)
        allocc = [(s, i) for s in range(2) for i in occ[s]]
        for (s, i) in allocc:
            for (t, j) in allocc:
                e += 0.5 * Vmo[i, j, i, j]
                if s == t:
                    e -= 0.5 * Vmo[i, j, j, i]
        wk = O.init_walkers(sys, 3)
        el = O.local_energy(sys, wk.theta)
        assert np.allclose(el, e, rtol=1e-12, atol=0)


def test_taylor_truncation_bound():
    """P4: the order-K Taylor propagator differs from the converged (order 40,
    itself pinned by the FCI quadrature test) by at most the remainder bound
    ||A||^{K+1}/(K+1)! e^{||A||} ||P Phi|| (then times ||P||)."""
    ham, sys6 = tiny_system(12, 36, 3, 2, dt=0.05, K=6)
    sys40 = O.System(ham.h, ham.chol, ham.e_core, sys6.trial, 3, 2, 0.05, taylor_order=40)
    wk = O.init_walkers(sys6, 5)
    x = np.random.default_rng(2).standard_normal((5, 36)) * 3
    p6 = O.propagate(sys6, wk.phi, wk.lnov, wk.theta, x)[0]
    p40 = O.propagate(sys40, wk.phi, wk.lnov, wk.theta, x)[0]
    xbar = O.xbar_of(sys6, O.force_bias_f(sys6, wk.theta))
    c = x - xbar
    nP = np.linalg.norm(sys6.P, 2)
    for k in range(5):
        A = 1j * np.sqrt(0.05) * np.tensordot(c[k], ham.chol, axes=1)
        nA = np.linalg.norm(A, 2)
        bound = nA ** 7 / 5040.0 * np.exp(nA) * nP * np.linalg.norm(sys6.P @ wk.phi[k], 2)
        err = np.linalg.norm(p6[k] - p40[k], 2)
        assert err <= bound
        assert err > 1e-3 * bound  # the bound is not vacuous here


def test_one_body_limit_matches_fci():
    """P6: with no Cholesky vectors the step is deterministic and exact
    (P P = e^{-dt h}); E(tau) must equal <phi_T|H e^{-tau H}|phi_0> /
    <phi_T|e^{-tau H}|phi_0> from the dense FCI Hamiltonian, all weights equal.
    A rotated (non-eigenvector) trial makes E(tau) non-constant."""
    M, na, nb, dt = 5, 2, 2, 0.05
    ham = make_hamiltonian(M, 0, seed=2, e_core=0.1)
    rng = np.random.default_rng(1)
    q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    trial = np.concatenate([q[:, :na], q[:, :nb]], axis=1)
    sys = O.System(ham.h, ham.chol, ham.e_core, trial, na, nb, dt)
    init = make_trial(ham.h + 0.3 * np.diag(np.arange(M)), na, nb)
    wk = O.init_walkers(sys, 3, init_phi=init)
    sec = fci.Sector(M, na, nb)
    H = fci.hamiltonian(sec, ham.h, ham.chol, ham.e_core)
    vt, v0 = sec.slater(trial), sec.slater(init)
    es = []
    for n in range(1, 21):
        O.step(sys, wk, np.zeros((3, 0)))
        e = O.mixed_energy(wk, O.local_energy(sys, wk.theta))
        prop = fci.expm(-n * dt * H) @ v0
        e_ex = (vt @ H @ prop) / (vt @ prop)
        assert abs(e - e_ex) < 1e-11 * abs(e_ex)
        assert np.ptp(wk.weight) == 0.0
        es.append(e)
    assert np.ptp(es) > 1e-3


def test_mgs_invariance():
    """P7: MGS leaves every weight and local energy unchanged (Eq. 6) and
    makes each spin block orthonormal."""
    ham, sys = tiny_system(12, 36, 3, 2)
    wk = O.init_walkers(sys, 8)
    for t in range(6):
        O.step(sys, wk, np.random.default_rng(t).standard_normal((8, 36)))
    e_before = O.local_energy(sys, wk.theta)
    w_before = wk.weight.copy()
    O.orthonormalize(sys, wk)
    e_after = O.local_energy(sys, wk.theta)
    assert np.allclose(e_after, e_before, rtol=1e-12, atol=0)
    assert np.array_equal(wk.weight, w_before)
    for off, n in sys.spins:
        b = wk.phi[:, :, off:off + n]
        g = np.matmul(np.conj(np.swapaxes(b, 1, 2)), b)
        assert np.allclose(g, np.eye(n)[None], atol=1e-13)


def test_identical_pair_zero_difference():
    """P5: identical primary and secondary systems give exactly zero energy
    difference at every measurement (Sec. III.C discussion)."""
    ham, sa = tiny_system(12, 36, 3, 3)
    _, sb = tiny_system(12, 36, 3, 3)
    wa, wb = O.init_walkers(sa, 16), O.init_walkers(sb, 16)
    out = O.run_pair(sa, sb, wa, wb, O.PhiloxFields(0, 0, 36), 30, 5, 3)
    assert len(out["dE"]) == 10
    assert all(d == 0.0 for d in out["dE"])


def test_frozen_walker_keeps_others_unchanged():
    """A walker whose weight reaches zero is frozen; every other walker's
    trajectory is identical to a run in which it was never present
    (Sec. II.B: the fields of the other pairs are unaffected)."""
    ham, sys = tiny_system(12, 36, 3, 2, dt=0.01)
    wk = O.init_walkers(sys, 6)
    fields = O.PhiloxFields(5, 1, 36)
    kill = 2
    for t in range(12):
        x = fields(wk.t, 6)
        if t == 3:
            x = x.copy()
            x[kill] = 0.0
        O.step(sys, wk, x)
        if t == 3:
            wk.weight[kill] = 0.0
            wk.alive[kill] = False
    ref = O.init_walkers(sys, 6)
    keep = np.array([0, 1, 3, 4, 5])
    sub = O.Walkers(ref.phi[keep].copy(), ref.weight[keep].copy(), ref.lnov[keep].copy(),
                    ref.theta[keep].copy(), ref.alive[keep].copy(), 0, ref.e_shift)
    f2 = O.PhiloxFields(5, 1, 36, walkers=keep)
    for t in range(12):
        O.step(sys, sub, f2(sub.t, 5))
    assert np.array_equal(sub.phi, wk.phi[keep])
    assert np.array_equal(sub.weight, wk.weight[keep])


def test_oracle_rounding_floor_cfg0_shape():
    """Reading of the summation-order question: permuting the Cholesky
    vectors (and their fields) changes only the rounding order.  Over 200
    steps of the M=12 pair the energies move by far less than the 1e-10
    parity tolerance."""
    ham, sa = tiny_system(12, 36, 3, 3, dt=0.01, seed=0, e_core=0.0)
    trial_b = make_trial(ham.h, 3, 2)
    sb = O.System(ham.h, ham.chol, 0.0, trial_b, 3, 2, 0.01)
    perm = np.random.default_rng(0).permutation(36)
    sa2 = O.System(ham.h, ham.chol[perm], 0.0, sa.trial, 3, 3, 0.01)
    sb2 = O.System(ham.h, ham.chol[perm], 0.0, trial_b, 3, 2, 0.01)
    f = O.PhiloxFields(0, 0, 36)
    nw = 16
    out1 = O.run_pair(sa, sb, O.init_walkers(sa, nw), O.init_walkers(sb, nw), f, 200, 5, 20)

    def fperm(t, n):
        return f(t, n)[:, perm]

    out2 = O.run_pair(sa2, sb2, O.init_walkers(sa2, nw), O.init_walkers(sb2, nw), fperm, 200, 5, 20)
    for k in ("EA", "EB"):
        a, b = np.array(out1[k]), np.array(out2[k])
        assert np.max(np.abs(a - b) / np.abs(a)) < 1e-12


def test_force_bias_cap_definition():
    """The optional force-bias cap (a bounding condition the paper cites
    without stating; parity unpinned beyond this definition): a threshold above
    every |xbar| changes nothing; an applied cap leaves every |xbar| at most
    the cap with its phase unchanged and counts exactly the entries above it;
    counting alone changes nothing."""
    c_ham = make_hamiltonian(12, 36, seed=0)
    trial = make_trial(c_ham.h, 3, 3)
    f = O.PhiloxFields(3, 0, 36)
    runs = {}
    for name, cap, apply in (("off", 0.0, False), ("huge", 1e3, True), ("count", 0.03, False),
                             ("apply", 0.03, True)):
        s = O.System(c_ham.h, c_ham.chol, 0.0, trial, 3, 3, 0.01, fb_cap=cap, cap_apply=apply)
        wk = O.init_walkers(s, 16)
        raw_over = 0
        for _ in range(20):
            raw = O.xbar_of(s, O.force_bias_f(s, wk.theta))
            raw_over += int(np.sum((np.abs(raw) > 0.03) & wk.alive[:, None]))
            used = O.propagate(s, wk.phi, wk.lnov, wk.theta, f(wk.t, 16))[5]
            if name == "apply":
                assert np.all(np.abs(used) <= 0.03 * (1 + 1e-15))
                big = np.abs(raw) > 0.03
                assert np.allclose(np.angle(used[big]), np.angle(raw[big]), atol=1e-13)
                assert np.array_equal(used[~big], raw[~big])
            O.step(s, wk, f(wk.t, 16))
        runs[name] = (wk, raw_over)
    base = runs["off"][0]
    assert runs["off"][0].cap_events == 0 and runs["huge"][0].cap_events == 0
    for name in ("huge", "count"):
        assert np.array_equal(runs[name][0].phi, base.phi)
        assert np.array_equal(runs[name][0].weight, base.weight)
    assert runs["count"][0].cap_events == runs["count"][1] > 0
    assert runs["apply"][0].cap_events > 0
    assert not np.array_equal(runs["apply"][0].weight, base.weight)
