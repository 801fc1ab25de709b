"""Pins of the oracle's population control (the comb) and of the start of the
secondary system in the preliminary equilibration scheme (Sec. II.B)."""
import numpy as np

from oracle import afqmc as O
from oracle import fci
from synth import make_hamiltonian, make_trial, random_walkers


def _population(nw=12, seed=3, kill=(4,)):
    ham = make_hamiltonian(8, 10, seed=seed)
    sys_ = O.System(ham.h, ham.chol, 0.0, make_trial(ham.h, 2, 2), 2, 2, 0.02)
    wk = O.init_walkers(sys_, nw)
    f = O.PhiloxFields(seed, 0, 10)
    for _ in range(6):
        O.step(sys_, wk, f(wk.t, nw))
    wk.weight = wk.weight * np.random.default_rng(seed).uniform(0.2, 3.0, nw)
    for k in kill:
        wk.weight[k] = 0.0
        wk.alive[k] = False
    return sys_, wk


def _copies(sel, nw):
    return np.bincount(sel, minlength=nw)


def test_comb_counts_total_weight_and_frozen_walkers():
    """Each walker gets floor or ceil of nw w_k / W copies, the total weight is
    kept, frozen walkers are never copied and every new walker is live."""
    sys_, wk = _population()
    W = wk.weight[wk.alive].sum()
    expect = 12 * np.where(wk.alive, wk.weight, 0.0) / W
    for xi in (0.0, 0.137, 0.5, 0.999):
        w2 = wk.copy()
        # each walker is tagged by its first element to recover the selection
        tags = w2.phi[:, 0, 0].copy()
        assert len(set(tags.tolist())) == 12
        O.comb(w2, xi)
        sel = np.array([int(np.nonzero(tags == v)[0][0]) for v in w2.phi[:, 0, 0]])
        n = _copies(sel, 12)
        assert np.all(n >= np.floor(expect) - 1e-12) and np.all(n <= np.ceil(expect) + 1e-12)
        assert n[4] == 0
        assert w2.alive.all()
        assert abs(w2.weight.sum() - W) < 1e-13 * W
        assert np.ptp(w2.weight) == 0.0
        # copies carry their walker's overlap and Theta unchanged
        assert np.array_equal(w2.lnov, wk.lnov[sel])
        assert np.array_equal(w2.theta, wk.theta[sel])


def test_comb_is_unbiased_for_the_mixed_estimator():
    """Averaged over xi uniform in [0, 1), the comb keeps the expected number
    of copies nw w_k / W of every walker, so the equal-weight estimate after
    the comb averages to the weighted estimate of Eq. 7 before it.  The
    midpoint rule over 4096 values of xi integrates these step functions to
    within (jumps) / 4096."""
    sys_, wk = _population()
    el = O.local_energy(sys_, wk.theta).real
    e_before = O.mixed_energy(wk, O.local_energy(sys_, wk.theta))
    tags = wk.phi[:, 0, 0].copy()
    G = 4096
    counts = np.zeros(12)
    e_after = 0.0
    for i in range(G):
        w2 = wk.copy()
        O.comb(w2, (i + 0.5) / G)
        sel = np.array([int(np.nonzero(tags == v)[0][0]) for v in w2.phi[:, 0, 0]])
        counts += _copies(sel, 12)
        e_after += el[sel].mean()
    W = wk.weight[wk.alive].sum()
    expect = 12 * np.where(wk.alive, wk.weight, 0.0) / W
    assert np.max(np.abs(counts / G - expect)) < 13.0 / G
    assert abs(e_after / G - e_before) < 13.0 / G * np.ptp(el)
    # a single comb is not the weighted estimate (the test is not vacuous)
    w1 = wk.copy()
    O.comb(w1, 0.5)
    assert abs(O.mixed_energy(w1, O.local_energy(sys_, w1.theta)) - e_before) > 1e-6


def test_secondary_start_weights_from_fci_overlaps():
    """The secondary walker (the primary's determinant with one beta column
    fewer) gets w_pri |r| max(0, cos arg r), r the ratio of its overlap with
    the secondary trial to the primary's overlap with the primary trial, both
    computed from FCI-sector vectors (Cauchy-Binet: no determinant of the
    overlap matrix is formed)."""
    M, dt = 5, 0.02
    ham = make_hamiltonian(M, 4, seed=6)
    tp, ts = make_trial(ham.h, 2, 2), make_trial(ham.h, 2, 1)
    pri = O.System(ham.h, ham.chol, 0.0, tp, 2, 2, dt)
    sec = O.System(ham.h, ham.chol, 0.0, ts, 2, 1, dt)
    phis = random_walkers(M, 4, 6, seed=2)
    wk = O.init_walkers(pri, 6)
    wk.phi = phis.copy()
    wk.lnov, wk.theta = O.overlap(pri, wk.phi)
    wk.weight = np.linspace(0.5, 2.0, 6)
    ws = O.init_from_primary(sec, pri, wk)
    sp, ss = fci.Sector(M, 2, 2), fci.Sector(M, 2, 1)
    seen = set()
    for k in range(6):
        ov_p = sp.slater(tp) @ sp.slater(phis[k])
        ov_s = ss.slater(ts) @ ss.slater(phis[k][:, [0, 1, 2]])
        r = ov_s / ov_p
        expect = wk.weight[k] * abs(r) * max(0.0, np.cos(np.angle(r)))
        assert abs(ws.weight[k] - expect) <= 1e-12 * max(expect, 1.0)
        assert bool(ws.alive[k]) == (expect > 0)
        assert np.allclose(ws.phi[k], phis[k][:, [0, 1, 2]], rtol=0, atol=0)
        seen.add(expect > 0)
    assert seen == {True, False}


def test_secondary_start_identical_system_is_a_copy():
    """With the secondary equal to the primary the ratio is 1: weights, overlaps
    and determinants are unchanged, and a correlated pair started this way
    has an energy difference of exactly zero."""
    ham = make_hamiltonian(10, 20, seed=1)
    trial = make_trial(ham.h, 3, 3)
    pri = O.System(ham.h, ham.chol, 0.0, trial, 3, 3, 0.01)
    sec = O.System(ham.h, ham.chol, 0.0, trial, 3, 3, 0.01)
    wk = O.init_walkers(pri, 8)
    f = O.PhiloxFields(9, 0, 20)
    for _ in range(10):
        O.step(pri, wk, f(wk.t, 8))
    O.comb(wk, 0.3)
    ws = O.init_from_primary(sec, pri, wk)
    assert np.array_equal(ws.weight, wk.weight)
    assert np.array_equal(ws.phi, wk.phi)
    out = O.run_pair(pri, sec, wk, ws, f, 10, 5, 5)
    assert all(d == 0.0 for d in out["dE"])
