"""Population control (the comb) and the preliminary equilibration scheme on
the GPU against the oracle (Sec. II.B)."""
import numpy as np
import pytest

from oracle import afqmc as O
from synth import config

from tests.gpu_helpers import Workload, banner, phase_diff, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1703_01545_amd import afqmc
    return afqmc


def _compare(g, wk, tol=TOL):
    got = g.walkers()
    assert np.array_equal(got["alive"], wk.alive)
    live = wk.alive
    assert rel(got["weight"][live], wk.weight[live]) < tol
    assert rel(got["lnov"].real[live], wk.lnov.real[live]) < tol
    assert np.max(phase_diff(got["lnov"].imag[live], wk.lnov.imag[live]), initial=0) < tol
    for k in np.nonzero(live)[0]:
        assert rel(got["phi"][k], wk.phi[k]) < tol


def test_comb_matches_oracle(lib):
    """64 walkers of the M = 12 neutral system, 15 steps (weights spread),
    one walker frozen by a non-finite field, then the comb at xi = 0.37 and
    10 more steps: the same copies (selection is exact), weights W / nw and
    the same walkers afterwards."""
    import torch
    c = config(0)
    nw = 64
    banner("comb vs oracle")
    wl = Workload(c.M, c.n_chol, c.na_a, c.nb_a, c.na_b, c.nb_b, nw, 0.02)
    x = wl.fields(25, seed=8) * 1.5
    x[3, 9, 0] = np.nan
    sa, _ = wl.oracle_systems()
    wk = O.init_walkers(sa, nw)
    H = lib.Hamiltonian(wl.ham.h, wl.ham.chol, wl.ham.e_core)
    g = lib.System(H, c.na_a, c.nb_a, wl.trials[0], nw, 0.02, ortho_every=5, measure_every=0)
    dev = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    g.step(15, fields=dev[:15].contiguous())
    for t in range(15):
        O.step(sa, wk, x[t])
        if wk.t % 5 == 0:
            O.orthonormalize(sa, wk)
    assert not wk.alive[9] and np.ptp(wk.weight[wk.alive]) > 0.05 * wk.weight[wk.alive].max()
    _compare(g, wk)
    g.population_control(0.37)
    O.comb(wk, 0.37)
    _compare(g, wk)
    assert g.walkers()["alive"].all()
    g.step(10, fields=dev[15:].contiguous())
    for t in range(15, 25):
        O.step(sa, wk, x[t])
        if wk.t % 5 == 0:
            O.orthonormalize(sa, wk)
    _compare(g, wk)


def test_preliminary_equilibration_matches_oracle(lib):
    """The primary (3/3 electrons) equilibrated 20 steps with the comb every
    10, the secondary (3/2) started from it, then 20 correlated steps with
    energies every 5: the secondary's start and the pair's trace against the
    oracle."""
    from paper_1703_01545_amd import pes
    c = config(0)
    nw, seed = 32, 5
    banner("preliminary equilibration vs oracle")
    wl = Workload(c.M, c.n_chol, c.na_a, c.nb_a, c.na_b, c.nb_b, nw, c.dt)
    H = lib.Hamiltonian(wl.ham.h, wl.ham.chol, wl.ham.e_core)
    ga, gb = (lib.System(H, na, nb, t, nw, c.dt, ortho_every=5, measure_every=5)
              for t, (na, nb) in zip(wl.trials, wl.spins))
    pes.preliminary_equilibration(ga, gb, 20, 10, seed=seed, xi_seed=11)
    assert gb.info()["step"] == 20
    sa, sb = wl.oracle_systems()
    wa = O.init_walkers(sa, nw)
    f = O.PhiloxFields(seed, 0, c.n_chol)
    rng = np.random.default_rng(11)
    for t in range(20):
        O.step(sa, wa, f(wa.t, nw))
        if wa.t % 5 == 0:
            O.orthonormalize(sa, wa)
        if wa.t % 10 == 0:
            O.comb(wa, float(rng.random()))
    wb = O.init_from_primary(sb, sa, wa)
    _compare(ga, wa)
    _compare(gb, wb)
    tr = lib.pair_step(ga, gb, 20, seed=seed)
    ref = O.run_pair(sa, sb, wa, wb, f, 20, 5, 5)
    for col, key in enumerate(("EA", "EB", "dE")):
        r = np.asarray(ref[key])
        assert np.max(np.abs(tr[:, col] - r) / np.maximum(np.abs(r), 1e-3)) < TOL, key


def test_population_errors(lib):
    banner("population control errors")
    wl = Workload(12, 10, 3, 3, 3, 2, 8, 0.01)
    H = lib.Hamiltonian(wl.ham.h, wl.ham.chol, wl.ham.e_core)
    a = lib.System(H, 3, 3, wl.trials[0], 8, 0.01)
    b = lib.System(H, 3, 2, wl.trials[1], 8, 0.01)
    for bad in (-0.1, 1.0, float("nan")):
        with pytest.raises(lib.AfqmcError) as e:
            a.population_control(bad)
        assert e.value.status == lib.E_INVALID
    with pytest.raises(lib.AfqmcError) as e:
        a.init_from_primary(b)  # the secondary may not have more electrons
    assert e.value.status == lib.E_SHAPE
    f = lib.System(H, 3, 3, wl.trials[0], 8, 0.01, mode="free")
    with pytest.raises(lib.AfqmcError) as e:
        f.population_control(0.5)
    assert e.value.status == lib.E_STATE
