"""Multi-determinant trial (Sec. II.D, the CASSCF trial) on the GPU against
the oracle: overlaps, force bias, weights and mixed energies of
phi_T = sum_i c_i D_i."""
import numpy as np
import pytest

from oracle import afqmc as O
from synth import make_expansion, make_hamiltonian

from tests.gpu_helpers import banner, phase_diff, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1703_01545_amd import afqmc
    return afqmc


def _pair(M, nc, spins, n_dets, ham_seed=0, e_core=0.0):
    ham = make_hamiltonian(M, nc, seed=ham_seed, e_core=e_core)
    exps = [make_expansion(ham.h, na, nb, nd, seed=7 + k)
            for k, ((na, nb), nd) in enumerate(zip(spins, n_dets))]
    return ham, exps


def _run(lib, ham, exps, spins, nw, dt, n_steps, oe, me, seed, precision="fp64"):
    osys = [O.System(ham.h, ham.chol, ham.e_core, e[1][0], na, nb, dt, expansion=e)
            for e, (na, nb) in zip(exps, spins)]
    wa, wb = (O.init_walkers(s, nw) for s in osys)
    ref = O.run_pair(osys[0], osys[1], wa, wb, O.PhiloxFields(seed, 0, ham.chol.shape[0]), n_steps,
                     oe, me)
    H = lib.Hamiltonian(ham.h, ham.chol, ham.e_core)
    g = [lib.System(H, na, nb, None, nw, dt, ortho_every=oe, measure_every=me,
                    precision=precision, expansion=e) for e, (na, nb) in zip(exps, spins)]
    tr = lib.pair_step(g[0], g[1], n_steps, seed=seed)
    return ref, tr, (wa, wb), g, osys, H


def test_msd_pair_m12_matches_oracle(lib):
    """M = 12 pair: the neutral (3/3) with a 5-determinant expansion, the ion
    (3/2) with 4; 32 walkers, 60 steps, Gram-Schmidt every 5, energies every
    5, Philox fields; every energy, weight, ln overlap and determinant at
    1e-10."""
    spins = ((3, 3), (3, 2))
    banner("multi-determinant pair M=12 vs oracle")
    ham, exps = _pair(12, 36, spins, (5, 4))
    ref, tr, (wa, wb), g, _, H = _run(lib, ham, exps, spins, 32, 0.01, 60, 5, 5, seed=4)
    assert tr.shape == (12, 3)
    for col, key in enumerate(("EA", "EB", "dE")):
        r = np.asarray(ref[key])
        assert np.max(np.abs(tr[:, col] - r) / np.maximum(np.abs(r), 1e-3)) < TOL, key
    for gs, wk in zip(g, (wa, wb)):
        got = gs.walkers()
        assert np.array_equal(got["alive"], wk.alive)
        live = wk.alive
        assert rel(got["weight"][live], wk.weight[live]) < TOL
        assert rel(got["lnov"].real[live], wk.lnov.real[live]) < TOL
        assert np.max(phase_diff(got["lnov"].imag[live], wk.lnov.imag[live])) < TOL
        for k in np.nonzero(live)[0]:
            assert rel(got["phi"][k], wk.phi[k]) < TOL


@pytest.mark.parametrize("precision,tol", [("fp64", TOL), ("bf16x3", 1e-5)])
def test_msd_pair_ragged_matches_oracle(lib, precision, tol):
    """M = 37 pair (7/6 vs 7/5), 6 and 3 determinants, n_chol = 75, 24
    walkers, 24 steps: FP64 at 1e-10, the split-BF16 plan within the bound
    of the single-determinant reduced-precision tests."""
    spins = ((7, 6), (7, 5))
    banner(f"multi-determinant pair M=37 {precision} vs oracle")
    ham, exps = _pair(37, 75, spins, (6, 3), ham_seed=3, e_core=1.25)
    ref, tr, _, _, _, H = _run(lib, ham, exps, spins, 24, 0.01, 24, 4, 3, seed=9,
                               precision=precision)
    scale = max(np.max(np.abs(ref["EA"])), np.max(np.abs(ref["EB"])))
    for col, key in enumerate(("EA", "EB", "dE")):
        err = np.max(np.abs(tr[:, col] - np.asarray(ref[key])))
        assert err <= tol * scale, (key, err, scale)


def test_msd_one_determinant_and_checkpoint(lib):
    """A one-determinant expansion is the single-determinant system bit for
    bit; a snapshot of a multi-determinant system restores bit for bit; the
    adjoint refuses the expansion."""
    banner("multi-determinant: one determinant, checkpoint, adjoint refusal")
    ham, exps = _pair(20, 40, ((4, 4), (4, 3)), (1, 4), ham_seed=2)
    H = lib.Hamiltonian(ham.h, ham.chol, ham.e_core)
    kw = dict(ortho_every=5, measure_every=5)
    one = exps[0]
    a1 = lib.System(H, 4, 4, one[1][0], 16, 0.01, **kw)
    a2 = lib.System(H, 4, 4, None, 16, 0.01, expansion=one, **kw)
    b1 = lib.System(H, 4, 3, exps[1][1][0], 16, 0.01, **kw)
    b2 = lib.System(H, 4, 3, exps[1][1][0], 16, 0.01, **kw)
    assert np.array_equal(lib.pair_step(a1, b1, 15, seed=2), lib.pair_step(a2, b2, 15, seed=2))
    m = lib.System(H, 4, 3, None, 16, 0.01, expansion=exps[1], **kw)
    n = lib.System(H, 4, 4, one[1][0], 16, 0.01, **kw)
    lib.pair_step(n, m, 10, seed=5)
    cm, cn = m.checkpoint(), n.checkpoint()
    t1 = lib.pair_step(n, m, 10, seed=5)
    m.restore(cm)
    n.restore(cn)
    t2 = lib.pair_step(n, m, 10, seed=5)
    assert np.array_equal(t1, t2)
    with pytest.raises(lib.AfqmcError) as e:
        m.adjoint_forward(np.eye(20) * 0.01, 5)
    assert e.value.status == lib.E_STATE
