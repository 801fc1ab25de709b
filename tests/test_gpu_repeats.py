"""Repeats of correlated and uncorrelated pairs on the GPU (Sec. II.B): the
batched repeat runner reproduces each repeat's standalone pair run bit for
bit, the uncorrelated variant leaves the primary system's energies unchanged,
and correlating the fields shrinks the standard error of the energy
difference over repeats."""
import numpy as np
import pytest

from synth import config

from tests.gpu_helpers import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1703_01545_amd import afqmc
    return afqmc


def _setup(lib):
    c = config(0)
    ham = c.hamiltonian()
    H = lib.Hamiltonian(ham.h, ham.chol, ham.e_core)
    spec_a = (c.na_a, c.nb_a, c.trial_a())
    spec_b = (c.na_b, c.nb_b, c.trial_b())
    return c, H, spec_a, spec_b


def test_correlated_repeats_equal_standalone_pairs(lib):
    from paper_1703_01545_amd import repeats
    banner("repeat runner vs standalone pairs")
    c, H, sa, sb = _setup(lib)
    kw = dict(ortho_every=5, measure_every=5)
    tr = repeats.correlated_repeats(H, sa, sb, 16, 3, 40, c.dt, seed0=7, **kw)
    assert tr.shape == (3, 8, 3)
    for r in range(3):
        a = lib.System(H, sa[0], sa[1], sa[2], 16, c.dt, **kw)
        b = lib.System(H, sb[0], sb[1], sb[2], 16, c.dt, **kw)
        assert np.array_equal(lib.pair_step(a, b, 40, seed=7 + r), tr[r])


def test_uncorrelated_repeats_keep_primary_and_lose_the_correlation(lib):
    from paper_1703_01545_amd import repeats, stats
    banner("correlated vs uncorrelated standard error over 11 repeats")
    c, H, sa, sb = _setup(lib)
    kw = dict(ortho_every=5, measure_every=10)
    cor = repeats.correlated_repeats(H, sa, sb, 32, 11, 100, c.dt, seed0=3, **kw)
    unc = repeats.uncorrelated_repeats(H, sa, sb, 32, 11, 100, c.dt, seed0=3, **kw)
    assert np.array_equal(cor[:, :, 0], unc[:, :, 0])
    assert not np.array_equal(cor[:, :, 1], unc[:, :, 1])
    e_cor = stats.final_estimate(cor[:, :, 2], 2)
    e_unc = stats.final_estimate(unc[:, :, 2], 2)
    banner(f"  dE correlated {e_cor.value:.5f} +- {e_cor.se:.5f}, uncorrelated "
           f"{e_unc.value:.5f} +- {e_unc.se:.5f}")
    assert e_cor.se < 0.5 * e_unc.se
    assert abs(e_cor.value - e_unc.value) < 4 * np.hypot(e_cor.se, e_unc.se)
