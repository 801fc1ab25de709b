"""The allocation-free pair step against afqmc_pair_step: the same trace and
walkers, bit for bit, on two calls in a row (the second on a smaller pair
and fewer steps, so stale staging rows of the first call would show), and a
clear error past the staging limit."""
import numpy as np
import pytest

from tests.gpu_helpers import Workload, banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1703_01545_amd import afqmc
    return afqmc


def _both(lib, wl, n_steps, seed, oe, me):
    out = []
    for fn in (lib.pair_step, lib.pair_step_noalloc):
        H, (a, b) = wl.gpu_systems(lib, ortho_every=oe, measure_every=me)
        tr = fn(a, b, n_steps, seed=seed)
        out.append((tr, a.walkers(), b.walkers()))
    return out


def test_noalloc_pair_step_matches_pair_step_twice(lib):
    banner("pair_step_noalloc: first call, M=37 pair, 36 steps, 12 measurements")
    big = Workload(37, 75, 7, 6, 7, 5, 24, 0.01, ham_seed=3, e_core=1.25)
    (t1, a1, b1), (t2, a2, b2) = _both(lib, big, 36, 5, 4, 3)
    assert t1.shape == (12, 3) and np.all(np.isfinite(t1))
    assert np.array_equal(t1, t2)
    for x, y in ((a1, a2), (b1, b2)):
        for k in ("phi", "weight", "lnov", "alive"):
            assert np.array_equal(x[k], y[k]), k
    banner("pair_step_noalloc: second call, M=12 pair, 10 steps, 2 measurements")
    small = Workload(12, 36, 3, 3, 3, 2, 8, 0.01, ham_seed=0)
    (s1, c1, d1), (s2, c2, d2) = _both(lib, small, 10, 7, 5, 5)
    assert s1.shape == (2, 3)
    assert np.array_equal(s1, s2)
    for x, y in ((c1, c2), (d1, d2)):
        for k in ("phi", "weight", "lnov", "alive"):
            assert np.array_equal(x[k], y[k]), k


def test_noalloc_pair_step_rejects_too_many_measurements(lib):
    banner("pair_step_noalloc: staging limit")
    wl = Workload(12, 36, 3, 3, 3, 2, 4, 0.01, ham_seed=0)
    H, (a, b) = wl.gpu_systems(lib, ortho_every=5, measure_every=1)
    n = lib.NOALLOC_MAX_MEASUREMENTS + 1
    with pytest.raises(lib.AfqmcError) as e:
        lib.pair_step_noalloc(a, b, n, seed=1)
    assert e.value.status == lib.E_INVALID
    assert "staging limit" in str(e.value)
    assert a.info()["step"] == 0 and b.info()["step"] == 0
