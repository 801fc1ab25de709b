"""Batched correlated pairs (graph-replayed) and the launch-shape autotuner.

Pair p of a batch must run exactly what a standalone afqmc_pair_step of that
pair runs: the traces and the final walker states are compared bit for bit,
for graph replay over several lanes, one lane, and direct launches, across
calls that start and end off the graph period.
"""
import numpy as np
import pytest

from oracle import afqmc as O

from tests.gpu_helpers import Workload, banner, rel

pytestmark = pytest.mark.gpu

# (M, n_chol, na_a, nb_a, na_b, nb_b, walkers, ham_seed)
PAIRS = [(12, 36, 3, 3, 3, 2, 64, 0), (20, 60, 4, 4, 4, 3, 40, 1), (37, 100, 7, 6, 7, 5, 96, 2)]
CHUNKS = [25, 7, 20]
DT = 0.01


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1703_01545_amd import afqmc
    return afqmc


def _make(lib, precision):
    out = []
    for (M, nc, naa, nba, nab, nbb, nw, hs) in PAIRS:
        wl = Workload(M, nc, naa, nba, nab, nbb, nw, DT, ham_seed=hs)
        H, (a, b) = wl.gpu_systems(lib, precision=precision, ortho_every=5, measure_every=2)
        out.append((wl, H, a, b))
    return out


def _state(s):
    w = s.walkers()
    return [w["phi"], w["weight"], w["lnov"], w["alive"]]


def _standalone(lib, precision, seeds):
    sys_ = _make(lib, precision)
    traces = []
    for (wl, H, a, b), sd in zip(sys_, seeds):
        traces.append(np.concatenate([lib.pair_step(a, b, n, seed=sd) for n in CHUNKS]))
    return sys_, traces


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lanes,graph", [(3, True), (1, True), (2, False)])
def test_batch_matches_standalone_pairs(lib, precision, lanes, graph):
    banner(f"batch {precision} lanes={lanes} graph={graph}")
    seeds = [11, 12, 13]
    ref_sys, ref_tr = _standalone(lib, precision, seeds)
    sys_ = _make(lib, precision)
    pairs = [(a, b) for (_, _, a, b) in sys_]
    tr = [lib.pair_batch_step(pairs, seeds, n, lanes=lanes, graph=graph) for n in CHUNKS]
    tr = np.concatenate(tr, axis=1)
    for p in range(len(PAIRS)):
        assert np.array_equal(tr[p], ref_tr[p]), f"pair {p} trace differs"
        for x, y in ((sys_[p][2], ref_sys[p][2]), (sys_[p][3], ref_sys[p][3])):
            for u, v in zip(_state(x), _state(y)):
                assert np.array_equal(u, v, equal_nan=True), f"pair {p} walker state differs"
    assert tr.shape[1] == sum(CHUNKS) // 2


def test_batch_fp64_pair_matches_oracle(lib):
    """The first pair of a graph-replayed FP64 batch against the oracle."""
    banner("batch fp64 vs oracle")
    from oracle.afqmc import PhiloxFields
    sys_ = _make(lib, "fp64")
    pairs = [(a, b) for (_, _, a, b) in sys_]
    tr = lib.pair_batch_step(pairs, [5, 6, 7], 40, lanes=2)
    wl = sys_[0][0]
    sa, sb = wl.oracle_systems()
    wa, wb = O.init_walkers(sa, wl.nw), O.init_walkers(sb, wl.nw)
    ref = O.run_pair(sa, sb, wa, wb, PhiloxFields(5, 0, wl.n_chol), 40, 5, 2)
    assert rel(tr[0][:, 0], ref["EA"]) < 1e-10
    assert rel(tr[0][:, 1], ref["EB"]) < 1e-10
    assert np.max(np.abs(tr[0][:, 2] - np.asarray(ref["dE"]))) < 1e-10 * np.max(np.abs(ref["EA"]))


def test_autotune_keeps_results(lib):
    banner("autotune bitwise")
    outs = []
    for tune in (False, True):
        sys_ = _make(lib, "fp32")
        wl, H, a, b = sys_[2]
        if tune:
            for s in (a, b):
                ch = lib.autotune(s)
                assert ch[0] in (1, 2, 3) and ch[1] in (1, 2, 3)
                assert 0 <= ch[2] < 13
        outs.append((lib.pair_step(a, b, 12, seed=3), _state(a), _state(b)))
    assert np.array_equal(outs[0][0], outs[1][0])
    for u, v in zip(outs[0][1] + outs[0][2], outs[1][1] + outs[1][2]):
        assert np.array_equal(u, v)


def test_unrelated_hamiltonians_from_two_host_threads(lib):
    """Two host threads, each with its own Hamiltonian and pair, autotune and
    step at the same time (ctypes releases the interpreter lock during a
    call): the shared cache of tuned launch shapes is guarded, and tuning
    never changes a bit, so each pair ends bitwise where it ends when the two
    run one after the other."""
    import threading
    banner("two host threads, unrelated Hamiltonians")
    wls = [Workload(20, 40, 4, 4, 4, 3, 48, 0.01, ham_seed=s) for s in (5, 6)]

    def run(wl, out, i):
        try:
            H, (a, b) = wl.gpu_systems(lib, precision="bf16x3", ortho_every=5, measure_every=5)
            lib.autotune(a)
            lib.autotune(b)
            tr = lib.pair_step(a, b, 20, seed=9)
            out[i] = (tr, a.walkers()["phi"], b.walkers()["weight"])
        except Exception as e:  # surfaced in the main thread
            out[i] = e

    seq = [None, None]
    for i, wl in enumerate(wls):
        run(wl, seq, i)
    par = [None, None]
    th = [threading.Thread(target=run, args=(wl, par, i)) for i, wl in enumerate(wls)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    for i in range(2):
        for r in (seq[i], par[i]):
            if isinstance(r, Exception):
                raise r
            assert r is not None
        for u, v in zip(seq[i], par[i]):
            assert np.array_equal(u, v)


def test_tune_cache_carries_choices(lib, tmp_path):
    """Tune one system and save the table; clear it, change the file's GEMM
    tiles to other valid tiles and load it: a new system of the same shape
    gets exactly those tiles (taken from the file, not timed).  A file tagged
    with another device or holding a choice no tuner could make is refused and
    leaves the table as it was."""
    banner("tune cache save / clear / load")
    wl = Workload(40, 80, 8, 8, 8, 7, 64, 0.01, ham_seed=4)
    path = str(tmp_path / "tune.txt")
    H, (a, _) = wl.gpu_systems(lib, precision="bf16x3")
    c1 = [int(x) for x in lib.autotune(a)]
    lib.tune_cache_save(path)
    lines = open(path).read().splitlines()
    head, rows = lines[:2], [l.split() for l in lines[2:] if l.strip()]
    planted = {}
    for r in rows:
        if r[0] in ("0", "1") and int(r[1]) == 2 * wl.nw:  # this system's GEMMs
            r[-1] = "2" if r[-1] != "2" else "1"
            planted[int(r[0])] = int(r[-1])
    assert set(planted) == {0, 1}, lines

    def write(first, second, body):
        open(path, "w").write("\n".join([first, second] + [" ".join(r) for r in body]) + "\n")

    lib.tune_cache_clear()
    write(head[0], "another device", rows)
    with pytest.raises(lib.AfqmcError) as e:
        lib.tune_cache_load(path)
    assert e.value.status == lib.E_INVALID
    bad = [list(r) for r in rows]
    bad[0][-1] = "99"
    write(head[0], head[1], bad)
    with pytest.raises(lib.AfqmcError) as e:
        lib.tune_cache_load(path)
    assert e.value.status == lib.E_INVALID
    write(head[0], head[1], rows)
    lib.tune_cache_load(path)
    H2, (a2, _) = wl.gpu_systems(lib, precision="bf16x3")
    c2 = [int(x) for x in lib.autotune(a2)]
    assert c2 == [planted[0], planted[1], c1[2]], (c1, c2)
    lib.tune_cache_clear()


def test_batch_errors(lib):
    banner("batch errors")
    sys_ = _make(lib, "fp64")
    (_, _, a0, b0), (_, _, a1, b1) = sys_[0], sys_[1]
    with pytest.raises(lib.AfqmcError) as e:
        lib.pair_batch_step([(a0, b0), (a0, b1)], [1, 2], 4)
    assert e.value.status == lib.E_INVALID
    lib.pair_step(a1, b1, 1)
    with pytest.raises(lib.AfqmcError) as e:
        lib.pair_batch_step([(a0, b0), (a1, b1)], [1, 2], 4)
    assert e.value.status == lib.E_STATE
    with pytest.raises(lib.AfqmcError) as e:
        lib.pair_batch_step([(a0, b1)], [1], 4)
    assert e.value.status == lib.E_SHAPE
