"""GPU (HIP) path vs the FP64 oracle on identical seeded inputs.

FP64 parity bar: 1e-10 relative in every measured energy and per-walker
weight, log-overlap (imaginary part compared modulo 2 pi) and determinant.
"""
import numpy as np
import pytest

from oracle import afqmc as O
from oracle import philox
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


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _bf16_round(x):
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = ((f + 0x7FFF + ((f >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("shape", [(1, 1, 1), (37, 53, 29), (200, 160, 333), (300, 260, 64),
                                   (1000, 700, 96)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_gemm_kernel(lib, shape, prec):
    banner(f"gemm {prec} {shape}")
    m, n, k = shape
    rng = np.random.default_rng(m * 7 + n + k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((n, k))
    # inputs made exactly representable in the compute precision, so the test
    # checks the MFMA arithmetic and tiling, not the device's tie rounding
    if prec == "fp32":
        A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    elif prec == "bf16":
        A, B = _bf16_round(A), _bf16_round(B)
    got = lib.selftest_gemm(A, B, prec)
    ref = A @ B.T
    tol = 1e-13 if prec == "fp64" else 2e-6
    scale = np.abs(A) @ np.abs(B).T
    assert np.max(np.abs(got - ref) / scale) < tol


# Every workgroup tile of the contraction GEMM on operands stored as the walker
# step stores them (FP32 for the fp32 and split-BF16 products, FP64 for fp64):
# ragged m and n (rows past the operands), K a whole number of 32-wide tiles
# (the two-set fetch path of the split products) or not, one or several K
# ranges, and K ranges left empty (K = 40 in four ranges of 32).  The tile
# shapes sum in the same order, so they agree bitwise for each number of K
# ranges; the result matches the product of the stored operands within the
# rounding of the precision (split BF16: a few 2^-17 per product).
@pytest.mark.parametrize("shape,ks", [((300, 141, 4096), 3), ((517, 260, 1000), 1),
                                      ((256, 128, 96), 1), ((700, 333, 2080), 4),
                                      ((64, 801, 3648), 3), ((150, 70, 40), 4)])
@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp64"])
def test_gemm_tile_shapes_agree(lib, prec, shape, ks):
    banner(f"gemm tiles {prec} {shape} ksplit {ks}")
    m, n, k = shape
    rng = np.random.default_rng(m + 3 * n + k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((n, k))
    if prec != "fp64":
        A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    outs = [lib.selftest_gemm_shape(A, B, prec, tile, ks) for tile in (1, 2, 3, 4)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ref = A @ B.T
    scale = np.abs(A) @ np.abs(B).T
    tol = {"fp64": 1e-13, "fp32": 1e-5, "bf16": 5e-5}[prec]
    assert np.max(np.abs(outs[0] - ref) / scale) < tol


def test_device_fields_match_oracle_generator(lib):
    banner("philox fields")
    for (seed, stream, t, nw, nc) in [(0, 0, 0, 64, 36), (2 ** 40 + 5, 3, 123457, 33, 401)]:
        got = lib.selftest_fields(seed, stream, t, nw, nc)
        ref = philox.normals(seed, stream, t, np.arange(nw), nc)
        assert np.max(np.abs(got - ref)) < 1e-14 * 8


def _run_pair_both(lib, torch, wl: Workload, n_steps, ortho, meas, fields=None, philox_seed=None,
                   K=6, walkers_sub=None, precision="fp64"):
    sa, sb = wl.oracle_systems(K)
    wa, wb = O.init_walkers(sa, wl.nw if walkers_sub is None else len(walkers_sub)), None
    wb = O.init_walkers(sb, wl.nw if walkers_sub is None else len(walkers_sub))
    if fields is not None:
        ff = O.ExplicitFields(fields, walkers=walkers_sub)
        dev = torch.from_numpy(np.ascontiguousarray(fields)).cuda()
    else:
        ff = O.PhiloxFields(philox_seed, 0, wl.n_chol, walkers=walkers_sub)
        dev = None
    ref = O.run_pair(sa, sb, wa, wb, ff, n_steps, ortho, meas)
    H, (ga, gb) = wl.gpu_systems(lib, precision=precision, K=K, ortho_every=ortho,
                                 measure_every=meas)
    tr = lib.pair_step(ga, gb, n_steps, seed=philox_seed or 0, fields=dev)
    torch.cuda.synchronize()
    return ref, tr, (wa, wb), (ga, gb), (sa, sb)


def _compare_walkers(gpu_sys, wk, sub=None, tol=TOL):
    g = gpu_sys.walkers()
    idx = np.arange(len(wk.weight)) if sub is None else np.asarray(sub)
    alive = g["alive"][idx]
    assert np.array_equal(alive, wk.alive)
    live = wk.alive
    assert rel(g["weight"][idx][live], wk.weight[live]) < tol
    assert np.all(g["weight"][idx][~live] == 0.0)
    assert rel(g["lnov"][idx].real[live], wk.lnov.real[live]) < tol
    assert np.max(phase_diff(g["lnov"][idx].imag[live], wk.lnov.imag[live]), initial=0) < tol
    for k in np.nonzero(live)[0]:
        assert rel(g["phi"][idx[k]], wk.phi[k]) < tol


def test_parity_pair_m12_explicit_fields(lib, torch_mod):
    """M=12 pair (3/3 vs 3/2), 64 walkers, 200 steps, MGS every 5, measured
    every step, explicit N(0,1) fields."""
    c = config(0)
    banner("parity M=12 explicit fields")
    wl = Workload(c.M, c.n_chol, c.na_a, c.nb_a, c.na_b, c.nb_b, c.n_walkers, c.dt)
    x = wl.fields(c.n_steps, seed=0)
    ref, tr, (wa, wb), (ga, gb), _ = _run_pair_both(lib, torch_mod, wl, c.n_steps, c.ortho_every,
                                                    1, fields=x)
    assert tr.shape == (c.n_steps, 3)
    for col, key in enumerate(("EA", "EB", "dE")):
        r = np.asarray(ref[key])
        assert np.max(np.abs(tr[:, col] - r) / np.maximum(np.abs(r), 1e-3)) < TOL, key
    _compare_walkers(ga, wa)
    _compare_walkers(gb, wb)


def test_parity_pair_m12_device_philox(lib, torch_mod):
    c = config(0)
    banner("parity M=12 philox")
    wl = Workload(c.M, c.n_chol, c.na_a, c.nb_a, c.na_b, c.nb_b, c.n_walkers, c.dt)
    ref, tr, (wa, wb), (ga, gb), _ = _run_pair_both(lib, torch_mod, wl, 100, c.ortho_every, 10,
                                                    philox_seed=1234)
    for col, key in enumerate(("EA", "EB")):
        assert rel(tr[:, col], np.asarray(ref[key])) < TOL
    _compare_walkers(ga, wa)
    _compare_walkers(gb, wb)


@pytest.mark.parametrize("dims", [(37, 75, 7, 6, 7, 5, 37), (19, 9, 4, 0, 3, 0, 70),
                                  (64, 130, 16, 16, 16, 15, 5), (60, 90, 44, 41, 44, 40, 6),
                                  (70, 100, 56, 50, 56, 49, 4)])
def test_parity_ragged(lib, torch_mod, dims):
    """Sizes that leave ragged tails in every tile dimension."""
    M, nc, a1, b1, a2, b2, nw = dims
    banner(f"parity ragged {dims}")
    wl = Workload(M, nc, a1, b1, a2, b2, nw, 0.01, ham_seed=3, e_core=1.25)
    x = wl.fields(24, seed=5)
    ref, tr, (wa, wb), (ga, gb), _ = _run_pair_both(lib, torch_mod, wl, 24, 4, 3, fields=x)
    for col, key in enumerate(("EA", "EB", "dE")):
        r = np.asarray(ref[key])
        assert np.max(np.abs(tr[:, col] - r) / np.maximum(np.abs(r), 1e-3)) < TOL, key
    _compare_walkers(ga, wa)
    _compare_walkers(gb, wb)


# Reduced-precision plans against the FP64 oracle on the same fields.  FP32
# storage (unit roundoff 6e-8) and split-BF16 products (about 2^-17 relative
# per product, averaged over the contractions) leave about 1e-6 relative in
# the energies over 40 steps; the bound 1e-5 keeps a 10x margin and still
# fails on a dropped split term (plain BF16 products: about 4e-4).
@pytest.mark.parametrize("dims", [(37, 75, 7, 6, 7, 5, 37), (64, 130, 16, 16, 16, 15, 16),
                                  (40, 120, 20, 20, 20, 19, 16), (60, 90, 44, 33, 44, 32, 6)])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 1e-5), ("bf16x3", 1e-5),
                                      ("bf16_plain", 5e-3)])
def test_reduced_precision_close_to_oracle(lib, torch_mod, dims, prec, tol):
    M, nc, a1, b1, a2, b2, nw = dims
    banner(f"{prec} vs oracle {dims}")
    wl = Workload(M, nc, a1, b1, a2, b2, nw, 0.01, ham_seed=3, e_core=1.25)
    x = wl.fields(40, seed=5)
    ref, tr, _, _, _ = _run_pair_both(lib, torch_mod, wl, 40, 5, 4, fields=x, precision=prec)
    scale = max(np.max(np.abs(ref["EA"])), np.max(np.abs(ref["EB"])))
    for col, key in enumerate(("EA", "EB", "dE")):
        err = np.max(np.abs(tr[:, col] - np.asarray(ref[key])))
        assert err <= tol * scale, (key, err, scale)


# The largest basis the split plan serves (M = 256: the one-plane unpack holds
# a 131 KB triangle in LDS, the 32-orbital propagation shapes) and the largest
# the 80-orbital shape serves (M = 224), as whole pairs against the oracle at
# the bound above; Philox fields, one measurement after 10 steps.
@pytest.mark.parametrize("dims", [(256, 384, 12, 12, 12, 11, 6), (224, 448, 40, 40, 40, 39, 3)])
def test_split_plan_largest_bases(lib, torch_mod, dims):
    M, nc, a1, b1, a2, b2, nw = dims
    banner(f"bf16x3 vs oracle, large basis {dims}")
    wl = Workload(M, nc, a1, b1, a2, b2, nw, 0.005, ham_seed=5)
    ref, tr, _, (ga, gb), _ = _run_pair_both(lib, torch_mod, wl, 10, 5, 10, philox_seed=3,
                                             precision="bf16x3")
    assert tr.shape == (1, 3)
    scale = max(np.max(np.abs(ref["EA"])), np.max(np.abs(ref["EB"])))
    for col, key in enumerate(("EA", "EB", "dE")):
        err = np.max(np.abs(tr[:, col] - np.asarray(ref[key])))
        assert err <= 1e-5 * scale, (key, err, scale)
    # the energy difference against the oracle in the target's unit
    err_kcal = abs(tr[0, 2] - ref["dE"][0]) * 627.5095
    banner(f"  dE split-BF16 vs FP64 oracle: {err_kcal:.2e} kcal/mol")
    assert err_kcal <= 0.05


def test_parity_m100_sampled_walkers(lib, torch_mod):
    """M=100 pair at its full walker count (1024), device Philox fields; the
    oracle recomputes a sample of walkers one by one (walkers are independent
    under correlated sampling without population control)."""
    c = config(1)
    banner("parity M=100 full batch, sampled walkers")
    n_steps = 40
    wl = Workload(c.M, c.n_chol, c.na_a, c.nb_a, c.na_b, c.nb_b, c.n_walkers, c.dt)
    sub = np.array([0, 1, 511, 1023])
    sa, sb = wl.oracle_systems()
    wa, wb = O.init_walkers(sa, len(sub)), O.init_walkers(sb, len(sub))
    O.run_pair(sa, sb, wa, wb, O.PhiloxFields(7, 0, c.n_chol, walkers=sub), n_steps, 10, 20)
    H, (ga, gb) = wl.gpu_systems(lib, ortho_every=10, measure_every=20)
    lib.pair_step(ga, gb, n_steps, seed=7)
    _compare_walkers(ga, wa, sub)
    _compare_walkers(gb, wb, sub)
    el_a, w_a, _ = ga.local_energy()
    ref_el = O.local_energy(sa, wa.theta)
    assert rel(el_a[sub], ref_el) < TOL


def test_walker_count_beyond_grid_y_limit(lib):
    """40 000 walkers per system: 80 000 walker planes, more than a launch
    grid takes in its y or z dimension (65 535 blocks), so every per-plane
    launch (the FP64 plan's unpack of the field sums among them) must put the
    planes on x.  Sampled walkers, on both sides of 32 768, match the oracle."""
    c = config(0)
    nw = 40000
    banner(f"walker count {nw} (planes beyond the grid's y limit)")
    wl = Workload(c.M, c.n_chol, c.na_a, c.nb_a, c.na_b, c.nb_b, nw, c.dt)
    sub = np.array([0, 32767, 32768, nw - 1])
    sa, sb = wl.oracle_systems()
    wa, wb = O.init_walkers(sa, len(sub)), O.init_walkers(sb, len(sub))
    O.run_pair(sa, sb, wa, wb, O.PhiloxFields(3, 0, c.n_chol, walkers=sub), 10, 5, 5)
    H, (ga, gb) = wl.gpu_systems(lib, ortho_every=5, measure_every=5)
    lib.pair_step(ga, gb, 10, seed=3)
    _compare_walkers(ga, wa, sub)
    _compare_walkers(gb, wb, sub)


def test_bench_config_sampled_walkers(lib, torch_mod):
    """The timed workload as bench.py runs it: the M=200 pair (40/40 vs 40/39,
    n_chol = 800) at its full 2048 walkers per system, autotuned shapes,
    graph-replayed batch path, device Philox fields, in the split-BF16 plan
    and in FP64.  The FP64 oracle recomputes three walkers one by one: the
    FP64 run must match them to 1e-10, the split-BF16 run within the bound
    below; the pair's energy difference of the split-BF16 run must meet the
    0.05 kcal/mol target against the FP64 run on the same fields.

    Bound of the split-BF16 run: each split-BF16 product carries a relative
    error of a few 2^-17 (< 3e-5), and a step applies ten dense products to a
    walker (force bias, field sum, two one-body halves, six Taylor terms), so
    20 steps bound the relative error of a walker's orbitals and of its
    weight (a product of 20 overlap ratios) by 20 x 10 x 3e-5 = 6e-3; the
    local energy of a walker, formed from its orbitals by two more split
    contractions, is checked at the same bound."""
    cfg = config(2)
    n_steps, seed = 20, 9
    banner(f"bench workload M={cfg.M} Nw={cfg.n_walkers}, sampled walkers")
    ham = cfg.hamiltonian()
    trials = (cfg.trial_a(), cfg.trial_b())
    spins = ((cfg.na_a, cfg.nb_a), (cfg.na_b, cfg.nb_b))
    sub = np.array([0, 777, cfg.n_walkers - 1])
    osys = [O.System(ham.h, ham.chol, ham.e_core, t, na, nb, cfg.dt,
                     taylor_order=cfg.taylor_order) for t, (na, nb) in zip(trials, spins)]
    wa, wb = (O.init_walkers(s, len(sub)) for s in osys)
    O.run_pair(osys[0], osys[1], wa, wb, O.PhiloxFields(seed, 0, cfg.n_chol, walkers=sub),
               n_steps, cfg.ortho_every, cfg.measure_every)
    ref_el = [O.local_energy(s, wk.theta) for s, wk in zip(osys, (wa, wb))]
    traces = {}
    for prec, tol in (("fp64", TOL), ("bf16x3", 6e-3)):
        H = lib.Hamiltonian(ham.h, ham.chol, ham.e_core)
        kw = dict(taylor_order=cfg.taylor_order, ortho_every=cfg.ortho_every,
                  measure_every=cfg.measure_every, precision=prec)
        ga, gb = (lib.System(H, na, nb, t, cfg.n_walkers, cfg.dt, **kw)
                  for t, (na, nb) in zip(trials, spins))
        traces[prec] = lib.pair_batch_step([(ga, gb)], [seed], n_steps, lanes=1)[0]
        for g, wk, ref in zip((ga, gb), (wa, wb), ref_el):
            w = g.walkers()
            el = g.local_energy()[0][sub]
            banner(f"  {prec}: weight {rel(w['weight'][sub], wk.weight):.2e}  phi "
                   f"{max(rel(w['phi'][k], wk.phi[i]) for i, k in enumerate(sub)):.2e}  "
                   f"local energy {rel(el, ref):.2e}")
            _compare_walkers(g, wk, sub, tol=tol)
            assert rel(el, ref) < tol
    err = np.abs(traces["bf16x3"][:, 2] - traces["fp64"][:, 2]) * 627.5095
    banner(f"  dE split-BF16 vs FP64 (kcal/mol) {np.max(err):.2e}")
    assert traces["fp64"].shape[0] == n_steps // cfg.measure_every
    assert np.max(err) < 0.05


# The exchange kernel that keeps whole gamma blocks in each wavefront serves
# spin blocks of 17..48 orbitals, padded to 24, 32, 40 or 48 (split-BF16
# contractions, M a multiple of 4); one case per padding, with ragged spin
# blocks.  After a few steps the local energy of every walker is compared with
# the oracle's on the walker's own orbitals (the split products of T and of
# the force-bias-like half contraction: a few 2^-17 relative; 3e-7 to 5e-7
# measured).
@pytest.mark.parametrize("M,na,nb", [(60, 20, 19), (76, 29, 27), (84, 37, 33), (100, 45, 42)])
def test_exchange_blocks_local_energy_matches_oracle(lib, M, na, nb):
    banner(f"exchange blocks M={M} spins {na}/{nb}")
    wl = Workload(M, 2 * M, na, nb, na, nb, 24, 0.01, ham_seed=M)
    H, (ga, gb) = wl.gpu_systems(lib, precision="bf16", ortho_every=3, measure_every=3)
    lib.pair_step(ga, gb, 6, seed=4)
    el = ga.local_energy()[0]
    osys = wl.oracle_systems()[0]
    _, theta = O.overlap(osys, ga.walkers()["phi"])
    ref = O.local_energy(osys, theta)
    banner(f"  local energy split-BF16 vs oracle on the same orbitals: {rel(el, ref):.2e}")
    assert rel(el, ref) < 2e-5


def _gs_expected(phi, na, nb):
    """Per (walker, spin block): ell = max_k 1/2 ln(S_kk / D_k) and
    ln |det R| = 1/2 sum_k ln D_k from S = Phi^H Phi = C C^H (D_k = |C_kk|^2)."""
    ell, lnd = [], []
    for w in range(phi.shape[0]):
        for sl in (slice(0, na), slice(na, na + nb)):
            P = phi[w][:, sl]
            S = P.conj().T @ P
            D = np.abs(np.diag(np.linalg.cholesky(S))) ** 2
            ell.append(np.max(0.5 * np.log(np.real(np.diag(S)) / D)))
            lnd.append(0.5 * np.sum(np.log(D)))
    return np.array(ell), np.array(lnd)


# The Gram-Schmidt monitor against the loss of orthogonality computed from
# the walkers' own orbitals: steps without orthonormalisation, then one
# afqmc_orthonormalize; the Gram-matrix factorisation (spin blocks up to 48)
# and the column-by-column one (52/50 orbitals).
@pytest.mark.parametrize("M,na,nb", [(12, 4, 3), (64, 52, 50)])
def test_gs_monitor_matches_the_orbitals(lib, M, na, nb):
    banner(f"Gram-Schmidt monitor M={M} {na}/{nb}")
    wl = Workload(M, 2 * M, na, nb, na, nb, 24, 0.02, ham_seed=3)
    H, (ga, gb) = wl.gpu_systems(lib, ortho_every=0, measure_every=10)
    ga.gs_monitor()  # clears what the set-up recorded
    lib.pair_step(ga, gb, 30, seed=2)
    w = ga.walkers()
    assert w["alive"].all()
    ell, lnd = _gs_expected(w["phi"], na, nb)
    ga.orthonormalize()
    me, ml, trips = ga.gs_monitor(threshold=float(np.max(ell)) * 0.999)
    banner(f"  ell {me:.6e} (orbitals {np.max(ell):.6e}), |ln det R| {ml:.6e} "
           f"(orbitals {np.max(np.abs(lnd)):.6e}), trips {trips}")
    assert abs(me - np.max(ell)) < 1e-9 * max(1.0, np.max(ell))
    assert abs(ml - np.max(np.abs(lnd))) < 1e-9 * max(1.0, np.max(np.abs(lnd)))
    assert trips == int(np.sum(ell > np.max(ell) * 0.999)) and trips >= 1
    assert ga.gs_monitor() == (0.0, 0.0, 0)  # the record was cleared


def test_gs_monitor_trips_without_orthonormalisation(lib):
    """Free projection keeps every walker; 120 steps at dt = 0.05 without
    Gram-Schmidt leave the orbitals of most spin blocks more than 9 nepers
    from orthogonal (the factorisation loses about 8 digits), while every
    orthonormalisation of a run with Gram-Schmidt every 5 steps finds them
    close."""
    banner("Gram-Schmidt monitor trips")
    wl = Workload(12, 24, 4, 4, 4, 3, 16, 0.05, ham_seed=7)
    H = lib.Hamiltonian(wl.ham.h, wl.ham.chol, wl.ham.e_core)
    res = {}
    for oe in (0, 5):
        ga, gb = (lib.System(H, na, nb, t, wl.nw, wl.dt, ortho_every=oe, measure_every=10,
                             mode="free") for t, (na, nb) in zip(wl.trials, wl.spins))
        ga.gs_monitor()
        lib.pair_step(ga, gb, 120, seed=5)
        assert ga.walkers()["alive"].all()
        if not oe:
            ga.orthonormalize()
        # without Gram-Schmidt: the one orthonormalisation at the end; with
        # it: the 24 periodic ones of the run
        res[oe] = ga.gs_monitor(threshold=9.0)
        banner(f"  ortho_every {oe}: ell {res[oe][0]:.3f}, trips {res[oe][2]}")
    assert res[0][2] >= wl.nw // 2 and res[0][0] > 9.0
    assert res[5][2] == 0 and res[5][0] < 2.0


def test_identical_pair_exact_zero(lib):
    banner("identical pair")
    wl = Workload(20, 40, 4, 4, 4, 4, 32, 0.01, ham_seed=2)
    H, (ga, gb) = wl.gpu_systems(lib, ortho_every=5, measure_every=5)
    tr = lib.pair_step(ga, gb, 40, seed=11)
    assert tr.shape == (8, 3)
    assert np.all(tr[:, 2] == 0.0)


def test_mgs_invariance_and_determinism(lib):
    banner("mgs invariance / determinism")
    wl = Workload(30, 60, 6, 5, 6, 4, 24, 0.01, ham_seed=4)
    H, (ga, gb) = wl.gpu_systems(lib, ortho_every=0, measure_every=0)
    ga.step(15, seed=3)
    e0, w0, m0 = ga.local_energy()
    ga.orthonormalize()
    e1, w1, m1 = ga.local_energy()
    assert rel(e1, e0) < 1e-12 and np.array_equal(w0, w1)
    H2, (ha, hb) = wl.gpu_systems(lib, ortho_every=0, measure_every=0)
    ha.step(15, seed=3)
    ha.orthonormalize()
    e2, w2, m2 = ha.local_energy()
    assert np.array_equal(e2, e1) and np.array_equal(w2, w1) and m2 == m1


def test_checkpoint_restore_bitwise(lib):
    banner("checkpoint/restore")
    wl = Workload(24, 48, 5, 5, 5, 4, 16, 0.01, ham_seed=6)
    H, (ga, gb) = wl.gpu_systems(lib, ortho_every=5, measure_every=5)
    lib.pair_step(ga, gb, 10, seed=9)
    ca, cb = ga.checkpoint(), gb.checkpoint()
    t1 = lib.pair_step(ga, gb, 10, seed=9)
    ga.restore(ca)
    gb.restore(cb)
    t2 = lib.pair_step(ga, gb, 10, seed=9)
    assert np.array_equal(t1, t2)


def test_nan_field_freezes_only_that_walker(lib, torch_mod):
    """A non-finite field kills one walker; every other walker is bitwise
    identical to a run without it, and the oracle agrees (Sec. II.B)."""
    banner("nan field")
    wl = Workload(18, 30, 4, 3, 4, 2, 12, 0.01, ham_seed=8)
    x = wl.fields(8, seed=2)
    xbad = x.copy()
    xbad[3, 5, 7] = np.nan
    outs = []
    for arr in (x, xbad):
        H, (ga, gb) = wl.gpu_systems(lib, ortho_every=4, measure_every=0)
        ga.step(8, fields=torch_mod.from_numpy(arr).cuda())
        outs.append(ga.walkers())
    assert outs[0]["alive"].all()
    assert not outs[1]["alive"][5] and outs[1]["weight"][5] == 0.0
    keep = np.arange(12) != 5
    assert np.array_equal(outs[0]["phi"][keep], outs[1]["phi"][keep])
    assert np.array_equal(outs[0]["weight"][keep], outs[1]["weight"][keep])
    sa, _ = wl.oracle_systems()
    wk = O.init_walkers(sa, 12)
    for t in range(8):
        O.step(sa, wk, xbad[t])
        if wk.t % 4 == 0:
            O.orthonormalize(sa, wk)
    assert np.array_equal(wk.alive, outs[1]["alive"])


def test_errors(lib):
    banner("error paths")
    wl = Workload(12, 10, 3, 3, 3, 2, 8, 0.01)
    H, (ga, gb) = wl.gpu_systems(lib)
    wl2 = Workload(12, 11, 3, 3, 3, 2, 8, 0.01)
    H2, (ha, hb) = wl2.gpu_systems(lib)
    with pytest.raises(lib.AfqmcError) as e:
        lib.pair_step(ga, hb, 2)
    assert e.value.status == lib.E_SHAPE
    ga.step(1)
    with pytest.raises(lib.AfqmcError) as e:
        lib.pair_step(ga, gb, 2)
    assert e.value.status == lib.E_STATE
    # walkers exactly orthogonal to the trial -> zero overlap -> singular
    eye = np.eye(12)
    trial = np.concatenate([eye[:, :3], eye[:, :3]], axis=1)
    init = np.concatenate([eye[:, 3:6], eye[:, 3:6]], axis=1)
    with pytest.raises(lib.AfqmcError) as e:
        lib.System(H, 3, 3, trial, 4, 0.01, init_phi=init)
    assert e.value.status == lib.E_SINGULAR
    gb.free()
    import ctypes
    st = lib._lib.afqmc_step(gb._s if gb._s else ctypes.c_void_p(), 0, 0, 1, None)
    assert st == lib.E_INVALID


@pytest.mark.parametrize("dims", [(12, 6, 3), (37, 13, 5), (200, 80, 3), (64, 16, 2), (41, 17, 4),
                                  (96, 33, 2), (256, 20, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_propagation_kernel(lib, dims, prec):
    """Fused P T_K(A) P kernel vs the same products in numpy (K = 6)."""
    M, N, nw = dims
    banner(f"propagate kernel {prec} {dims}")
    rng = np.random.default_rng(M + N)
    phi = rng.standard_normal((nw, M, N)) + 1j * rng.standard_normal((nw, M, N))
    P = rng.standard_normal((M, M)) * 0.05
    P = np.eye(M) + 0.5 * (P + P.T)
    A = (rng.standard_normal((nw, M, M)) + 1j * rng.standard_normal((nw, M, M))) * (0.4 / np.sqrt(M))
    A = 0.5 * (A + np.swapaxes(A, 1, 2))
    got = lib.selftest_propagate(phi, P, A, 6, prec)
    ref = np.empty_like(phi)
    for k in range(nw):
        y = P @ phi[k]
        term, acc = y, y.copy()
        for n in range(1, 7):
            term = A[k] @ term / n
            acc = acc + term
        ref[k] = P @ acc
    tol = {"fp64": 1e-12, "fp32": 2e-5, "bf16x3": 5e-5}[prec]
    assert rel(got, ref) < tol


@pytest.mark.parametrize("dims", [(12, 6, 3), (37, 13, 5), (130, 40, 3), (200, 80, 2), (64, 17, 2),
                                  (128, 24, 2), (224, 100, 2), (232, 20, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_propagation_shapes_bitwise(lib, dims, prec):
    """Every workgroup shape the autotuner may pick gives bitwise the result
    of the default shape (same summation order per output element)."""
    M, N, nw = dims
    banner(f"propagate shapes {prec} {dims}")
    rng = np.random.default_rng(7 * M + N)
    phi = rng.standard_normal((nw, M, N)) + 1j * rng.standard_normal((nw, M, N))
    P = rng.standard_normal((M, M)) * 0.05
    P = np.eye(M) + 0.5 * (P + P.T)
    A = (rng.standard_normal((nw, M, M)) + 1j * rng.standard_normal((nw, M, M))) * (0.4 / np.sqrt(M))
    A = 0.5 * (A + np.swapaxes(A, 1, 2))
    base = lib.selftest_propagate(phi, P, A, 6, prec, variant=0)
    # variant: (waves, column blocks per wave, prefetch, row blocks per workgroup)
    shapes = {0: (8, 2, 1, 1), 1: (4, 2, 1, 1), 2: (4, 1, 1, 1), 3: (2, 2, 1, 1), 4: (8, 2, 0, 1),
              5: (4, 2, 0, 1), 6: (4, 1, 0, 1), 7: (2, 2, 0, 1), 8: (16, 1, 0, 2), 9: (8, 1, 0, 2),
              10: (8, 2, 0, 2), 11: (4, 2, 0, 2), 12: (8, 2, 0, 5), 13: (16, 1, 0, 5)}
    ran = 0
    for v, (waves, blocks, pf, rows) in shapes.items():
        ok = ((M + 15) // 16 <= waves * blocks and not (prec == "fp64" and not pf)
              and not (rows > 1 and prec != "bf16x3")
              and not (rows == 5 and (M + 31) // 32 * 32 > 224))
        if not ok:
            with pytest.raises(lib.AfqmcError):
                lib.selftest_propagate(phi, P, A, 6, prec, variant=v)
            continue
        got = lib.selftest_propagate(phi, P, A, 6, prec, variant=v)
        assert np.array_equal(got, base), f"shape {v} differs"
        ran += 1
    assert ran >= 1
