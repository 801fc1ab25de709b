"""Pins of the oracle's multi-determinant trial (Sec. II.D, the CASSCF
trial): every quantity against the FCI-sector vector of the expansion
sum_i c_i |D_i>."""
import numpy as np
import pytest

from oracle import afqmc as O
from oracle import fci
from synth import make_expansion, make_hamiltonian, random_walkers


@pytest.fixture(scope="module", params=[(5, 2, 2, 4, 5), (6, 3, 2, 5, 6), (5, 2, 1, 3, 4)])
def msd_case(request):
    M, na, nb, nch, nd = request.param
    ham = make_hamiltonian(M, nch, seed=20 + M, e_core=0.4)
    ham.chol *= 2.0
    coeffs, dets = make_expansion(ham.h, na, nb, nd, seed=M + na, n_act=2)
    sys_ = O.System(ham.h, ham.chol, ham.e_core, dets[0], na, nb, 0.05, taylor_order=40,
                    expansion=(coeffs, dets))
    sec = fci.Sector(M, na, nb)
    ops = sec.one_body_ops()
    vt = sum(c * sec.slater(d) for c, d in zip(coeffs, dets))
    return dict(ham=ham, sys=sys_, sec=sec, ops=ops, vt=vt,
                H=fci.hamiltonian(sec, ham.h, ham.chol, ham.e_core, ops))


def test_expansion_is_a_set_of_distinct_orthonormal_determinants(msd_case):
    s = msd_case["sys"]
    assert s.n_det >= 4 and s.coeffs[0] == 1.0
    vecs = np.array([msd_case["sec"].slater(d) for d in s.dets])
    # distinct excitations of one orthonormal orbital set: orthonormal FCI vectors
    assert np.allclose(vecs @ vecs.T, np.eye(len(vecs)), atol=1e-12)


def test_overlap_force_bias_energy_against_fci(msd_case):
    s, sec, vt, H = msd_case["sys"], msd_case["sec"], msd_case["vt"], msd_case["H"]
    rho = fci.rho_ops(msd_case["ops"], msd_case["ham"].chol)
    phis = random_walkers(sec.M, s.N, 4, seed=3)
    lnov, theta = O.overlap(s, phis)
    f = O.force_bias_f(s, theta)
    el = O.local_energy(s, theta)
    for k in range(4):
        v = sec.slater(phis[k])
        ov = vt @ v
        assert abs(np.exp(lnov[k]) - ov) < 1e-12 * abs(ov)
        f_fci = np.array([(vt @ r @ v) / ov for r in rho])
        assert np.allclose(f[k], f_fci, rtol=0, atol=1e-11 * max(1.0, np.abs(f_fci).max()))
        e_fci = (vt @ H @ v) / ov
        assert abs(el[k] - e_fci) < 1e-11 * max(1.0, abs(e_fci))
    a_fci = np.array([(vt @ r @ vt) / (vt @ vt) for r in rho])
    assert np.allclose(s.a, a_fci, atol=1e-12)


def test_hs_quadrature_with_the_expansion(msd_case):
    """One Cholesky vector: the Gauss-Hermite average of the hybrid weight I(x)
    with the multi-determinant force bias equals the dense Trotter product
    against the expansion, up to the dropped constant e^{dt c0}."""
    M, na, nb, dt = 5, 2, 1, 0.05
    ham = make_hamiltonian(M, 1, seed=4, e_core=0.2)
    ham.chol *= 4.0
    coeffs, dets = make_expansion(ham.h, na, nb, 4, seed=2, n_act=2)
    s = O.System(ham.h, ham.chol, ham.e_core, dets[0], na, nb, dt, taylor_order=40,
                 expansion=(coeffs, dets))
    sec = fci.Sector(M, na, nb)
    ops = sec.one_body_ops()
    vt = sum(c * sec.slater(d) for c, d in zip(coeffs, dets))
    Hf = fci.hamiltonian(sec, ham.h, ham.chol, ham.e_core, ops)
    r0 = fci.rho_ops(ops, ham.chol)[0]
    a = (vt @ r0 @ vt) / (vt @ vt)
    assert abs(a - s.a[0]) < 1e-12
    eye = np.eye(sec.dim)
    H2 = 0.5 * (r0 - a * eye) @ (r0 - a * eye)
    half = fci.expm(-0.5 * dt * (Hf - H2))
    trotter = half @ fci.expm(-dt * H2) @ half
    c0 = ham.e_core - 0.5 * a * a
    nodes, wts = np.polynomial.hermite_e.hermegauss(80)
    wts = wts / np.sqrt(2 * np.pi)
    for phi in random_walkers(M, na + nb, 2, seed=9):
        lnov, theta = O.overlap(s, phi[None])
        acc = 0.0
        for xq, wq in zip(nodes, wts):
            lnI = O.propagate(s, phi[None], lnov, theta, np.array([[xq]]))[4]
            acc += wq * np.exp(lnI[0])
        v = sec.slater(phi)
        exact = (vt @ trotter @ v) / (vt @ v)
        assert abs(acc / exact - np.exp(dt * c0)) < 1e-10


def test_one_determinant_expansion_is_the_single_determinant_trial():
    ham = make_hamiltonian(8, 12, seed=1)
    coeffs, dets = make_expansion(ham.h, 3, 2, 1, seed=0)
    s1 = O.System(ham.h, ham.chol, 0.0, dets[0], 3, 2, 0.01)
    s2 = O.System(ham.h, ham.chol, 0.0, dets[0], 3, 2, 0.01, expansion=(2.0 * coeffs, dets))
    assert s2.n_det == 1 and np.array_equal(s1.a, s2.a) and np.array_equal(s1.P, s2.P)
