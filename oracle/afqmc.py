"""Plain FP64 oracle of the correlated-sampling ph-AFQMC walker step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (the readings of the paper this oracle takes):

* Hamiltonian, Eq. 1: H = sum_ij h_ij E_ij + 1/2 sum_ijkl V_ijkl
  sum_{s,t} c+_is c+_jt c_lt c_ks + e_core, V_ijkl = sum_g L^g_ik L^g_jl,
  L^g real symmetric.  v_g = i rho_g with rho_g = sum_ik L^g_ik E_ik.
* Mean-field subtraction, Eq. 2: <v_g> = i a_g, a_g = <phi_T|rho_g|phi_T>.
  The one-body remainder H_1 (the paper leaves it implicit) is
  h~ = h - 1/2 sum_g L_g L_g + sum_g a_g L_g plus a constant that is a
  uniform factor on every walker and is dropped.
* Walker step, Eq. 3, 4, 11: B(x - xbar) = e^{-dt H1/2} e^{sqrt(dt)(x-xbar)
  (v - <v>)} e^{-dt H1/2}.  Acting on a determinant (Thouless theorem) it is
  Phi -> P T_K(A) P Phi times the c-number e^{s}, with P = expm(-dt h~/2),
  A = i sqrt(dt) sum_g c_g L_g, s = -i sqrt(dt) sum_g c_g a_g, c = x - xbar,
  and T_K the Taylor polynomial of order K (term_n = A term_{n-1} / n).
  The B(x) printed after Eq. 5 lacks the 1/2 on H_1; Eq. 3 and Eq. 11 have
  it, and they are followed.
* Force bias, Eq. 8-9: xbar_g = -sqrt(dt)(vbar_g - <v_g>) with
  vbar_g = i f_g, f_g = sum_s Tr(L^half_{g s} Theta^s), evaluated on the
  walker at the start of the step.  Eq. 8's "x_alpha xbar" is read as
  x_alpha xbar_alpha summed over alpha.
* Hybrid weight, Sec. II.D: I = R e^{sum_g (x_g xbar_g - xbar_g^2/2)},
  R = <phi_T|B|phi>/<phi_T|phi> (c-number included).  Phaseless update,
  Sec. II.A: w <- w |I| max(0, cos(Im ln R)).  A walker whose weight is no
  longer positive is frozen for the rest of the run (Sec. II.B).
* Energy shift (the paper is silent): every weight update carries the
  constant factor e^{dt e_shift}, e_shift = Re E_L(phi_init) - c0 with
  c0 = e_core - 1/2 sum_g a_g^2 the constant of H_1.  It is the same for
  every walker of a system, so it cancels in Eq. 7; it keeps weights O(1)
  over long runs (without it they grow like e^{-dt (E_L - c0) t} and leave
  the FP64 range within a few hundred steps).
* Mixed estimator, Eq. 7 and Eq. 10: E = sum_k w_k Re E_L(phi_k) / sum_k w_k
  over live walkers; E_L = e_core + sum_s Tr(h^half_s Theta^s)
  + 1/2 sum_g [(sum_s Tr T_gs)^2 - sum_s Tr(T_gs T_gs)], T_gs = L^half_gs Theta^s.
* Modified Gram-Schmidt, Sec. II.D: each spin block of each walker, columns
  in index order (normalise column j, then remove its projection q_j^H v
  from every later column); the overlap and Theta are recomputed and the
  weight is left unchanged (the walker representation of Eq. 6 is invariant
  under Phi -> Phi R).  MGS runs before a measurement that falls on the same
  step.
* Free projection, Sec. II.A: xbar = 0, complex weights W <- W R, no
  projection; importance-sampled free projection: W <- W I.  Estimator
  Re(sum W E_L / sum W).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Dict, List, Optional

import numpy as np
import scipy.linalg

from . import philox

PHASELESS = "phaseless"
FREE = "free"
IS_FREE = "is_free"


class System:
    """Per-system quantities fixed for a run (the precompute of the step)."""

    def __init__(self, h, chol, e_core, trial, n_alpha, n_beta, dt, taylor_order=6,
                 h_pert: Optional[np.ndarray] = None, lam: float = 0.0, fb_cap: float = 0.0,
                 cap_apply: bool = False, expansion=None):
        h = np.asarray(h, dtype=np.float64)
        if h_pert is not None:
            h = h + lam * np.asarray(h_pert, dtype=np.float64)
        self.h = h
        self.chol = np.asarray(chol, dtype=np.float64)
        self.e_core = float(e_core)
        self.trial = np.asarray(trial, dtype=np.float64)
        self.na, self.nb = int(n_alpha), int(n_beta)
        self.N = self.na + self.nb
        self.M = h.shape[0]
        self.n_chol = self.chol.shape[0]
        self.dt = float(dt)
        self.K = int(taylor_order)
        # optional force-bias cap (a bounding condition the paper cites in
        # Sec. II.D without stating it): |xbar_g| > fb_cap is counted and,
        # with cap_apply, scaled to modulus fb_cap keeping its phase
        self.fb_cap = float(fb_cap)
        self.cap_apply = bool(cap_apply)
        assert self.trial.shape == (self.M, self.N)
        # spin blocks: (offset, count)
        self.spins = [(0, self.na), (self.na, self.nb)]
        # Multi-determinant trial (Sec. II.D, the CASSCF trial): expansion =
        # (coefficients c_i, determinants D_i of shape (M, N)); the trial is
        # sum_i c_i |D_i>.  Without it the trial is the one determinant `trial`.
        if expansion is not None:
            coeffs, dets = expansion
            self.coeffs = np.asarray(coeffs, dtype=np.float64)
            self.dets = np.asarray(dets, dtype=np.float64)
            assert self.dets.shape == (len(self.coeffs), self.M, self.N)
            self.trial = self.dets[0]
        else:
            self.coeffs = np.ones(1)
            self.dets = self.trial[None]
        self.n_det = len(self.coeffs)
        # Half-rotated tensors of every determinant: L^half_{g s} = D^{sT} L_g,
        # h^half_s = D^{sT} h.
        self.lhalf_d, self.hhalf_d = [], []
        for d in self.dets:
            lh, hh = [], []
            for off, n in self.spins:
                t = d[:, off:off + n]
                lh.append(np.matmul(t.T[None], self.chol))
                hh.append(t.T @ h)
            self.lhalf_d.append(lh)
            self.hhalf_d.append(hh)
        if self.n_det == 1:
            # Trial density G_T^s = Phi_T (Phi_T^T Phi_T)^{-1} Phi_T^T and
            # a_g = sum_s Tr(L_g G_T^s): <v_g> = i a_g (Eq. 2, Eq. 9).
            self.a = np.zeros(self.n_chol)
            for off, n in self.spins:
                if n == 0:
                    continue
                t = self.trial[:, off:off + n]
                g_t = t @ np.linalg.solve(t.T @ t, t.T)
                self.a += self.chol.reshape(self.n_chol, self.M * self.M) @ g_t.T.reshape(-1)
        else:
            # a_g = <phi_T|rho_g|phi_T>/<phi_T|phi_T> = sum_j c_j <phi_T|D_j> f_g(D_j)
            # / sum_j c_j <phi_T|D_j>, with f_g(D_j) = <phi_T|rho_g|D_j>/<phi_T|D_j>
            # the mixed estimate at the determinant D_j.
            lnov_d, theta_d = overlap(self, self.dets.astype(np.complex128))
            fd = force_bias_f(self, theta_d)
            wgt = self.coeffs * np.exp(lnov_d - np.max(lnov_d.real))
            self.a = (np.sum(wgt[:, None] * fd, axis=0) / np.sum(wgt)).real
        # One-body part after mean-field subtraction (Eq. 2).
        M_, G_ = self.M, self.n_chol
        l2 = (np.swapaxes(self.chol, 0, 1).reshape(M_, G_ * M_) @ self.chol.reshape(G_ * M_, M_)
              if G_ else np.zeros((M_, M_)))
        self.htilde = h - 0.5 * l2 + np.einsum("g,gij->ij", self.a, self.chol)
        self.P = scipy.linalg.expm(-0.5 * self.dt * self.htilde)
        self.lhalf = self.lhalf_d[0]
        self.hhalf = self.hhalf_d[0]


@dataclass
class Walkers:
    phi: np.ndarray       # (nw, M, N) complex
    weight: np.ndarray    # (nw,) float (phaseless) or complex (free modes)
    lnov: np.ndarray      # (nw,) complex: sum_s ln det(Phi_T^{sT} Phi^s)
    theta: np.ndarray     # (nw, M, N) complex: Phi^s (Phi_T^{sT} Phi^s)^{-1}
    alive: np.ndarray     # (nw,) bool
    t: int = 0            # absolute step counter (feeds the field generator)
    e_shift: float = 0.0  # constant energy shift of the weight factor
    cap_events: int = 0   # (live walker, step, gamma) with |xbar| above the cap

    def copy(self) -> "Walkers":
        return Walkers(self.phi.copy(), self.weight.copy(), self.lnov.copy(),
                       self.theta.copy(), self.alive.copy(), self.t, self.e_shift,
                       self.cap_events)


class MsdTheta:
    """Per-walker data of a multi-determinant trial: th[k, i] = Theta of walker
    k against determinant D_i (Phi^s (D_i^{sT} Phi^s)^{-1} per spin block) and
    ld[k, i] = ln <D_i|phi_k> (without c_i)."""

    def __init__(self, th: np.ndarray, ld: np.ndarray):
        self.th, self.ld = th, ld

    def __getitem__(self, idx) -> "MsdTheta":
        return MsdTheta(self.th[idx], self.ld[idx])

    def __setitem__(self, idx, other: "MsdTheta"):
        self.th[idx] = other.th
        self.ld[idx] = other.ld

    def copy(self) -> "MsdTheta":
        return MsdTheta(self.th.copy(), self.ld.copy())


def _det_overlap(trial: np.ndarray, spins, phi: np.ndarray):
    """ln det(D^{sT} Phi^s) summed over spins, and Theta against one
    determinant D."""
    nw = phi.shape[0]
    lndet = np.zeros(nw, dtype=np.complex128)
    theta = np.zeros_like(phi)
    for off, n in spins:
        if n == 0:
            continue
        t = trial[:, off:off + n]
        ps = phi[:, :, off:off + n]
        o = np.matmul(t.T[None], ps)
        sign, logabs = np.linalg.slogdet(o)
        lndet += logabs + 1j * np.angle(sign)
        theta[:, :, off:off + n] = np.swapaxes(
            np.linalg.solve(np.swapaxes(o, 1, 2), np.swapaxes(ps, 1, 2)), 1, 2)
    return lndet, theta


def det_weights(sys: System, ld: np.ndarray):
    """ln <phi_T|phi> = ln sum_i c_i <D_i|phi> and r_i = c_i <D_i|phi> / <phi_T|phi>
    from the per-determinant log overlaps ld (nw, n_det)."""
    top = np.max(ld.real, axis=1, keepdims=True)
    terms = sys.coeffs[None, :] * np.exp(ld - top)
    tot = np.sum(terms, axis=1)
    return np.log(tot) + top[:, 0], terms / tot[:, None]


def overlap(sys: System, phi: np.ndarray):
    """ln <phi_T|phi> = sum_s ln det(Phi_T^{sT} Phi^s) by LU with partial
    pivoting, and Theta^s = Phi^s (Phi_T^{sT} Phi^s)^{-1}.  With a
    multi-determinant trial: ln sum_i c_i <D_i|phi> and an MsdTheta."""
    if sys.n_det > 1:
        nw = phi.shape[0]
        th = np.zeros((nw, sys.n_det) + phi.shape[1:], dtype=np.complex128)
        ld = np.zeros((nw, sys.n_det), dtype=np.complex128)
        for i, d in enumerate(sys.dets):
            ld[:, i], th[:, i] = _det_overlap(d, sys.spins, phi)
        return det_weights(sys, ld)[0], MsdTheta(th, ld)
    nw = phi.shape[0]
    lndet = np.zeros(nw, dtype=np.complex128)
    theta = np.zeros_like(phi)
    for off, n in sys.spins:
        if n == 0:
            continue
        t = sys.trial[:, off:off + n]
        ps = phi[:, :, off:off + n]
        o = np.matmul(t.T[None], ps)                    # (nw, n, n)
        sign, logabs = np.linalg.slogdet(o)
        lndet += logabs + 1j * np.angle(sign)
        # Theta = Phi O^{-1}  <=>  Theta^T = solve(O^T, Phi^T)
        theta[:, :, off:off + n] = np.swapaxes(
            np.linalg.solve(np.swapaxes(o, 1, 2), np.swapaxes(ps, 1, 2)), 1, 2)
    return lndet, theta


def init_walkers(sys: System, nw: int, init_phi: Optional[np.ndarray] = None,
                 complex_weights: bool = False) -> Walkers:
    """Walkers start from the trial (or a given determinant) with weight 1."""
    src = sys.trial if init_phi is None else np.asarray(init_phi)
    phi = np.broadcast_to(src.astype(np.complex128), (nw, sys.M, sys.N)).copy()
    lnov, theta = overlap(sys, phi)
    w = np.ones(nw, dtype=np.complex128 if complex_weights else np.float64)
    e_t = local_energy(sys, theta[:1])[0].real
    c0 = sys.e_core - 0.5 * float(np.sum(sys.a * sys.a))
    return Walkers(phi, w, lnov, theta, np.ones(nw, dtype=bool), 0, e_t - c0)


def force_bias_f(sys: System, theta) -> np.ndarray:
    """f_g = sum_s Tr(L^half_{g s} Theta^s) = <phi_T|rho_g|phi>/<phi_T|phi>;
    with a multi-determinant trial sum_i r_i f_g^{(i)}, r_i = c_i <D_i|phi> /
    <phi_T|phi>."""
    if isinstance(theta, MsdTheta):
        r = det_weights(sys, theta.ld)[1]
        return sum(r[:, i, None] * _det_force_bias(sys.spins, sys.lhalf_d[i], theta.th[:, i],
                                                     sys.n_chol, sys.M)
                   for i in range(sys.n_det))
    return _det_force_bias(sys.spins, sys.lhalf, theta, sys.n_chol, sys.M)


def _det_force_bias(spins, lhalf, theta, n_chol, M) -> np.ndarray:
    nw = theta.shape[0]
    f = np.zeros((nw, n_chol), dtype=np.complex128)
    for (off, n), lh in zip(spins, lhalf):
        if n == 0:
            continue
        th = np.swapaxes(theta[:, :, off:off + n], 1, 2).reshape(nw, -1)   # (nw, n*M) as (i, m)
        f += th @ lh.reshape(n_chol, n * M).T
    return f


def xbar_of(sys: System, f: np.ndarray) -> np.ndarray:
    """Optimal force bias, Eq. 9: xbar = -sqrt(dt) (i f - i a)."""
    return -np.sqrt(sys.dt) * (1j * f - 1j * sys.a[None, :])


def cap_xbar(xbar: np.ndarray, cap: float) -> np.ndarray:
    """Entries with |xbar| > cap scaled to modulus cap, phase kept."""
    mag = np.abs(xbar)
    over = mag > cap
    return np.where(over, xbar * (cap / np.where(over, mag, 1.0)), xbar)


def propagate(sys: System, phi: np.ndarray, lnov: np.ndarray, theta: np.ndarray,
              x: np.ndarray, mode: str = PHASELESS, taylor_order: Optional[int] = None):
    """One application of B(x - xbar) to each walker (no weight bookkeeping).

    Returns the propagated determinants, their ln overlap and Theta, ln R and
    ln I of the hybrid weight, and xbar."""
    K = sys.K if taylor_order is None else int(taylor_order)
    nw = phi.shape[0]
    sq = np.sqrt(sys.dt)
    if mode == FREE:
        xbar = np.zeros((nw, sys.n_chol), dtype=np.complex128)
    else:
        xbar = xbar_of(sys, force_bias_f(sys, theta))
        if sys.fb_cap > 0.0 and sys.cap_apply:
            xbar = cap_xbar(xbar, sys.fb_cap)
    c = x - xbar
    A = (1j * sq * (c @ sys.chol.reshape(sys.n_chol, sys.M * sys.M))).reshape(nw, sys.M, sys.M)
    s = -1j * sq * (c @ sys.a)
    p = np.matmul(sys.P[None], phi)
    term = p
    acc = p.copy()
    for n in range(1, K + 1):
        term = np.matmul(A, term) / n
        acc = acc + term
    new_phi = np.matmul(sys.P[None], acc)
    new_lnov, new_theta = overlap(sys, new_phi)
    lnR = new_lnov - lnov + s
    lnI = lnR + np.sum(x * xbar - 0.5 * xbar * xbar, axis=1)
    return new_phi, new_lnov, new_theta, lnR, lnI, xbar


def step(sys: System, wk: Walkers, x: np.ndarray, mode: str = PHASELESS) -> Walkers:
    """Advance all live walkers one time step with fields x (nw, n_chol)."""
    live = wk.alive
    if sys.fb_cap > 0.0 and mode != FREE:
        raw = xbar_of(sys, force_bias_f(sys, wk.theta))
        wk.cap_events += int(np.sum((np.abs(raw) > sys.fb_cap) & live[:, None]))
    new_phi, new_lnov, new_theta, lnR, lnI, _ = propagate(sys, wk.phi, wk.lnov, wk.theta, x, mode)
    shift = sys.dt * wk.e_shift
    if mode == PHASELESS:
        fac = np.exp(lnI.real + shift) * np.maximum(0.0, np.cos(lnR.imag))
        w_new = wk.weight * fac
        ok = np.isfinite(w_new) & (w_new > 0.0)
        w_new = np.where(ok, w_new, 0.0)
        still = live & ok
    elif mode == FREE:
        w_new = wk.weight * np.exp(lnR + shift)
        still = live.copy()
    elif mode == IS_FREE:
        w_new = wk.weight * np.exp(lnI + shift)
        still = live.copy()
    else:
        raise ValueError(mode)
    upd = live
    wk.phi[upd] = new_phi[upd]
    wk.lnov[upd] = new_lnov[upd]
    wk.theta[upd] = new_theta[upd]
    wk.weight[upd] = w_new[upd]
    wk.alive = still
    wk.t += 1
    return wk


def orthonormalize(sys: System, wk: Walkers) -> Walkers:
    """Modified Gram-Schmidt on each spin block of each live walker."""
    live = wk.alive
    phi = wk.phi[live].copy()
    for off, n in sys.spins:
        for j in range(n):
            q = phi[:, :, off + j]
            nrm = np.sqrt(np.sum((q.conj() * q).real, axis=1))
            q = q / nrm[:, None]
            phi[:, :, off + j] = q
            if j + 1 < n:
                rest = phi[:, :, off + j + 1:off + n]
                proj = np.einsum("wm,wml->wl", q.conj(), rest)
                phi[:, :, off + j + 1:off + n] = rest - q[:, :, None] * proj[:, None, :]
    lnov, theta = overlap(sys, phi)
    wk.phi[live] = phi
    wk.lnov[live] = lnov
    wk.theta[live] = theta
    return wk


def local_energy(sys: System, theta, chunk: int = 8) -> np.ndarray:
    """Mixed local energy E_L = <phi_T|H|phi>/<phi_T|phi> (Eq. 7), complex;
    with a multi-determinant trial sum_i r_i E_L^{(i)}, E_L^{(i)} the energy
    against D_i."""
    if isinstance(theta, MsdTheta):
        r = det_weights(sys, theta.ld)[1]
        return sum(r[:, i] * _det_local_energy(sys, sys.lhalf_d[i], sys.hhalf_d[i],
                                               theta.th[:, i], chunk)
                   for i in range(sys.n_det))
    return _det_local_energy(sys, sys.lhalf, sys.hhalf, theta, chunk)


def _det_local_energy(sys: System, lhalf, hhalf, theta: np.ndarray, chunk: int) -> np.ndarray:
    nw = theta.shape[0]
    f = _det_force_bias(sys.spins, lhalf, theta, sys.n_chol, sys.M)
    e1 = np.zeros(nw, dtype=np.complex128)
    exch = np.zeros(nw, dtype=np.complex128)
    for (off, n), lh, hh in zip(sys.spins, lhalf, hhalf):
        if n == 0:
            continue
        th = theta[:, :, off:off + n]
        e1 += np.einsum("im,wmi->w", hh, th)
        for w0 in range(0, nw, chunk):
            tt = np.matmul(lh[None], th[w0:w0 + chunk, None])    # (c, g, n, n)
            exch[w0:w0 + chunk] += np.sum(tt * np.swapaxes(tt, 2, 3), axis=(1, 2, 3))
    return sys.e_core + e1 + 0.5 * (np.sum(f * f, axis=1) - exch)


def mixed_energy(wk: Walkers, e_local: np.ndarray, mode: str = PHASELESS):
    """Eq. 7 over live walkers; phaseless uses Re E_L (Eq. 10)."""
    if mode == PHASELESS:
        m = wk.alive
        den = np.sum(wk.weight[m])
        return float(np.sum(wk.weight[m] * e_local[m].real) / den) if den > 0 else float("nan")
    return complex(np.sum(wk.weight * e_local) / np.sum(wk.weight)).real


# ------------------------------------------- population control and PES

def comb(wk: Walkers, xi: float) -> Walkers:
    """Population control by the comb (Sec. II.B: walkers with large weights
    are replicated, small ones stochastically removed), keeping the walker
    count: with C the running sum of the live weights in walker order and
    W = C[-1], the j-th new walker copies the first walker k with
    C[k] > (j + xi) W / Nw (xi in [0, 1) drawn once per call); every new
    walker is live with weight W / Nw, so the total weight is kept.  A point
    that rounding puts at or past W takes the last walker of positive weight.
    Phaseless mode only."""
    w = np.where(wk.alive, wk.weight, 0.0)
    nw = w.shape[0]
    C = np.cumsum(w)
    W = C[-1]
    if not W > 0:
        raise ValueError("no walker of positive weight")
    z = (np.arange(nw, dtype=np.float64) + xi) * W / nw
    sel = np.searchsorted(C, z, side="right")
    last = int(np.nonzero(w > 0)[0][-1])
    sel = np.where(sel >= nw, last, sel)
    wk.phi = wk.phi[sel].copy()
    wk.lnov = wk.lnov[sel].copy()
    wk.theta = wk.theta[sel].copy()
    wk.weight = np.full(nw, W / nw)
    wk.alive = np.ones(nw, dtype=bool)
    return wk


def init_from_primary(sec: System, pri: System, wk_pri: Walkers) -> Walkers:
    """Preliminary equilibration scheme (Sec. II.B): the secondary system's
    walkers start from the primary's determinants (the first N_alpha and
    N_beta orbital columns of each spin block when the secondary has fewer
    electrons) with weights scaled by <phi_T^sec|phi>/<phi_T^pri|phi>, the
    phase of that ratio projected as in the phaseless step:
    w_sec = w_pri |ratio| max(0, cos arg ratio)."""
    assert sec.M == pri.M and sec.na <= pri.na and sec.nb <= pri.nb
    cols = list(range(sec.na)) + [pri.na + j for j in range(sec.nb)]
    phi = wk_pri.phi[:, :, cols].copy()
    lnov, theta = overlap(sec, phi)
    ln_ratio = lnov - wk_pri.lnov
    w = wk_pri.weight * np.exp(ln_ratio.real) * np.maximum(0.0, np.cos(ln_ratio.imag))
    alive = wk_pri.alive & (w > 0)
    w = np.where(alive, w, 0.0)
    e_t = local_energy(sec, overlap(sec, sec.trial[None].astype(np.complex128))[1])[0].real
    c0 = sec.e_core - 0.5 * float(np.sum(sec.a * sec.a))
    return Walkers(phi, w, lnov, theta, alive, wk_pri.t, e_t - c0)


# --------------------------------------------------------------------- fields

class ExplicitFields:
    """Fields given as an array x[t, k, gamma] (absolute step t)."""

    def __init__(self, x: np.ndarray, walkers=None):
        self.x = np.asarray(x, dtype=np.float64)
        self.walkers = None if walkers is None else np.asarray(walkers)

    def __call__(self, t: int, nw: int) -> np.ndarray:
        x = self.x[t]
        return x if self.walkers is None else x[self.walkers]


class PhiloxFields:
    """Counter-based fields: walker k of every system sees the same draws."""

    def __init__(self, seed: int, stream: int, n_chol: int, walkers=None):
        self.seed, self.stream, self.n_chol = int(seed), int(stream), int(n_chol)
        self.walkers = None if walkers is None else np.asarray(walkers)

    def __call__(self, t: int, nw: int) -> np.ndarray:
        idx = np.arange(nw) if self.walkers is None else self.walkers
        return philox.normals(self.seed, self.stream, t, idx, self.n_chol)


def run(sys: System, wk: Walkers, fields: Callable, n_steps: int, ortho_every: int,
        measure_every: int, mode: str = PHASELESS) -> Dict[str, List]:
    """Single-system run; returns the measured mixed energies."""
    out = {"t": [], "E": []}
    for _ in range(n_steps):
        x = fields(wk.t, wk.phi.shape[0])
        step(sys, wk, x, mode)
        if ortho_every > 0 and wk.t % ortho_every == 0:
            orthonormalize(sys, wk)
        if measure_every > 0 and wk.t % measure_every == 0:
            out["t"].append(wk.t)
            out["E"].append(mixed_energy(wk, local_energy(sys, wk.theta), mode))
    return out


def run_pair(sa: System, sb: System, wa: Walkers, wb: Walkers, fields: Callable, n_steps: int,
             ortho_every: int, measure_every: int, mode: str = PHASELESS) -> Dict[str, List]:
    """Correlated pair (Sec. II.B): walker k of A and of B use the same fields
    x[t, k, :] at every step; no population control."""
    assert sa.n_chol == sb.n_chol and sa.M == sb.M
    assert wa.phi.shape[0] == wb.phi.shape[0] and wa.t == wb.t
    out = {"t": [], "EA": [], "EB": [], "dE": []}
    for _ in range(n_steps):
        x = fields(wa.t, wa.phi.shape[0])
        step(sa, wa, x, mode)
        step(sb, wb, x, mode)
        for s, w in ((sa, wa), (sb, wb)):
            if ortho_every > 0 and w.t % ortho_every == 0:
                orthonormalize(s, w)
        if measure_every > 0 and wa.t % measure_every == 0:
            ea = mixed_energy(wa, local_energy(sa, wa.theta), mode)
            eb = mixed_energy(wb, local_energy(sb, wb.theta), mode)
            out["t"].append(wa.t)
            out["EA"].append(ea)
            out["EB"].append(eb)
            out["dE"].append(eb - ea)
    return out
