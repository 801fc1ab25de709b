"""Tangent-linear (forward-mode) derivative of the mixed energy for a
one-body perturbation h -> h + lambda V, on given fields.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The derivative is pathwise: the fields x are held fixed, so d/dlambda acts on
the deterministic map from (fields, initial walkers) to the mixed energy of
Eq. 7 after the window of steps.  lambda enters through the one-body half
propagator P = expm(-dt (h~ + lambda V) / 2) of every step in the window
(Eq. 3, Eq. 11) and through h^half = Phi_T^T (h + lambda V) in the final local
energy (Eq. 10); a_g and the Cholesky tensor do not depend on it.  The
constant energy shift of the weights is held at its value before the window
(it multiplies every weight of the system alike and cancels in Eq. 7).

Every quantity of one step (force bias, xbar, the Taylor terms, the overlap,
Theta, ln R, ln I, the phaseless weight) is differentiated along with its
value, in the order the step computes it.  A walker whose weight is set to
zero by the phase projection has zero derivative from then on (the
projection is locally constant there).

Gram-Schmidt (Sec. II.D) replaces Phi by Q = Phi R^{-1} with R upper
triangular; every later quantity depends on Q only through expressions that
are unchanged by Q -> Q U for invertible U (Theta, differences of ln
overlaps, the propagated determinants up to the same U), so the tangent may
drop the change of R: dQ = dPhi R^{-1}, with R = Q^H Phi.
"""
from __future__ import annotations

from typing import Callable, Tuple

import numpy as np
import scipy.linalg

from .afqmc import (PHASELESS, System, Walkers, force_bias_f, local_energy, orthonormalize,
                    overlap, xbar_of)


def d_overlap(sys: System, phi: np.ndarray, theta: np.ndarray, dphi: np.ndarray):
    """Tangents of ln <phi_T|phi> and Theta: d ln det O = Tr(O^{-1} dO),
    dTheta = (dPhi - Theta dO) O^{-1}, dO = Phi_T^T dPhi, per spin block."""
    nw = phi.shape[0]
    dlnov = np.zeros(nw, dtype=np.complex128)
    dtheta = np.zeros_like(phi)
    for off, n in sys.spins:
        if n == 0:
            continue
        t = sys.trial[:, off:off + n]
        o = np.matmul(t.T[None], phi[:, :, off:off + n])
        do = np.matmul(t.T[None], dphi[:, :, off:off + n])
        dlnov += np.trace(np.linalg.solve(o, do), axis1=1, axis2=2)
        rhs = dphi[:, :, off:off + n] - np.matmul(theta[:, :, off:off + n], do)
        dtheta[:, :, off:off + n] = np.swapaxes(
            np.linalg.solve(np.swapaxes(o, 1, 2), np.swapaxes(rhs, 1, 2)), 1, 2)
    return dlnov, dtheta


class Tangent:
    """dPhi, dw, d ln overlap and dTheta of every walker."""

    def __init__(self, wk: Walkers):
        self.phi = np.zeros_like(wk.phi)
        self.weight = np.zeros(wk.weight.shape)
        self.lnov = np.zeros_like(wk.lnov)
        self.theta = np.zeros_like(wk.theta)


def tangent_step(sys: System, dP: np.ndarray, wk: Walkers, d: Tangent, x: np.ndarray):
    """One phaseless step of the walkers and of their tangents (in place)."""
    live = wk.alive
    nw = wk.phi.shape[0]
    sq = np.sqrt(sys.dt)
    G, M = sys.n_chol, sys.M
    f = force_bias_f(sys, wk.theta)
    df = force_bias_f(sys, d.theta)                 # f is linear in Theta
    xbar = xbar_of(sys, f)
    dxbar = -sq * 1j * df
    c = x - xbar
    dc = -dxbar
    lflat = sys.chol.reshape(G, M * M)
    A = (1j * sq * (c @ lflat)).reshape(nw, M, M)
    dA = (1j * sq * (dc @ lflat)).reshape(nw, M, M)
    s = -1j * sq * (c @ sys.a)
    ds = -1j * sq * (dc @ sys.a)
    p = np.matmul(sys.P[None], wk.phi)
    dp = np.matmul(dP[None], wk.phi) + np.matmul(sys.P[None], d.phi)
    term, dterm = p, dp
    acc, dacc = p.copy(), dp.copy()
    for n in range(1, sys.K + 1):
        dterm = (np.matmul(dA, term) + np.matmul(A, dterm)) / n
        term = np.matmul(A, term) / n
        acc = acc + term
        dacc = dacc + dterm
    new_phi = np.matmul(sys.P[None], acc)
    dnew_phi = np.matmul(dP[None], acc) + np.matmul(sys.P[None], dacc)
    new_lnov, new_theta = overlap(sys, new_phi)
    dnew_lnov, dnew_theta = d_overlap(sys, new_phi, new_theta, dnew_phi)
    lnR = new_lnov - wk.lnov + s
    dlnR = dnew_lnov - d.lnov + ds
    lnI = lnR + np.sum(x * xbar - 0.5 * xbar * xbar, axis=1)
    dlnI = dlnR + np.sum((x - xbar) * dxbar, axis=1)
    g = np.exp(lnI.real + sys.dt * wk.e_shift)
    cs = np.cos(lnR.imag)
    fac = g * np.maximum(0.0, cs)
    dfac = np.where(cs > 0.0, g * (dlnI.real * cs - np.sin(lnR.imag) * dlnR.imag), 0.0)
    w_new = wk.weight * fac
    dw_new = d.weight * fac + wk.weight * dfac
    ok = np.isfinite(w_new) & (w_new > 0.0)
    w_new = np.where(ok, w_new, 0.0)
    dw_new = np.where(ok, dw_new, 0.0)
    upd = live
    wk.phi[upd], d.phi[upd] = new_phi[upd], dnew_phi[upd]
    wk.lnov[upd], d.lnov[upd] = new_lnov[upd], dnew_lnov[upd]
    wk.theta[upd], d.theta[upd] = new_theta[upd], dnew_theta[upd]
    wk.weight[upd], d.weight[upd] = w_new[upd], dw_new[upd]
    wk.alive = live & ok
    wk.t += 1


def tangent_orthonormalize(sys: System, wk: Walkers, d: Tangent):
    """Gram-Schmidt of the walkers; the tangent follows as dPhi R^{-1}."""
    live = wk.alive
    before = wk.phi[live].copy()
    orthonormalize(sys, wk)
    q = wk.phi[live]
    dq = d.phi[live].copy()
    for off, n in sys.spins:
        if n == 0:
            continue
        r = np.matmul(np.conj(np.swapaxes(q[:, :, off:off + n], 1, 2)), before[:, :, off:off + n])
        # dQ = dPhi R^{-1}  <=>  dQ^T = solve(R^T, dPhi^T)
        dq[:, :, off:off + n] = np.swapaxes(
            np.linalg.solve(np.swapaxes(r, 1, 2), np.swapaxes(dq[:, :, off:off + n], 1, 2)), 1, 2)
    dlnov, dtheta = d_overlap(sys, q, wk.theta[live], dq)
    d.phi[live] = dq
    d.lnov[live] = dlnov
    d.theta[live] = dtheta


def d_local_energy(sys: System, V: np.ndarray, theta: np.ndarray, dtheta: np.ndarray):
    """Tangent of E_L (Eq. 7, 10): the explicit h^half term plus the chain
    through Theta (one-body, Coulomb f^2 and exchange Tr(T T))."""
    nw = theta.shape[0]
    f = force_bias_f(sys, theta)
    df = force_bias_f(sys, dtheta)
    de = np.sum(f * df, axis=1)
    for (off, n), lh, hh in zip(sys.spins, sys.lhalf, sys.hhalf):
        if n == 0:
            continue
        t = sys.trial[:, off:off + n]
        th = theta[:, :, off:off + n]
        dth = dtheta[:, :, off:off + n]
        de += np.einsum("im,wmi->w", t.T @ V, th) + np.einsum("im,wmi->w", hh, dth)
        for w in range(nw):
            tt = np.matmul(lh, th[w])            # (g, n, n)
            dtt = np.matmul(lh, dth[w])
            de[w] -= np.sum(tt * np.swapaxes(dtt, 1, 2))
    return de


def energy_and_tangent(sys: System, V: np.ndarray, wk: Walkers, d: Tangent) -> Tuple[float, float]:
    """E = sum w Re E_L / sum w over live walkers, and its tangent."""
    m = wk.alive
    el = local_energy(sys, wk.theta)
    dl = d_local_energy(sys, V, wk.theta, d.theta)
    w, dw = wk.weight[m], d.weight[m]
    W = np.sum(w)
    E = float(np.sum(w * el[m].real) / W)
    dE = float((np.sum(dw * el[m].real) + np.sum(w * dl[m].real)) / W - E * np.sum(dw) / W)
    return E, dE


def window_tangent(sys: System, V: np.ndarray, wk: Walkers, fields: Callable, n_steps: int,
                   ortho_every: int) -> Tuple[float, float, Walkers]:
    """Advance a copy of the walkers n_steps (Gram-Schmidt every ortho_every
    steps) with their tangents from zero, and return the mixed energy at the
    end, dE/dlambda, and the advanced walkers."""
    V = np.asarray(V, dtype=np.float64)
    wk = wk.copy()
    d = Tangent(wk)
    X = -0.5 * sys.dt * sys.htilde
    dP = scipy.linalg.expm_frechet(X, -0.5 * sys.dt * V, compute_expm=False)
    for _ in range(n_steps):
        x = fields(wk.t, wk.phi.shape[0])
        tangent_step(sys, dP, wk, d, x)
        if ortho_every > 0 and wk.t % ortho_every == 0:
            tangent_orthonormalize(sys, wk, d)
    E, dE = energy_and_tangent(sys, V, wk, d)
    return E, dE, wk


def window_energy(sys: System, wk: Walkers, fields: Callable, n_steps: int,
                  ortho_every: int) -> float:
    """Mixed energy after n_steps more plain steps of a copy of the walkers
    (the quantity window_tangent differentiates)."""
    from .afqmc import mixed_energy, step
    wk = wk.copy()
    for _ in range(n_steps):
        step(sys, wk, fields(wk.t, wk.phi.shape[0]), PHASELESS)
        if ortho_every > 0 and wk.t % ortho_every == 0:
            orthonormalize(sys, wk)
    return mixed_energy(wk, local_energy(sys, wk.theta), PHASELESS)
