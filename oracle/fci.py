"""Dense determinant-space (FCI) tools for tiny systems; test pins only.

TEST INFRASTRUCTURE ONLY.  Builds the second-quantised Hamiltonian of Eq. 1
directly from V_ijkl = sum_g L^g_ik L^g_jl in the sector of fixed (N_alpha,
N_beta), with fermionic signs from explicit occupation bitstrings.  Nothing
here uses the Cholesky/Wick shortcuts of the walker step, so it pins them.

Basis ordering: spin-orbitals 0..M-1 are alpha, M..2M-1 are beta; a basis
determinant is c+_{p1} ... c+_{pN}|0> with p1 < ... < pN.  The amplitude of
the Slater determinant prod_i (sum_m Phi^a_mi c+_ma) prod_j (sum_m Phi^b_mj
c+_mb)|0> on that basis state is det(Phi^a[occ_a]) det(Phi^b[occ_b]).
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.linalg


class Sector:
    def __init__(self, M: int, na: int, nb: int):
        self.M, self.na, self.nb = M, na, nb
        self.alpha = list(combinations(range(M), na))
        self.beta = list(combinations(range(M), nb))
        self.dets = [(a, b) for a in self.alpha for b in self.beta]
        self.index = {d: i for i, d in enumerate(self.dets)}
        self.dim = len(self.dets)

    def _excite(self, occ, p, q):
        """c+_p c_q on one spin string (sorted tuple); returns (sign, occ') or None."""
        if q not in occ:
            return None
        if p != q and p in occ:
            return None
        lst = list(occ)
        iq = lst.index(q)
        sign = (-1) ** iq
        lst.pop(iq)
        ip = sum(1 for o in lst if o < p)
        sign *= (-1) ** ip
        lst.insert(ip, p)
        return sign, tuple(lst)

    def excitation(self, spin: int, p: int, q: int) -> np.ndarray:
        """Matrix of E^spin_pq = c+_{p spin} c_{q spin} in this sector.

        The beta string sits after the full alpha string, so the sign from
        moving past the alpha block is the same for c+ and c and cancels."""
        E = np.zeros((self.dim, self.dim))
        for col, (a, b) in enumerate(self.dets):
            occ = a if spin == 0 else b
            r = self._excite(occ, p, q)
            if r is None:
                continue
            sign, new = r
            d = (new, b) if spin == 0 else (a, new)
            E[self.index[d], col] += sign
        return E

    def one_body_ops(self) -> np.ndarray:
        """E_pq = sum_spin E^spin_pq, shape (M, M, dim, dim)."""
        M = self.M
        ops = np.zeros((M, M, self.dim, self.dim))
        for p in range(M):
            for q in range(M):
                ops[p, q] = self.excitation(0, p, q) + self.excitation(1, p, q)
        return ops

    def slater(self, phi: np.ndarray) -> np.ndarray:
        """FCI vector of the determinant with orbitals phi (M x (na+nb))."""
        pa, pb = phi[:, :self.na], phi[:, self.na:]
        v = np.zeros(self.dim, dtype=np.result_type(phi, np.float64))
        for i, (a, b) in enumerate(self.dets):
            da = np.linalg.det(pa[list(a), :]) if self.na else 1.0
            db = np.linalg.det(pb[list(b), :]) if self.nb else 1.0
            v[i] = da * db
        return v


def one_body_operator(ops: np.ndarray, mat: np.ndarray) -> np.ndarray:
    """sum_pq mat_pq E_pq."""
    return np.tensordot(mat, ops, axes=([0, 1], [0, 1]))


def hamiltonian(sec: Sector, h: np.ndarray, chol: np.ndarray, e_core: float = 0.0,
                ops: np.ndarray = None) -> np.ndarray:
    """Eq. 1 in the sector: sum h_ij E_ij + 1/2 sum V_ijkl sum_st c+_is c+_jt
    c_lt c_ks, using c+_i c+_j c_l c_k = E_ik E_jl - delta_jk E_il for the
    spin-summed operators (canonical anticommutation)."""
    if ops is None:
        ops = sec.one_body_ops()
    M = sec.M
    V = np.einsum("gik,gjl->ijkl", chol, chol)
    H = one_body_operator(ops, h) + e_core * np.eye(sec.dim)
    # 1/2 sum_ijkl V_ijkl E_ik E_jl
    W = np.tensordot(V, ops, axes=([1, 3], [0, 1]))        # (i, k, dim, dim) = sum_jl V_ijkl E_jl
    for i in range(M):
        for k in range(M):
            H += 0.5 * ops[i, k] @ W[i, k]
    # -1/2 sum_ijl V_ijjl E_il
    H -= 0.5 * one_body_operator(ops, np.einsum("ijjl->il", V))
    return H


def rho_ops(ops: np.ndarray, chol: np.ndarray) -> np.ndarray:
    """rho_g = sum_ik L^g_ik E_ik; v_g = i rho_g (Eq. 1)."""
    return np.stack([one_body_operator(ops, L) for L in chol])


def expm(a: np.ndarray) -> np.ndarray:
    return scipy.linalg.expm(a)


def ground_state(H: np.ndarray):
    w, v = np.linalg.eigh(H)
    return w[0], v[:, 0]
