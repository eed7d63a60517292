"""Brute-force projection of exp(-T) H_N exp(T).  TEST INFRASTRUCTURE.

The plain definition of the coupled-cluster energy and residual
(Eq. eq:amp) evaluated in the space of all N-electron determinants of a
tiny system, with no diagrams at all:

* Orbitals 0..o-1 are occupied in the reference |Phi_0>; N = o.
* E_pq = a+_p a_q is built as a dense matrix on the determinant basis, with
  the usual fermion sign (-1)^(number of occupied orbitals below the index).
* H = sum h_pq E_pq + 1/4 sum <pq||rs> a+_p a+_q a_s a_r  (Eq. ham2q) with
  a+_p a+_q a_s a_r = E_pr E_qs - delta_qr E_ps, and the one-body part
  recovered from the Fock operator, h_pq = f_pq - sum_k <pk||qk>.
* T1 = sum t_i^a E_ai and T2 = 1/4 sum t_ij^ab a+_a a+_b a_j a_i
  = 1/4 sum t_ij^ab E_ai E_bj (cluster operators of the CC section).
* Hbar = exp(-T) H exp(T); exp is the terminating power series (T is
  nilpotent on the N-electron space).
* `cluster_general` / `evaluate_general` extend the same construction to
  cluster operators and projections of any excitation level:
  T_m = sum over i1<..<im, a1<..<am of t_{i1..im}^{a1..am} E_{a1 i1}..E_{am im},
  |Phi_{i1..im}^{a1..am}> = E_{a1 i1}..E_{am im} |Phi_0>.
* E - E_HF = <Phi_0|Hbar|Phi_0> - <Phi_0|H|Phi_0>;
  R_i^a = <Phi_i^a|Hbar|Phi_0>, |Phi_i^a> = E_ai |Phi_0>;
  R_ij^ab = <Phi_ij^ab|Hbar|Phi_0>, |Phi_ij^ab> = a+_a a+_b a_j a_i |Phi_0>.

Intended for o + v <= 10.
"""
from __future__ import annotations

import itertools

import numpy as np


def determinants(n: int, N: int):
    dets = [sum(1 << p for p in occ) for occ in itertools.combinations(range(n), N)]
    return dets, {d: k for k, d in enumerate(dets)}


def _apply_E(p: int, q: int, det: int):
    """a+_p a_q |det> -> (sign, new_det) or None."""
    if not (det >> q) & 1:
        return None
    s = bin(det & ((1 << q) - 1)).count("1")
    d1 = det & ~(1 << q)
    if (d1 >> p) & 1:
        return None
    s += bin(d1 & ((1 << p) - 1)).count("1")
    return (-1) ** s, d1 | (1 << p)


def excitation_matrices(n: int, N: int):
    dets, index = determinants(n, N)
    dim = len(dets)
    E = np.zeros((n, n, dim, dim))
    for p in range(n):
        for q in range(n):
            for k, d in enumerate(dets):
                r = _apply_E(p, q, d)
                if r is not None:
                    E[p, q, index[r[1]], k] = r[0]
    return E, dets, index


def hamiltonian(E, fock, g, o):
    """Determinant-space H from the Fock matrix and <pq||rs> (full tensors)."""
    n = fock.shape[0]
    occ = np.arange(o)
    h = fock - np.einsum("pkqk->pq", g[:, occ][:, :, :, occ])
    dim = E.shape[2]
    H = np.zeros((dim, dim), dtype=np.result_type(fock.dtype, g.dtype))
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0:
                H += h[p, q] * E[p, q]
    for p in range(n):
        for r in range(n):
            M = np.tensordot(g[p, :, r, :], E, axes=([0, 1], [0, 1]))  # sum_qs g_pqrs E_qs
            H += 0.25 * (E[p, r] @ M)
    # - 1/4 sum_pqs g_pqqs E_ps
    G = np.einsum("pqqs->ps", g)
    H -= 0.25 * np.tensordot(G, E, axes=([0, 1], [0, 1]))
    return H


def _expm_nilpotent(A):
    out = np.eye(A.shape[0], dtype=A.dtype)
    term = out.copy()
    for k in range(1, A.shape[0] + 1):
        term = term @ A / k
        if not np.any(term):
            break
        out = out + term
    return out


class Projector:
    """Precomputes E_pq and H for one tiny system."""

    def __init__(self, fock, g, o):
        n = fock.shape[0]
        self.o, self.v, self.n = o, n - o, n
        self.E, self.dets, self.index = excitation_matrices(n, o)
        self.H = hamiltonian(self.E, fock, g, o)
        self.ref = self.index[(1 << o) - 1]
        self.e_hf = self.H[self.ref, self.ref]

    def cluster(self, t1, t2):
        o, E = self.o, self.E
        T = np.zeros(self.H.shape, dtype=np.result_type(self.H.dtype, t2.dtype))
        vir = range(o, self.n)
        if t1 is not None:
            for i in range(o):
                for a in vir:
                    T += t1[i, a - o] * E[a, i]
        for i in range(o):
            for j in range(o):
                for a in vir:
                    for b in vir:
                        c = t2[i, j, a - o, b - o]
                        if c != 0:
                            T += 0.25 * c * (E[a, i] @ E[b, j])
        return T

    def excitation(self, holes, parts):
        """E_{a1 i1} ... E_{am im} as a matrix (|Phi_{i1..im}^{a1..am}> = this applied to |Phi_0>)."""
        M = np.eye(self.H.shape[0])
        for i, a in zip(holes, parts):
            M = M @ self.E[a + self.o, i]
        return M

    def cluster_general(self, amps):
        """T = sum_m T_m, T_m = (1/m!)^2 sum t_{i1..im}^{a1..am} a+_a1..a+_am a_im..a_i1
        = sum over i1<..<im, a1<..<am of t E_{a1 i1}..E_{am im}; amps maps m to an
        antisymmetric tensor t[i1..im, a1..am] (any level, generalising T1 and T2)."""
        o, v = self.o, self.v
        dt = np.result_type(self.H.dtype, *[a.dtype for a in amps.values() if a is not None])
        T = np.zeros(self.H.shape, dtype=dt)
        for m, t in amps.items():
            if t is None:
                continue
            for holes in itertools.combinations(range(o), m):
                for parts in itertools.combinations(range(v), m):
                    c = t[holes + parts]
                    if c != 0:
                        T += c * self.excitation(holes, parts)
        return T

    def evaluate_general(self, amps, levels):
        """(E - E_HF, {k: R_k[i1..ik, a1..ak]}) with R_k = <Phi_k| exp(-T) H exp(T) |Phi_0>
        for the projection levels k in `levels` (Eq. eq:amp), T from cluster_general."""
        T = self.cluster_general(amps)
        Hb = _expm_nilpotent(-T) @ self.H @ _expm_nilpotent(T)
        col = Hb[:, self.ref]
        phi0 = np.zeros(Hb.shape[0])
        phi0[self.ref] = 1.0
        out = {}
        o, v = self.o, self.v
        for k in levels:
            R = np.zeros((o,) * k + (v,) * k, dtype=col.dtype)
            for holes in itertools.product(range(o), repeat=k):
                if len(set(holes)) < k:
                    continue
                for parts in itertools.product(range(v), repeat=k):
                    if len(set(parts)) < k:
                        continue
                    R[holes + parts] = (self.excitation(holes, parts) @ phi0) @ col
            out[k] = R
        return col[self.ref] - self.e_hf, out

    def hbar(self, t1, t2):
        T = self.cluster(t1, t2)
        return _expm_nilpotent(-T) @ self.H @ _expm_nilpotent(T)

    def evaluate(self, t1, t2):
        """(E - E_HF, R1[i][a] or None, R2[i][j][a][b])."""
        o, v, E = self.o, self.v, self.E
        Hb = self.hbar(t1, t2)
        col = Hb[:, self.ref]
        phi0 = np.zeros(Hb.shape[0])
        phi0[self.ref] = 1.0
        e = col[self.ref] - self.e_hf
        R1 = None
        if t1 is not None:
            R1 = np.zeros((o, v), dtype=col.dtype)
            for i in range(o):
                for a in range(v):
                    R1[i, a] = (E[a + o, i] @ phi0) @ col
        R2 = np.zeros((o, o, v, v), dtype=col.dtype)
        for i in range(o):
            for j in range(o):
                for a in range(v):
                    for b in range(v):
                        bra = E[a + o, i] @ (E[b + o, j] @ phi0)
                        R2[i, j, a, b] = bra @ col
        return e, R1, R2
