"""Unfactorised spin-orbital CCD / CCSD equations.  TEST INFRASTRUCTURE.

What is computed (Sec. "Coupled cluster amplitude equations", Eq. eq:amp):

    E - E_HF  = <Phi_0| exp(-T) H_N exp(T) |Phi_0>
    R_l       = <Phi_l| exp(-T) H_N exp(T) |Phi_0>,  l = singles, doubles

with T = T1 + T2 as defined in the same section (T1 = sum t_i^a a+_a a_i,
T2 = 1/4 sum t_ij^ab a+_a a+_b a_j a_i) and H_N the normal-ordered form of
the Hamiltonian of Eq. ham2q.  CCD drops T1 and the singles projection.

Each diagram is one ``einsum`` line below (a library contraction used as a
step; no intermediates are shared between diagrams).  Counting the energy
equation, CCD has 11 diagrams and CCSD 48 (3 energy + 14 singles + 31
doubles), the numbers the paper's generator reports for these two methods
(Table "gener").  The signs and factors are pinned independently by the
brute-force projection in ``oracle.projection``.

Index convention of every integral written below: in <pq||rs>, p and q are
the indices of creation operators of H_N and r, s those of annihilation
operators.  External virtual indices and summed occupied indices therefore
sit in the bra, external occupied and summed virtual indices in the ket.
For real integrals this is immaterial; for complex Hermitian integrals it
fixes the orientation (e.g. the doubles driver is <ab||ij> and the singles
driver f_ai).

P(ij) X_ij = X_ij - X_ji and P(ab) X^ab = X^ab - X^ba.

The residual contains the diagonal Fock terms, so R = 0 at the solution and
the Jacobi step is t <- t + R / D with D_i^a = f_ii - f_aa and
D_ij^ab = f_ii + f_jj - f_aa - f_bb.
"""
from __future__ import annotations

import itertools

import numpy as np

from .integrals import Integrals


def _es(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


def P_ij(x):
    return x - x.swapaxes(0, 1)


def P_ab(x):
    return x - x.swapaxes(2, 3)


def P_ijab(x):
    return P_ab(P_ij(x))


class Fock:
    def __init__(self, f_oo, f_ov, f_vv):
        self.oo = f_oo
        self.ov = f_ov
        self.vv = f_vv
        self.vo = np.conj(f_ov.T)

    @classmethod
    def from_system(cls, s):
        return cls(s.f_oo, s.f_ov, s.f_vv)


def denominators(F: Fock):
    eo = np.real(np.diag(F.oo))
    ev = np.real(np.diag(F.vv))
    d1 = eo[:, None] - ev[None, :]
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return d1, d2


# ---------------------------------------------------------------- energy --
def energy_terms(F: Fock, V: Integrals, t1, t2):
    """The three energy diagrams (one when t1 is None)."""
    oovv = V.get("oovv")
    out = [0.25 * _es("ijab,ijab->", oovv, t2)]
    if t1 is not None:
        out.append(_es("ia,ia->", F.ov, t1))
        out.append(0.5 * _es("ijab,ia,jb->", oovv, t1, t1))
    return out


def energy(F, V, t1, t2):
    return complex(sum(energy_terms(F, V, t1, t2))) if np.iscomplexobj(t2) or np.iscomplexobj(V.get("oovv")) \
        else float(sum(energy_terms(F, V, t1, t2)))


# --------------------------------------------------------------- singles --
def singles_terms(F: Fock, V: Integrals, t1, t2):
    """The fourteen singles diagrams, each as an [i][a] array."""
    ovvo, ovvv, oovo, oovv = V.get("ovvo"), V.get("ovvv"), V.get("oovo"), V.get("oovv")
    return [
        F.vo.T.copy(),                                             # f_ai
        _es("ac,ic->ia", F.vv, t1),                                # f_ac t_i^c
        -_es("ki,ka->ia", F.oo, t1),                               # -f_ki t_k^a
        _es("kaci,kc->ia", ovvo, t1),                              # <ka||ci> t_k^c
        _es("kc,ikac->ia", F.ov, t2),                              # f_kc t_ik^ac
        0.5 * _es("kacd,kicd->ia", ovvv, t2),                      # 1/2 <ka||cd> t_ki^cd
        -0.5 * _es("klci,klca->ia", oovo, t2),                     # -1/2 <kl||ci> t_kl^ca
        -_es("kc,ic,ka->ia", F.ov, t1, t1),                        # -f_kc t_i^c t_k^a
        -_es("klci,kc,la->ia", oovo, t1, t1),                      # -<kl||ci> t_k^c t_l^a
        _es("kacd,kc,id->ia", ovvv, t1, t1),                       # <ka||cd> t_k^c t_i^d
        -_es("klcd,kc,id,la->ia", oovv, t1, t1, t1),               # -<kl||cd> t_k^c t_i^d t_l^a
        _es("klcd,kc,lida->ia", oovv, t1, t2),                     # <kl||cd> t_k^c t_li^da
        -0.5 * _es("klcd,kicd,la->ia", oovv, t2, t1),              # -1/2 <kl||cd> t_ki^cd t_l^a
        -0.5 * _es("klcd,klca,id->ia", oovv, t2, t1),              # -1/2 <kl||cd> t_kl^ca t_i^d
    ]


# --------------------------------------------------------------- doubles --
def doubles_terms_ccd(F: Fock, V: Integrals, t2):
    """The ten doubles diagrams that survive when T1 = 0 (a list)."""
    return list(_doubles_ccd(F, V, t2))


def _doubles_ccd(F: Fock, V: Integrals, t2):
    """The same diagrams, produced one at a time (a generator)."""
    oooo, vvvv, ovvo, oovv = V.get("oooo"), V.get("vvvv"), V.get("ovvo"), V.get("oovv")
    yield V.get("vvoo").transpose(2, 3, 0, 1).copy()                                # <ab||ij>
    yield P_ab(_es("bc,ijac->ijab", F.vv, t2))                                      # P(ab) f_bc t_ij^ac
    yield -P_ij(_es("kj,ikab->ijab", F.oo, t2))                                     # -P(ij) f_kj t_ik^ab
    yield 0.5 * _es("klij,klab->ijab", oooo, t2)                                    # 1/2 <kl||ij> t_kl^ab
    yield 0.5 * _es("abcd,ijcd->ijab", vvvv, t2)                                    # 1/2 <ab||cd> t_ij^cd
    yield P_ijab(_es("kbcj,ikac->ijab", ovvo, t2))                                  # P(ij)P(ab) <kb||cj> t_ik^ac
    yield 0.25 * _es("klcd,ijcd,klab->ijab", oovv, t2, t2)                          # 1/4 <kl||cd> t_ij^cd t_kl^ab
    yield P_ij(_es("klcd,ikac,jlbd->ijab", oovv, t2, t2))                           # P(ij) <kl||cd> t_ik^ac t_jl^bd
    yield -0.5 * P_ij(_es("klcd,ikdc,ljab->ijab", oovv, t2, t2))                    # -1/2 P(ij) <kl||cd> t_ik^dc t_lj^ab
    yield -0.5 * P_ab(_es("klcd,lkac,ijdb->ijab", oovv, t2, t2))                    # -1/2 P(ab) <kl||cd> t_lk^ac t_ij^db


def doubles_terms_t1(F: Fock, V: Integrals, t1, t2):
    """The twenty-one doubles diagrams that contain at least one t1 (a list)."""
    return list(_doubles_t1(F, V, t1, t2))


def _doubles_t1(F: Fock, V: Integrals, t1, t2):
    """The same diagrams, produced one at a time (a generator)."""
    oooo, vvvv, oovv = V.get("oooo"), V.get("vvvv"), V.get("oovv")
    ovvv, ooov, oovo = V.get("ovvv"), V.get("ooov"), V.get("oovo")
    yield P_ij(_es("abcj,ic->ijab", V.get("vvvo"), t1))                             # P(ij) <ab||cj> t_i^c
    yield -P_ab(_es("kbij,ka->ijab", V.get("ovoo"), t1))                            # -P(ab) <kb||ij> t_k^a
    yield 0.5 * P_ab(_es("klij,ka,lb->ijab", oooo, t1, t1))                         # 1/2 P(ab) <kl||ij> t_k^a t_l^b
    # 1/2 P(ij) <ab||cd> t_i^c t_j^d, with t_i^c t_j^d formed first: contracting
    # vvvv with one t1 at a time would transpose vvvv into a temporary as large
    yield 0.5 * P_ij(_es("abcd,ijcd->ijab", vvvv, _es("ic,jd->ijcd", t1, t1)))
    yield -P_ijab(_es("kbic,ka,jc->ijab", V.get("ovov"), t1, t1))                   # -P(ij)P(ab) <kb||ic> t_k^a t_j^c
    yield P_ab(_es("kc,ka,ijbc->ijab", F.ov, t1, t2))                               # P(ab) f_kc t_k^a t_ij^bc
    yield P_ij(_es("kc,ic,jkab->ijab", F.ov, t1, t2))                               # P(ij) f_kc t_i^c t_jk^ab
    yield -P_ij(_es("klci,kc,ljab->ijab", oovo, t1, t2))                            # -P(ij) <kl||ci> t_k^c t_lj^ab
    yield P_ab(_es("kacd,kc,ijdb->ijab", ovvv, t1, t2))                             # P(ab) <ka||cd> t_k^c t_ij^db
    yield P_ijab(_es("akdc,id,jkbc->ijab", V.get("vovv"), t1, t2))                  # P(ij)P(ab) <ak||dc> t_i^d t_jk^bc
    yield P_ijab(_es("klic,la,jkbc->ijab", ooov, t1, t2))                           # P(ij)P(ab) <kl||ic> t_l^a t_jk^bc
    yield 0.5 * P_ij(_es("klcj,ic,klab->ijab", oovo, t1, t2))                       # 1/2 P(ij) <kl||cj> t_i^c t_kl^ab
    yield -0.5 * P_ab(_es("kbcd,ka,ijcd->ijab", ovvv, t1, t2))                      # -1/2 P(ab) <kb||cd> t_k^a t_ij^cd
    yield -0.5 * P_ijab(_es("kbcd,ic,ka,jd->ijab", ovvv, t1, t1, t1))               # -1/2 P(ij)P(ab) <kb||cd> t_i^c t_k^a t_j^d
    yield 0.5 * P_ijab(_es("klcj,ic,ka,lb->ijab", oovo, t1, t1, t1))                # 1/2 P(ij)P(ab) <kl||cj> t_i^c t_k^a t_l^b
    yield -P_ij(_es("klcd,kc,id,ljab->ijab", oovv, t1, t1, t2))                     # -P(ij) <kl||cd> t_k^c t_i^d t_lj^ab
    yield -P_ab(_es("klcd,kc,la,ijdb->ijab", oovv, t1, t1, t2))                     # -P(ab) <kl||cd> t_k^c t_l^a t_ij^db
    yield 0.25 * P_ij(_es("klcd,ic,jd,klab->ijab", oovv, t1, t1, t2))               # 1/4 P(ij) <kl||cd> t_i^c t_j^d t_kl^ab
    yield 0.25 * P_ab(_es("klcd,ka,lb,ijcd->ijab", oovv, t1, t1, t2))               # 1/4 P(ab) <kl||cd> t_k^a t_l^b t_ij^cd
    yield P_ijab(_es("klcd,ic,lb,kjad->ijab", oovv, t1, t1, t2))                    # P(ij)P(ab) <kl||cd> t_i^c t_l^b t_kj^ad
    yield 0.25 * P_ijab(_es("klcd,ic,ka,jd,lb->ijab", oovv, t1, t1, t1, t1))        # 1/4 P(ij)P(ab) <kl||cd> t_i^c t_k^a t_j^d t_l^b


def _sum(terms):
    """Sum of the terms in their order (a list or a generator: each term of
    a generator is added before the next one is formed)."""
    it = iter(terms)
    acc = next(it).copy()
    for x in it:
        acc += x
    return acc


def residual(F: Fock, V: Integrals, t1, t2):
    """(R1, R2) for CCSD, or (None, R2) for CCD when t1 is None.  The doubles
    diagrams are summed as they are formed, in the order listed."""
    if t1 is None:
        return None, _sum(_doubles_ccd(F, V, t2))
    r2 = _sum(itertools.chain(_doubles_ccd(F, V, t2), _doubles_t1(F, V, t1, t2)))
    return _sum(singles_terms(F, V, t1, t2)), r2


def diagram_count(method: str) -> int:
    """Number of distinct diagrams listed above (energy equation included)."""
    o, v = 1, 1
    z1, z2 = np.zeros((o, v)), np.zeros((o, o, v, v))
    F = Fock(np.zeros((o, o)), np.zeros((o, v)), np.zeros((v, v)))
    V = Integrals({b: np.zeros(tuple(o if c == "o" else v for c in b))
                   for b in ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")}, o, v)
    if method == "ccd":
        return 1 + len(doubles_terms_ccd(F, V, z2))
    if method == "ccsd":
        return (len(energy_terms(F, V, z1, z2)) + len(singles_terms(F, V, z1, z2))
                + len(doubles_terms_ccd(F, V, z2)) + len(doubles_terms_t1(F, V, z1, z2)))
    raise ValueError(method)


def dressed_diagonals(F: Fock, V: Integrals, t1, t2):
    """Diagonals of the T-dressed one-body intermediates.

    F~_ae = f_ae - 1/2 f_me t_m^a + t_m^f <ma||fe> - 1/2 taut_mn^af <mn||ef>
    F~_mi = f_mi + 1/2 f_me t_i^e + t_n^e <mn||ie> + 1/2 taut_in^ef <mn||ef>
    F~_me = f_me + t_n^f <mn||ef>,   taut = t2 + 1/2 (t1 t1 - t1 t1)
    and the operators that multiply t2 in the doubles residual,
    Fv = F~_ae - 1/2 t_m^b F~_me (at a = e = b), Fo = F~_mi + 1/2 F~_me t_i^e (at m = i).
    Returned: (diag F~_oo, diag F~_vv, diag Fo, diag Fv); t1 None means CCD.
    Only diagonal elements are formed (einsum over the repeated index).
    """
    oovv = V.get("oovv")
    taut = t2
    if t1 is not None:
        x = _es("ia,jb->ijab", t1, t1)
        taut = t2 + 0.5 * (x - x.transpose(0, 1, 3, 2))
    fv = np.diag(F.vv).copy() - 0.5 * _es("mnaf,mnaf->a", taut, oovv)
    fo = np.diag(F.oo).copy() + 0.5 * _es("inef,inef->i", oovv, taut)
    if t1 is None:
        return fo, fv, fo.copy(), fv.copy()
    fv += -0.5 * _es("ma,ma->a", F.ov, t1) + _es("mafa,mf->a", V.get("ovvv"), t1)
    fo += 0.5 * _es("ie,ie->i", F.ov, t1) + _es("inie,ne->i", V.get("ooov"), t1)
    fme = F.ov + _es("mnef,nf->me", oovv, t1)
    return fo, fv, fo + 0.5 * _es("ie,ie->i", fme, t1), fv - 0.5 * _es("mb,mb->b", t1, fme)


def residual_norm(r1, r2):
    """Frobenius norm over every stored element of R1 and R2."""
    s = float(np.sum(np.abs(r2) ** 2))
    if r1 is not None:
        s += float(np.sum(np.abs(r1) ** 2))
    return s ** 0.5


def jacobi(F: Fock, V: Integrals, method: str = "ccsd", tol: float = 1e-8, max_iter: int = 200,
           t1=None, t2=None, callback=None, level_shift: float = 0.0, dressed: bool = False):
    """Jacobi iteration t <- t + R(t)/(D - s) from t = 0 (or the given guess).

    s >= 0 is a level shift (s = 0: the plain denominator update).  With
    ``dressed`` the denominators are rebuilt every iteration from the
    diagonals of the dressed one-body operators (``dressed_diagonals``):
    D_ij^ab = Fo_i + Fo_j - Fv_a - Fv_b, D_i^a = F~_ii - F~_aa.
    Iteration n evaluates R(t_n), records ||R(t_n)|| and E(t_n), stops if
    ||R(t_n)|| < tol and otherwise updates.  Returns a dict with the final
    amplitudes and the per-iteration history; E(t_1) is the MP2 energy when
    the start is t = 0.
    """
    o, v = F.oo.shape[0], F.vv.shape[0]
    dt = np.result_type(F.oo.dtype, V.get("oovv").dtype)
    d1, d2 = denominators(F)
    d1 = d1 - level_shift
    d2 = d2 - level_shift
    if t2 is None:
        t2 = np.zeros((o, o, v, v), dtype=dt)
    if method == "ccsd" and t1 is None:
        t1 = np.zeros((o, v), dtype=dt)
    if method == "ccd":
        t1 = None
    hist_e, hist_r = [], []
    converged = False
    for it in range(max_iter):
        r1, r2 = residual(F, V, t1, t2)
        rn = residual_norm(r1, r2)
        e = energy(F, V, t1, t2)
        hist_e.append(e)
        hist_r.append(rn)
        if callback is not None:
            callback(it, e, rn)
        if rn < tol:
            converged = True
            break
        if not np.isfinite(rn):
            break
        if dressed:
            fo1, fv1, fo2, fv2 = dressed_diagonals(F, V, t1, t2)
            e1 = np.real(fo1)[:, None] - np.real(fv1)[None, :] - level_shift
            e2 = (np.real(fo2)[:, None, None, None] + np.real(fo2)[None, :, None, None]) - (
                np.real(fv2)[None, None, :, None] + np.real(fv2)[None, None, None, :]) - level_shift
        else:
            e1, e2 = d1, d2
        t2 = t2 + r2 / e2
        if t1 is not None:
            t1 = t1 + r1 / e1
    return {"t1": t1, "t2": t2, "energy": hist_e[-1], "rnorm": hist_r[-1], "hist_e": hist_e,
            "hist_r": hist_r, "iters": len(hist_e), "converged": converged}
