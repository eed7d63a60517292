"""Pins of ``oracle.cc.denominators`` and ``oracle.cc.dressed_diagonals``
against the projection-pinned diagrams (CPU only).

Neither function is checked by retyping its formula.  Both are tied to the
unfactorised singles and doubles diagrams of ``oracle.cc``, which
``test_oracle.test_equations_match_projection`` pins to the brute-force
projection of Eq. eq:amp:

* Bare denominators.  With a diagonal Fock operator the two Fock diagrams of
  the doubles equation add up to -D_ij^ab t_ij^ab and the two of the singles
  equation to -D_i^a t_i^a.  D is read off from these diagrams element by
  element.
* Dressed denominators.  A dressed one-body operator is the matrix that
  multiplies the amplitudes in a diagram where it leaves one amplitude's
  external indices in place.
  * In the doubles equation, the selected diagrams must have the form
    P(ab) t_ij^ae Fv_be - P(ij) t_im^ab Fo_mj.  Fv and Fo are found from the
    diagrams by least squares, where the residual must vanish.  They are
    unique up to Fv + cI, Fo + cI, which leaves
    D~ij^ab = Fo_ii + Fo_jj - Fv_aa - Fv_bb unchanged.
  * In the singles equation, with o = v and an invertible t1, the selected
    diagrams give F~_ae from t_i^e F~_ae and F~_mi from -t_m^a F~_mi by a
    solve.  Two singles diagrams, -f_kc t_i^c t_k^a and the t1^3 term, have
    both forms; they are split evenly between the two operators (a reading
    of the factorised singles equation).
  * ``dressed_diagonals`` must return exactly these diagonals.
* One-token mutations of either function fail these checks.  The mutants are
  built from the function's own source on the CPU.
"""
import inspect

import numpy as np
import pytest

import oracle.cc as occ
from ccinputs.synth import make_system
from oracle.cc import Fock, doubles_terms_ccd, doubles_terms_t1, singles_terms
from oracle.integrals import Integrals


def _case(o, v, cplx, seed, diagonal_fock=False):
    """Random amplitudes and (unless diagonal_fock) a random Hermitian Fock
    operator with nonzero occupied-virtual block."""
    s = make_system(o, v, 300 + seed, is_complex=cplx, sigma=0.1)
    rng = np.random.default_rng(seed)
    n = o + v
    F = s.fock()
    if not diagonal_fock:
        X = rng.normal(size=(n, n)) * 0.1
        if cplx:
            X = X + 1j * rng.normal(size=(n, n)) * 0.1
        F = F + X + X.conj().T
    t1 = rng.normal(size=(o, v)) * 0.3
    t2 = rng.normal(size=(o, o, v, v)) * 0.3
    if cplx:
        t1 = t1 + 1j * rng.normal(size=(o, v)) * 0.3
        t2 = t2 + 1j * rng.normal(size=(o, o, v, v)) * 0.3
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return Fock(F[:o, :o], F[:o, o:], F[o:, o:]), Integrals.from_system(s), t1, t2


# ------------------------------------------------------ bare denominators --
def check_denominators(fn, o=4, v=6, cplx=False, seed=1):
    F, V, t1, t2 = _case(o, v, cplx, seed, diagonal_fock=True)
    d1, d2 = fn(F)
    # singles: f_ac t_i^c - f_ki t_k^a = -D_i^a t_i^a  (diagrams 1 and 2)
    s = singles_terms(F, V, t1, t2)
    d1_diag = -(s[1] + s[2]) / t1
    # doubles: P(ab) f_bc t_ij^ac - P(ij) f_kj t_ik^ab = -D_ij^ab t_ij^ab
    d = doubles_terms_ccd(F, V, t2)
    fock2 = d[1] + d[2]
    off = np.ones((o, o, v, v), bool)
    off[np.arange(o), np.arange(o)] = False
    off[:, :, np.arange(v), np.arange(v)] = False
    err1 = np.abs(d1 - d1_diag).max()
    err2 = np.abs(d2[off] - (-fock2[off] / t2[off])).max()
    # elements with i = j or a = b (t2 is zero there): D is the sum of the
    # two singles denominators, each pinned above
    err3 = np.abs(d2 - (d1_diag[:, None, :, None] + d1_diag[None, :, None, :])).max()
    return max(err1, err2, err3)


@pytest.mark.parametrize("cplx", [False, True])
def test_denominators_from_fock_diagrams(cplx):
    assert check_denominators(occ.denominators, cplx=cplx) < 1e-13


# --------------------------------------------------- dressed denominators --
def _doubles_one_body_map(t2):
    """Columns: the image of each unit Fv_be (then each unit Fo_mj) under
    X -> P(ab) t_ij^ae Fv_be - P(ij) t_im^ab Fo_mj."""
    o, v = t2.shape[0], t2.shape[2]
    cols = []
    for b in range(v):
        for e in range(v):
            y = np.zeros_like(t2)
            y[:, :, :, b] += t2[:, :, :, e]          # t_ij^ae Fv_be
            y[:, :, b, :] -= t2[:, :, :, e]          # - t_ij^be Fv_ae  (a <-> b)
            cols.append(y.ravel())
    for m in range(o):
        for j in range(o):
            y = np.zeros_like(t2)
            y[:, j] -= t2[:, m]                      # - t_im^ab Fo_mj
            y[j, :] += t2[:, m]                      # + t_jm^ab Fo_mi  (i <-> j)
            cols.append(y.ravel())
    return np.stack(cols, axis=1)


def dressed_doubles_from_diagrams(F, V, t1, t2):
    """Fv, Fo (up to Fv + cI, Fo + cI) and the least-squares misfit from the
    doubles diagrams that keep one amplitude's external pair in place."""
    d0 = doubles_terms_ccd(F, V, t2)
    d1 = doubles_terms_t1(F, V, t1, t2)
    # Fv side: f_bc, the t2-t2 term with t_ij^db, and the t1 terms
    # f_kc t_k^a t_ij^bc, <ka||cd> t_k^c t_ij^db, <kl||cd> t_k^c t_l^a t_ij^db
    # Fo side: f_kj, the t2-t2 term with t_lj^ab, and the t1 terms
    # f_kc t_i^c t_jk^ab, <kl||ci> t_k^c t_lj^ab, <kl||cd> t_k^c t_i^d t_lj^ab
    S = d0[1] + d0[9] + d1[5] + d1[8] + d1[16] + d0[2] + d0[8] + d1[6] + d1[7] + d1[15]
    o, v = t2.shape[0], t2.shape[2]
    A = _doubles_one_body_map(t2)
    x, *_ = np.linalg.lstsq(A, S.ravel(), rcond=None)
    misfit = np.abs(A @ x - S.ravel()).max()
    Fv = x[: v * v].reshape(v, v)
    Fo = x[v * v:].reshape(o, o)
    return Fv, Fo, misfit


def dressed_singles_from_diagrams(F, V, t1, t2):
    """F~_ae and F~_mi from the singles diagrams (o = v, t1 invertible)."""
    s = singles_terms(F, V, t1, t2)
    shared = 0.5 * (s[7] + s[10])
    # t_i^e F~_ae: f_ac t_i^c, <ka||cd> t_k^c t_i^d, <kl||cd> t_kl^ca t_i^d
    SX = s[1] + s[9] + s[13] + shared
    # -t_m^a F~_mi: f_ki t_k^a, <kl||ci> t_k^c t_l^a, <kl||cd> t_ki^cd t_l^a
    SY = s[2] + s[8] + s[12] + shared
    X = np.linalg.solve(t1, SX).T        # SX = t1 X^T
    Y = -np.linalg.solve(t1.T, SY.T)     # SY = -Y^T t1
    return X, Y


def check_dressed(fn, cplx, seed, o=4, v=4, method="ccsd"):
    """Largest deviation of fn's dressed denominators from those read off the
    diagrams (doubles: D~ij^ab; singles: F~_ii - F~_aa)."""
    F, V, t1, t2 = _case(o, v, cplx, seed)
    if method == "ccd":
        t1 = np.zeros((o, v), dtype=t2.dtype)
    Fv, Fo, misfit = dressed_doubles_from_diagrams(F, V, t1, t2)
    assert misfit < 1e-12, "the selected doubles diagrams are not of one-body form"
    fo1, fv1, fo2, fv2 = fn(F, V, None if method == "ccd" else t1, t2)
    fo, fvv = np.diag(Fo), np.diag(Fv)
    D_ref = fo[:, None, None, None] + fo[None, :, None, None] - fvv[None, None, :, None] - fvv[None, None, None, :]
    D = fo2[:, None, None, None] + fo2[None, :, None, None] - fv2[None, None, :, None] - fv2[None, None, None, :]
    err = np.abs(D - D_ref).max()
    if method == "ccsd":
        X, Y = dressed_singles_from_diagrams(F, V, t1, t2)
        err = max(err, np.abs(fv1 - np.diag(X)).max(), np.abs(fo1 - np.diag(Y)).max())
    return err


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("seed", [2, 3])
def test_dressed_diagonals_from_diagrams(cplx, seed):
    assert check_dressed(occ.dressed_diagonals, cplx, seed) < 1e-12


def test_dressed_diagonals_ccd():
    # CCD: t1 = 0, the two operators reduce to the f and t2-t2 parts
    assert check_dressed(occ.dressed_diagonals, False, 4, o=4, v=5, method="ccd") < 1e-12


@pytest.mark.parametrize("ov", [(4, 4), (4, 5)])
def test_doubles_map_has_only_the_constant_gauge(ov):
    """At the sizes used above the least-squares problem fixes Fv and Fo up
    to Fv + cI, Fo + cI (rank = v^2 + o^2 - 1), so D~ is determined by the
    diagrams.  (With o = 3 the hole side has more null directions.)"""
    _, _, _, t2 = _case(*ov, False, 2)
    A = _doubles_one_body_map(t2)
    assert np.linalg.matrix_rank(A) == A.shape[1] - 1


# ------------------------------------------------------ planted mistakes --
_DRESSED_MUTANTS = [
    ("taut = t2 + 0.5 * (x", "taut = t2 + 1.0 * (x"),
    ('- 0.5 * _es("mnaf,mnaf->a"', '- 1.0 * _es("mnaf,mnaf->a"'),
    ('+ 0.5 * _es("inef,inef->i"', '- 0.5 * _es("inef,inef->i"'),
    ('-0.5 * _es("ma,ma->a"', '+0.5 * _es("ma,ma->a"'),
    ('0.5 * _es("ie,ie->i", F.ov, t1)', '1.0 * _es("ie,ie->i", F.ov, t1)'),
    ('+ _es("mafa,mf->a"', '- _es("mafa,mf->a"'),
    ('+ _es("inie,ne->i"', '- _es("inie,ne->i"'),
    ('F.ov + _es("mnef,nf->me"', 'F.ov - _es("mnef,nf->me"'),
    ('fo + 0.5 * _es("ie,ie->i", fme', 'fo + 1.0 * _es("ie,ie->i", fme'),
    ('fv - 0.5 * _es("mb,mb->b"', 'fv + 0.5 * _es("mb,mb->b"'),
    ('(x - x.transpose(0, 1, 3, 2))', '(x + x.transpose(0, 1, 3, 2))'),
]

_DENOM_MUTANTS = [
    ("d1 = eo[:, None] - ev[None, :]", "d1 = ev[None, :] - eo[:, None]"),
    ("+ eo[None, :, None, None]", "- eo[None, :, None, None]"),
    ("- ev[None, None, None, :]", "+ ev[None, None, None, :]"),
    ("ev = np.real(np.diag(F.vv))", "ev = np.real(np.diag(F.oo))[:1]"),
]


def _mutant(fn, old, new):
    src = inspect.getsource(fn)
    assert src.count(old) == 1, old
    ns = dict(vars(occ))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns[fn.__name__]


@pytest.mark.parametrize("old,new", _DRESSED_MUTANTS)
def test_planted_mistake_in_dressed_diagonals_is_caught(old, new):
    bad = _mutant(occ.dressed_diagonals, old, new)
    errs = []
    for cplx, seed in ((False, 2), (True, 3)):
        try:
            errs.append(check_dressed(bad, cplx, seed))
        except (ValueError, AssertionError):
            errs.append(np.inf)
    assert max(errs) > 1e-6


@pytest.mark.parametrize("old,new", _DENOM_MUTANTS)
def test_planted_mistake_in_denominators_is_caught(old, new):
    bad = _mutant(occ.denominators, old, new)
    try:
        err = check_denominators(bad)
    except (ValueError, IndexError):
        err = np.inf
    assert err > 1e-6
