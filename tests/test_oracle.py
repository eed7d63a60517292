"""Pins of the CPU oracle against things other than itself (CPU only).

* the input generator's symmetries;
* Slater-Condon closed forms for the brute-force determinant Hamiltonian;
* the unfactorised 48-/11-diagram equations against the brute-force
  projection of Eq. eq:amp at random amplitudes (real and complex, with
  off-diagonal Fock operators);
* the diagram counts 11 (CCD) and 48 (CCSD) of the paper's Table "gener";
* first iteration = MP2 (closed form);
* linear CCD at iteration 2 = MP2 + MP3 (textbook closed form);
* CCSD = FCI for two electrons;
* invariance of the converged energy under occupied-occupied and
  virtual-virtual orbital rotations.
"""
import numpy as np
import pytest

from ccinputs.synth import batch_shapes, integral_block, make_system
from oracle.cc import Fock, diagram_count, doubles_terms_ccd, energy, jacobi, residual
from oracle.integrals import Integrals
from oracle.projection import Projector, determinants


def _random_case(o, v, cplx, seed=1, sigma=0.1):
    s = make_system(o, v, 100 + seed, is_complex=cplx, sigma=sigma)
    rng = np.random.default_rng(seed)
    n = o + v
    F = s.fock()
    X = rng.normal(size=(n, n)) * 0.1
    if cplx:
        X = X + 1j * rng.normal(size=(n, n)) * 0.1
    F = F + X + X.conj().T
    t1 = rng.normal(size=(o, v)) * 0.1
    t2 = rng.normal(size=(o, o, v, v)) * 0.1
    if cplx:
        t1 = t1 + 1j * rng.normal(size=(o, v)) * 0.1
        t2 = t2 + 1j * rng.normal(size=(o, o, v, v)) * 0.1
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return s, F, t1, t2


# ------------------------------------------------------------- generator --
@pytest.mark.parametrize("cplx", [False, True])
def test_generator_symmetries(cplx):
    s = make_system(3, 4, 11, is_complex=cplx)
    g = s.full_integrals()
    n = 7
    assert np.array_equal(g, -g.transpose(1, 0, 2, 3))
    assert np.array_equal(g, -g.transpose(0, 1, 3, 2))
    assert np.array_equal(g, np.conj(g.transpose(2, 3, 0, 1)))
    for b in ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv"):
        sl = tuple(slice(0, 3) if c == "o" else slice(3, n) for c in b)
        assert np.array_equal(s.block(b), g[sl])
    # deterministic
    assert np.array_equal(integral_block(3, 4, "ovvv", 11, cplx), s.block("ovvv"))


def test_generator_moments():
    s = make_system(6, 30, 5)
    canon = s.block("vvvv").reshape(900, 900)  # [(ab)][(cd)]
    mask = np.zeros((30, 30), bool)
    mask[np.triu_indices(30, 1)] = True
    G = canon[mask.ravel()][:, mask.ravel()]
    vals = G[np.triu_indices(G.shape[0])]
    assert abs(vals.mean()) < 3 * 0.01 / np.sqrt(vals.size)
    assert abs(vals.std() / 0.01 - 1) < 0.01
    eo, ev = np.diag(s.f_oo), np.diag(s.f_vv)
    assert eo.min() >= -2 and eo.max() <= -0.5 and np.all(np.diff(eo) >= 0)
    assert ev.min() >= 0.5 and ev.max() <= 3 and np.all(np.diff(ev) >= 0)


def test_batch_shapes_ranges():
    sh = batch_shapes(64)
    assert len(sh) == 64
    assert all(4 <= o <= 16 and 20 <= v <= 60 for o, v, _ in sh)
    assert len({s for _, _, s in sh}) == 64


@pytest.mark.parametrize("cplx", [False, True])
def test_integral_orientations(cplx):
    o, v = 3, 4
    s = make_system(o, v, 12, is_complex=cplx)
    g = s.full_integrals()
    V = Integrals.from_system(s)
    for b in ["oooo", "ooov", "oovo", "ovoo", "vooo", "oovv", "vvoo", "ovov", "voov", "vovo", "ovvo",
              "ovvv", "vovv", "vvov", "vvvo", "vvvv"]:
        sl = tuple(slice(0, o) if c == "o" else slice(o, o + v) for c in b)
        assert np.array_equal(V.get(b), g[sl]), b


# ------------------------------------------------- brute-force Hamiltonian --
@pytest.mark.parametrize("cplx", [False, True])
def test_hamiltonian_slater_condon(cplx):
    o, v = 3, 3
    s, F, _, _ = _random_case(o, v, cplx, seed=3)
    g = s.full_integrals()
    P = Projector(F, g, o)
    n = o + v
    occ = np.arange(o)
    h = F - np.einsum("pkqk->pq", g[:, occ][:, :, :, occ])
    assert np.allclose(P.H, P.H.conj().T, atol=1e-14)
    dets, index = determinants(n, o)
    for k, d in enumerate(dets):
        orbs = [p for p in range(n) if (d >> p) & 1]
        diag = sum(h[p, p] for p in orbs) + 0.5 * sum(g[p, q, p, q] for p in orbs for q in orbs)
        assert abs(P.H[k, k] - diag) < 1e-13
    # E_HF = sum_i f_ii - 1/2 sum_ij <ij||ij>
    e_hf = np.trace(F[:o, :o]) - 0.5 * np.einsum("ijij->", g[:o, :o, :o, :o])
    assert abs(P.e_hf - e_hf) < 1e-13
    ref = P.ref
    phi0 = np.zeros(len(dets))
    phi0[ref] = 1
    for i in range(o):
        for a in range(o, n):
            bra = P.E[a, i] @ phi0
            assert abs(bra @ P.H[:, ref] - F[a, i]) < 1e-13  # <Phi_i^a|H|Phi_0> = f_ai
    for i in range(o):
        for j in range(o):
            for a in range(o, n):
                for b in range(o, n):
                    bra = P.E[a, i] @ (P.E[b, j] @ phi0)
                    assert abs(bra @ P.H[:, ref] - g[a, b, i, j]) < 1e-13  # = <ab||ij>


# ------------------------------------------- equations vs the definition --
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("ov", [(2, 3), (3, 4), (4, 4)])
def test_equations_match_projection(cplx, ov):
    o, v = ov
    s, F, t1, t2 = _random_case(o, v, cplx, seed=o + v)
    P = Projector(F, s.full_integrals(), o)
    V = Integrals.from_system(s)
    Fk = Fock(F[:o, :o], F[:o, o:], F[o:, o:])
    e_ref, r1_ref, r2_ref = P.evaluate(t1, t2)
    r1, r2 = residual(Fk, V, t1, t2)
    assert abs(energy(Fk, V, t1, t2) - e_ref) < 1e-12
    assert np.abs(r1 - r1_ref).max() < 1e-12
    assert np.abs(r2 - r2_ref).max() < 1e-12
    e_ref, _, r2_ref = P.evaluate(None, t2)
    _, r2 = residual(Fk, V, None, t2)
    assert abs(energy(Fk, V, None, t2) - e_ref) < 1e-12
    assert np.abs(r2 - r2_ref).max() < 1e-12


def test_diagram_counts_match_paper_table():
    # Table "gener": CCD 11 diagrams, CCSD 48 (energy equation included)
    assert diagram_count("ccd") == 11
    assert diagram_count("ccsd") == 48


def test_residual_antisymmetric():
    o, v = 3, 5
    s, F, t1, t2 = _random_case(o, v, False, seed=9)
    V = Integrals.from_system(s)
    _, r2 = residual(Fock(F[:o, :o], F[:o, o:], F[o:, o:]), V, t1, t2)
    assert np.abs(r2 + r2.transpose(1, 0, 2, 3)).max() < 1e-14
    assert np.abs(r2 + r2.transpose(0, 1, 3, 2)).max() < 1e-14


# ------------------------------------------------------------ closed forms --
def _orbital_energy_denominators(s):
    """D_ij^ab = e_i + e_j - e_a - e_b written out from the orbital energies
    of the diagonal Fock operator (independent of ``oracle.cc``)."""
    eo, ev = np.real(np.diag(s.f_oo)), np.real(np.diag(s.f_vv))
    o, v = len(eo), len(ev)
    D = np.empty((o, o, v, v))
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    D[i, j, a, b] = eo[i] + eo[j] - ev[a] - ev[b]
    return D


@pytest.mark.parametrize("method", ["ccd", "ccsd"])
@pytest.mark.parametrize("cplx", [False, True])
def test_first_iteration_is_mp2(method, cplx):
    o, v = 4, 9
    s = make_system(o, v, 21, is_complex=cplx)
    V, F = Integrals.from_system(s), Fock.from_system(s)
    res = jacobi(F, V, method, tol=0.0, max_iter=2)
    d2 = _orbital_energy_denominators(s)
    vvoo = V.get("vvoo").transpose(2, 3, 0, 1)
    e_mp2 = 0.25 * np.sum(np.abs(vvoo) ** 2 / d2)
    assert res["hist_e"][0] == 0
    assert abs(res["hist_e"][1] - e_mp2) < 1e-15 * max(1.0, abs(e_mp2)) * 10
    assert abs(np.imag(res["hist_e"][1])) < 1e-15


def test_linear_ccd_second_iteration_is_mp3():
    o, v = 4, 8
    s = make_system(o, v, 33, sigma=0.05)
    V, F = Integrals.from_system(s), Fock.from_system(s)
    D = _orbital_energy_denominators(s)
    g = V.get("oovv")  # <ij||ab>; real integrals: <ab||ij> = <ij||ab>

    def linear_residual(t2):  # driver + Fock + the three linear diagrams
        return sum(doubles_terms_ccd(F, V, t2)[:6])

    t = np.zeros((o, o, v, v))
    t = t + linear_residual(t) / D
    e2 = 0.25 * np.sum(g * t)
    t = t + linear_residual(t) / D
    e3 = 0.25 * np.sum(g * t)
    oooo, vvvv, ovvo = V.get("oooo"), V.get("vvvv"), V.get("ovvo")
    Dik = D  # D[i,k,a,c]
    mp2 = 0.25 * np.sum(g * g / D)
    pp = 0.125 * np.einsum("ijab,abcd,ijcd,ijab,ijcd->", g, vvvv, g, 1 / D, 1 / D)
    hh = 0.125 * np.einsum("ijab,klij,klab,ijab,klab->", g, oooo, g, 1 / D, 1 / D)
    ring = np.einsum("ijab,kbcj,ikac,ijab,ikac->", g, ovvo, g, 1 / D, 1 / Dik)
    assert abs(e2 - mp2) < 1e-15
    assert abs(e3 - (mp2 + pp + hh + ring)) < 1e-14


def test_two_electron_ccsd_equals_fci():
    o, v = 2, 5
    s = make_system(o, v, 44, sigma=0.3)
    V, F = Integrals.from_system(s), Fock.from_system(s)
    res = jacobi(F, V, "ccsd", tol=1e-13, max_iter=400)
    assert res["converged"]
    P = Projector(s.fock(), s.full_integrals(), o)
    w, U = np.linalg.eigh(P.H)
    k = int(np.argmax(np.abs(U[P.ref, :]) ** 2))  # root with the dominant reference weight
    assert abs(U[P.ref, k]) ** 2 > 0.5
    assert abs(res["energy"] - (w[k] - P.e_hf)) < 1e-11


@pytest.mark.parametrize("method", ["ccd", "ccsd"])
def test_orbital_rotation_invariance(method):
    o, v = 4, 8
    s = make_system(o, v, 55, sigma=0.05)
    g = s.full_integrals()
    F = s.fock()
    ref = jacobi(Fock.from_system(s), Integrals.from_system(s), method, tol=1e-12, max_iter=300)
    rng = np.random.default_rng(0)

    def small_rotation(k, eps):
        A = rng.normal(size=(k, k)) * eps
        A = A - A.T
        w, Q = np.linalg.eigh(1j * A)
        return np.real(Q @ np.diag(np.exp(-1j * w)) @ Q.conj().T)

    U = np.zeros((o + v, o + v))
    U[:o, :o] = small_rotation(o, 0.05)
    U[o:, o:] = small_rotation(v, 0.05)
    g2 = np.einsum("pqrs,pa,qb,rc,sd->abcd", g, U, U, U, U, optimize=True)
    F2 = U.T @ F @ U
    blocks = {b: g2[tuple(slice(0, o) if c == "o" else slice(o, o + v) for c in b)]
              for b in ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")}
    res = jacobi(Fock(F2[:o, :o], F2[:o, o:], F2[o:, o:]), Integrals(blocks, o, v), method,
                 tol=1e-12, max_iter=300)
    assert ref["converged"] and res["converged"]
    assert abs(res["energy"] - ref["energy"]) < 1e-10


def test_stored_c1_trajectory_is_the_oracles():
    """tests/golden/c1_ccd_trajectory.json equals a fresh oracle run."""
    import json
    import pathlib
    gold = json.loads((pathlib.Path(__file__).resolve().parent / "golden" / "c1_ccd_trajectory.json").read_text())
    s = make_system(8, 24)
    r = jacobi(Fock.from_system(s), Integrals.from_system(s), "ccd", tol=0.0, max_iter=10)
    assert np.allclose(r["hist_e"], gold["hist_e"], rtol=0, atol=1e-14)
    assert np.allclose(r["hist_r"], gold["hist_rnorm"], rtol=1e-12, atol=0)


# ---- the projection at any excitation level (cluster_general) -------------

def _antisym(x, m):
    import itertools
    out = np.zeros_like(x)
    for ph in itertools.permutations(range(m)):
        for pp in itertools.permutations(range(m)):
            sg = round(np.linalg.det(np.eye(m)[list(ph)]) * np.linalg.det(np.eye(m)[list(pp)]))
            out = out + sg * np.transpose(x, list(ph) + [m + q for q in pp])
    return out


def test_general_projection_reduces_to_singles_doubles():
    o, v = 2, 4
    s = make_system(o, v, 21, sigma=0.1)
    P = Projector(s.fock(), s.full_integrals(), o)
    rng = np.random.default_rng(4)
    t1 = rng.normal(size=(o, v)) * 0.1
    t2 = _antisym(rng.normal(size=(o, o, v, v)) * 0.1, 2)
    assert np.array_equal(P.cluster_general({1: t1, 2: t2}), P.cluster(t1, t2)) or np.allclose(
        P.cluster_general({1: t1, 2: t2}), P.cluster(t1, t2), atol=1e-15)
    e, R1, R2 = P.evaluate(t1, t2)
    e_g, R = P.evaluate_general({1: t1, 2: t2}, (1, 2))
    assert abs(e - e_g) < 1e-14 and np.abs(R[1] - R1).max() < 1e-14 and np.abs(R[2] - R2).max() < 1e-14


def test_triples_cluster_operator_normalisation():
    """<Phi_ijk^abc| T3 |Phi_0> = t_ijk^abc for every index triple (the 1/36
    and the operator order of T3 and of the triply excited bra)."""
    o, v = 3, 3
    s = make_system(o, v, 22, sigma=0.1)
    P = Projector(s.fock(), s.full_integrals(), o)
    t3 = _antisym(np.random.default_rng(5).normal(size=(o,) * 3 + (v,) * 3), 3)
    T = P.cluster_general({3: t3})
    phi0 = np.zeros(T.shape[0])
    phi0[P.ref] = 1.0
    import itertools
    for holes in itertools.product(range(o), repeat=3):
        for parts in itertools.product(range(v), repeat=3):
            bra = P.excitation(holes, parts) @ phi0
            assert abs(bra @ (T @ phi0) - t3[holes + parts]) < 1e-13


def test_ccsdt_is_exact_for_three_electrons():
    """CCSDT (projection residuals, Jacobi) reproduces the FCI correlation
    energy of a three-electron system."""
    import itertools
    o, v = 3, 3
    s = make_system(o, v, 11, sigma=0.05)
    P = Projector(s.fock(), s.full_integrals(), o)
    eo, ev = np.diag(s.fock())[:o], np.diag(s.fock())[o:]
    D = {}
    for m in (1, 2, 3):
        d = np.zeros((o,) * m + (v,) * m)
        for idx in itertools.product(*([range(o)] * m + [range(v)] * m)):
            d[idx] = sum(eo[q] for q in idx[:m]) - sum(ev[q] for q in idx[m:])
        D[m] = d
    amps = {m: np.zeros((o,) * m + (v,) * m) for m in (1, 2, 3)}
    for _ in range(200):
        e, R = P.evaluate_general(amps, (1, 2, 3))
        if np.sqrt(sum(np.sum(R[m] ** 2) for m in R)) < 1e-11:
            break
        for m in (1, 2, 3):
            amps[m] = amps[m] + R[m] / D[m]
    e_fci = np.linalg.eigvalsh(P.H)[0] - P.e_hf
    assert abs(e - e_fci) < 1e-11
