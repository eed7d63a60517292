"""The diagrammatic derivation (paper_2409_06759_amd.codegen) against the
paper's diagram counts and, numerically, against the oracle: the derived
CCD/CCSD equations equal the oracle's equations (which are pinned to the
brute-force projection), and the derived CCSDT and CCSDTQ equations equal
the brute-force projection itself at random amplitudes."""
import itertools

import numpy as np
import pytest

from ccinputs.synth import make_system
from oracle.cc import Fock, energy, residual
from oracle.integrals import Integrals
from oracle.projection import Projector
from paper_2409_06759_amd.codegen import diagram_count, equations, method_diagrams
from derived_eval import evaluate


def test_diagram_counts_of_table_gener():
    """Numbers of diagrams of Table "gener": 11, 48, 102, 183, 289."""
    counts = {m: diagram_count(m) for m in ("ccd", "ccsd", "ccsdt", "ccsdtq", "ccsdtqp")}
    assert counts == {"ccd": 11, "ccsd": 48, "ccsdt": 102, "ccsdtq": 183, "ccsdtqp": 289}


def test_ccsd_counts_per_equation_and_unique_strings():
    d = method_diagrams("ccsd")
    assert [len(d[k]) for k in (0, 1, 2)] == [3, 14, 31]
    strings = [x.string() for ds in d.values() for x in ds]
    assert len(set(strings)) == len(strings)


def _antisym(x, m):
    out = np.zeros_like(x)
    for ph in itertools.permutations(range(m)):
        for pp in itertools.permutations(range(m)):
            sg = round(np.linalg.det(np.eye(m)[list(ph)]) * np.linalg.det(np.eye(m)[list(pp)]))
            out = out + sg * np.transpose(x, list(ph) + [m + q for q in pp])
    return out


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("method", ["ccd", "ccsd"])
def test_derived_equations_equal_oracle(method, cplx):
    o, v = 3, 5
    s = make_system(o, v, 3, is_complex=cplx, sigma=0.1)
    rng = np.random.default_rng(1)
    n = o + v
    F = s.fock()
    X = rng.normal(size=(n, n)) * 0.1 + (1j * rng.normal(size=(n, n)) * 0.1 if cplx else 0)
    F = F + X + X.conj().T  # off-diagonal Fock blocks exercise the non-canonical diagrams
    Fk = Fock(F[:o, :o], F[:o, o:], F[o:, o:])
    V = Integrals.from_system(s)
    t1 = rng.normal(size=(o, v)) * 0.1 + (1j * rng.normal(size=(o, v)) * 0.1 if cplx else 0)
    t2 = _antisym(rng.normal(size=(o, o, v, v)) * 0.1 + (1j * rng.normal(size=(o, o, v, v)) * 0.1 if cplx else 0), 2)
    if method == "ccd":
        t1 = None
    sl = {"o": slice(0, o), "v": slice(o, n)}
    fock = lambda b: F[sl[b[0]], sl[b[1]]]  # noqa: E731
    eq = equations(method)
    amps = {1: t1, 2: t2}
    r1, r2 = residual(Fk, V, t1, t2)
    assert abs(evaluate(eq[0], fock, V.get, amps) - energy(Fk, V, t1, t2)) < 1e-13
    assert np.abs(evaluate(eq[2], fock, V.get, amps) - r2).max() < 1e-13
    if method == "ccsd":
        assert np.abs(evaluate(eq[1], fock, V.get, amps) - r1).max() < 1e-13


@pytest.mark.parametrize("method,o,v", [("ccsdt", 3, 4), ("ccsdtq", 4, 4)])
def test_derived_higher_order_equations_equal_projection(method, o, v):
    levels = {"ccsdt": (1, 2, 3), "ccsdtq": (1, 2, 3, 4)}[method]
    s = make_system(o, v, 5, sigma=0.1)
    rng = np.random.default_rng(2)
    n = o + v
    X = rng.normal(size=(n, n)) * 0.05
    F = s.fock() + X + X.T
    P = Projector(F, s.full_integrals(), o)
    amps = {m: _antisym(rng.normal(size=(o,) * m + (v,) * m) * 0.05, m) for m in levels}
    e, R = P.evaluate_general(amps, levels)
    V = Integrals.from_system(s)
    sl = {"o": slice(0, o), "v": slice(o, n)}
    fock = lambda b: F[sl[b[0]], sl[b[1]]]  # noqa: E731
    eq = equations(method)
    assert abs(evaluate(eq[0], fock, V.get, amps) - e) < 1e-13
    for k in levels:
        got = evaluate(eq[k], fock, V.get, amps)
        assert np.abs(got - R[k]).max() < 1e-12 * max(1.0, np.abs(R[k]).max()), k


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("ov", [(4, 7), (3, 5), (1, 3), (2, 2)])
def test_emitted_op_list_plans_reproduce_oracle(method, cplx, ov):
    """The binary contraction list emitted from the derived equations, laid
    out by the engine's planner (cc_plan_describe_ops_dry) and executed by
    the NumPy interpreter of the listing, equals the oracle residual."""
    from plan_interp import run_listing
    from paper_2409_06759_amd import _lib as L
    from paper_2409_06759_amd.codegen.emit import op_list
    lib = L.load()
    o, v = ov
    text = op_list("ccsd" if method else "ccd", o, v)
    listing = lib.cc_plan_describe_ops_dry(o, v, method, 1 if cplx else 0, text.encode()).decode()
    assert not listing.startswith("error"), listing[:200]
    R1, R2, r1_ref, r2_ref = run_listing(listing, o, v, method, cplx)
    assert np.abs(R2 - r2_ref).max() < 1e-13
    if method:
        assert np.abs(R1 - r1_ref).max() < 1e-13


def test_op_list_errors_name_the_line():
    from paper_2409_06759_amd import _lib as L
    lib = L.load()
    bad = b"work G1 oo\nop x XP ijab 1.0 oovv ijab\n"
    assert lib.cc_plan_describe_ops_dry(3, 4, 1, 0, bad).decode().startswith("error: op list line 2")
    assert b"unknown tensor" in lib.cc_plan_describe_ops_dry(3, 4, 1, 0, b"op x XP ijab 1.0 nope ijab - -\n")
    assert b"reads t1" in lib.cc_plan_describe_ops_dry(3, 4, 0, 0, b"op x R1 ia 1.0 t1 ia - -\n")


def test_emitted_ccsdt_plan_reproduces_projection():
    """CCSDT: the emitted list (singles, doubles and triples into Y3), laid
    out by the planner and executed in NumPy, equals the brute-force
    projection at random amplitudes; R3 is the antisymmetriser of Y3."""
    from plan_interp import doubles, execute, triples
    from paper_2409_06759_amd import _lib as L
    from paper_2409_06759_amd.codegen.emit import op_list
    lib = L.load()
    o, v = 3, 4
    s = make_system(o, v, 8, sigma=0.1)
    rng = np.random.default_rng(3)
    n = o + v
    X = rng.normal(size=(n, n)) * 0.05
    F = s.fock() + X + X.T
    P = Projector(F, s.full_integrals(), o)
    amps = {m: _antisym(rng.normal(size=(o,) * m + (v,) * m) * 0.05, m) for m in (1, 2, 3)}
    e, R = P.evaluate_general(amps, (1, 2, 3))
    listing = lib.cc_plan_describe_ops_dry(o, v, 1, 0, op_list("ccsdt", o, v).encode()).decode()
    assert not listing.startswith("error"), listing[:200]
    V = Integrals.from_system(s)
    inputs = {"foo": F[:o, :o], "fov": F[:o, o:], "fvv": F[o:, o:], "t1": amps[1], "t2": amps[2], "t3": amps[3]}
    inputs.update({b: V.get(b) for b in ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")})
    get = execute(listing, inputs, o, v, False, 1)
    assert np.abs(get("R1").reshape(o, v) - R[1]).max() < 1e-13
    assert np.abs(doubles(get, o, v) - R[2]).max() < 1e-13
    assert np.abs(triples(get, o, v) - R[3]).max() < 1e-12
