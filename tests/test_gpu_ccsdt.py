"""CCSDT on the GPU from the diagram generator's contraction list
(cc_plan_create_ops + cc_plan_set_triples) against the brute-force
projection, the NumPy evaluation of the derived terms, and FCI."""
import itertools

import numpy as np
import pytest

from ccinputs.synth import make_system
from oracle.integrals import Integrals
from oracle.projection import Projector

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    from paper_2409_06759_amd import engine
    return engine


@pytest.fixture(scope="module")
def ctx(E):
    c = E.Context(0)
    yield c
    c.close()


def _antisym(x, m):
    out = np.zeros_like(x)
    for ph in itertools.permutations(range(m)):
        for pp in itertools.permutations(range(m)):
            sg = round(np.linalg.det(np.eye(m)[list(ph)]) * np.linalg.det(np.eye(m)[list(pp)]))
            out = out + sg * np.transpose(x, list(ph) + [m + q for q in pp])
    return out


def _residuals(E, ctx, s, amps):
    from paper_2409_06759_amd.codegen.emit import op_list
    o, v = s.o, s.v
    d = E.DeviceSystem(s)
    T = {m: torch.from_numpy(np.ascontiguousarray(amps[m])).cuda() for m in (1, 2, 3)}
    r3 = torch.zeros_like(T[3])
    with E.Plan(ctx, d, E.CCSD, ops=op_list("ccsdt", o, v)) as p:
        p.set_triples(T[3], r3)
        r1, r2, rn = p.residual(T[1], T[2])
        _, e, _ = p.scalars()
    return e, r1.cpu().numpy(), r2.cpu().numpy(), r3.cpu().numpy(), rn


@pytest.mark.parametrize("ov", [(3, 4), (4, 5)])
def test_ccsdt_residual_matches_projection(E, ctx, ov):
    o, v = ov
    print(f"CCSDT residual o={o} v={v} vs projection", flush=True)
    s = make_system(o, v, 9, sigma=0.1)
    rng = np.random.default_rng(4)
    amps = {m: _antisym(rng.normal(size=(o,) * m + (v,) * m) * 0.05, m) for m in (1, 2, 3)}
    P = Projector(s.fock(), s.full_integrals(), o)
    e_ref, R = P.evaluate_general(amps, (1, 2, 3))
    e, r1, r2, r3, rn = _residuals(E, ctx, s, amps)
    assert abs(e - e_ref) < 1e-13
    assert np.abs(r1 - R[1]).max() < 1e-12 and np.abs(r2 - R[2]).max() < 1e-12
    assert np.abs(r3 - R[3]).max() < 1e-12
    nref = np.sqrt(sum(np.sum(R[m] ** 2) for m in R))
    assert abs(rn - nref) < 1e-12 * nref


def test_ccsdt_residual_matches_derived_terms_larger(E, ctx):
    """Several tiles in every dimension: against the NumPy evaluation of the
    derived CCSDT terms (themselves pinned to the projection on the CPU)."""
    from paper_2409_06759_amd.codegen import equations
    from derived_eval import evaluate
    o, v = 6, 21
    s = make_system(o, v, 10, sigma=0.05)
    rng = np.random.default_rng(5)
    amps = {m: _antisym(rng.normal(size=(o,) * m + (v,) * m) * 0.02, m) for m in (1, 2, 3)}
    F = s.fock()
    V = Integrals.from_system(s)
    sl = {"o": slice(0, o), "v": slice(o, o + v)}
    fock = lambda b: F[sl[b[0]], sl[b[1]]]  # noqa: E731
    eq = equations("ccsdt")
    e, r1, r2, r3, _ = _residuals(E, ctx, s, amps)
    assert abs(e - evaluate(eq[0], fock, V.get, amps)) < 1e-13
    for k, r in ((1, r1), (2, r2), (3, r3)):
        ref = evaluate(eq[k], fock, V.get, amps)
        assert np.abs(r - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), k


def test_ccsdt_is_exact_for_three_electrons_on_gpu(E, ctx):
    """Bare Jacobi with the generated CCSDT plan converges to the FCI
    correlation energy of a three-electron system."""
    from paper_2409_06759_amd.codegen.emit import op_list
    o, v = 3, 5
    s = make_system(o, v, 11, sigma=0.05)
    P = Projector(s.fock(), s.full_integrals(), o)
    e_fci = np.linalg.eigvalsh(P.H)[0] - P.e_hf
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    t3 = torch.zeros((o,) * 3 + (v,) * 3, dtype=torch.float64, device="cuda")
    with E.Plan(ctx, d, E.CCSD, ops=op_list("ccsdt", o, v)) as p:
        p.set_triples(t3)
        for it in range(200):
            p.step(t1, t2, 0.0, False)
            rn, e, _ = p.scalars()
            if rn < 1e-11:
                break
    print(f"CCSDT {it + 1} iterations: E = {e:.14f}, FCI {e_fci:.14f}", flush=True)
    assert rn < 1e-11
    assert abs(e - e_fci) < 1e-10
