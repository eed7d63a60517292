"""Plans built from the diagram generator's contraction list (derived
equations -> binary ops -> cc_plan_create_ops) on the GPU against the
oracle, and against the built-in factorised table."""
import numpy as np
import pytest

from ccinputs.synth import make_system
from oracle.cc import Fock, energy, jacobi, residual
from oracle.integrals import Integrals

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


def _amps(o, v, seed, cplx=False):
    rng = np.random.default_rng(seed)
    t1 = rng.normal(size=(o, v)) * 0.02
    t2 = rng.normal(size=(o, o, v, v)) * 0.02
    if cplx:
        t1 = t1 + 1j * rng.normal(size=(o, v)) * 0.02
        t2 = t2 + 1j * rng.normal(size=(o, o, v, v)) * 0.02
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return t1, t2


@pytest.mark.parametrize("method", ["ccd", "ccsd"])
@pytest.mark.parametrize("ov,cplx", [((3, 5), False), ((8, 24), False), ((5, 70), False), ((4, 19), True),
                                     ((1, 4), False)])
def test_generated_plan_residual_matches_oracle(E, ctx, method, ov, cplx):
    from paper_2409_06759_amd.codegen.emit import op_list
    o, v = ov
    print(f"generated {method} o={o} v={v} complex={cplx}", flush=True)
    s = make_system(o, v, 77 + o, is_complex=cplx)
    t1, t2 = _amps(o, v, o * v, cplx)
    if method == "ccd":
        t1 = None
    F, V = Fock.from_system(s), Integrals.from_system(s)
    r1_ref, r2_ref = residual(F, V, t1, t2)
    d = E.DeviceSystem(s)
    T1 = torch.from_numpy(t1).cuda() if t1 is not None else None
    T2 = torch.from_numpy(t2).cuda()
    with E.Plan(ctx, d, E.METHODS[method], ops=op_list(method, o, v)) as p:
        r1, r2, rn = p.residual(T1, T2)
        _, e, ei = p.scalars()
    r2 = r2.cpu().numpy()
    assert np.abs(r2 - r2_ref).max() < 1e-12
    assert np.array_equal(r2, -r2.transpose(1, 0, 2, 3)) and np.array_equal(r2, -r2.transpose(0, 1, 3, 2))
    if method == "ccsd":
        assert np.abs(r1.cpu().numpy() - r1_ref).max() < 1e-12
    e_ref = energy(F, V, t1, t2)
    assert abs(complex(e, ei) - e_ref) < 1e-13


def test_generated_plan_trajectory_matches_oracle(E, ctx):
    """Bare-denominator Jacobi steps with the generated plan follow the oracle."""
    from paper_2409_06759_amd.codegen.emit import op_list
    o, v = 6, 22
    s = make_system(o, v, 5)
    ref = jacobi(Fock.from_system(s), Integrals.from_system(s), "ccsd", tol=0.0, max_iter=6)
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    es = []
    with E.Plan(ctx, d, E.CCSD, ops=op_list("ccsd", o, v)) as p:
        for _ in range(6):
            p.step(t1, t2, 0.0, False)
            es.append(p.scalars()[1])
        with pytest.raises(Exception):
            p.step(t1, t2, 0.0, True)  # dressed denominators need the built-in table
    assert np.allclose(es, ref["hist_e"], rtol=0, atol=1e-12)
