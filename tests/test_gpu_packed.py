"""Contractions over packed index pairs (the ladder over i<j, a<b, e<f, the
hole-hole ladder over m<n and Z over e<f; CC_PLAN_PACKED_LADDER) against
the dense plan and the oracle."""
import json
import pathlib

import numpy as np
import pytest

from ccinputs.synth import make_system
from oracle.cc import Fock, residual
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


def _amps(o, v, seed, cplx):
    rng = np.random.default_rng(seed)
    t1 = rng.normal(size=(o, v)) * 0.03
    t2 = rng.normal(size=(o, o, v, v)) * 0.03
    if cplx:
        t1 = t1 + 1j * rng.normal(size=(o, v)) * 0.03
        t2 = t2 + 1j * rng.normal(size=(o, o, v, v)) * 0.03
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return t1, t2


@pytest.mark.parametrize("method", ["ccd", "ccsd"])
@pytest.mark.parametrize("ov,cplx", [((8, 24), False), ((12, 37), False), ((5, 70), False), ((4, 19), True),
                                     ((1, 4), False), ((3, 1), False), ((2, 2), False)])
def test_packed_ladder_equals_oracle_and_dense(E, ctx, method, ov, cplx):
    o, v = ov
    print(f"packed {method} o={o} v={v} complex={cplx}", flush=True)
    s = make_system(o, v, 40 + v, is_complex=cplx)
    t1, t2 = _amps(o, v, 3 * o + v, cplx)
    if method == "ccd":
        t1 = None
    r1_ref, r2_ref = residual(Fock.from_system(s), Integrals.from_system(s), t1, t2)
    d = E.DeviceSystem(s)
    m = E.METHODS[method]
    T1 = torch.from_numpy(t1).cuda() if t1 is not None else None
    T2 = torch.from_numpy(t2).cuda()
    out = {}
    for packed in (False, True):
        with E.Plan(ctx, d, m, packed=packed) as p:
            r1, r2, rn = p.residual(T1, T2)
            out[packed] = (r1, r2.cpu().numpy(), rn, p.flops(), p.flops(ladder_only=True))
    r2p = out[True][1]
    assert np.abs(r2p - r2_ref).max() < 1e-12
    assert np.array_equal(r2p, -r2p.transpose(1, 0, 2, 3)) and np.array_equal(r2p, -r2p.transpose(0, 1, 3, 2))
    assert np.abs(r2p - out[False][1]).max() < 1e-13
    if method == "ccsd":
        assert np.abs(out[True][0].cpu().numpy() - r1_ref).max() < 1e-12
    assert abs(out[True][2] - out[False][2]) < 1e-12 * max(1.0, out[False][2])
    # flop accounting: the packed ladder has o(o-1)/2 x [v(v-1)/2]^2 MACs, the
    # packed hh ladder [o(o-1)/2]^2 v(v-1)/2 and the packed Z o(o-1)/2 x ov x v(v-1)/2
    no, nv = o * (o - 1) // 2, v * (v - 1) // 2
    mul = 8 if cplx else 2
    assert out[True][4] == mul * no * nv * nv
    dense_hh, dense_z = mul * o ** 4 * v ** 2, (mul * o ** 3 * v ** 3 if method == "ccsd" else 0)
    packed_hh = mul * no * no * nv if no and nv else 0
    packed_z = (mul * no * o * v * nv if no and nv else 0) if method == "ccsd" else 0
    expect = out[False][3] - out[False][4] - dense_hh - dense_z + out[True][4] + packed_hh + packed_z
    assert abs(out[True][3] - expect) < 1e-6 * out[False][3]


def test_packed_iteration_matches_dense(E, ctx):
    o, v = 8, 30
    s = make_system(o, v, 12)
    d = E.DeviceSystem(s)
    res = {}
    for packed in (False, True):
        t1, t2 = E.zeros_amps(d, E.CCSD)
        res[packed] = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-10, max_iter=100, dressed=True, packed=packed)
    assert res[True]["converged"] and res[True]["iters"] == res[False]["iters"]
    assert np.allclose(res[True]["hist_e"], res[False]["hist_e"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_packed_c2_converges_to_oracle(E, ctx, prec):
    """o=32, v=160 with the packed ladder: FP64, and split-bf16 with the
    FP64 refinement, against the stored oracle run."""
    ref = json.loads((pathlib.Path(__file__).resolve().parent / "golden" / "c2_ccsd_energy.json").read_text())
    d = E.DeviceSystem(make_system(32, 160), drop_host=True)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-8, max_iter=400, dressed=True, autotune=True,
                    prec=E.PRECS[prec], packed=True)
    print(f"packed {prec}: {out['iters']} it, {out['seconds']:.2f}s, |dE|={abs(out['energy'] - ref['energy']):.2e}",
          flush=True)
    assert out["converged"]
    assert abs(out["energy"] - ref["energy"]) < (1e-10 if prec == "f64" else 1e-6)
