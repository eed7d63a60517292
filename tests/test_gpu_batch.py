"""Batched evaluation of uneven systems (one grouped launch per step) against
single-system plans and the oracle (GPU)."""
import numpy as np
import pytest

from ccinputs.synth import batch_shapes, make_system
from oracle.cc import Fock, jacobi
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


SHAPES = [(4, 20, 11), (7, 33, 12), (5, 26, 13), (9, 21, 14), (6, 41, 15)]


@pytest.mark.parametrize("packed", [True, False])
@pytest.mark.parametrize("method", ["ccd", "ccsd"])
def test_batch_steps_equal_single_system_steps(E, ctx, monkeypatch, method, packed):
    """Batches of real systems run the ladder, the hole-hole ladder and Z over
    packed pairs (CC_BATCH_DENSE keeps them dense): against single-system
    plans of the same layout."""
    m = E.METHODS[method]
    systems = [make_system(o, v, seed) for o, v, seed in SHAPES]
    ds = [E.DeviceSystem(s) for s in systems]
    if not packed:
        monkeypatch.setenv("CC_BATCH_DENSE", "1")
    with E.Batch(ctx, ds, m) as B:
        for _ in range(4):
            B.step(0.0, True)
        rn_b, e_b, _ = B.scalars()
        amps_b = B.amps
        for b, d in enumerate(ds):
            t1, t2 = E.zeros_amps(d, m)
            with E.Plan(ctx, d, m, packed=packed) as p:
                for _ in range(4):
                    p.step(t1, t2, 0.0, True)
                rn, e, _ = p.scalars()
            print(f"system {b}: dE={abs(e - e_b[b]):.3e} drn={abs(rn - rn_b[b]):.3e}", flush=True)
            assert abs(e - e_b[b]) < 1e-13 and abs(rn - rn_b[b]) < 1e-12
            assert (amps_b[b][1] - t2).abs().max().item() < 1e-14


def test_batch_iterate_matches_oracle_per_system(E, ctx):
    systems = [make_system(o, v, seed) for o, v, seed in SHAPES]
    ds = [E.DeviceSystem(s) for s in systems]
    with E.Batch(ctx, ds, E.CCSD) as B:
        B.autotune(1)
        out = B.iterate(tol=1e-10, max_iter=100, dressed=True)
    assert out["n_converged"] == len(SHAPES)
    for s, rec in zip(systems, out["systems"]):
        ref = jacobi(Fock.from_system(s), Integrals.from_system(s), "ccsd", tol=1e-10, max_iter=100,
                     dressed=True)
        assert rec["iters"] == ref["iters"]
        assert abs(rec["energy"] - ref["energy"]) < 1e-11


def test_batch_c4_shapes_run(E, ctx):
    """The 64-system workload's shapes (o in [4,16], v in [20,60]) build and step."""
    shapes = batch_shapes(64)[:16]
    ds = [E.DeviceSystem(make_system(o, v, seed)) for o, v, seed in shapes]
    with E.Batch(ctx, ds, E.CCSD) as B:
        B.step(0.0, True)
        B.step(0.0, True)
        rn, e, _ = B.scalars()
    assert all(np.isfinite(rn)) and all(x < 0 for x in e)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_batch_reduced_precision_equals_single_system(E, ctx, prec):
    """Grouped reduced-precision GEMMs (K-contiguous operands read from
    copies made by grouped conversions, the others converted while staging)
    against single-system plans (operands converted once into copies): the
    same products in the same order, so equal to FP64 rounding of the
    epilogues."""
    systems = [make_system(o, v, seed) for o, v, seed in SHAPES]
    ds = [E.DeviceSystem(s) for s in systems]
    P = E.PRECS[prec]
    with E.Batch(ctx, ds, E.CCSD, prec=P) as B:
        B.autotune(1)
        for _ in range(3):
            B.step(0.0, True)
        rn_b, e_b, _ = B.scalars()
        amps_b = B.amps
        for b, d in enumerate(ds):
            t1, t2 = E.zeros_amps(d, E.CCSD)
            with E.Plan(ctx, d, E.CCSD, prec=P, lowp_all=True, packed=True) as p:  # as the batch
                for _ in range(3):
                    p.step(t1, t2, 0.0, True)
                rn, e, _ = p.scalars()
            print(f"{prec} system {b}: dE={abs(e - e_b[b]):.3e} drn={abs(rn - rn_b[b]):.3e}", flush=True)
            assert abs(e - e_b[b]) < 1e-12 * max(1.0, abs(e)) and abs(rn - rn_b[b]) < 1e-12
            assert (amps_b[b][1] - t2).abs().max().item() < 1e-13


def test_batch_c4_full_workload(E, ctx, monkeypatch):
    """All 64 systems of the batched workload iterated together to 1e-10.
    With the split-K factors each system's own plan chose
    (CC_BATCH_OWN_SPLITS=1) every system equals its own single-system solve
    (over packed pairs, as the batch) bitwise. With the batch's factors (the default; fewer K-slices, since
    the systems fill the GPU together) the sums are ordered differently:
    the same iteration counts and energies within 1e-12 Eh. Three systems
    (the smallest, a middle and the largest) equal the oracle's converged
    energy."""
    shapes = batch_shapes(64)
    systems = [make_system(o, v, seed) for o, v, seed in shapes]
    ds = [E.DeviceSystem(s) for s in systems]
    monkeypatch.setenv("CC_BATCH_OWN_SPLITS", "1")
    with E.Batch(ctx, ds, E.CCSD) as B:
        own = B.iterate(tol=1e-10, max_iter=200, dressed=True)
    monkeypatch.delenv("CC_BATCH_OWN_SPLITS")
    with E.Batch(ctx, ds, E.CCSD) as B:
        out = B.iterate(tol=1e-10, max_iter=200, dressed=True)
    assert own["n_converged"] == 64 and out["n_converged"] == 64
    size = [o * o * v * v for o, v, _ in shapes]
    order = np.argsort(size)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    worst = 0.0
    for b in range(64):
        t1, t2 = E.zeros_amps(ds[b], E.CCSD)
        single = E.iterate(ctx, ds[b], E.CCSD, t1, t2, tol=1e-10, max_iter=200, dressed=True, packed=True)
        assert single["iters"] == own["systems"][b]["iters"] == out["systems"][b]["iters"]
        assert single["energy"] == own["systems"][b]["energy"]
        worst = max(worst, abs(single["energy"] - out["systems"][b]["energy"]))
    print(f"batch split-K factors: largest energy difference {worst:.2e} Eh", flush=True)
    assert worst < 1e-12
    for b in pick:
        o, v, _ = shapes[b]
        print(f"oracle check: system {b} o={o} v={v}", flush=True)
        ref = jacobi(Fock.from_system(systems[b]), Integrals.from_system(systems[b]), "ccsd", tol=1e-10,
                     max_iter=200, dressed=True)
        assert abs(ref["energy"] - out["systems"][b]["energy"]) < 1e-10
