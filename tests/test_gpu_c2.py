"""The o=32, v=160 CCSD workload against the FP64 oracle's stored Jacobi run
(tests/golden/c2_ccsd_energy.json, written by make_reference.py from the
oracle alone): iteration-by-iteration energies, the converged energy in FP64
and with reduced-precision contractions."""
import json
import pathlib

import numpy as np
import pytest

from ccinputs.synth import make_system

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = pathlib.Path(__file__).resolve().parent / "golden" / "c2_ccsd_energy.json"


@pytest.fixture(scope="module")
def E():
    from paper_2409_06759_amd import engine
    return engine


@pytest.fixture(scope="module")
def ref():
    return json.loads(GOLD.read_text())


@pytest.fixture(scope="module")
def setup(E):
    ctx = E.Context(0)
    d = E.DeviceSystem(make_system(32, 160), drop_host=True)
    yield ctx, d
    ctx.close()


def test_c2_fp64_trajectory_and_converged_energy(E, setup, ref):
    ctx, d = setup
    t1, t2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-8, max_iter=400, dressed=True, autotune=True)
    print(f"FP64: {out['iters']} it, {out['seconds']:.2f}s, E={out['energy']:.12f}, oracle {ref['energy']:.12f}",
          flush=True)
    assert out["converged"] and out["iters"] == ref["iterations"]
    # same iteration, same energy (the oracle records E(t_n) for n = 0..)
    he = np.array(out["hist_e"])
    ho = np.array(ref["hist_e"][:len(he)])
    hr, hro = np.array(out["hist_rnorm"]), np.array(ref["hist_rnorm"][:len(he)])
    print(f"max |dE| per iteration {np.abs(he - ho).max():.2e}; max rel |d||R||| "
          f"{np.max(np.abs(hr - hro) / hro):.2e}", flush=True)
    assert np.abs(he - ho).max() < 1e-11
    assert np.max(np.abs(hr - hro) / hro) < 1e-6
    assert abs(out["energy"] - ref["energy"]) < 1e-10
    if "energy_tight" in ref:
        assert abs(out["energy"] - ref["energy_tight"]) < 1e-8


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_c2_mixed_precision_converged_energy(E, setup, ref, prec):
    ctx, d = setup
    t1, t2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-8, max_iter=400, dressed=True, autotune=True,
                    prec=E.PRECS[prec])
    print(f"{prec}: {out['iters']} it ({out['lowp_iters']} reduced, {out['corr_iters']} corrected), "
          f"{out['seconds']:.2f}s, |dE|={abs(out['energy'] - ref['energy']):.2e}", flush=True)
    assert out["converged"]
    assert abs(out["energy"] - ref["energy"]) < 1e-6


def test_c2_split_bf16_residual_on_blocked_copies(E, setup):
    """One split-bf16 residual at o=32, v=160 in the configuration the bench
    times (plan created in split bf16, autotuned, so the ladder, Z and the
    ring terms run on the blocked copies with the full-size tail cut),
    against the FP64 residual at the same random amplitudes. Terms are
    O(1e-2) with up to v^2 = 25,600 products: split bf16 (hi*hi + hi*lo +
    lo*hi, FP32 accumulation) stays within 1e-4 of the largest |R|."""
    ctx, d = setup
    o, v = 32, 160
    g = torch.Generator(device="cuda")
    g.manual_seed(21)
    t1 = torch.randn(o, v, dtype=torch.float64, device="cuda", generator=g) * 0.01
    t2 = torch.randn(o, o, v, v, dtype=torch.float64, device="cuda", generator=g) * 0.01
    t2 = t2 - t2.transpose(0, 1)
    t2 = (t2 - t2.transpose(2, 3)).contiguous()
    with E.Plan(ctx, d, E.CCSD) as p64:
        e1, e2, _ = p64.residual(t1, t2)
        e1, e2 = e1.clone(), e2.clone()
    with E.Plan(ctx, d, E.CCSD, prec=E.PRECS["bf16x3"]) as p:
        p.autotune(t1, t2)
        p.profile(True)
        r1, r2, _ = p.residual(t1, t2)
        tags = [row[2] for row in p.profile_table() if row[1] == "GEMM"]
    scale = max(float(e2.abs().max()), float(e1.abs().max()))
    err = max(float((r2 - e2).abs().max()), float((r1 - e1).abs().max()))
    blk = [t for t in tags if t.endswith("/blk")]
    print(f"split bf16 at C2: max err {err:.2e} (|R| {scale:.2e}); blocked: {blk}", flush=True)
    assert any(t.startswith("ladder@") for t in blk)
    assert err < 1e-4 * scale
    assert err > 1e-12 * scale  # reduced-precision rounding is there
