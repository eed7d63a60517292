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
