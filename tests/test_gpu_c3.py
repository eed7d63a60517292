"""Full-size checks of the complex128 workload (CCSD, o=40, v=200, vvvv
25.6 GB) through the C ABI, by properties that hold at any size: the first
Jacobi iterate and energy in closed form (MP2), bitwise antisymmetry of the
residual, and equality with the real path when the imaginary parts vanish."""
import numpy as np
import pytest

from ccinputs.synth import make_system

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

O, V = 40, 200


@pytest.fixture(scope="module")
def E():
    from paper_2409_06759_amd import engine
    return engine


@pytest.fixture(scope="module")
def ctx(E):
    c = E.Context(0)
    yield c
    c.close()


def _antisym(x):
    return bool(torch.equal(x, -x.transpose(0, 1)) and torch.equal(x, -x.transpose(2, 3)))


def test_c3_complex_first_iterate_is_mp2_and_residual_antisymmetric(E, ctx):
    print(f"complex CCSD o={O} v={V}: generating", flush=True)
    s = make_system(O, V, is_complex=True)
    oovv = s.block("oovv")
    eo, ev = np.real(np.diag(s.f_oo)), np.real(np.diag(s.f_vv))
    D = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        t2_mp2 = np.where(D != 0, np.conj(oovv) / D, 0)
    e_mp2 = 0.25 * np.sum(np.abs(oovv) ** 2 / D)  # closed form, real
    d = E.DeviceSystem(s, drop_host=True)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-30, max_iter=2)
    print(f"E(t1) = {out['hist_e'][1]:.12f}, MP2 closed form {e_mp2:.12f}", flush=True)
    assert abs(out["hist_e"][1] - e_mp2) < 1e-12 * abs(e_mp2)
    with E.Plan(ctx, d, E.CCSD) as plan:
        # t after one plain step from zero: <ab||ij> / D, t1 = 0 (f_ov = 0)
        a1, a2 = E.zeros_amps(d, E.CCSD)
        plan.step(a1, a2, 0.0, False)
        got = a2.cpu().numpy()
        assert np.abs(got - t2_mp2).max() < 1e-15 * max(1.0, np.abs(t2_mp2).max())
        assert torch.all(a1 == 0)
        r1, r2, rn = plan.residual(t1, t2)  # at the iterate of the two dressed-free steps
        assert _antisym(r2) and np.isfinite(rn)
        _, e, ei = plan.scalars()
        assert np.isfinite(e) and np.isfinite(ei)


def test_c3_zero_imaginary_equals_real_path(E, ctx):
    print(f"real and zero-imaginary complex CCSD o={O} v={V}", flush=True)
    s = make_system(O, V)
    dr = E.DeviceSystem(s, drop_host=True)
    tc = {n: dr.t[n].to(torch.complex128) for n in E.DeviceSystem.NAMES}
    dc = E.DeviceSystem.from_tensors(O, V, tc)
    rng = np.random.default_rng(5)
    t2 = rng.normal(size=(O, O, V, V)) * 1e-3
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    t1 = rng.normal(size=(O, V)) * 1e-3
    T1, T2 = torch.from_numpy(t1).cuda(), torch.from_numpy(t2).cuda()
    r1, r2, rn = E.residual(ctx, dr, E.CCSD, T1, T2)
    z1, z2, zn = E.residual(ctx, dc, E.CCSD, T1.to(torch.complex128), T2.to(torch.complex128))
    assert torch.all(z2.imag == 0) and torch.all(z1.imag == 0)
    scale = r2.abs().max().item()
    err = (z2.real - r2).abs().max().item()
    print(f"max |R_complex - R_real| = {err:.3e} (|R| {scale:.3e}), norms {zn:.12e} {rn:.12e}", flush=True)
    assert err < 1e-13 * max(1.0, scale)
    assert abs(zn - rn) < 1e-12 * rn


def test_c3_complex_residual_matches_oracle_sample(E, ctx):
    """R1, R2, the norm and the energy at seeded random complex amplitudes
    (genuinely complex, every term of the residual contributing), against
    the oracle's values stored by tests/golden/make_reference.py c3, after
    the autotuner has picked the launch configurations the benchmark times."""
    import json
    import pathlib

    from ccinputs.synth import random_amplitudes
    g = json.loads((pathlib.Path(__file__).parent / "golden" / f"c3_complex_o{O}_v{V}_sample.json").read_text())
    print(f"complex CCSD o={O} v={V}: residual against the oracle sample", flush=True)
    s = make_system(O, V, is_complex=True)
    assert complex(*g["fingerprint"]["vvvv_0123"]) == s.block("vvvv")[0, 1, 2, 3]
    t1, t2 = random_amplitudes(O, V, g["amp_seed"], g["amp_scale"], is_complex=True)
    assert abs(np.abs(t2).sum() - g["fingerprint"]["t2_sum_abs"]) <= 1e-12 * g["fingerprint"]["t2_sum_abs"]
    d = E.DeviceSystem(s, drop_host=True)
    T1, T2 = torch.from_numpy(t1).cuda(), torch.from_numpy(t2).cuda()
    del t2
    with E.Plan(ctx, d, E.CCSD) as plan:
        plan.autotune(T1, T2, 1)
        r1, r2, rn = plan.residual(T1, T2)
        _, er, ei = plan.scalars()
    i2 = torch.tensor(g["r2_index"], device="cuda")
    i1 = torch.tensor(g["r1_index"], device="cuda")
    got2 = r2.reshape(-1)[i2].cpu().numpy()
    got1 = r1.reshape(-1)[i1].cpu().numpy()
    want2 = np.array([complex(*z) for z in g["r2"]])
    want1 = np.array([complex(*z) for z in g["r1"]])
    e2 = np.abs(got2 - want2).max() / g["r2_max_abs"]
    e1 = np.abs(got1 - want1).max() / g["r1_max_abs"]
    ew = complex(*g["energy"])
    print(f"max |dR2|/max|R2| {e2:.2e}, |dR1|/max|R1| {e1:.2e}, norm {rn:.15e} vs {g['rnorm']:.15e}, "
          f"E {er:.15f}{ei:+.3e}i vs {ew:.15f}", flush=True)
    assert np.abs(want2.imag).max() > 0.1 * np.abs(want2.real).max()  # genuinely complex
    assert e2 < 1e-12 and e1 < 1e-12
    assert abs(rn - g["rnorm"]) < 1e-12 * g["rnorm"]
    assert abs(complex(er, ei) - ew) < 1e-12 * max(1.0, abs(ew))
