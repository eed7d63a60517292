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
