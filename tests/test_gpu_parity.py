"""HIP path against the CPU oracle through the C ABI (GPU).

Tolerances (FP64 everywhere): residual elements agree to 1e-12 absolute
(terms are O(1e-2); summation order differs between einsum and the
MFMA tiles); energies along a Jacobi trajectory agree to 1e-12 Eh; the
residual's (ij) and (ab) antisymmetry holds bitwise.
"""
import json
import pathlib

import numpy as np
import pytest

from ccinputs.synth import make_system
from oracle.cc import Fock, denominators, energy, jacobi, residual
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


def _amps(o, v, seed, scale=0.01, cplx=False):
    rng = np.random.default_rng(seed)
    t1 = rng.normal(size=(o, v)) * scale
    t2 = rng.normal(size=(o, o, v, v)) * scale
    if cplx:
        t1 = t1 + 1j * rng.normal(size=(o, v)) * scale
        t2 = t2 + 1j * rng.normal(size=(o, o, v, v)) * scale
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return t1, t2


@pytest.mark.parametrize("method", ["ccd", "ccsd"])
@pytest.mark.parametrize("ov", [(3, 5), (8, 24), (12, 37), (5, 70), (1, 4), (2, 1), (1, 1), (2, 3)])
def test_residual_matches_oracle(E, ctx, method, ov):
    o, v = ov
    print(f"residual {method} o={o} v={v}", flush=True)
    s = make_system(o, v, 1000 + o * v)
    t1, t2 = _amps(o, v, o + v)
    if method == "ccd":
        t1 = None
    F, V = Fock.from_system(s), Integrals.from_system(s)
    r1_ref, r2_ref = residual(F, V, t1, t2)
    d = E.DeviceSystem(s)
    T1 = torch.from_numpy(t1).cuda() if t1 is not None else None
    T2 = torch.from_numpy(t2).cuda()
    r1, r2, rn = E.residual(ctx, d, E.METHODS[method], T1, T2)
    r2 = r2.cpu().numpy()
    assert np.abs(r2 - r2_ref).max() < 1e-12
    if method == "ccsd":
        assert np.abs(r1.cpu().numpy() - r1_ref).max() < 1e-12
    # bitwise antisymmetry and exact zeros on the diagonals
    assert np.array_equal(r2, -r2.transpose(1, 0, 2, 3))
    assert np.array_equal(r2, -r2.transpose(0, 1, 3, 2))
    nref = np.sqrt(np.sum(np.abs(r2_ref) ** 2) + (np.sum(np.abs(r1_ref) ** 2) if r1_ref is not None else 0))
    assert abs(rn - nref) < 1e-12 * max(1.0, nref)
    e = E.energy(ctx, d, E.METHODS[method], T1, T2)
    assert abs(e - energy(F, V, t1, t2)) < 1e-13


def test_complex_batch_reduced_precision_rejected(E, ctx):
    """Batches of complex systems keep FP64 contractions (their grouped
    launches have no realified complex path)."""
    from paper_2409_06759_amd import _lib as L
    s = make_system(3, 5, 9, is_complex=True)
    d = E.DeviceSystem(s)
    with pytest.raises(L.CCError) as ei:
        E.Batch(ctx, [d], E.CCSD, prec=E.F32)
    assert ei.value.status == L.CC_EUNSUPPORTED


@pytest.mark.parametrize("prec,tol", [("f32", 2e-6), ("bf16x3", 5e-5)])
@pytest.mark.parametrize("ov", [(3, 5), (8, 24), (6, 40)])
def test_complex_reduced_precision_residual(E, ctx, prec, tol, ov):
    """Complex residual with the large contractions as real reduced-precision
    GEMMs on realified operands, against the FP64 oracle.  As for real
    systems, terms are O(1e-2) with at most 2 v^2 real products each (the
    realified sum has twice the length), so FP32 gives about
    2 * 1600 * 2^-24 * 1e-2 ~ 2e-6 at v = 40 in the worst case, split bf16 adds
    3 * 2^-17 * 1e-2; the plan's flags show which contractions took that path."""
    o, v = ov
    s = make_system(o, v, 2100 + o * v, is_complex=True)
    t1, t2 = _amps(o, v, o * v + 1, cplx=True)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    r1_ref, r2_ref = residual(F, V, t1, t2)
    d = E.DeviceSystem(s)
    T1, T2 = torch.from_numpy(t1).cuda(), torch.from_numpy(t2).cuda()
    with E.Plan(ctx, d, E.CCSD, prec=E.PRECS[prec]) as p:
        r1, r2, rn = p.residual(T1, T2)
    r2 = r2.cpu().numpy()
    err = max(np.abs(r2 - r2_ref).max(), np.abs(r1.cpu().numpy() - r1_ref).max())
    print(f"complex {prec} o={o} v={v}: max err {err:.2e} (tol {tol:.0e})", flush=True)
    assert err < tol
    assert err > 1e-11  # reduced-precision rounding, far above FP64's (1e-12 tests above)
    assert np.array_equal(r2, -r2.transpose(1, 0, 2, 3))


@pytest.mark.parametrize("method", ["ccd", "ccsd"])
@pytest.mark.parametrize("ov", [(3, 5), (7, 23), (4, 40)])
def test_complex_residual_matches_oracle(E, ctx, method, ov):
    """Hermitian complex integrals: driver <ab||ij> = conj <ij||ab>, every
    non-stored block a conjugated view; parity 1e-12 as in the real case."""
    o, v = ov
    s = make_system(o, v, 3000 + o * v, is_complex=True)
    t1, t2 = _amps(o, v, 7 * o + v, cplx=True)
    if method == "ccd":
        t1 = None
    F, V = Fock.from_system(s), Integrals.from_system(s)
    r1_ref, r2_ref = residual(F, V, t1, t2)
    d = E.DeviceSystem(s)
    T1 = torch.from_numpy(t1).cuda() if t1 is not None else None
    r1, r2, rn = E.residual(ctx, d, E.METHODS[method], T1, torch.from_numpy(t2).cuda())
    r2 = r2.cpu().numpy()
    assert np.abs(r2 - r2_ref).max() < 1e-12
    if t1 is not None:
        assert np.abs(r1.cpu().numpy() - r1_ref).max() < 1e-12
    assert np.array_equal(r2, -r2.transpose(1, 0, 2, 3))
    e = E.energy(ctx, d, E.METHODS[method], T1, torch.from_numpy(t2).cuda())
    e_ref = energy(F, V, t1, t2)
    assert abs(e.real - e_ref.real) < 1e-13 and abs(e.imag - e_ref.imag) < 1e-13


def test_complex_with_zero_imaginary_equals_real(E, ctx):
    o, v = 5, 17
    s = make_system(o, v, 4)
    sc = make_system(o, v, 4, is_complex=True)
    for b in ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv"):
        sc._blocks[b] = s.block(b).astype(np.complex128)
    t1, t2 = _amps(o, v, 11)
    d, dc = E.DeviceSystem(s), E.DeviceSystem(sc)
    r1, r2, rn = E.residual(ctx, d, E.CCSD, torch.from_numpy(t1).cuda(), torch.from_numpy(t2).cuda())
    z1, z2, zn = E.residual(ctx, dc, E.CCSD, torch.from_numpy(t1.astype(complex)).cuda(),
                            torch.from_numpy(t2.astype(complex)).cuda())
    assert torch.all(z2.imag == 0) and torch.all(z1.imag == 0)
    assert np.abs(z2.real.cpu().numpy() - r2.cpu().numpy()).max() < 1e-14
    assert abs(zn - rn) < 1e-12


def test_complex_dressed_trajectory(E, ctx):
    o, v = 6, 26
    s = make_system(o, v, 79, is_complex=True)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    ref = jacobi(F, V, "ccsd", tol=0.0, max_iter=6, dressed=True)
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-30, max_iter=6, dressed=True)
    assert np.allclose(out["hist_e"], np.real(ref["hist_e"]), rtol=0, atol=1e-12)
    assert abs(out["energy"] - ref["hist_e"][-1]) < 1e-12  # complex: Re and Im
    assert np.abs(t2.cpu().numpy() - ref["t2"]).max() < 1e-12


def test_ccd_c1_trajectory(E, ctx):
    """o=8, v=24 CCD: ten Jacobi iterations from t = 0 (first = MP2)."""
    o, v = 8, 24
    s = make_system(o, v)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    ref = jacobi(F, V, "ccd", tol=0.0, max_iter=10)
    d = E.DeviceSystem(s)
    _, t2 = E.zeros_amps(d, E.CCD)
    out = E.iterate(ctx, d, E.CCD, None, t2, tol=1e-30, max_iter=10, use_graph=True)
    assert out["iters"] == 10
    assert np.allclose(out["hist_e"], ref["hist_e"], rtol=0, atol=1e-12)
    assert np.allclose(out["hist_rnorm"], ref["hist_r"], rtol=1e-10, atol=1e-14)
    _, d2 = denominators(F)
    g = V.get("oovv")
    assert abs(out["hist_e"][1] - 0.25 * np.sum(g * g / d2)) < 1e-13
    # the stored oracle trajectory (tests/golden, written from the oracle alone)
    gold = json.loads((pathlib.Path(__file__).resolve().parent / "golden" / "c1_ccd_trajectory.json").read_text())
    assert np.allclose(out["hist_e"], gold["hist_e"], rtol=0, atol=1e-12)
    assert np.allclose(out["hist_rnorm"], gold["hist_rnorm"], rtol=1e-10, atol=1e-14)


def test_ccsd_converges_like_oracle(E, ctx):
    o, v = 8, 24
    s = make_system(o, v)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    ref = jacobi(F, V, "ccsd", tol=1e-8, max_iter=60)
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-8, max_iter=60)
    assert out["converged"] and ref["converged"]
    assert out["iters"] == ref["iters"]
    assert abs(out["energy"] - ref["energy"]) < 1e-12
    assert np.allclose(out["hist_e"], ref["hist_e"], rtol=0, atol=1e-12)


def test_level_shift_trajectory(E, ctx):
    o, v = 6, 30
    s = make_system(o, v, 77)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    ref = jacobi(F, V, "ccsd", tol=0.0, max_iter=6, level_shift=1.5)
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-30, max_iter=6, level_shift=1.5, use_graph=False)
    assert np.allclose(out["hist_e"], ref["hist_e"], rtol=0, atol=1e-12)
    assert np.abs(t2.cpu().numpy() - ref["t2"]).max() < 1e-12  # t_6 on both sides
    assert np.abs(t1.cpu().numpy() - ref["t1"]).max() < 1e-12


def test_graph_replay_is_bitwise_eager(E, ctx):
    o, v = 6, 22
    s = make_system(o, v, 5)
    d = E.DeviceSystem(s)
    a1, a2 = E.zeros_amps(d, E.CCSD)
    b1, b2 = E.zeros_amps(d, E.CCSD)
    ra = E.iterate(ctx, d, E.CCSD, a1, a2, tol=1e-30, max_iter=5, use_graph=True)
    rb = E.iterate(ctx, d, E.CCSD, b1, b2, tol=1e-30, max_iter=5, use_graph=False)
    assert ra["hist_e"] == rb["hist_e"] and ra["hist_rnorm"] == rb["hist_rnorm"]
    assert torch.equal(a2, b2) and torch.equal(a1, b1)


def test_autotune_choices_written_to_the_cache_file(E, ctx, tmp_path, monkeypatch):
    """With CC_AUTOTUNE_CACHE set, each new per-shape choice is appended to
    the file as "key tile" (a split-bf16 choice on blocked copies as tile +
    1000), and a second plan of the same shapes takes the same tiles."""
    f = tmp_path / "tune.txt"
    monkeypatch.setenv("CC_AUTOTUNE_CACHE", str(f))
    o, v = 7, 29  # shapes no other test tunes, so the choices are new
    d = E.DeviceSystem(make_system(o, v, 12))
    t1, t2 = E.zeros_amps(d, E.CCSD)
    tags = []
    for _ in range(2):
        with E.Plan(ctx, d, E.CCSD) as p:
            p.autotune(t1, t2)
            p.profile(True)
            p.residual(t1, t2)
            tags.append([r[2] for r in p.profile_table() if r[1] == "GEMM"])
    lines = f.read_text().split("\n")
    entries = [ln.split() for ln in lines if ln.strip()]
    assert entries and all(len(e) == 2 and ":" in e[0] and 0 <= int(e[1]) < 1000 for e in entries)
    assert len({e[0] for e in entries}) == len(entries)  # each shape tuned once
    assert tags[0] == tags[1]


def test_plan_step_matches_iterate(E, ctx):
    o, v = 5, 19
    s = make_system(o, v, 8)
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    with E.Plan(ctx, d, E.CCSD) as p:
        hist = []
        for _ in range(4):
            p.step(t1, t2, 0.0)
            hist.append(p.scalars()[1])
    u1, u2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, u1, u2, tol=1e-30, max_iter=4, use_graph=False)
    assert hist == out["hist_e"]
    assert torch.equal(t2, u2)


def test_abi_errors_on_device(E, ctx):
    from paper_2409_06759_amd import _lib as L
    s = make_system(3, 5, 1)
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    with pytest.raises(L.CCError) as ei:  # CCD must not get t1
        E.residual(ctx, d, E.CCD, t1, t2)
    assert ei.value.status == L.CC_EINVAL
    bad = torch.zeros(3 * 3 * 5 * 5 + 1, dtype=torch.float64, device="cuda")[1:].view(3, 3, 5, 5)
    with pytest.raises(L.CCError) as ei:  # misaligned pointer
        E.residual(ctx, d, E.CCD, None, bad)
    assert ei.value.status == L.CC_EINVAL
    nan_sys = make_system(3, 5, 1)
    blk = nan_sys.block("oovv").copy()
    blk[0, 1, 0, 1] = np.nan
    nan_sys._blocks["oovv"] = blk
    dn = E.DeviceSystem(nan_sys)
    u1, u2 = E.zeros_amps(dn, E.CCSD)
    out = E.iterate(ctx, dn, E.CCSD, u1, u2, tol=1e-8, max_iter=5)
    assert out["status"] == L.CC_EDIVERGED
    u1, u2 = E.zeros_amps(d, E.CCSD)
    out = E.iterate(ctx, d, E.CCSD, u1, u2, tol=1e-8, max_iter=1)
    assert out["status"] == L.CC_ENOTCONV


@pytest.mark.parametrize("method", ["ccd", "ccsd"])
def test_dressed_denominator_trajectory(E, ctx, method):
    o, v = 6, 30
    s = make_system(o, v, 78)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    ref = jacobi(F, V, method, tol=0.0, max_iter=7, dressed=True, level_shift=0.25)
    d = E.DeviceSystem(s)
    m = E.METHODS[method]
    t1, t2 = E.zeros_amps(d, m)
    out = E.iterate(ctx, d, m, t1, t2, tol=1e-30, max_iter=7, level_shift=0.25, dressed=True)
    assert np.allclose(out["hist_e"], ref["hist_e"], rtol=0, atol=1e-12)
    assert np.abs(t2.cpu().numpy() - ref["t2"]).max() < 1e-12
    if method == "ccsd":
        assert np.abs(t1.cpu().numpy() - ref["t1"]).max() < 1e-12


@pytest.mark.parametrize("prec,tol", [("f32", 2e-6), ("bf16x3", 5e-5)])
@pytest.mark.parametrize("ov", [(3, 5), (8, 24)])
def test_reduced_precision_residual(E, ctx, prec, tol, ov):
    """Residual with reduced-precision contractions against the FP64 oracle.
    Terms are O(1e-2) with at most v^2 = 576 products each: FP32 gives
    <= 576 * 2^-24 * 1e-2 ~ 3e-7 per GEMM, split-bf16 adds ~3 * 2^-17 * 1e-2."""
    o, v = ov
    s = make_system(o, v, 2000 + o * v)
    t1, t2 = _amps(o, v, o * v)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    r1_ref, r2_ref = residual(F, V, t1, t2)
    d = E.DeviceSystem(s)
    r1, r2, rn = E.residual(ctx, d, E.CCSD, torch.from_numpy(t1).cuda(), torch.from_numpy(t2).cuda(),
                            prec=E.PRECS[prec])
    r2 = r2.cpu().numpy()
    assert np.abs(r2 - r2_ref).max() < tol
    assert np.abs(r1.cpu().numpy() - r1_ref).max() < tol
    assert np.array_equal(r2, -r2.transpose(1, 0, 2, 3))


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_mixed_precision_refines_to_fp64_solution(E, ctx, prec):
    o, v = 8, 24
    s = make_system(o, v)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    ref = jacobi(F, V, "ccsd", tol=1e-11, max_iter=100, dressed=True)
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    for corr in (False, True):
        t1, t2 = E.zeros_amps(d, E.CCSD)
        out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-10, max_iter=100, prec=E.PRECS[prec], dressed=True,
                        correction=corr)
        print(f"{prec} correction={corr}: {out['iters']} it, {out['lowp_iters']} reduced, "
              f"{out['corr_iters']} corrected, dE={abs(out['energy'] - ref['energy']):.2e}", flush=True)
        assert out["converged"]
        assert 0 < out["lowp_iters"] < out["iters"]
        assert (out["corr_iters"] > 0) == corr
        assert abs(out["energy"] - ref["energy"]) < 1e-10


@pytest.mark.parametrize("cplx", [False, True])
def test_blocked_split_bf16_copies_in_plans(E, ctx, cplx):
    """At o=16, v=64 the ladder, Z, the ring terms and W_mnij's tau term are
    large enough for the split-bf16 copies in 16 x 32 blocks (complex: of
    the realified operands); after autotuning, the plain split-bf16 residual
    and the reference + correction one keep the errors they have with
    row-major copies (a wrong block layout would make them of the order of
    the residual itself)."""
    o, v = 16, 64
    s = make_system(o, v, 43, is_complex=cplx)
    d = E.DeviceSystem(s)
    rng = np.random.default_rng(10)

    def amps(scale):
        a1 = rng.normal(size=(o, v)) * scale
        a2 = rng.normal(size=(o, o, v, v)) * scale
        if cplx:
            a1 = a1 + 1j * rng.normal(size=(o, v)) * scale
            a2 = a2 + 1j * rng.normal(size=(o, o, v, v)) * scale
        a2 = a2 - a2.transpose(1, 0, 2, 3)
        a2 = a2 - a2.transpose(0, 1, 3, 2)
        return a1, a2

    r1, r2 = amps(0.02)
    d1, d2 = amps(1e-6)
    t_ref = [torch.from_numpy(x).cuda() for x in (r1, r2)]
    t_new = [torch.from_numpy(x).cuda() for x in (r1 + d1, r2 + d2)]

    def res(plan, t):
        q1, q2, _ = plan.residual(t[0], t[1])
        return torch.cat([q1.flatten(), q2.flatten()]).cpu().numpy()

    with E.Plan(ctx, d, E.CCSD) as p64:
        exact_ref, exact_new = res(p64, t_ref), res(p64, t_new)
    scale = np.abs(exact_new).max()
    with E.Plan(ctx, d, E.CCSD, prec=E.PRECS["bf16x3"]) as p:
        p.autotune(t_ref[0], t_ref[1])
        p.profile(True)
        plain = res(p, t_new)
        tags = [row[2] for row in p.profile_table() if row[1] == "GEMM"]
        p.profile(False)
        plain_err = np.abs(plain - exact_new).max()
        p.set_precision(E.F64)
        p.set_correction(1, E.PRECS["bf16x3"])
        at_ref = res(p, t_ref)
        corrected = res(p, t_new)
    print(f"complex {cplx}: blocked tags {[t for t in tags if t.endswith('/blk')]}; plain {plain_err:.2e}, "
          f"corrected {np.abs(corrected - exact_new).max():.2e} (|R| {scale:.2e})", flush=True)
    assert any(t.endswith("/blk") for t in tags)
    assert plain_err < 1e-4 * scale
    assert np.abs(at_ref - exact_ref).max() < 1e-13 * max(1.0, scale)
    assert np.abs(corrected - exact_new).max() < 1e-3 * plain_err


@pytest.mark.parametrize("prec,eps", [("f32", 2.0 ** -24), ("bf16x3", 2.0 ** -16)])
def test_correction_form_error_scales_with_the_change(E, ctx, prec, eps):
    """Reference + correction: at the reference amplitudes the residual is
    the FP64 one; at t_ref + delta its error is about eps * |delta| terms,
    far below the plain reduced-precision residual's error."""
    o, v = 6, 28
    s = make_system(o, v, 41)
    d = E.DeviceSystem(s)
    rng = np.random.default_rng(9)

    def amps(scale):
        a1 = rng.normal(size=(o, v)) * scale
        a2 = rng.normal(size=(o, o, v, v)) * scale
        a2 = a2 - a2.transpose(1, 0, 2, 3)
        a2 = a2 - a2.transpose(0, 1, 3, 2)
        return a1, a2

    r1, r2 = amps(0.05)
    d1, d2 = amps(1e-6)
    t_ref = [torch.from_numpy(x).cuda() for x in (r1, r2)]
    t_new = [torch.from_numpy(x).cuda() for x in (r1 + d1, r2 + d2)]

    def res(plan, t):
        q1, q2, _ = plan.residual(t[0], t[1])
        return torch.cat([q1.flatten(), q2.flatten()]).cpu().numpy()

    with E.Plan(ctx, d, E.CCSD) as p64:
        exact_ref, exact_new = res(p64, t_ref), res(p64, t_new)
    with E.Plan(ctx, d, E.CCSD, prec=E.PRECS[prec]) as p:
        plain_err = np.abs(res(p, t_new) - exact_new).max()
        p.set_precision(E.F64)
        p.set_correction(1, E.PRECS[prec])
        at_ref = res(p, t_ref)      # stores the reference
        corrected = res(p, t_new)   # reference + correction
    scale = np.abs(exact_new).max()
    print(f"{prec}: plain {plain_err:.2e}, at ref {np.abs(at_ref - exact_ref).max():.2e}, "
          f"corrected {np.abs(corrected - exact_new).max():.2e} (|R| {scale:.2e})", flush=True)
    assert np.abs(at_ref - exact_ref).max() < 1e-13 * max(1.0, scale)
    assert np.abs(corrected - exact_new).max() < 1e-3 * plain_err
    assert np.abs(corrected - exact_new).max() < 1e3 * eps * 1e-6 * max(1.0, scale)


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_batched_norm_readback_reports_the_same_convergence(E, ctx, prec):
    """check_every = 5 launches five steps per synchronisation.  In FP64 the
    reported iteration count, norm, energy and history are those of
    check_every = 1; with reduced precision the switch to FP64 acts from the
    next batch, so the path differs by a few steps but not the solution."""
    o, v = 8, 30
    s = make_system(o, v, 14)
    d = E.DeviceSystem(s)
    out = {}
    for k in (1, 5):
        t1, t2 = E.zeros_amps(d, E.CCSD)
        out[k] = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-10, max_iter=200, dressed=True, prec=E.PRECS[prec],
                           check_every=k)
    assert out[5]["converged"] and out[1]["converged"]
    if prec == "f64":
        assert out[5]["iters"] == out[1]["iters"]
        assert out[5]["energy"] == out[1]["energy"] and out[5]["rnorm"] == out[1]["rnorm"]
        assert out[5]["hist_e"] == out[1]["hist_e"]
    else:
        assert abs(out[5]["iters"] - out[1]["iters"]) <= 10
        assert abs(out[5]["energy"] - out[1]["energy"]) < 1e-10


@pytest.mark.parametrize("prec,kc", [("f64", False), ("f32", True), ("bf16x3", True)])
def test_hole_hole_ladder_layout_follows_plan_precision(E, ctx, prec, kc):
    """Plans made for a reduced precision read both operands of the hole-hole
    ladder K-contiguous (tau permuted to [ab][mn], W to [ij][mn]); FP64 plans
    read the stored [mn][ij] and [mn][ab] layouts."""
    d = E.DeviceSystem(make_system(4, 12))
    with E.Plan(ctx, d, E.CCSD, E.PRECS[prec]) as p:
        line = next(s for s in p.describe().splitlines() if s.startswith("GEMM hh_ladder "))
    assert (" sak=1 " in line and " sbk=1 " in line) == kc, line


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_complex_mixed_precision_refines_to_fp64_solution(E, ctx, prec):
    """Complex CCSD with reduced-precision contractions, then the FP64 phase
    (plain and in reference + correction form): the converged energy equals
    the FP64 solve's."""
    o, v = 6, 20
    s = make_system(o, v, 77, is_complex=True)
    d = E.DeviceSystem(s)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    ref = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-11, max_iter=200, dressed=True)
    assert ref["converged"]
    for corr in (False, True):
        t1, t2 = E.zeros_amps(d, E.CCSD)
        out = E.iterate(ctx, d, E.CCSD, t1, t2, tol=1e-10, max_iter=200, prec=E.PRECS[prec], dressed=True,
                        correction=corr)
        print(f"complex {prec} correction={corr}: {out['iters']} it, {out['lowp_iters']} reduced, "
              f"{out['corr_iters']} corrected, dE={abs(out['energy'] - ref['energy']):.2e}", flush=True)
        assert out["converged"]
        assert 0 < out["lowp_iters"] < out["iters"]
        assert (out["corr_iters"] > 0) == corr
        assert abs(out["energy"] - ref["energy"]) < 1e-10


@pytest.mark.parametrize("prec,eps", [("f32", 2.0 ** -24), ("bf16x3", 2.0 ** -16)])
def test_complex_correction_form_error_scales_with_the_change(E, ctx, prec, eps):
    """Complex reference + correction: exact at the reference; at t_ref + delta
    the error is about eps * |delta| terms, far below the plain error."""
    o, v = 6, 28
    s = make_system(o, v, 43, is_complex=True)
    d = E.DeviceSystem(s)
    r1, r2 = _amps(o, v, 11, scale=0.05, cplx=True)
    d1, d2 = _amps(o, v, 12, scale=1e-6, cplx=True)
    t_ref = [torch.from_numpy(x).cuda() for x in (r1, r2)]
    t_new = [torch.from_numpy(x).cuda() for x in (r1 + d1, r2 + d2)]

    def res(plan, t):
        q1, q2, _ = plan.residual(t[0], t[1])
        return torch.cat([q1.flatten(), q2.flatten()]).cpu().numpy()

    with E.Plan(ctx, d, E.CCSD) as p64:
        exact_ref, exact_new = res(p64, t_ref), res(p64, t_new)
    with E.Plan(ctx, d, E.CCSD, prec=E.PRECS[prec]) as p:
        plain_err = np.abs(res(p, t_new) - exact_new).max()
        p.set_precision(E.F64)
        p.set_correction(1, E.PRECS[prec])
        at_ref = res(p, t_ref)
        corrected = res(p, t_new)
    scale = np.abs(exact_new).max()
    print(f"complex {prec}: plain {plain_err:.2e}, at ref {np.abs(at_ref - exact_ref).max():.2e}, "
          f"corrected {np.abs(corrected - exact_new).max():.2e} (|R| {scale:.2e})", flush=True)
    assert np.abs(at_ref - exact_ref).max() < 1e-13 * max(1.0, scale)
    assert np.abs(corrected - exact_new).max() < 1e-3 * plain_err
    assert np.abs(corrected - exact_new).max() < 1e3 * eps * 1e-6 * max(1.0, scale)
