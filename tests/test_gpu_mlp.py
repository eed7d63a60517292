"""Amplitude-guess network on the GPU against the FP64 oracle network, and
what the trained network gains over the plain MP2 guess."""
import numpy as np
import pytest

from ccinputs.synth import make_system
from oracle import mlp as ref
from oracle.cc import Fock, denominators
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


def _stats():
    return dict(sx=0.01, mD=-5.0, sD=2.0, me=-0.05, se=0.03, st=0.002)


def test_features_match_oracle(E, ctx):
    o, v = 5, 13
    s = make_system(o, v, 31)
    d = E.DeviceSystem(s)
    got = E.MLP.raw_features(ctx, d).cpu().numpy()
    _, d2 = denominators(Fock.from_system(s))
    want = ref.raw_features(Integrals.from_system(s).get("oovv"), d2)
    assert np.allclose(got, want, rtol=1e-14, atol=1e-18)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-5)])
def test_forward_and_gradient_match_oracle(E, ctx, prec, tol):
    """FP64 dense layers agree to rounding; FP32 MFMA layers to ~K 2^-24."""
    rng = np.random.default_rng(3)
    p = ref.init_params(5)
    z = rng.normal(size=(700, 3))
    y = rng.normal(size=700) * 0.5
    P = torch.from_numpy(ref.flatten(p)).cuda()
    net = E.MLP(ctx, P, _stats(), E.PRECS[prec])
    f = net.forward(torch.from_numpy(z).cuda()).cpu().numpy()
    f_ref = ref.forward(p, z)
    assert np.abs(f - f_ref).max() < tol * max(1.0, np.abs(f_ref).max())
    loss, g = net.loss_grad(torch.from_numpy(z).cuda(), torch.from_numpy(y).cuda())
    loss_ref, g_ref = ref.loss_and_grad(p, z, y)
    gv, gr = g.cpu().numpy(), ref.flatten(g_ref)
    assert abs(loss - loss_ref) < tol * max(1.0, loss_ref)
    assert np.abs(gv - gr).max() < tol * max(1.0, np.abs(gr).max())


def test_adam_training_matches_oracle(E, ctx):
    rng = np.random.default_rng(4)
    p = ref.init_params(6)
    z = rng.normal(size=(96, 3))
    y = rng.normal(size=96) * 0.3
    net = E.MLP(ctx, torch.from_numpy(ref.flatten(p)).cuda(), _stats(), E.F64)
    hist = net.train(torch.from_numpy(z).cuda(), torch.from_numpy(y).cuda(), epochs=3, batch=32, lr=1e-3)
    opt = ref.Adam(lr=1e-3)
    vec = ref.flatten(p)
    losses = []
    for _ in range(3):
        ep = []
        for s0 in range(0, 96, 32):
            l_, g_ = ref.loss_and_grad(ref.unflatten(vec), z[s0:s0 + 32], y[s0:s0 + 32])
            ep.append(l_)
            vec = opt.step(vec, ref.flatten(g_))
        losses.append(np.mean(ep))
    got = net.params.cpu().numpy()
    # b3 (last parameter) cancels in f = (g(z) - g(-z))/2, so its gradient is
    # zero up to summation rounding, which Adam's normalisation magnifies to
    # ~lr * noise / eps on both sides independently; it stays near zero.
    assert np.abs(got[:-1] - vec[:-1]).max() < 1e-11
    assert abs(got[-1]) < 1e-9 and abs(vec[-1]) < 1e-9
    assert np.allclose(hist, losses, rtol=1e-11, atol=0)


def test_guess_matches_oracle_and_is_antisymmetric(E, ctx):
    o, v = 6, 15
    s = make_system(o, v, 32)
    d = E.DeviceSystem(s)
    p = ref.init_params(7)
    net = E.MLP(ctx, torch.from_numpy(ref.flatten(p)).cuda(), _stats(), E.F64)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    t1.fill_(1.0)
    net.guess(d, t1, t2)
    g = t2.cpu().numpy()
    _, d2 = denominators(Fock.from_system(s))
    want = ref.predict_t2(p, _stats(), Integrals.from_system(s).get("oovv"), d2)
    assert np.abs(g - want).max() < 1e-12
    assert np.array_equal(g, -g.transpose(1, 0, 2, 3)) and np.array_equal(g, -g.transpose(0, 1, 3, 2))
    assert torch.all(t1 == 0)


def test_trained_network_gains_over_mp2(E, ctx):
    """Train on converged amplitudes of small generated systems, then start a
    held-out system from the network's guess and from MP2: the network's
    guess has the smaller residual and needs no more iterations."""
    from paper_2409_06759_amd import learned
    shapes = learned.training_shapes(24, o_range=(4, 8), v_range=(16, 32))
    raw, y = learned.generate(ctx, shapes, tol=1e-9, group=12)
    net, hist = learned.train(ctx, raw, y, epochs=30, batch=4096, lr=2e-3, prec=E.F32)
    assert hist[-1] < 0.5 * hist[0]
    res = learned.evaluate(ctx, net, o=8, v=34, seed=424242, tol=1e-8, max_iter=300)
    print("gain:", res["iterations_saved"], "iterations;", res["rnorm_guess"], flush=True)
    assert res["mlp"]["converged"] and res["mp2"]["converged"]
    assert abs(res["mlp"]["energy"] - res["mp2"]["energy"]) < 1e-8
    assert res["rnorm_guess"]["mlp"] < res["rnorm_guess"]["mp2"]
    # weakly correlated small systems: most of t - t_MP2 comes from ladder and
    # ring sums that per-amplitude features cannot see, so the gain in
    # iterations is small; it must not be a loss
    assert res["mlp"]["iterations"] <= res["mp2"]["iterations"]


def test_iterate_guess_option(E, ctx):
    """cc_iterate's guess option.  MP2: the start is the zero start's first
    iterate, so the run is the zero-start run shifted by one iteration.  MLP:
    the network's amplitudes unless the MP2 ones have the smaller FP64
    residual norm; both candidate norms are reported and the first iteration
    evaluates the chosen one."""
    o, v = 8, 24
    s = make_system(o, v)
    d = E.DeviceSystem(s)
    z1, z2 = E.zeros_amps(d, E.CCSD)
    ref_run = E.iterate(ctx, d, E.CCSD, z1, z2, tol=1e-10, max_iter=200, dressed=True)
    g1, g2 = E.zeros_amps(d, E.CCSD)
    g2.fill_(1.0)  # overwritten by the guess
    mp = E.iterate(ctx, d, E.CCSD, g1, g2, tol=1e-10, max_iter=200, dressed=True, guess="mp2")
    assert mp["guess_used"] == "mp2"
    assert abs(mp["hist_rnorm"][0] - ref_run["hist_rnorm"][1]) < 1e-12 * ref_run["hist_rnorm"][1]
    assert mp["iters"] == ref_run["iters"] - 1
    assert abs(mp["energy"] - ref_run["energy"]) < 1e-12
    params = E.MLP.init_params(3, "cuda")
    # output scale 0: the network's t2 is exactly zero, whose norm is the zero start's
    zero_net = E.MLP(ctx, params, dict(_stats(), st=0.0), E.F64)
    a1, a2 = E.zeros_amps(d, E.CCSD)
    r = E.iterate(ctx, d, E.CCSD, a1, a2, tol=1e-10, max_iter=200, dressed=True, guess="mlp", mlp=zero_net)
    assert abs(r["guess_rnorm"]["mlp"] - ref_run["hist_rnorm"][0]) < 1e-12 * ref_run["hist_rnorm"][0]
    assert abs(r["guess_rnorm"]["mp2"] - ref_run["hist_rnorm"][1]) < 1e-12 * ref_run["hist_rnorm"][1]
    want = "mlp" if r["guess_rnorm"]["mlp"] <= r["guess_rnorm"]["mp2"] else "mp2"
    assert r["guess_used"] == want
    assert abs(r["hist_rnorm"][0] - min(r["guess_rnorm"].values())) < 1e-12 * r["hist_rnorm"][0]
    assert abs(r["energy"] - ref_run["energy"]) < 1e-12
    # an output scale far beyond the amplitudes: the MP2 start is kept
    wild = E.MLP(ctx, params, dict(_stats(), st=1e3), E.F32)
    b1, b2 = E.zeros_amps(d, E.CCSD)
    w = E.iterate(ctx, d, E.CCSD, b1, b2, tol=1e-10, max_iter=200, dressed=True, guess="mlp", mlp=wild)
    assert w["guess_used"] == "mp2" and w["guess_rnorm"]["mlp"] > w["guess_rnorm"]["mp2"]
    assert w["iters"] == mp["iters"] and abs(w["energy"] - ref_run["energy"]) < 1e-12
    assert w["guess_seconds"] > 0


@pytest.mark.parametrize("n", [1, 17, 50017])
def test_fused_fp32_forward_matches_oracle(E, ctx, n):
    """FP32 inference is one fused launch (layer 1 in registers, layer 2 on
    FP32 MFMA with W2 in LDS, bias, ReLU and the output layer on the
    accumulators): against the FP64 oracle network to ~K 2^-24, for sample
    counts that leave a ragged last group of 16 and span many workgroups."""
    rng = np.random.default_rng(n)
    p = ref.init_params(8)
    z = rng.normal(size=(n, 3))
    net = E.MLP(ctx, torch.from_numpy(ref.flatten(p)).cuda(), _stats(), E.F32)
    f = net.forward(torch.from_numpy(z).cuda()).cpu().numpy()
    f_ref = ref.forward(p, z)
    assert f.shape == f_ref.shape
    assert np.abs(f - f_ref).max() < 2e-5 * max(1.0, np.abs(f_ref).max())


def test_fp32_guess_matches_oracle(E, ctx):
    o, v = 7, 19
    s = make_system(o, v, 33)
    d = E.DeviceSystem(s)
    p = ref.init_params(9)
    net = E.MLP(ctx, torch.from_numpy(ref.flatten(p)).cuda(), _stats(), E.F32)
    t1, t2 = E.zeros_amps(d, E.CCSD)
    net.guess(d, t1, t2)
    g = t2.cpu().numpy()
    _, d2 = denominators(Fock.from_system(s))
    want = ref.predict_t2(p, _stats(), Integrals.from_system(s).get("oovv"), d2)
    assert np.abs(g - want).max() < 2e-5 * np.abs(want).max()
    assert np.array_equal(g, -g.transpose(1, 0, 2, 3)) and np.array_equal(g, -g.transpose(0, 1, 3, 2))
