"""Pins of the FP64 amplitude-guess network (CPU): analytic gradients
against central finite differences, exact oddness in <ij||ab>, the pair
energies against the MP2 closed form, the first Adam step against its
closed form, and the parameter count."""
import numpy as np

from ccinputs.synth import make_system
from oracle import mlp
from oracle.cc import Fock, denominators
from oracle.integrals import Integrals


def _data(n=40, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 3)), rng.normal(size=n) * 0.3


def test_parameter_count():
    assert mlp.N_PARAMS == 17153


def test_gradient_matches_finite_differences():
    p = mlp.init_params(3)
    z, y = _data()
    _, g = mlp.loss_and_grad(p, z, y)
    vec = mlp.flatten(p)
    gvec = mlp.flatten(g)
    rng = np.random.default_rng(1)
    idx = rng.choice(vec.size, 60, replace=False)
    h = 1e-6
    for k in idx:
        vp, vm = vec.copy(), vec.copy()
        vp[k] += h
        vm[k] -= h
        lp, _ = mlp.loss_and_grad(mlp.unflatten(vp), z, y)
        lm, _ = mlp.loss_and_grad(mlp.unflatten(vm), z, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gvec[k]) < 1e-7 * max(1.0, abs(fd)), (k, fd, gvec[k])


def test_network_is_odd_in_the_integral():
    p = mlp.init_params(4)
    p["b3"][:] = 0.7  # the bias cancels in f
    z, _ = _data(25, 2)
    zn = z.copy()
    zn[:, 0] = -zn[:, 0]
    assert np.array_equal(mlp.forward(p, zn), -mlp.forward(p, z))


def test_pair_energies_sum_to_mp2_and_t2_antisymmetric():
    o, v = 4, 9
    s = make_system(o, v, 5)
    F, V = Fock.from_system(s), Integrals.from_system(s)
    _, d2 = denominators(F)
    g = V.get("oovv")
    raw = mlp.raw_features(g, d2)
    n_ab = v * (v - 1) // 2
    e_pairs = raw[::n_ab, 2]
    assert abs(e_pairs.sum() - 0.25 * np.sum(g * g / d2)) < 1e-15
    stats = dict(sx=0.01, mD=-5.0, sD=2.0, me=-0.1, se=0.05, st=0.002)
    t2 = mlp.predict_t2(mlp.init_params(0), stats, g, d2)
    assert np.array_equal(t2, -t2.transpose(1, 0, 2, 3))
    assert np.array_equal(t2, -t2.transpose(0, 1, 3, 2))


def test_adam_first_step_closed_form():
    opt = mlp.Adam(lr=0.01)
    x = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    x1 = opt.step(x, g)
    assert np.allclose(x1, x - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
