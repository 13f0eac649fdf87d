"""Pins of the oracle's forward models and analytic Jacobians: closed forms
(Eq. 3), special cases that reduce to another model or to a library
routine, invariances, and central finite differences."""
import math

import numpy as np
import pytest
from scipy import special

TE12 = 2.0 + 4.0 * np.arange(12)


def test_monoexp_closed_form(orc):
    te = np.array([0.0, 30.0, 60.0])
    th = np.array([[1.7], [30.0]])
    s = orc.forward("monoexp_t2s", orc.Acq(te=te), th)[:, 0]
    assert s[0] == pytest.approx(1.7, rel=1e-15)
    assert s[1] == pytest.approx(1.7 / math.e, rel=1e-14)
    assert s[2] == pytest.approx(1.7 / math.e**2, rel=1e-14)


def test_r2s_is_t2s_with_reciprocal_rate(orc):
    th_t = np.array([[1.2, 0.8], [25.0, 60.0]])
    th_r = np.array([[1.2, 0.8], [1000.0 / 25.0, 1000.0 / 60.0]])
    a = orc.forward("monoexp_t2s", orc.Acq(te=TE12), th_t)
    b = orc.forward("monoexp_r2s", orc.Acq(te=TE12), th_r)
    np.testing.assert_allclose(a, b, rtol=1e-13)


def test_linear3_is_matrix_product_and_linear(orc):
    rng = np.random.default_rng(0)
    A = rng.uniform(-1, 1, (3, 7))
    s = orc.forward("linear3", orc.Acq(te=TE12), A)
    # a single active basis function is a mono-exponential with T2 = tau
    for k, tau in enumerate((10.0, 30.0, 80.0)):
        e = np.zeros((3, 1))
        e[k, 0] = 1.0
        ref = orc.forward("monoexp_t2s", orc.Acq(te=TE12), np.array([[1.0], [tau]]))
        np.testing.assert_allclose(orc.forward("linear3", orc.Acq(te=TE12), e), ref, rtol=1e-14)
    # and the model is the product of the Jacobian (the basis) with A
    Phi = orc.jacobian("linear3", orc.Acq(te=TE12), A[:, :1])[0]
    np.testing.assert_allclose(s, Phi @ A, rtol=1e-13)
    B = rng.uniform(-1, 1, (3, 7))
    np.testing.assert_allclose(orc.forward("linear3", orc.Acq(te=TE12), A + 2 * B),
                               s + 2 * orc.forward("linear3", orc.Acq(te=TE12), B),
                               rtol=1e-12, atol=1e-14)


def test_gre3_single_pool_reduces_to_monoexp(orc):
    te = 2.0 + 2.0 * np.arange(24)
    th = np.array([0.7, 0, 0, 12.0, 50.0, 30.0, 0.0, 3.0, -2.0])[:, None]
    s = orc.forward("gre3", orc.Acq(te=te), th)
    ref = orc.forward("monoexp_t2s", orc.Acq(te=te), np.array([[0.7], [12.0]]))
    np.testing.assert_allclose(s[:24], ref, rtol=1e-14)
    np.testing.assert_allclose(s[24:], 0.0, atol=1e-16)


def test_gre3_phase_sign_and_units(orc):
    # 25 Hz for 10 ms is a quarter turn: positive frequency -> +i
    th = np.array([0.5, 0, 0, 20.0, 50.0, 30.0, 25.0, 0.0, 0.0])[:, None]
    s = orc.forward("gre3", orc.Acq(te=np.array([10.0, 20.0])), th)
    mag = 0.5 * math.exp(-10.0 / 20.0)
    assert s[0, 0] == pytest.approx(0.0, abs=1e-15)
    assert s[2, 0] == pytest.approx(mag, rel=1e-14)
    # 20 ms is half a turn: -1 times the magnitude
    assert s[1, 0] == pytest.approx(-0.5 * math.exp(-1.0), rel=1e-14)
    assert s[3, 0] == pytest.approx(0.0, abs=1e-15)


def test_gre3_pools_superpose(orc):
    te = 2.0 + 2.0 * np.arange(24)
    th = np.array([0.2, 0.5, 0.3, 10.0, 55.0, 30.0, 4.0, -3.0, 1.5])
    tot = orc.forward("gre3", orc.Acq(te=te), th[:, None])
    parts = 0
    for k in range(3):
        t = th.copy()
        t[[j for j in range(3) if j != k]] = 0.0
        parts = parts + orc.forward("gre3", orc.Acq(te=te), t[:, None])
        # each pool alone keeps |s| = A exp(-TE/T2*) whatever its frequency
        one = orc.forward("gre3", orc.Acq(te=te), t[:, None])
        np.testing.assert_allclose(np.hypot(one[:24, 0], one[24:, 0]),
                                   th[k] * np.exp(-te / th[3 + k]), rtol=1e-13)
    np.testing.assert_allclose(tot, parts, rtol=1e-13, atol=1e-16)


def _dwi(orc, b, g):
    return orc.Acq(bval=np.asarray(b, float), bvec=np.asarray(g, float))


def test_dwi2_special_cases(orc):
    g = np.array([[0, 0, 1.0], [1.0, 0, 0], [0, 1.0, 0]])
    b = np.array([1000.0, 2000.0, 3000.0])
    # fibre along z (theta = 0)
    th = np.array([[1.0], [2.0], [1.0], [0.0], [0.3]])
    s = orc.forward("dwi2", _dwi(orc, b, g), th)[:, 0]
    assert s[0] == pytest.approx(math.exp(-1000e-3 * 2.0), rel=1e-14)   # g parallel n
    assert s[1] == pytest.approx(1.0, abs=1e-15)                          # g perpendicular
    assert s[2] == pytest.approx(1.0, abs=1e-15)
    # ball only: isotropic
    th0 = np.array([[0.0], [2.0], [1.5], [0.7], [1.1]])
    s0 = orc.forward("dwi2", _dwi(orc, b, g), th0)[:, 0]
    np.testing.assert_allclose(s0, np.exp(-b * 1e-3 * 1.5), rtol=1e-14)


def test_dwi2_antipodal_symmetry(orc):
    rng = np.random.default_rng(1)
    g = rng.standard_normal((40, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    b = np.full(40, 2000.0)
    th = np.array([[0.6], [2.2], [0.9], [0.4], [1.0]])
    th2 = th.copy()
    th2[3] = math.pi - th[3]
    th2[4] = th[4] + math.pi
    np.testing.assert_allclose(orc.forward("dwi2", _dwi(orc, b, g), th),
                               orc.forward("dwi2", _dwi(orc, b, g), th2), rtol=1e-13)


def test_dwi2_stick_spherical_mean(orc):
    # mean over directions of exp(-bD (g.n)^2) = sqrt(pi/(4bD)) erf(sqrt(bD))
    nd = 20000
    k = np.arange(nd) + 0.5
    zc = 1 - 2 * k / nd
    ph = math.pi * (1 + 5 ** 0.5) * k
    rr = np.sqrt(1 - zc**2)
    g = np.stack([rr * np.cos(ph), rr * np.sin(ph), zc], 1)    # Fibonacci sphere
    for bval, D in [(1000.0, 2.0), (3000.0, 1.2)]:
        s = orc.forward("dwi2", _dwi(orc, np.full(nd, bval), g),
                        np.array([[1.0], [D], [1.0], [0.3], [0.8]]))
        bd = bval * 1e-3 * D
        ref = math.sqrt(math.pi / (4 * bd)) * special.erf(math.sqrt(bd))
        assert s.mean() == pytest.approx(ref, rel=2e-6)


MODELS = {
    "monoexp_t2s": (dict(te=TE12), [1.1, 37.0]),
    "monoexp_r2s": (dict(te=TE12), [0.9, 31.0]),
    "linear3": (dict(te=TE12), [0.3, -0.4, 0.8]),
    "gre3": (dict(te=2.0 + 2.0 * np.arange(24)), [0.2, 0.5, 0.3, 9.0, 55.0, 31.0, 3.0, -4.0, 1.2]),
}


def _dwi_acq(seed=2):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((30, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return dict(bval=np.repeat([1000.0, 2000.0, 3000.0], 10), bvec=g)


@pytest.mark.parametrize("model", ["monoexp_t2s", "monoexp_r2s", "linear3", "gre3", "dwi2"])
def test_jacobian_matches_central_fd(orc, model):
    if model == "dwi2":
        acq, th = _dwi_acq(), [0.55, 2.1, 0.8, 0.7, -1.3]
    else:
        acq, th = MODELS[model]
    acq = orc.Acq(**acq)
    th = np.array(th, dtype=float)
    J = orc.jacobian(model, acq, th[:, None])[0]
    for p in range(len(th)):
        h = 1e-6 * max(1.0, abs(th[p]))
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (orc.forward(model, acq, tp[:, None]) - orc.forward(model, acq, tm[:, None]))[:, 0] / (2 * h)
        scale = max(np.abs(J[:, p]).max(), 1e-12)
        assert np.abs(fd - J[:, p]).max() / scale < 1e-6, (model, p)


def test_vjp_is_jacobian_transpose(orc):
    acq, th = MODELS["gre3"]
    acq = orc.Acq(**acq)
    rng = np.random.default_rng(3)
    thn = np.array(th)[:, None] * (1 + 0.01 * rng.standard_normal((9, 5)))
    ds = rng.standard_normal((48, 5))
    g = orc.vjp("gre3", acq, thn, ds)
    J = orc.jacobian("gre3", acq, thn)
    np.testing.assert_allclose(g, np.einsum("nmp,mn->pn", J, ds), rtol=1e-12, atol=1e-14)
