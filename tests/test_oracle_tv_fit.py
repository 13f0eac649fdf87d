"""Pins of the oracle's total-variation term (Eq. 5) and of the askadam
solver (Eq. 2/4 with Adam, SGDM, RMSProp and the stopping rules)."""
import math

import numpy as np
import pytest

from paper_2511_22094_amd import synth


# ---------------------------------------------------------------- TV
def test_tv_constant_is_zero(orc):
    mask = np.ones((3, 4, 5), np.uint8)
    R, dR = orc.tv(mask, np.full(mask.shape, 0.3))
    assert R == 0.0 and np.all(dR == 0.0)


def test_tv_ramps_closed_form(orc):
    nz, ny, nx = 4, 5, 6
    mask = np.ones((nz, ny, nx), np.uint8)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c = 0.3, -0.7, 0.11
    u = a * x + b * y + c * z
    R3, _ = orc.tv(mask, u, 3)
    R2, _ = orc.tv(mask, u, 2)
    ex = abs(a) * (nx - 1) * ny * nz
    ey = abs(b) * nx * (ny - 1) * nz
    ez = abs(c) * nx * ny * (nz - 1)
    assert R3 == pytest.approx(ex + ey + ez, rel=1e-13)
    assert R2 == pytest.approx(ex + ey, rel=1e-13)


def test_tv_counts_only_pairs_inside_mask(orc):
    mask = np.zeros((3, 3, 3), np.uint8)
    mask[1, 1, 1] = 1          # isolated voxel: no pair
    mask[0, 0, 0] = mask[0, 0, 1] = 1   # one x pair
    u = np.random.default_rng(0).uniform(size=mask.shape)
    R, dR = orc.tv(mask, u, 3)
    assert R == pytest.approx(abs(u[0, 0, 1] - u[0, 0, 0]), rel=1e-14)
    assert dR[1, 1, 1] == 0.0
    assert np.count_nonzero(dR) == 2


@pytest.mark.parametrize("dim", [2, 3])
def test_tv_subgradient_matches_fd(orc, dim):
    rng = np.random.default_rng(dim)
    mask = np.ones((3, 3, 3), np.uint8)
    mask[0, 2, 2] = 0
    u = rng.uniform(size=mask.shape)
    R, dR = orc.tv(mask, u, dim)
    h = 1e-7
    for idx in np.ndindex(mask.shape):
        up, um = u.copy(), u.copy()
        up[idx] += h
        um[idx] -= h
        fd = (orc.tv(mask, up, dim)[0] - orc.tv(mask, um, dim)[0]) / (2 * h)
        assert fd == pytest.approx(dR[idx], abs=1e-6)


# ---------------------------------------------------------------- askadam
def _one_voxel():
    acq = synth.Acq(te=synth.echo_times(2.0, 4.0, 12))
    th = np.array([[1.1], [45.0]])
    return acq, th


def test_optimizer_first_steps(orc):
    acq, th = _one_voxel()
    lb, ub = synth.bounds("monoexp_t2s")
    mask = np.ones((1, 1, 1), np.uint8)
    y = orc.forward("monoexp_t2s", acq, th).reshape(12, 1, 1, 1) + 0.01
    # gradient at the midpoint in normalised coordinates
    mid = 0.5 * (lb + ub)
    _, g = orc.loss_grad("monoexp_t2s", acq, mid[:, None], y.reshape(12, 1), p=2,
                         scale=1.0 / 12)
    gu = (ub - lb) * g[:, 0]
    lr = 0.01
    r = orc.askadam("monoexp_t2s", acq, mask, y, lb, ub, n_iter=1, lr=lr)
    u1 = (r["maps"][:, 0, 0, 0] - lb) / (ub - lb)
    # bias-corrected first Adam step has length lr |g| / (|g| + eps), opposite to g
    np.testing.assert_allclose(u1 - 0.5, -lr * gu / (np.abs(gu) + 1e-8), rtol=1e-9)
    r = orc.askadam("monoexp_t2s", acq, mask, y, lb, ub, n_iter=1, lr=lr, optimizer="sgdm")
    u1 = (r["maps"][:, 0, 0, 0] - lb) / (ub - lb)
    np.testing.assert_allclose(u1 - 0.5, -lr * gu, rtol=1e-9)
    r = orc.askadam("monoexp_t2s", acq, mask, y, lb, ub, n_iter=1, lr=lr, optimizer="rmsprop",
                    rho=0.9)
    u1 = (r["maps"][:, 0, 0, 0] - lb) / (ub - lb)
    np.testing.assert_allclose(u1 - 0.5, -lr * gu / (math.sqrt(0.1) * np.abs(gu) + 1e-8),
                               rtol=1e-9)


def test_adam_linear3_reaches_least_squares(orc):
    rng = np.random.default_rng(4)
    acq = synth.Acq(te=synth.echo_times(2.0, 4.0, 12))
    A = rng.uniform(0.2, 1.0, (3, 6))
    y = orc.forward("linear3", acq, A) + 0.01 * rng.standard_normal((12, 6))
    y32 = y.astype(np.float32)
    mask = np.ones((1, 2, 3), np.uint8)
    lb, ub = np.full(3, -10.0), np.full(3, 10.0)
    r = orc.askadam("linear3", acq, mask, y32.reshape(12, 1, 2, 3), lb, ub, n_iter=20000,
                    lr=2e-3)
    Phi = orc.jacobian("linear3", acq, A[:, :1])[0]
    ols = np.linalg.lstsq(Phi, y32.astype(np.float64), rcond=None)[0]
    # constant-step Adam settles within ~1e-5 of the minimiser of this badly
    # conditioned quadratic (three correlated exponentials)
    fit = r["maps"].reshape(3, 6)
    np.testing.assert_allclose(fit, ols, atol=5e-5)
    res_fit = ((y32 - Phi @ fit) ** 2).sum(0)
    res_ols = ((y32 - Phi @ ols) ** 2).sum(0)
    np.testing.assert_allclose(res_fit, res_ols, rtol=5e-5)


def test_adam_noiseless_monoexp_recovers_truth(orc):
    d = synth.make_draw("monoexp_t2s", (1, 2, 4), 0, 0.0)
    y = orc.forward("monoexp_t2s", d.acq, d.truth).astype(np.float32)
    r = orc.askadam("monoexp_t2s", d.acq, d.mask, synth.scatter(y, d.mask), d.lb, d.ub,
                    n_iter=6000, lr=0.01)
    np.testing.assert_allclose(r["maps"].reshape(2, -1), d.truth, rtol=1e-4)


def test_no_regulariser_fits_voxels_independently(orc):
    # with eps = 0 Adam is invariant to the gradient scale, so the 1/N of the
    # whole-volume mean does not couple voxels
    d = synth.make_draw("monoexp_t2s", (1, 1, 3), 5, 0.01)
    y = (orc.forward("monoexp_t2s", d.acq, d.truth) + d.sigma * d.noise).astype(np.float32)
    whole = orc.askadam("monoexp_t2s", d.acq, d.mask, synth.scatter(y, d.mask), d.lb, d.ub,
                        n_iter=150, eps=0.0)["maps"].reshape(2, -1)
    for i in range(3):
        one = orc.askadam("monoexp_t2s", d.acq, np.ones((1, 1, 1), np.uint8),
                          y[:, i].reshape(12, 1, 1, 1), d.lb, d.ub, n_iter=150, eps=0.0)
        np.testing.assert_allclose(one["maps"].reshape(2), whole[:, i], rtol=1e-12)


def test_tv_pulls_neighbours_together(orc):
    d = synth.make_draw("monoexp_t2s", (2, 3, 3), 6, 0.05)
    y = (orc.forward("monoexp_t2s", d.acq, d.truth) + d.sigma * d.noise).astype(np.float32)
    yg = synth.scatter(y, d.mask)
    plain = orc.askadam("monoexp_t2s", d.acq, d.mask, yg, d.lb, d.ub, n_iter=300)
    reg = orc.askadam("monoexp_t2s", d.acq, d.mask, yg, d.lb, d.ub, n_iter=300, lam=0.05,
                      tv_mask=0b10)
    u_plain = (plain["maps"][1] - d.lb[1]) / (d.ub[1] - d.lb[1])
    u_reg = (reg["maps"][1] - d.lb[1]) / (d.ub[1] - d.lb[1])
    assert orc.tv(d.mask, u_reg)[0] < orc.tv(d.mask, u_plain)[0]
    # the start is a constant map, so the regulariser adds nothing to the first loss
    assert reg["loss"][0] == plain["loss"][0]
    assert reg["loss"][1] > plain["loss"][1]


def test_stopping_tol_and_window(orc):
    d = synth.make_draw("monoexp_t2s", (1, 2, 2), 7, 0.01)
    y = synth.scatter((orc.forward("monoexp_t2s", d.acq, d.truth) +
                       d.sigma * d.noise).astype(np.float32), d.mask)
    full = orc.askadam("monoexp_t2s", d.acq, d.mask, y, d.lb, d.ub, n_iter=400)
    assert full["iters_run"] == 400 and full["stop_reason"] == 0
    L = full["loss"]
    tol = float(np.quantile(L, 0.5))
    first = int(np.argmax(L < tol))       # first iteration index with L < tol
    r = orc.askadam("monoexp_t2s", d.acq, d.mask, y, d.lb, d.ub, n_iter=400, tol=tol)
    assert r["stop_reason"] == 1 and r["iters_run"] == first + 1
    np.testing.assert_array_equal(r["loss"], L[: first + 1])
    # window rule: |least-squares slope| of the last W losses below the value
    W = 20
    slopes = np.array([np.polyfit(np.arange(t - W + 1, t + 1), L[t - W:t], 1)[0]
                       for t in range(W, 401)])
    srt = np.sort(np.abs(slopes))
    j = len(srt) // 3
    cv = float(0.5 * (srt[j] + srt[j + 1]))      # a threshold between two slopes
    t_stop = W + int(np.argmax(np.abs(slopes) < cv))
    r = orc.askadam("monoexp_t2s", d.acq, d.mask, y, d.lb, d.ub, n_iter=400, conv_value=cv,
                    conv_window=W)
    assert r["stop_reason"] == 2 and r["iters_run"] == t_stop
