"""Pins of the oracle's optimiser recurrences beyond the first step
(paper §2.2.1: Adam, SGDM and RMSProp drive the askadam fit).

Constant-gradient problem.  The linear model s = Phi A (Phi_jk =
exp(-TE_j / tau_k), tau = 10, 30, 80 ms) with data far above anything the
box can produce (y = 1000, A in [-1, 1]) keeps every residual y - s positive,
so the L1 loss mean_j |y_j - s_j| has the same gradient at every iterate:
dL/dA_k = -(1/M) sum_j Phi_jk, and g = (ub - lb) dL/dA in the normalised
coordinates the fit works in.  For a constant gradient each optimiser has a
closed form after t steps (no clamping: the total move stays inside [0, 1]):

* Adam (Kingma & Ba, bias-corrected moments): m_t = (1 - b1^t) g and
  v_t = (1 - b2^t) g^2, so m_t / (1 - b1^t) = g and v_t / (1 - b2^t) = g^2
  exactly, and every step is lr g / (|g| + eps):
  u_t = u_0 - t lr g / (|g| + eps).
* SGDM (velocity form): vel_t = -lr g (1 - mu^t) / (1 - mu), so
  u_t = u_0 - lr g / (1 - mu) (t - mu (1 - mu^t) / (1 - mu)).
* RMSProp (no bias correction): v_t = (1 - rho^t) g^2, step t is
  lr g / (sqrt(1 - rho^t) |g| + eps).

A wrong power of beta, rho or mu, a bias correction applied outside the
square root, a missing (1 - beta) factor or eps inside the root changes
these sums after the first step; the tests use eps comparable to |g| so that
its placement matters too.

Changing gradients.  For the L2 loss of the same linear model the gradient
is the closed form 2/M Phi^T (Phi A - y) (times ub - lb in u); three Adam
steps are rebuilt from it with the published "efficient" form of the update
(step size lr sqrt(1 - b2^t) / (1 - b1^t) on the raw moments, with
eps sqrt(1 - b2^t)), a different arrangement of the same arithmetic than the
oracle's bias-corrected moments.
"""
import math

import numpy as np
import pytest

from paper_2511_22094_amd import synth

TAU = np.array([10.0, 30.0, 80.0])


def _phi(te):
    return np.exp(-np.asarray(te)[:, None] / TAU[None, :])


def _const_grad_problem():
    acq = synth.Acq(te=synth.echo_times(2.0, 4.0, 12))
    M = 12
    y = np.full((M, 1, 1, 1), 1000.0, np.float32)
    mask = np.ones((1, 1, 1), np.uint8)
    lb, ub = np.full(3, -1.0), np.full(3, 1.0)
    Phi = _phi(acq.te)
    gA = -Phi.sum(0) / M                 # d/dA of mean_j |y_j - (Phi A)_j|, residuals > 0
    g = (ub - lb) * gA                   # in u = (A - lb) / (ub - lb)
    return acq, y, mask, lb, ub, g


def _u(r, lb, ub):
    return (r["maps"][:, 0, 0, 0] - lb) / (ub - lb)


@pytest.mark.parametrize("t", [1, 2, 3, 7, 25])
def test_adam_constant_gradient_closed_form(orc, t):
    acq, y, mask, lb, ub, g = _const_grad_problem()
    lr = 0.004
    eps = 0.5 * float(np.abs(g).min())
    r = orc.askadam("linear3", acq, mask, y, lb, ub, n_iter=t, loss=1, lr=lr, eps=eps,
                    beta1=0.9, beta2=0.999)
    expect = 0.5 - t * lr * g / (np.abs(g) + eps)
    np.testing.assert_allclose(_u(r, lb, ub), expect, rtol=0, atol=1e-12)


@pytest.mark.parametrize("b1,b2", [(0.9, 0.999), (0.5, 0.75), (0.0, 0.9)])
def test_adam_constant_gradient_other_decays(orc, b1, b2):
    acq, y, mask, lb, ub, g = _const_grad_problem()
    lr, eps, t = 0.01, 0.3 * float(np.abs(g).max()), 9
    r = orc.askadam("linear3", acq, mask, y, lb, ub, n_iter=t, loss=1, lr=lr, eps=eps,
                    beta1=b1, beta2=b2)
    expect = 0.5 - t * lr * g / (np.abs(g) + eps)
    np.testing.assert_allclose(_u(r, lb, ub), expect, rtol=0, atol=1e-12)


@pytest.mark.parametrize("t", [1, 2, 5, 12])
@pytest.mark.parametrize("mu", [0.9, 0.5])
def test_sgdm_constant_gradient_closed_form(orc, t, mu):
    acq, y, mask, lb, ub, g = _const_grad_problem()
    lr = 0.002
    r = orc.askadam("linear3", acq, mask, y, lb, ub, n_iter=t, loss=1, lr=lr,
                    optimizer="sgdm", momentum=mu)
    disp = lr * g / (1 - mu) * (t - mu * (1 - mu ** t) / (1 - mu))
    np.testing.assert_allclose(_u(r, lb, ub), 0.5 - disp, rtol=0, atol=1e-12)


@pytest.mark.parametrize("t", [1, 2, 4, 10])
@pytest.mark.parametrize("rho", [0.9, 0.6])
def test_rmsprop_constant_gradient_closed_form(orc, t, rho):
    acq, y, mask, lb, ub, g = _const_grad_problem()
    lr = 0.003
    eps = 0.5 * float(np.abs(g).min())
    r = orc.askadam("linear3", acq, mask, y, lb, ub, n_iter=t, loss=1, lr=lr,
                    optimizer="rmsprop", rho=rho, eps=eps)
    disp = sum(lr * g / (math.sqrt(1 - rho ** s) * np.abs(g) + eps) for s in range(1, t + 1))
    np.testing.assert_allclose(_u(r, lb, ub), 0.5 - disp, rtol=0, atol=1e-12)


def test_adam_three_steps_changing_gradient(orc):
    """L2 fit of the linear model from the midpoint: the gradient changes at
    every step; the iterates follow the efficient form of the update."""
    acq = synth.Acq(te=synth.echo_times(2.0, 4.0, 12))
    M = 12
    Phi = _phi(acq.te)
    A_true = np.array([0.6, -0.3, 0.4])
    y = (Phi @ A_true + 0.05 * np.cos(np.arange(M))).astype(np.float32)
    mask = np.ones((1, 1, 1), np.uint8)
    lb, ub = np.full(3, -1.0), np.full(3, 2.0)
    lr, b1, b2, eps = 0.05, 0.8, 0.95, 1e-3
    u = np.full(3, 0.5)
    m = np.zeros(3)
    v = np.zeros(3)
    yd = y.astype(np.float64)
    for t in range(1, 4):
        A = lb + (ub - lb) * u
        gA = 2.0 / M * Phi.T @ (Phi @ A - yd)
        g = (ub - lb) * gA
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        a_t = lr * math.sqrt(1 - b2 ** t) / (1 - b1 ** t)
        eps_t = eps * math.sqrt(1 - b2 ** t)
        u = np.clip(u - a_t * m / (np.sqrt(v) + eps_t), 0.0, 1.0)
        r = orc.askadam("linear3", acq, mask, y.reshape(M, 1, 1, 1), lb, ub, n_iter=t, loss=2,
                        lr=lr, beta1=b1, beta2=b2, eps=eps)
        np.testing.assert_allclose(_u(r, lb, ub), u, rtol=0, atol=1e-12)
        # the loss recorded at step t is the one at the iterate before the update
        res = yd - Phi @ A
        assert r["loss"][t - 1] == pytest.approx(np.mean(res ** 2), rel=1e-12)
