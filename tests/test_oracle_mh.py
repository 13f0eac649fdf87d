"""Pins of the oracle's Metropolis-Hastings sampler: an analytic Gaussian
posterior (linear model, flat prior), a brute-force grid posterior (two
parameters), the prior-only limit (uniform on the box), the retention
arithmetic of the paper's Table 1, bounds, and determinism."""
import math

import numpy as np
import pytest

import mcstats
from paper_2511_22094_amd import synth

TE12 = synth.echo_times(2.0, 4.0, 12)


def test_linear_model_matches_analytic_posterior(orc):
    acq = orc.Acq(te=TE12)
    Phi = orc.jacobian("linear3", acq, np.ones((3, 1)))[0]
    sig = 0.01
    cov = sig**2 * np.linalg.inv(Phi.T @ Phi)
    sd = np.sqrt(np.diag(cov))
    n = 4
    rng = np.random.default_rng(0)
    A = rng.uniform(0.2, 1.0, (3, n))
    y = (orc.forward("linear3", acq, A) + sig * rng.standard_normal((12, n))).astype(np.float32)
    mu = np.linalg.solve(Phi.T @ Phi, Phi.T @ y.astype(np.float64))
    r = orc.mh("linear3", acq, y, np.full(3, -10.0), np.full(3, 10.0), 0.2 * sd, sig, 1,
               4, 200000, 2000, 10, x0=np.broadcast_to(mu[None], (4, 3, n)),
               keep_samples=True, n_threads=4)
    S = r["samples"]
    z_mean = (r["mean"] - mu) / mcstats.mcse_mean(S)
    z_sd = (r["std"] - sd[:, None]) / mcstats.mcse_std(S)
    assert np.abs(z_mean).max() < 4.5
    assert np.abs(z_sd).max() < 4.5
    # the test is sharp: the Monte-Carlo error is a few percent of the SD
    assert (mcstats.mcse_mean(S) / sd[:, None]).max() < 0.05


def _grid_moments(orc, acq, y, sig, s0, t2):
    G0, G1 = np.meshgrid(s0, t2, indexing="ij")
    th = np.stack([G0.ravel(), G1.ravel()])
    ll = orc.logl("monoexp_t2s", acq, th, np.repeat(y[:, None], th.shape[1], 1), sig)
    w = np.exp(ll - ll.max()).reshape(G0.shape)
    w /= w.sum()
    m0, m1 = (w * G0).sum(), (w * G1).sum()
    v0, v1 = (w * (G0 - m0) ** 2).sum(), (w * (G1 - m1) ** 2).sum()
    return np.array([m0, m1]), np.sqrt([v0, v1])


def test_monoexp_matches_brute_force_grid_posterior(orc):
    acq = orc.Acq(te=TE12)
    sig = 0.05
    truth = np.array([[0.9, 1.3, 0.7], [30.0, 55.0, 70.0]])
    rng = np.random.default_rng(2)
    y = (orc.forward("monoexp_t2s", acq, truth) + sig * rng.standard_normal((12, 3))).astype(
        np.float32)
    lb, ub = synth.bounds("monoexp_t2s")
    r = orc.mh("monoexp_t2s", acq, y, lb, ub, [0.03, 4.0], sig, 5, 4, 60000, 1000, 5,
               x0=np.broadcast_to(truth[None], (4, 2, 3)), keep_samples=True, n_threads=4)
    S = r["samples"]
    se_m = mcstats.mcse_mean(S)
    se_s = mcstats.mcse_std(S)
    for i in range(3):
        # grid over +-10 sd of the chain, fine enough for quadrature
        c, w = r["mean"][:, i], r["std"][:, i]
        s0 = np.linspace(c[0] - 10 * w[0], c[0] + 10 * w[0], 801)
        t2 = np.linspace(max(c[1] - 10 * w[1], 1.0), c[1] + 12 * w[1], 801)
        gm, gs = _grid_moments(orc, acq, y[:, i], sig, s0, t2)
        assert np.all(np.abs(r["mean"][:, i] - gm) / se_m[:, i] < 4.5), (i, r["mean"][:, i], gm)
        assert np.all(np.abs(r["std"][:, i] - gs) / se_s[:, i] < 4.5), (i, r["std"][:, i], gs)


def test_prior_only_is_uniform_on_box(orc):
    acq = orc.Acq(te=TE12)
    lb, ub = synth.bounds("monoexp_t2s")
    y = np.zeros((12, 3), np.float32)
    w = np.zeros(3, np.float32)          # zero weight: the likelihood is flat
    r = orc.mh("monoexp_t2s", acq, y, lb, ub, 0.3 * (ub - lb), 0.01, 8, 4, 40000, 100, 2,
               w=w, keep_samples=True, n_threads=4)
    S = r["samples"]
    mid = (0.5 * (lb + ub))[:, None]
    sd = ((ub - lb) / math.sqrt(12.0))[:, None]
    assert np.abs((r["mean"] - mid) / mcstats.mcse_mean(S)).max() < 4.5
    assert np.abs((r["std"] - sd) / mcstats.mcse_std(S)).max() < 4.5


def test_table1_sample_count_and_bounds(orc):
    # 4 chains x 25,000 iterations, 10 % burn-in, thinning 100 -> 900 samples
    burnin = math.floor(0.1 * 25000)
    assert orc.mh_nkeep(25000, burnin, 100) * 4 == 900
    # 50 walkers x 2,000 iterations with the same rule -> 900 as well
    assert orc.mh_nkeep(2000, math.floor(0.1 * 2000), 100) * 50 == 900
    acq = orc.Acq(te=TE12)
    lb, ub = synth.bounds("monoexp_t2s")
    y = orc.forward("monoexp_t2s", acq, np.array([[0.05], [2.0]])).astype(np.float32)
    r = orc.mh("monoexp_t2s", acq, y, lb, ub, [0.05, 3.0], 0.05, 3, 4, 25000, burnin, 100,
               keep_samples=True)
    S = r["samples"]
    assert S.shape == (4, 225, 2, 1)
    # truth near the lower bounds: many proposals leave the box, none is kept
    assert np.all(S >= lb[None, None, :, None]) and np.all(S <= ub[None, None, :, None])


def test_subset_and_threads_reproduce_full_run(orc):
    d = synth.cfg0()
    y = (orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise).astype(np.float32)
    step = synth.MH_STEP[d.model]
    kw = dict(n_chains=2, n_iter=300, burnin=100, thin=4)
    full = orc.mh(d.model, d.acq, y, d.lb, d.ub, step, d.sigma, 0, n_threads=8, **kw)
    one = orc.mh(d.model, d.acq, y, d.lb, d.ub, step, d.sigma, 0, n_threads=1, **kw)
    for k in ("mean", "std", "accept", "final"):
        np.testing.assert_array_equal(full[k], one[k])
    pick = np.array([3, 500, 999])
    sub = orc.mh(d.model, d.acq, y[:, pick], d.lb, d.ub, step, d.sigma, 0, vidx=pick, **kw)
    np.testing.assert_array_equal(sub["final"], full["final"][:, :, pick])
    np.testing.assert_array_equal(sub["accept"], full["accept"][:, pick])
    assert np.all(full["margin"] > 0)


def test_ensemble_matches_analytic_posterior(orc):
    # the stretch move is affine invariant: the strongly correlated linear
    # posterior (|rho| ~ 0.98) mixes as well as an isotropic one
    acq = orc.Acq(te=TE12)
    Phi = orc.jacobian("linear3", acq, np.ones((3, 1)))[0]
    sig = 0.01
    sd = np.sqrt(np.diag(sig**2 * np.linalg.inv(Phi.T @ Phi)))
    n = 4
    rng = np.random.default_rng(3)
    A = rng.uniform(0.2, 1.0, (3, n))
    y = (orc.forward("linear3", acq, A) + sig * rng.standard_normal((12, n))).astype(np.float32)
    mu = np.linalg.solve(Phi.T @ Phi, Phi.T @ y.astype(np.float64))
    r = orc.ensemble("linear3", acq, y, np.full(3, -10.0), np.full(3, 10.0), sig, 2, 32, 6000,
                     1000, 5, x0=mu, keep_samples=True, n_threads=4)
    S = r["samples"]
    assert np.abs((r["mean"] - mu) / mcstats.mcse_mean(S)).max() < 4.5
    assert np.abs((r["std"] - sd[:, None]) / mcstats.mcse_std(S)).max() < 4.5


def test_ensemble_prior_only_and_counts(orc):
    acq = orc.Acq(te=TE12)
    lb, ub = synth.bounds("monoexp_t2s")
    y = np.zeros((12, 2), np.float32)
    r = orc.ensemble("monoexp_t2s", acq, y, lb, ub, 0.01, 4, 50, 2000, 200, 100, x0_mode=1,
                     w=np.zeros(2, np.float32), keep_samples=True)
    S = r["samples"]
    assert S.shape[0] * S.shape[1] == 900      # 50 walkers x 18 retained = Table 1's 900
    assert np.all(S >= lb[None, None, :, None]) and np.all(S <= ub[None, None, :, None])
    mid = (0.5 * (lb + ub))[:, None]
    sd = ((ub - lb) / math.sqrt(12.0))[:, None]
    # walkers are nearly independent draws here: compare with plain standard errors
    assert np.all(np.abs(r["mean"] - mid) < 5 * sd / math.sqrt(900))
