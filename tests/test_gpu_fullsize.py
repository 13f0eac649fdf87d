"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times, on sampled outputs the oracle computes voxel by voxel.

* MH, 3-pool GRE, 128x128x64 voxels, 4 chains x 5000 (burn-in 500, thin 100):
  FP32 chains (device-resident data, as benchmarked) against the FP64 oracle
  on sampled voxels (same random streams, statistical comparison), and the
  FP64 instantiation bit-exact on sampled voxels.
* MH, 3-pool GRE, 240x240x180 grid with the ellipsoid mask (1.2 M voxels),
  8 chains x 10000 (burn-in 1000, thin 10): FP32 against the oracle on
  sampled voxels.
* Adam, stick + ball, 64^3, 500 iterations without TV (voxels independent):
  sampled voxels against the oracle; with 3D TV (voxels coupled): the whole
  volume against the oracle over the first iterations, and properties of the
  full 500-iteration fit.
"""
import time

import numpy as np
import pytest

import mcstats
from gpu_util import G, say
from paper_2511_22094_amd import synth

pytestmark = pytest.mark.gpu


def _y(orc, d):
    """Measured data of a draw (oracle forward model + seeded noise), FP32 [Meff, n]."""
    return (orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise).astype(np.float32)


def _sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def _z_vs_oracle(mean_g, std_g, ref, S_g):
    """z-scores of GPU moments against the oracle's, each side's Monte-Carlo
    error from its own retained samples (the GPU's streamed for the sampled
    voxels)."""
    S = ref["samples"]
    zm = mcstats.zscores(mean_g, ref["mean"], mcstats.mcse_mean(S_g), mcstats.mcse_mean(S))
    zs = mcstats.zscores(std_g, ref["std"], mcstats.mcse_std(S_g), mcstats.mcse_std(S))
    return zm, zs


class _SampleTap:
    """Sample sink keeping the streamed draws of a few voxels: [C, K, P, k]."""

    def __init__(self, C, K, P, sel):
        self.sel = sel
        self.buf = np.empty((C, K, P, sel.size), np.float64)

    def __call__(self, k_first, s):
        self.buf[:, k_first:k_first + s.shape[1]] = s[:, :, :, self.sel]
        return True


def _run_mh_device(g, torch, d, y, kw, seed, precision="fp32", accept=False, tap=None):
    """gc_mcmc with device-resident data and outputs, as the benchmark calls it
    (with `tap`, the retained draws of its voxels stream to the host)."""
    dev = torch.device("cuda:0")
    nz, ny, nx = d.shape
    yg = torch.zeros((y.shape[0], nz * ny * nx), dtype=torch.float32, device=dev)
    idx = torch.from_numpy(np.flatnonzero(d.mask.reshape(-1))).to(dev)
    yg[:, idx] = torch.from_numpy(y).to(dev)
    yg = yg.reshape(y.shape[0], nz, ny, nx).contiguous()
    mask = torch.from_numpy(d.mask).to(dev)
    P = d.lb.size
    mean = torch.empty((P, nz, ny, nx), dtype=torch.float64, device=dev)
    std = torch.empty_like(mean)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    extra = {} if tap is None else dict(sample_sink=tap)
    out = g.gc_mcmc(g.Model.from_acq(d.model, d.acq), yg, mask, d.lb, d.ub, sigma=d.sigma,
                    step=synth.MH_STEP[d.model], seed=seed, precision=precision,
                    accept=accept, out_mean=mean, out_std=std, **extra, **kw)
    torch.cuda.synchronize()
    say(f"  gpu {precision} mcmc {time.perf_counter() - t0:.2f} s")
    m = mean.reshape(P, -1)[:, idx].cpu().numpy()
    s = std.reshape(P, -1)[:, idx].cpu().numpy()
    acc = None
    if accept:
        acc = out["accept"].reshape(kw["n_chains"], -1)[:, idx].cpu().numpy()
    return m, s, acc


def _check_statistical(zm, zs, tag):
    say(f"  {tag}: |z|>3 {(np.abs(zm) > 3).mean():.4f} {(np.abs(zs) > 3).mean():.4f} "
        f"max {np.abs(zm).max():.2f} {np.abs(zs).max():.2f}")
    # the posterior-moment rule: at most 1 % of (voxel, parameter) pairs
    # beyond |z| = 3 and none beyond 6 (both sides share their random streams,
    # which only makes the differences smaller)
    assert (np.abs(zm) > 3).mean() <= 0.01 and (np.abs(zs) > 3).mean() <= 0.01
    assert np.abs(zm).max() < 6 and np.abs(zs).max() < 6


def test_mh_gre3_128x128x64_fp32_sampled(orc):
    import torch
    g = G()
    d = synth.cfg1()
    kw = synth.CFG1_MCMC
    say("cfg gre3 128x128x64 fp32", kw)
    y = _y(orc, d)
    sel = _sample(d.n, 64, 11)
    tap = _SampleTap(kw["n_chains"], (kw["n_iter"] - kw["burnin"]) // kw["thin"], 9, sel)
    mean, std, _ = _run_mh_device(g, torch, d, y, kw, seed=1, tap=tap)
    assert np.all(np.isfinite(mean)) and np.all(np.isfinite(std))
    assert np.all(mean >= d.lb[:, None]) and np.all(mean <= d.ub[:, None])
    ref = orc.mh(d.model, d.acq, y[:, sel], d.lb, d.ub, synth.MH_STEP[d.model], d.sigma, 1,
                 vidx=sel, keep_samples=True, n_threads=16, **kw)
    zm, zs = _z_vs_oracle(mean[:, sel], std[:, sel], ref, tap.buf)
    _check_statistical(zm, zs, "gre3 128x128x64")


def test_mh_gre3_128x128x64_fp64_bit_exact_sampled(orc):
    import torch
    g = G()
    d = synth.cfg1()
    kw = synth.CFG1_MCMC
    say("cfg gre3 128x128x64 fp64", kw)
    y = _y(orc, d)
    mean, std, acc = _run_mh_device(g, torch, d, y, kw, seed=1, precision="fp64", accept=True)
    sel = _sample(d.n, 24, 12)
    ref = orc.mh(d.model, d.acq, y[:, sel], d.lb, d.ub, synth.MH_STEP[d.model], d.sigma, 1,
                 vidx=sel, n_threads=8, **kw)
    assert ref["margin"].min() > 1e-9
    assert np.array_equal(acc[:, sel], ref["accept"])
    np.testing.assert_allclose(mean[:, sel], ref["mean"], rtol=1e-11)
    np.testing.assert_allclose(std[:, sel], ref["std"], rtol=1e-9)


def test_mh_gre3_240x240x180_ellipsoid_fp32_sampled(orc):
    import torch
    g = G()
    d = synth.cfg4()
    kw = synth.CFG4_MCMC
    say("cfg gre3 240x240x180 ellipsoid fp32", d.n, kw)
    assert d.n == 1199888
    y = _y(orc, d)
    sel = _sample(d.n, 64, 13)
    tap = _SampleTap(kw["n_chains"], (kw["n_iter"] - kw["burnin"]) // kw["thin"], 9, sel)
    mean, std, _ = _run_mh_device(g, torch, d, y, kw, seed=4, tap=tap)
    assert np.all(np.isfinite(mean)) and np.all(np.isfinite(std))
    ref = orc.mh(d.model, d.acq, y[:, sel], d.lb, d.ub, synth.MH_STEP[d.model], d.sigma, 4,
                 vidx=sel, keep_samples=True, n_threads=16, **kw)
    zm, zs = _z_vs_oracle(mean[:, sel], std[:, sel], ref, tap.buf)
    _check_statistical(zm, zs, "gre3 240x240x180")


def _adam_device(g, torch, d, y, n_iter, lam, tv_params, x0_map=None):
    dev = torch.device("cuda:0")
    nz, ny, nx = d.shape
    yg = torch.from_numpy(synth.scatter(y, d.mask)).to(dev)
    mask = torch.from_numpy(d.mask).to(dev)
    out = torch.empty((d.lb.size, nz, ny, nx), dtype=torch.float32, device=dev)
    tvp = tuple(synth.PARAM_NAMES[d.model].index(p) for p in tv_params)
    x0 = None if x0_map is None else torch.from_numpy(x0_map).to(dev)
    t0 = time.perf_counter()
    r = g.gc_fit_askadam(g.Model.from_acq(d.model, d.acq), yg, mask, d.lb, d.ub, n_iter=n_iter,
                         loss=2, lam=lam, tv_params=tvp, tv_dim=3, out=out, x0_map=x0,
                         loss_history=True)
    torch.cuda.synchronize()
    say(f"  gpu adam {n_iter} it {time.perf_counter() - t0:.2f} s")
    return out.cpu().numpy(), r


def test_adam_dwi2_64cubed_no_tv_sampled(orc):
    import torch
    g = G()
    d = synth.cfg2()
    kw = synth.CFG2_ADAM
    say("cfg dwi2 64^3 adam, no TV", kw["n_iter"])
    y = _y(orc, d)
    maps, r = _adam_device(g, torch, d, y, kw["n_iter"], 0.0, ())
    sel = _sample(d.n, 64, 14)
    # the loss is a mean over all N voxels; the oracle fits the sampled voxels
    # alone, so each carries the weight sqrt(n_sample / N) to keep its gradient
    w = np.full(sel.size, np.sqrt(sel.size / d.n), np.float32)
    mk = np.ones((1, 1, sel.size), np.uint8)
    ref = orc.askadam(d.model, d.acq, mk, y[:, sel].reshape(-1, 1, 1, sel.size), d.lb, d.ub,
                      w=w.reshape(1, 1, -1), n_iter=kw["n_iter"], loss=2, n_threads=8)
    got = synth.gather(maps, d.mask)[:, sel]
    rng = (d.ub - d.lb)[:, None]
    err = np.abs(got - ref["maps"].reshape(d.lb.size, -1)) / rng
    say(f"  max err / range {err.max():.2e}")
    assert err.max() < 1e-4


def test_adam_dwi2_64cubed_tv_first_iterations_whole_volume(orc):
    import torch
    g = G()
    d = synth.cfg2()
    kw = synth.CFG2_ADAM
    y = _y(orc, d)
    # a non-uniform start, so that the TV term is active from the first step
    rng = np.random.default_rng(15)
    x0 = (d.lb[:, None] + (d.ub - d.lb)[:, None] * rng.uniform(0.2, 0.8, (d.lb.size, d.n)))
    x0_map = synth.scatter(x0.astype(np.float32), d.mask)
    n_it = 8
    say("cfg dwi2 64^3 adam + TV, whole volume", n_it)
    maps, r = _adam_device(g, torch, d, y, n_it, kw["lam"], kw["tv_params"], x0_map=x0_map)
    tvm = sum(1 << synth.PARAM_NAMES[d.model].index(p) for p in kw["tv_params"])
    ref = orc.askadam(d.model, d.acq, d.mask, synth.scatter(y, d.mask), d.lb, d.ub,
                      x0=x0_map.astype(np.float64), n_iter=n_it, loss=2, lam=kw["lam"],
                      tv_mask=tvm, tv_dim=3, n_threads=8)
    rng_ = (d.ub - d.lb)[:, None]
    err = np.abs(synth.gather(maps, d.mask) - synth.gather(ref["maps"], d.mask)) / rng_
    say(f"  err/range median {np.median(err):.2e} p99 {np.quantile(err, 0.99):.2e} "
        f"max {err.max():.2e}")
    assert np.median(err) < 1e-5 and np.quantile(err, 0.99) < 1e-4 and err.max() < 2e-2
    np.testing.assert_allclose(r["loss"], ref["loss"], rtol=1e-5)


def test_adam_dwi2_64cubed_tv_full_run_properties(orc):
    import torch
    g = G()
    d = synth.cfg2()
    kw = synth.CFG2_ADAM
    y = _y(orc, d)
    say("cfg dwi2 64^3 adam + TV, 500 iterations")
    maps, r = _adam_device(g, torch, d, y, kw["n_iter"], kw["lam"], kw["tv_params"])
    h = np.asarray(r["loss"])
    assert h.size == kw["n_iter"] and np.all(np.isfinite(h))
    assert r["final_loss"] == h[-1]
    # Adam on this smooth problem: the loss falls by orders of magnitude and
    # rises on few iterations only
    assert h[-1] < 0.05 * h[0]
    assert (np.diff(h) > 0).mean() < 0.2
    got = synth.gather(maps, d.mask)
    # maps are lb + (ub - lb) u in FP32 with u clamped to [0, 1]: within a
    # few FP32 ulps of the bounds
    tol = 4 * np.spacing(np.maximum(np.abs(d.lb), np.abs(d.ub)).astype(np.float32))[:, None]
    assert np.all(got >= d.lb[:, None] - tol) and np.all(got <= d.ub[:, None] + tol)
    # the volume fraction f is well determined at this noise level
    f_err = np.abs(got[0] - d.truth[0])
    say(f"  |f - truth| median {np.median(f_err):.3e}")
    assert np.median(f_err) < 0.05


def test_mh_gre3_240x240x180_streams_all_samples(orc):
    """The whole-brain volume with every retained sample kept: 8 chains x 900
    draws x 9 parameters x 1.2 M voxels (311 GB in FP32) stream through the
    sample sink in deliveries of one draw per chain (346 MB), never held at
    once; the streamed draws average to the posterior means the call reports,
    and the moments equal those of the call without samples."""
    import torch
    g = G()
    d = synth.cfg4()
    kw = synth.CFG4_MCMC
    y = _y(orc, d)
    mean0, std0, _ = _run_mh_device(g, torch, d, y, kw, seed=4)
    sel = _sample(d.n, 16, 17)
    K = (kw["n_iter"] - kw["burnin"]) // kw["thin"]
    C, P = kw["n_chains"], d.lb.size
    acc = np.zeros((P, sel.size))
    seen = []

    def sink(k_first, s):
        seen.append((k_first, s.shape[1]))
        x = s[:, :, :, sel].astype(np.float64)          # [C, k, P, 16]
        assert np.all(x >= d.lb[None, None, :, None]) and np.all(x <= d.ub[None, None, :, None])
        acc[:] += x.sum(axis=(0, 1))
        return True

    dev = torch.device("cuda:0")
    nz, ny, nx = d.shape
    yg = torch.zeros((y.shape[0], nz * ny * nx), dtype=torch.float32, device=dev)
    idx = torch.from_numpy(np.flatnonzero(d.mask.reshape(-1))).to(dev)
    yg[:, idx] = torch.from_numpy(y).to(dev)
    yg = yg.reshape(y.shape[0], nz, ny, nx).contiguous()
    mask = torch.from_numpy(d.mask).to(dev)
    mean = torch.empty((P, nz, ny, nx), dtype=torch.float64, device=dev)
    std = torch.empty_like(mean)
    t0 = time.perf_counter()
    g.gc_mcmc(g.Model.from_acq(d.model, d.acq), yg, mask, d.lb, d.ub, sigma=d.sigma,
              step=synth.MH_STEP[d.model], seed=4, accept=False, out_mean=mean, out_std=std,
              sample_sink=sink, **kw)
    torch.cuda.synchronize()
    say(f"  streamed {len(seen)} deliveries in {time.perf_counter() - t0:.1f} s")
    assert seen == [(k, 1) for k in range(K)]
    m = mean.reshape(P, -1)[:, idx].cpu().numpy()
    s = std.reshape(P, -1)[:, idx].cpu().numpy()
    assert np.array_equal(m, mean0) and np.array_equal(s, std0)
    # pooled mean of the streamed draws = the reported posterior mean
    # (Welford in FP64 of the same FP32 states against a plain FP64 sum)
    np.testing.assert_allclose(acc / (C * K), m[:, sel], rtol=1e-11, atol=1e-12)
