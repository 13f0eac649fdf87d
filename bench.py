#!/usr/bin/env python3
"""Throughput benchmark of the voxel-parallel fitting hot path on one MI355X.

Headline (``value``): Metropolis-Hastings voxel-chain-iterations per second
on the whole-brain-sized 3-pool complex GRE workload (240 x 240 x 180 grid,
1,199,888-voxel ellipsoid mask, 24 echoes, SNR 50, 8 chains x 10,000
iterations, burn-in 1,000, thinning 10, FP32 chains with FP64 moments).  One
step = one gc_mcmc call over the whole volume with the data already resident
in HBM (pack -> init -> fused MH chunks -> moment merge -> scatter to grid
maps).  The 128 x 128 x 64 volume (4 chains x 5,000) is a second MH leg.

Other legs: the whole-volume Adam fit with 3D TV on the stick + ball
diffusion workload (``adam``; 64^3 voxels, 96 measurements, 500 iterations);
image reconstruction with the same solver (``sense``); the ensemble sampler,
optimiser and regulariser variants (``next_rows``); and the serving loop
(``serving``): a trace of 256 fit / MCMC jobs through the batching server and
through the one-job-per-launch path, all jobs at once (saturated) and at the
trace's Poisson arrival times (paced), with p50 / p99 latency.

Each leg reports a roofline entry for its dominant kernel: algorithmic
FLOPs (MH, ALU bound) or bytes (Adam+TV step, HBM bound) per launch divided
by the launch time measured with HIP events on the launch stream.  The CPU
baseline times the FP64 oracle on a bounded voxel sample of the headline
workload, on one thread and on every thread the process may use.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operations of one gre3 MH step with the echo recurrence
# (add / mul = 1, FMA = 2, transcendental = 1):
#   proposal 9 x FMA                                   18
#   Box-Muller 5 pairs x (log, mul, sqrt, sin, cos, 2 mul)   35
#   acceptance log, subtract                            2
#   per pool set-up: rcp, one complex step factor q = exp(-dTE/T2 + i 2 pi df dTE)
#     (2 mul, exp, sin, cos, 2 mul) and the first echo z = A q (2 mul)   3 x 10 = 30
#   per echo: 3 complex updates (4 mul + 2 add) + 4 adds + 2 sub + 2 FMA: 28 x 24 = 672
#   likelihood scale                                    1
FLOP_PER_MH_STEP_GRE3 = 18 + 35 + 2 + 30 + 672 + 1      # = 758
# Algorithmic HBM bytes per voxel-iteration of the dwi2 Adam+TV step kernel:
#   data 96 x 4, iterate 5 x 4 in + out, Adam m, v 2 x 5 x 4 in + out,
#   neighbour table 6 x 4 (neighbour iterate values are re-reads of the
#   iterate and are not counted again)
BYTES_PER_ADAM_TV_VOXEL_ITER = 96 * 4 + 2 * 5 * 4 + 2 * 2 * 5 * 4 + 6 * 4   # = 528
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# The instruction mix of one gre3 MH step (from the kernel's ISA, confirmed by
# SQ_INSTS_VALU) priced with the issue costs measured on MI355X, in cycles per
# wave64 instruction per SIMD: 604 full-rate FP32 / integer instructions x 2.4,
# 42 half-rate (funnel shift, med3, select, 32-bit multiplies) x 4.2, 46
# 32x32->64 multiplies x 4.9, 32 transcendentals x 8.1 -> 2,110 cycles per
# wave-step.  At perfect issue the kernel then reaches 758 x 64 flops per
# 2,110 cycles of a SIMD's 64 flops per cycle at FP32 peak: the ceiling of
# `frac` for this mix.
MH_GRE3_ISSUE_CYCLES = 604 * 2.4 + 42 * 4.2 + 46 * 4.9 + 32 * 8.1     # = 2,110
MH_GRE3_MIX_CEILING = FLOP_PER_MH_STEP_GRE3 * 64 / MH_GRE3_ISSUE_CYCLES / 64.0   # = 0.36

# HBM bytes per launch of the dominant kernels, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE) of `bench.py --profile-only mh,adam,copy`
# (summaries under profiles/); FETCH_SIZE is scaled by the factor that a
# 256 MiB device copy in the same run gives (bytes it reads / its FETCH_SIZE),
# WRITE_SIZE likewise.  A figure holds only for the kernel sources it was
# taken on: when their sha256 differs, `traffic` is reported as null.
MEASURED_TRAFFIC = {
    "mh_chunk_cfg4": {"sources": ["gc_mh.hip", "gc_device.hpp", "gc_internal.hpp"],
        "sha256": "2a7f2115f4d2c0ea4d0fcb1baad656a7b299c2fb36fb568ecbb15fb0b7d02884",
        "read_bytes": 3767459368, "write_bytes": 1804631552,
        "profile": "profiles/mh_chunk_gre3_240x240x180_ellipsoid_8chains.md"},
    "mh_chunk_cfg1": {"sources": ["gc_mh.hip", "gc_device.hpp", "gc_internal.hpp"],
        "sha256": "2a7f2115f4d2c0ea4d0fcb1baad656a7b299c2fb36fb568ecbb15fb0b7d02884",
        "read_bytes": 1595956635, "write_bytes": 788529152,
        "profile": "profiles/mh_chunk_gre3_128x128x64_4chains.md"},
    "fit_step": {"sources": ["gc_fit.hip", "gc_device.hpp", "gc_internal.hpp"],
        "sha256": "430c4e215241d2ba3f0aeb73ce47ba6e06325f97500fcb6505679a7638c8740a",
        "read_bytes": 126856489, "write_bytes": 15728648,
        "profile": "profiles/fit_step_dwi2_64cubed_adam_tv.md"},
    "sense_ycols": {"sources": ["gc_sense.hip", "gc_fft.hpp", "gc_sense.hpp", "gc_device.hpp", "gc_internal.hpp"],
        "sha256": "4e8069406a18d2a669c4aa5424304a68ce821adc1e2ca5fece005d925b77ccaa",
        "read_bytes": 112252034, "write_bytes": 100663321,
        "profile": "profiles/sense_ycols_6x32_256x256.md"},
    "sense_zrows": {"sources": ["gc_sense.hip", "gc_fft.hpp", "gc_sense.hpp", "gc_device.hpp", "gc_internal.hpp"],
        "sha256": "4e8069406a18d2a669c4aa5424304a68ce821adc1e2ca5fece005d925b77ccaa",
        "read_bytes": 145928149, "write_bytes": 109899252,
        "profile": "profiles/sense_zrows_6x32_256x256.md"},
}


def measured_traffic(key):
    import hashlib
    e = MEASURED_TRAFFIC.get(key)
    if e is None:
        return None
    h = hashlib.sha256()
    for f in e["sources"]:
        with open(os.path.join(ROOT, "paper_2511_22094_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != e["sha256"]:
        return None
    return e["read_bytes"] + e["write_bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


MH_WORKLOADS = {
    # the whole-brain-sized 3-pool GRE volume: 240x240x180 grid, ellipsoid
    # mask (1,199,888 voxels), SNR 50, 8 chains x 10,000, burn-in 1,000, thin 10
    "cfg4": ("gre3 3-pool complex GRE MCMC, 240x240x180 grid, 1,199,888-voxel ellipsoid "
             "mask, 24 echoes, SNR 50, 8 chains x 10000 iters, burn-in 1000, thin 10, "
             "FP32 chains, FP64 moments", "cfg4", "CFG4_MCMC", 4),
    # the 128x128x64 volume, SNR 100, 4 chains x 5,000, burn-in 500, thin 100
    "cfg1": ("gre3 3-pool complex GRE MCMC, 128x128x64 voxels, 24 echoes, SNR 100, "
             "4 chains x 5000 iters, burn-in 500, thin 100, FP32 chains, FP64 moments",
             "cfg1", "CFG1_MCMC", 1),
}


def mh_draw(torch, g, which):
    """The workload's draw, its data on the GPU (HIP forward + seeded noise)
    and its model."""
    from paper_2511_22094_amd import synth
    _, fn, _, _ = MH_WORKLOADS[which]
    d = getattr(synth, fn)()
    m = g.Model.from_acq("gre3", d.acq)
    dev = torch.device("cuda:0")
    nz, ny, nx = d.shape
    truth = torch.tensor(d.truth, dtype=torch.float32, device=dev)
    s = g.gc_model_forward(m, truth)
    s += d.sigma * torch.from_numpy(d.noise).to(dev)
    del truth
    y = torch.zeros((48, nz * ny * nx), dtype=torch.float32, device=dev)
    idx = torch.from_numpy(np.flatnonzero(d.mask.reshape(-1))).to(dev)
    y[:, idx] = s
    del s
    return d, m, y.reshape(48, nz, ny, nx), torch.from_numpy(d.mask).to(dev), idx


def mh_leg(g, torch, steps, warmup, which="cfg4", sample=None):
    """Timed gc_mcmc calls over the whole volume, data and outputs resident on
    the GPU; the mh_chunk launches timed with HIP events on their stream."""
    from paper_2511_22094_amd import synth
    _, _, kwname, seed = MH_WORKLOADS[which]
    kw = getattr(synth, kwname)
    d, m, y, mask, idx = mh_draw(torch, g, which)
    dev = torch.device("cuda:0")
    nz, ny, nx = d.shape
    step = synth.MH_STEP["gre3"]
    mean = torch.empty((9, nz, ny, nx), dtype=torch.float64, device=dev)
    std = torch.empty_like(mean)

    def run():
        return g.gc_mcmc(m, y, mask, d.lb, d.ub, sigma=d.sigma, step=step, seed=seed,
                         accept=False, out_mean=mean, out_std=std, **kw)

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    g.gc_timing_reset()
    g.gc_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.gc_timing_enable(False)
    kms, nl = g.gc_timing_get("mh_chunk")
    gms, gnl = g.gc_timing_get("gather_rows")
    n = d.n
    units = n * kw["n_chains"] * kw["n_iter"]
    sec = (t1 - t0) / steps
    per_launch_s = kms / 1e3 / max(nl, 1)
    launches_per_step = nl / steps
    units_per_launch = units / launches_per_step
    achieved = FLOP_PER_MH_STEP_GRE3 * units_per_launch / per_launch_s / 1e12
    finite = bool(torch.isfinite(mean.reshape(9, -1)[:, idx]).all().item())
    moments = None
    if sample is not None:
        sidx = idx[torch.from_numpy(sample).to(dev)]
        moments = (mean.reshape(9, -1)[:, sidx].cpu().numpy(),
                   std.reshape(9, -1)[:, sidx].cpu().numpy())
    del y, mean, std
    torch.cuda.empty_cache()
    # the pack step's gather (a1): Meff rows of n masked voxels read and written,
    # plus the n-entry index
    gather = None
    if gnl > 0:
        gbytes = 2 * m.n_meas_eff * n * 4 + n * 4
        gus = gms * 1e3 / gnl
        gather = {"bound": "hbm", "kernel": "gather_rows", "launch_us": gus,
                  "bytes_per_launch": gbytes, "achieved": gbytes / (gus * 1e-6) / 1e9,
                  "peak": PEAK_HBM_GBS, "unit": "GB/s",
                  "frac": gbytes / (gus * 1e-6) / 1e9 / PEAK_HBM_GBS}
    return dict(units=units, sec=sec, value=units / sec, per_launch_ms=per_launch_s * 1e3,
                launches=launches_per_step, units_per_launch=units_per_launch,
                achieved_tflops=achieved, finite=finite, n=n, moments=moments, kw=kw,
                gather=gather)


def adam_leg(g, torch, steps, warmup):
    from paper_2511_22094_amd import synth
    d = synth.cfg2()
    kw = synth.CFG2_ADAM
    m = g.Model.from_acq("dwi2", d.acq)
    dev = torch.device("cuda:0")
    nz, ny, nx = d.shape
    truth = torch.tensor(d.truth, dtype=torch.float32, device=dev)
    s = g.gc_model_forward(m, truth)
    y = (s + d.sigma * torch.from_numpy(d.noise).to(dev)).reshape(96, nz, ny, nx).contiguous()
    out = torch.empty((5, nz, ny, nx), dtype=torch.float32, device=dev)
    mask = torch.from_numpy(d.mask).to(dev)
    tvp = tuple(synth.PARAM_NAMES["dwi2"].index(p) for p in kw["tv_params"])

    def run():
        return g.gc_fit_askadam(m, y, mask, d.lb, d.ub, n_iter=kw["n_iter"], loss=kw["loss"],
                                lam=kw["lam"], tv_params=tvp, tv_dim=kw["tv_dim"], out=out)

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    g.gc_timing_reset()
    # every 10th launch: the event records of timing would otherwise add
    # to the gaps between the 500 short per-iteration launches
    g.gc_timing_enable(True, every=10)
    t0 = time.perf_counter()
    for _ in range(steps):
        r = run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.gc_timing_enable(False)
    kms, nl = g.gc_timing_get("fit_step")
    n = d.n
    units = n * kw["n_iter"]
    sec = (t1 - t0) / steps
    per_launch_s = kms / 1e3 / max(nl, 1)
    gbs = BYTES_PER_ADAM_TV_VOXEL_ITER * n / per_launch_s / 1e9
    return dict(units=units, sec=sec, value=units / sec, per_launch_us=per_launch_s * 1e6,
                achieved_gbs=gbs, final_loss=r["final_loss"], n=n)


def sense_bytes(E, Nc, Ny, Nz, S):
    """Algorithmic HBM bytes of each reconstruction stage for one iteration
    (E echoes, Nc coils, N = Ny Nz pixels, S sampled (echo, y, z) entries):
    every array a stage must read or write, counted once; the measured
    samples count only the sampled entries, the mask one 4-byte word per row
    of each tile of G = min(16, 4096 / Ny) columns."""
    N = Ny * Nz
    G = min(16, 4096 // Ny)
    coil_imgs = 8 * E * Nc * N
    return {
        # y pass: coil images in and out, samples, tile row masks
        "sense_ycols": 2 * coil_imgs + 8 * Nc * S + 4 * E * Ny * (Nz // G),
        # z pass: coil images in and out, coil maps, image in and out, Adam m, v in and out
        "sense_zrows": 2 * coil_imgs + 8 * Nc * N + 16 * E * N + 32 * E * N,
    }


def sense_leg(g, torch, steps, warmup):
    from paper_2511_22094_amd import synth
    kw = synth.SENSE_RECON
    E, Nc, Ny, Nz = kw["n_echo"], kw["n_coil"], kw["ny"], kw["nz"]
    d = synth.sense_draw(41, E, Nc, Ny, Nz, sigma=kw["sigma"], noise=False)
    dev = torch.device("cuda:0")
    C = torch.from_numpy(d.coils.astype(np.complex64)).to(dev)
    M = torch.from_numpy(d.mask).to(dev)
    x = torch.from_numpy(d.truth.astype(np.complex64)).to(dev)
    gen = torch.Generator(device=dev).manual_seed(42)
    noise = torch.complex(torch.randn((E, Nc, Ny, Nz), generator=gen, device=dev),
                          torch.randn((E, Nc, Ny, Nz), generator=gen, device=dev))
    k = (g.gc_sense_forward(x, C, M) + kw["sigma"] * noise * M[:, None]).contiguous()
    out = torch.empty((E, Ny, Nz), dtype=torch.complex64, device=dev)

    def run():
        return g.gc_sense_recon(k, C, M, lr=kw["lr"], n_iter=kw["n_iter"], loss=kw["loss"],
                                lam=kw["lam"], out=out)

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    g.gc_timing_reset()
    g.gc_timing_enable(True, every=10)
    t0 = time.perf_counter()
    for _ in range(steps):
        r = run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.gc_timing_enable(False)
    S = int(d.mask.sum())
    nbytes = sense_bytes(E, Nc, Ny, Nz, S)
    stages = {}
    for fam, b in nbytes.items():
        kms, nl = g.gc_timing_get(fam)
        us = kms * 1e3 / max(nl, 1)
        stages[fam] = {"launch_us": us, "bytes": b, "achieved_gbs": b / (us * 1e-6) / 1e9}
    sec = (t1 - t0) / steps
    err = float((out - x).abs().pow(2).sum().sqrt() / x.abs().pow(2).sum().sqrt())
    return dict(sec=sec, iters=kw["n_iter"], value=kw["n_iter"] / sec, stages=stages,
                final_loss=r["final_loss"], rel_err=err)


# Algorithmic FP32 operations of one gre3 ensemble (stretch-move) walker step:
# the likelihood of the MH step (pool set-up 30, 24 echoes x 28, scale 1 = 703),
# the stretch z = ((a-1)u + 1)^2 / a (4), the proposal theta_j + z (theta_k -
# theta_j) over 9 parameters (27) and the acceptance (P-1) log z + dlogL (4).
FLOP_PER_ENS_STEP_GRE3 = 703 + 4 + 27 + 4   # = 738


def grid_csr(shape):
    """6-neighbourhood adjacency of a fully masked grid as CSR (vertex = voxel in
    grid order, neighbours in the order -x, +x, -y, +y, -z, +z)."""
    nz, ny, nx = shape
    g = np.arange(nz * ny * nx, dtype=np.int64).reshape(nz, ny, nx)
    src, dst = [], []
    for axis, step in ((2, -1), (2, 1), (1, -1), (1, 1), (0, -1), (0, 1)):
        a = np.roll(g, -step, axis=axis)
        ok = np.ones(g.shape, bool)
        idx = [slice(None)] * 3
        idx[axis] = -1 if step == 1 else 0
        ok[tuple(idx)] = False
        src.append(g[ok])
        dst.append(a[ok])
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    order = np.argsort(src, kind="stable")
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=g.size))]).astype(np.int64)
    return rowptr, dst[order].astype(np.int32)


def ens_leg(g, torch, warmup=1):
    """One timed run of the affine-invariant ensemble sampler: 50 walkers x
    1,800 iterations, thin 100 (900 retained samples per voxel, as in the
    paper's ensemble setting), gre3 on a 128x128x8 slab of the GRE volume."""
    from paper_2511_22094_amd import synth
    dev = torch.device("cuda:0")
    d = synth.cfg1(shape=(8, 128, 128))
    m = g.Model.from_acq("gre3", d.acq)
    nz, ny, nx = d.shape
    s_ = g.gc_model_forward(m, torch.tensor(d.truth, dtype=torch.float32, device=dev))
    y = (s_ + d.sigma * torch.from_numpy(d.noise).to(dev)).reshape(48, nz, ny, nx).contiguous()
    mean = torch.empty((9, nz, ny, nx), dtype=torch.float64, device=dev)
    std = torch.empty_like(mean)
    W, T = 50, 1800

    def ens():
        return g.gc_mcmc(m, y, None, d.lb, d.ub, 1, T, 0, 100, sigma=d.sigma, seed=1,
                         sampler="ensemble", n_walkers=W, stretch=2.0, accept=False,
                         out_mean=mean, out_std=std)

    for _ in range(warmup):
        ens()
    torch.cuda.synchronize()
    g.gc_timing_reset()
    g.gc_timing_enable(True)
    t0 = time.perf_counter()
    ens()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    g.gc_timing_enable(False)
    kms, nl = g.gc_timing_get("ens_chunk")
    units = d.n * W * T
    per = kms / 1e3 / max(nl, 1)
    tf = FLOP_PER_ENS_STEP_GRE3 * (units / max(nl, 1)) / per / 1e12
    return {
        "value": units / sec, "unit": "voxel-walker-iterations/s", "sec": sec,
        "workload": f"gre3, {d.n} voxels (128x128x8), {W} walkers x {T} iterations, thin 100",
        "roofline": {"bound": "alu", "kernel": "ens_chunk<gre3>", "achieved": tf,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_FP32_TFLOPS,
                     "flop_per_step": FLOP_PER_ENS_STEP_GRE3, "launch_ms": per * 1e3}}


def next_rows_leg(g, torch):
    """One timed run each of the rows built beyond the main path: the affine-
    invariant ensemble sampler (50 walkers x 1,800 iterations, thin 100, gre3 on
    a 128x128x8 slab of the GRE volume), Adam with isotropic TV, SGDM and
    RMSProp with TV, graph (mesh) TV and the Eq. 6 prior on the 64^3 diffusion
    workload (500 iterations each).  Kernel times from HIP events."""
    from paper_2511_22094_amd import synth
    dev = torch.device("cuda:0")
    out = {}
    # ---------------------------------------------------------- ensemble
    out["f1_ensemble"] = ens_leg(g, torch, warmup=1)
    # ------------------------------------------------ fit-step variants
    d = synth.cfg2()
    kw = synth.CFG2_ADAM
    m = g.Model.from_acq("dwi2", d.acq)
    nz, ny, nx = d.shape
    s_ = g.gc_model_forward(m, torch.tensor(d.truth, dtype=torch.float32, device=dev))
    y = (s_ + d.sigma * torch.from_numpy(d.noise).to(dev)).reshape(96, nz, ny, nx).contiguous()
    maps = torch.empty((5, nz, ny, nx), dtype=torch.float32, device=dev)
    tvp = tuple(synth.PARAM_NAMES["dwi2"].index(p) for p in kw["tv_params"])
    rowptr, col = grid_csr(d.shape)
    rng = np.random.default_rng(5)
    rngp = (d.ub - d.lb)[:, None, None, None]
    mu = torch.from_numpy((d.lb[:, None, None, None] + rngp * rng.uniform(0.3, 0.7, (5,) + d.shape))
                          .astype(np.float32)).to(dev)
    sg = torch.from_numpy((rngp * rng.uniform(0.05, 0.2, (5,) + d.shape)).astype(np.float32)).to(dev)
    base = dict(n_iter=kw["n_iter"], loss=kw["loss"], lam=kw["lam"], tv_params=tvp,
                tv_dim=kw["tv_dim"], out=maps)
    variants = [
        ("f2_adam_iso_tv", dict(base, tv_kind="iso"), 528 + 36,
         "Adam, isotropic 3D TV (+ 9 neighbour-table reads per voxel)"),
        ("f2_sgdm_tv", dict(base, optimizer="sgdm", lr=0.05), 528 - 40,
         "SGDM (momentum 0.9, lr 0.05), anisotropic 3D TV (one state array)"),
        ("f2_rmsprop_tv", dict(base, optimizer="rmsprop", lr=0.002), 528 - 40,
         "RMSProp (rho 0.9, lr 0.002), anisotropic 3D TV (one state array)"),
        ("f3_graph_tv", dict(base, tv_kind="graph", graph=(torch.from_numpy(rowptr).to(dev),
                                                           torch.from_numpy(col).to(dev))),
         528 - 24 + 8 + 24, "Adam, graph TV on the 6-neighbourhood mesh of the grid (CSR)"),
        ("f3_prior", dict(base, prior_lam=0.02, prior_params=(0, 1, 2), prior_mu=mu,
                          prior_sigma=sg), 528 + 24, "Adam, 3D TV and the Eq. 6 prior on f, Da, De"),
    ]
    for name, kwv, bpv, what in variants:
        def fit():
            return g.gc_fit_askadam(m, y, None, d.lb, d.ub, **kwv)
        fit()
        torch.cuda.synchronize()
        g.gc_timing_reset()
        g.gc_timing_enable(True, every=10)
        t0 = time.perf_counter()
        r = fit()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        g.gc_timing_enable(False)
        kms, nl = g.gc_timing_get("fit_step")
        per = kms / 1e3 / max(nl, 1)
        gbs = bpv * d.n / per / 1e9
        out[name] = {"value": d.n * kw["n_iter"] / sec, "unit": "voxel-iterations/s",
                     "workload": f"dwi2 64^3, 500 iterations; {what}",
                     "final_loss": r["final_loss"],
                     "roofline": {"bound": "hbm", "kernel": "fit_step<dwi2>", "achieved": gbs,
                                  "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                                  "bytes_per_voxel_iter": bpv, "launch_us": per * 1e6}}
    return out


def next_rows_oracle_error(g, torch):
    """The next-row legs against the FP64 oracle on small problems of the same
    recipes: the ensemble on 512 voxels of the GRE slab (same random streams,
    each side's own forward model for the data), in units of the oracle's
    posterior SD; each fit variant on a 16^3 volume of the diffusion recipe,
    |GPU - oracle| / (ub - lb) of the maps."""
    import oracle
    from paper_2511_22094_amd import synth
    threads = min(os.cpu_count() or 1, 16)
    out = {}
    d = synth.cfg1(shape=(8, 128, 128))
    idx = np.sort(np.random.default_rng(77).choice(d.n, 512, replace=False))
    W, T = 50, 1800
    y = (oracle.forward("gre3", d.acq, d.truth[:, idx]) + d.sigma * d.noise[:, idx]).astype(np.float32)
    ref = oracle.ensemble("gre3", d.acq, y, d.lb, d.ub, d.sigma, 1, W, T, 0, 100, stretch=2.0,
                          n_threads=threads)
    m = g.Model.from_acq("gre3", d.acq)
    r = g.gc_mcmc(m, y.reshape(48, 1, 1, idx.size), None, d.lb, d.ub, 1, T, 0, 100,
                  sigma=d.sigma, seed=1, sampler="ensemble", n_walkers=W, stretch=2.0,
                  accept=False)
    sd = np.maximum(ref["std"], 1e-300)
    dm = np.abs(r["mean"].reshape(9, -1) - ref["mean"]) / sd
    ds = np.abs(r["std"].reshape(9, -1) - ref["std"]) / sd
    out["f1_ensemble"] = {"what": "|GPU - oracle| of posterior mean / SD in units of the oracle's "
                                  "SD, 512 voxels x 9 parameters, FP32 vs FP64 walkers",
                          "mean_median": float(np.median(dm)), "mean_p99": float(np.quantile(dm, 0.99)),
                          "sd_median": float(np.median(ds)), "sd_p99": float(np.quantile(ds, 0.99))}
    d = synth.cfg2(shape=(16, 16, 16))
    kw = synth.CFG2_ADAM
    y = synth.scatter((oracle.forward("dwi2", d.acq, d.truth) + d.sigma * d.noise)
                      .astype(np.float32), d.mask)
    m = g.Model.from_acq("dwi2", d.acq)
    tvp = tuple(synth.PARAM_NAMES["dwi2"].index(p) for p in kw["tv_params"])
    tvm = sum(1 << p for p in tvp)
    rowptr, col = grid_csr(d.shape)
    rng = np.random.default_rng(5)
    rngp = (d.ub - d.lb)[:, None, None, None]
    mu = (d.lb[:, None, None, None] + rngp * rng.uniform(0.3, 0.7, (5,) + d.shape)).astype(np.float32)
    sg = (rngp * rng.uniform(0.05, 0.2, (5,) + d.shape)).astype(np.float32)
    base_g = dict(n_iter=kw["n_iter"], loss=kw["loss"], lam=kw["lam"], tv_params=tvp,
                  tv_dim=kw["tv_dim"])
    base_o = dict(n_iter=kw["n_iter"], loss=kw["loss"], lam=kw["lam"], tv_mask=tvm,
                  tv_dim=kw["tv_dim"], n_threads=threads)
    cases = [
        ("f2_adam_iso_tv", dict(tv_kind="iso"), dict(tv_kind="iso")),
        ("f2_sgdm_tv", dict(optimizer="sgdm", lr=0.05), dict(optimizer="sgdm", lr=0.05)),
        ("f2_rmsprop_tv", dict(optimizer="rmsprop", lr=0.002), dict(optimizer="rmsprop", lr=0.002)),
        ("f3_graph_tv", dict(tv_kind="graph", graph=(rowptr, col)),
         dict(tv_kind="graph", graph=(rowptr, col))),
        ("f3_prior", dict(prior_lam=0.02, prior_params=(0, 1, 2), prior_mu=mu, prior_sigma=sg),
         dict(prior_lam=0.02, prior_mask=0b111, prior_mu=mu.astype(np.float64),
              prior_sigma=sg.astype(np.float64))),
    ]
    for name, kg, ko in cases:
        r = g.gc_fit_askadam(m, y, d.mask, d.lb, d.ub, loss_history=True, **base_g, **kg)
        ref = oracle.askadam("dwi2", d.acq, d.mask, y, d.lb, d.ub, **base_o, **ko)
        err = np.abs(r["maps"] - ref["maps"]) / rngp
        out[name] = {"what": "|GPU - oracle| / (ub - lb) of the maps, 16^3 volume, 500 iterations",
                     "median": float(np.median(err)), "p99": float(np.quantile(err, 0.99)),
                     "max": float(err.max()),
                     "final_loss_rel": float(abs(r["loss"][-1] / ref["loss"][-1] - 1))}
    return out


def copy_leg(torch, mib=256, reps=3):
    """A plain device copy of known size (mib MiB read + mib MiB written per launch): the
    calibration launch for the HBM byte counters."""
    n = mib * 2 ** 20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return dict(bytes_read=n * 4, bytes_written=n * 4, launches=reps)


def bandwidth(torch):
    """Achievable bandwidth with plain torch kernels (copy, sum, axpy) on
    float32 arrays of 32 MiB to 1 GiB, GB/s of the bytes each must move, each
    kernel repeated back to back: the practical ceiling next to the 8 TB/s
    HBM peak.  Working sets up to a few hundred MiB can stay in the 256 MB
    Infinity Cache between repetitions; 1 GiB arrays cannot."""
    dev = torch.device("cuda:0")
    res = {}
    for mib in (32, 64, 128, 256, 1024):
        n = mib * 2 ** 20 // 4
        a = torch.ones(n, device=dev)
        b = torch.empty_like(a)
        for name, fn, nbytes in [("copy", lambda: b.copy_(a), 2 * n * 4),
                                 ("sum", lambda: a.sum(), n * 4),
                                 ("axpy", lambda: b.add_(a, alpha=0.5), 3 * n * 4)]:
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            res[f"{name}_{mib}MiB_GBs"] = round(nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9)
        del a, b
    print(json.dumps({"bandwidth": res}))


def sweep(g, torch, repeats=10):
    """Throughput against volume size (cf. the paper's scaling figure): for each
    model and N in {1e2, 1e3, 1e4, 1e5, 2.5e5, 1e6} voxels, the median wall
    time of one whole call (pack, solve, unpack; data resident on the GPU) for
    MH (4 chains x 1000 iterations, burn-in 100, thin 10, FP32) and Adam
    (200 iterations, no TV).  Prints one JSON line per point."""
    from paper_2511_22094_amd import synth
    acqs = {"monoexp_t2s": synth.Acq(te=synth.echo_times(2.0, 4.0, 12)),
            "gre3": synth.Acq(te=synth.echo_times(2.0, 2.0, 24)),
            "dwi2": synth.dwi_acq(np.random.default_rng(1002))}
    sigma = {"monoexp_t2s": 0.01, "gre3": 0.01, "dwi2": 0.02}
    dev = torch.device("cuda:0")
    for model, acq in acqs.items():
        m = g.Model.from_acq(model, acq)
        for N in (100, 1000, 10000, 100000, 250000, 1000000):
            d = synth.make_draw(model, (1, 1, N), 7, sigma[model], acq=acq)
            s_ = g.gc_model_forward(m, torch.tensor(d.truth, dtype=torch.float32, device=dev))
            y = (s_ + d.sigma * torch.from_numpy(d.noise).to(dev)).reshape(-1, 1, 1, N).contiguous()
            P = d.lb.size
            mean = torch.empty((P, 1, 1, N), dtype=torch.float64, device=dev)
            std = torch.empty_like(mean)
            maps = torch.empty((P, 1, 1, N), dtype=torch.float32, device=dev)
            runs = {
                "mh": (lambda: g.gc_mcmc(m, y, None, d.lb, d.ub, 4, 1000, 100, 10, sigma=d.sigma,
                                         step=synth.MH_STEP[model], seed=1, accept=False,
                                         out_mean=mean, out_std=std), N * 4 * 1000),
                "adam": (lambda: g.gc_fit_askadam(m, y, None, d.lb, d.ub, n_iter=200, out=maps),
                         N * 200),
            }
            for solver, (fn, units) in runs.items():
                fn()
                torch.cuda.synchronize()
                ts = []
                for _ in range(repeats):
                    t0 = time.perf_counter()
                    fn()
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                t = float(np.median(ts))
                print(json.dumps({"sweep": solver, "model": model, "voxels": N,
                                  "median_s": t, "mean_s": float(np.mean(ts)),
                                  "voxel_iter_per_s": units / t}), flush=True)
            del y, s_, mean, std, maps


SERVE_MODELS = {
    "monoexp_t2s": 0.01,
    "gre3": 0.01,
    "dwi2": 0.02,
}


def serve_trace_jobs(g, torch, n_jobs, vox_range, mcmc_iters, fit_iters, seed=3):
    """Host-side job inputs of a serving trace: parameters drawn per job on the
    host (the trace's seed per job), data made with the HIP forward model and
    noise from a seeded device generator, then copied to host memory (server
    jobs carry host buffers)."""
    from paper_2511_22094_amd import synth
    trace = synth.serving_trace(seed, n_jobs, 20.0, vox_range, mcmc_iters, fit_iters)
    acqs = {"monoexp_t2s": synth.Acq(te=synth.echo_times(2.0, 4.0, 12)),
            "gre3": synth.Acq(te=synth.echo_times(2.0, 2.0, 24)),
            "dwi2": synth.dwi_acq(np.random.default_rng(1002))}
    models = {k: g.Model.from_acq(k, a) for k, a in acqs.items()}
    dev = torch.device("cuda:0")
    jobs = []
    for j in trace:
        nx = 64
        ny = (j.n_vox + nx - 1) // nx
        mask = np.zeros((1, ny, nx), np.uint8)
        mask.reshape(-1)[: j.n_vox] = 1
        sigma = SERVE_MODELS[j.model]
        d = synth.make_draw(j.model, (1, ny, nx), j.seed, sigma, acq=acqs[j.model], mask=mask,
                            block=4 if j.model == "dwi2" else 0, noise=False)
        m = models[j.model]
        s = g.gc_model_forward(m, torch.tensor(d.truth, dtype=torch.float32, device=dev))
        gen = torch.Generator(device=dev)
        gen.manual_seed(j.seed)
        s += sigma * torch.randn(s.shape, generator=gen, device=dev, dtype=torch.float32)
        y = np.zeros((s.shape[0], 1, ny, nx), np.float32)
        y.reshape(s.shape[0], -1)[:, : j.n_vox] = s.cpu().numpy()
        del s
        jobs.append((j, d, y, m))
    return jobs


def _digest(r):
    import hashlib
    h = hashlib.sha1()
    for k in ("mean", "std", "maps"):
        if r.get(k) is not None:
            h.update(np.ascontiguousarray(r[k]).tobytes())
    return h.hexdigest()


def serve_run(g, jobs, baseline, saturated, chunk=256):
    """Submits the trace (paced by its arrival times, or all at once when
    saturated), waits for every job, and returns throughput, latency
    percentiles and a digest of every job's results."""
    from paper_2511_22094_amd import synth
    with g.Server(baseline=baseline, chunk_iters=chunk) as srv:
        ids = []
        t0 = time.perf_counter()
        for j, d, y, m in jobs:
            if not saturated:
                wait = j.arrival_s - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
            if j.kind == "mcmc":
                jid = srv.submit_mcmc(m, y, d.mask, d.lb, d.ub, j.n_chains, j.n_iter, j.burnin,
                                      j.thin, sigma=d.sigma, step=synth.MH_STEP[j.model],
                                      seed=j.seed, accept=False)
                work = d.n * j.n_chains * j.n_iter
            else:
                tv = (0, 1, 2) if j.tv else ()
                jid = srv.submit_fit(m, y, d.mask, d.lb, d.ub, n_iter=j.n_iter,
                                     lam=1e-3 if j.tv else 0.0, tv_params=tv)
                work = d.n * j.n_iter
            ids.append((jid, work))
        digests = []
        lat = []
        finite = True
        for k, (jid, _) in enumerate(ids):
            r = srv.wait(jid)
            lat.append(srv.latency(jid))
            digests.append(_digest(r))
            finite &= all(bool(np.isfinite(r[x]).all()) for x in ("mean", "std", "maps")
                          if r.get(x) is not None)
            if (k + 1) % 32 == 0:
                log(f"bench:   {k + 1}/{len(ids)} jobs done, {time.perf_counter() - t0:.1f} s")
        span = time.perf_counter() - t0
        st = srv.stats()
    total = sum(w for _, w in ids)
    return dict(makespan_s=span, value=total / span, p50_s=st["p50_latency_s"],
                p99_s=st["p99_latency_s"], jobs=len(ids), voxel_iters=total,
                finite=finite, latencies=lat, work=[w for _, w in ids]), digests


def batching_bound(jobs, base):
    """What batching can gain on a trace: in the saturated one-job-per-launch
    run jobs complete one after another, so job j's service time is its
    completion time minus the previous job's; the fastest rate any job of a
    (model, solver) class reaches alone stands for that class's full-GPU
    rate; the trace's work at those rates is the shortest time any schedule
    of these kernels can take.  Returns that time and the largest speed-up
    over the one-job-per-launch run it allows."""
    done = np.asarray(base["latencies"])
    order = np.argsort(done)
    service = np.empty_like(done)
    service[order] = np.diff(np.concatenate([[0.0], done[order]]))
    rate = {}
    for (j, d, y, m), w, t in zip(jobs, base["work"], service):
        key = (j.model, j.kind, bool(j.tv))
        if t > 0:
            rate[key] = max(rate.get(key, 0.0), w / t)
    ideal = sum(w / rate[(j.model, j.kind, bool(j.tv))]
                for (j, d, y, m), w in zip(jobs, base["work"]))
    return {"ideal_s": ideal, "max_speedup": base["makespan_s"] / ideal,
            "class_rates": {f"{k[0]}/{k[1]}{'+tv' if k[2] else ''}": v
                            for k, v in sorted(rate.items())}}


SERVE_TRACES = {
    # the serving workload: 256 jobs, voxels log-uniform in [1e3, 1e6], MCMC
    # 1-8 chains x 1k-10k iterations, Adam 200-500 iterations
    "full": (256, (1e3, 1e6), (1000, 10000), (200, 500)),
    # a smaller trace of the same mix (voxels up to 1e5, MCMC up to 4k iterations)
    "small": (64, (1e3, 1e5), (1000, 4000), (200, 500)),
    # the same mix of 256 jobs with voxel counts of single slices and ROIs
    # (log-uniform in [1e2, 1e4]): no job fills the GPU on its own
    "small_jobs": (256, (1e2, 1e4), (1000, 10000), (200, 500)),
}


def serve_leg(g, torch, trace="full", legs=("saturated", "paced")):
    """Saturated legs (every job submitted at once) give the batching ratio at
    full load; paced legs (Poisson arrivals at 20/s) give latency under the
    trace's own load.  Batched and one-job-per-launch results are compared
    job by job (digests of the result arrays)."""
    n_jobs, vr, mi, fi = SERVE_TRACES[trace]
    log(f"bench: serving trace {trace}: generating {n_jobs} jobs")
    t0 = time.perf_counter()
    jobs = serve_trace_jobs(g, torch, n_jobs, vr, mi, fi)
    log(f"bench:   inputs ready in {time.perf_counter() - t0:.1f} s")
    out = {}
    same = True
    for leg in legs:
        sat = leg == "saturated"
        res = {}
        dig = {}
        for mode in ("batched", "baseline"):
            log(f"bench: serving {leg} {mode}")
            res[mode], dig[mode] = serve_run(g, jobs, mode == "baseline", sat)
            log(f"bench:   { {k: v for k, v in res[mode].items() if k not in ('latencies', 'work')} }")
        res["speedup"] = res["batched"]["value"] / res["baseline"]["value"]
        res["identical_results"] = dig["batched"] == dig["baseline"]
        if sat:
            res["bound"] = batching_bound(jobs, res["baseline"])
        for mode in ("batched", "baseline"):
            res[mode].pop("latencies")
            res[mode].pop("work")
        same &= res["identical_results"]
        out[leg] = res
    out["identical_results"] = same
    out["trace"] = (f"Poisson arrivals 20/s, {n_jobs} jobs, models uniform over monoexp_t2s / "
                    f"gre3 / dwi2, voxels log-uniform in [{vr[0]:g}, {vr[1]:g}], 50/50 MCMC "
                    f"(1-8 chains, {mi[0]}-{mi[1]} iterations) / Adam ({fi[0]}-{fi[1]} "
                    "iterations, TV on dwi2); saturated = all submitted at t = 0")
    return out


def host_cpu():
    """Threads this process may run on, and the host CPU model (lscpu)."""
    import subprocess
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env_omp = os.environ.get("OMP_NUM_THREADS")
    if env_omp and env_omp.isdigit():
        threads = min(threads, int(env_omp))
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return threads, model, os.cpu_count()


def cpu_sample(n, k, seed=1234):
    """A fixed random sample of k of the workload's n (compacted) voxels."""
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


def cpu_baseline(which="cfg4", per_thread=64, gpu_moments=None, sample=None):
    """The FP64 oracle on a fixed voxel sample of the MH workload: once on one
    thread (per_thread voxels) and once on every thread this process may use
    (per_thread voxels per thread); the voxel indices of the sample key the
    random streams, so the sampled chains are the ones the GPU runs.  With
    gpu_moments = (mean, std) of the GPU run at `sample`, also the GPU result's
    error against the oracle on that sample."""
    import oracle
    from paper_2511_22094_amd import synth
    _, fn, kwname, seed = MH_WORKLOADS[which]
    d = getattr(synth, fn)()
    kw = getattr(synth, kwname)
    threads, cpu_model, ncpu = host_cpu()
    per_voxel = kw["n_chains"] * kw["n_iter"]

    def run(idx, nt):
        y = (oracle.forward("gre3", d.acq, d.truth[:, idx]) +
             d.sigma * d.noise[:, idx]).astype(np.float32)
        t0 = time.perf_counter()
        ref = oracle.mh("gre3", d.acq, y, d.lb, d.ub, synth.MH_STEP["gre3"], d.sigma, seed,
                        vidx=idx, n_threads=nt, **kw)
        return ref, time.perf_counter() - t0

    one = cpu_sample(d.n, per_thread, seed=4321)
    _, t1 = run(one, 1)
    alln = sample if sample is not None else cpu_sample(d.n, per_thread * threads)
    ref, ta = run(alln, threads)
    single = len(one) * per_voxel / t1
    allc = len(alln) * per_voxel / ta
    out = dict(value=allc, unit="voxel-iterations/s", cores=threads, kind="oracle",
               sample=f"{len(alln)} random voxels of the {which} volume "
                      f"({kw['n_chains']} chains x {kw['n_iter']} iterations each, FP64) on "
                      f"{threads} threads, {ta:.1f} s",
               single_thread={"value": single, "sample": f"{len(one)} voxels, {t1:.1f} s"},
               host={"cpu_model": cpu_model, "cpu_count": ncpu, "threads_used": threads})
    err = None
    if gpu_moments is not None:
        gm, gs = gpu_moments
        sd = np.maximum(ref["std"], 1e-300)
        dm = np.abs(gm - ref["mean"]) / sd
        ds = np.abs(gs - ref["std"]) / sd
        err = {"what": "|GPU - oracle| of the posterior mean and SD, in units of the "
                       "oracle's posterior SD, over the sampled voxels x 9 parameters "
                       "(FP32 chains vs FP64 chains on the same random streams)",
               "voxels": int(len(alln)),
               "mean_median": float(np.median(dm)), "mean_p99": float(np.quantile(dm, 0.99)),
               "sd_median": float(np.median(ds)), "sd_p99": float(np.quantile(ds, 0.99))}
    return out, err


def adam_oracle_error(g, torch, side=16):
    """The Adam+TV workload's recipe on a side^3 volume (TV couples voxels, so
    a cut-out of the 64^3 run would be another problem): GPU against the FP64
    oracle on the same FP32 data, same hyper-parameters."""
    import oracle
    from paper_2511_22094_amd import synth
    d = synth.cfg2(shape=(side, side, side))
    kw = synth.CFG2_ADAM
    y = synth.scatter((oracle.forward("dwi2", d.acq, d.truth) + d.sigma * d.noise)
                      .astype(np.float32), d.mask)
    names = synth.PARAM_NAMES["dwi2"]
    tvp = tuple(names.index(p) for p in kw["tv_params"])
    m = g.Model.from_acq("dwi2", d.acq)
    out = g.gc_fit_askadam(m, y, d.mask, d.lb, d.ub, n_iter=kw["n_iter"], loss=kw["loss"],
                           lam=kw["lam"], tv_params=tvp, tv_dim=kw["tv_dim"], loss_history=True)
    threads = host_cpu()[0]
    orc_kw = dict(loss=kw["loss"], lam=kw["lam"], tv_mask=sum(1 << p for p in tvp),
                  tv_dim=kw["tv_dim"])
    t0 = time.perf_counter()
    ref = oracle.askadam("dwi2", d.acq, d.mask, y, d.lb, d.ub, n_iter=kw["n_iter"],
                         n_threads=threads, **orc_kw)
    t_all = time.perf_counter() - t0
    n1 = 50
    t0 = time.perf_counter()
    oracle.askadam("dwi2", d.acq, d.mask, y, d.lb, d.ub, n_iter=n1, n_threads=1, **orc_kw)
    t_one = time.perf_counter() - t0
    err = np.abs(out["maps"] - ref["maps"]) / (d.ub - d.lb)[:, None, None, None]
    return {"what": f"|GPU - oracle| / (ub - lb) of the 5 maps after {kw['n_iter']} Adam "
                    f"iterations with 3D TV on a {side}^3 volume of the same recipe",
            "median": float(np.median(err)), "p99": float(np.quantile(err, 0.99)),
            "max": float(err.max()),
            "final_loss_rel": float(abs(out["loss"][-1] / ref["loss"][-1] - 1)),
            "cpu_oracle": {
                "value": d.n * kw["n_iter"] / t_all, "unit": "voxel-iterations/s",
                "cores": threads, "kind": "oracle",
                "sample": f"the {side}^3 volume, {kw['n_iter']} iterations, {threads} threads, "
                          f"{t_all:.1f} s",
                "single_thread": {"value": d.n * n1 / t_one,
                                  "sample": f"the {side}^3 volume, {n1} iterations, {t_one:.1f} s"}}}


def paper_context(mh, cpu, adam, adam_err):
    """Speed-ups over one host core of the FP64 oracle beside the ones the
    paper quotes for its own GPU framework against one CPU core (§3.1: an
    NVIDIA A40 against one AMD EPYC core, the NEXI model, 2.5e5 samples: MH
    14,380x, Adam 451x; its MH rate, derived from the quoted times, about
    5.1e7 voxel-chain-iterations/s).  Other models, hardware and code on each
    side: context, not a like-for-like comparison."""
    if cpu is None:
        return None
    out = {"mh_gre3_vs_one_oracle_core": mh["value"] / cpu["single_thread"]["value"],
           "paper_mh_nexi_vs_one_cpu_core": 14380,
           "paper_mh_rate_a40": 5.1e7,
           "paper_adam_nexi_vs_one_cpu_core": 451,
           "paper_setting": "NVIDIA A40 vs one AMD EPYC core, NEXI model, 2.5e5 samples"}
    if adam is not None and adam_err is not None and "cpu_oracle" in adam_err:
        out["adam_tv_dwi2_vs_one_oracle_core"] = (adam["value"] /
                                                   adam_err["cpu_oracle"]["single_thread"]["value"])
    return out


def sense_oracle_error(g, E=6, Nc=8, Ny=64, Nz=64):
    """The reconstruction workload's hyper-parameters on a smaller slice: GPU
    against the FP64 oracle on the same FP32 data."""
    from oracle import sense
    from paper_2511_22094_amd import synth
    kw = synth.SENSE_RECON
    d = synth.sense_draw(43, E, Nc, Ny, Nz, sigma=kw["sigma"])
    k = ((sense.forward(d.truth, d.coils) + d.sigma * d.noise) * d.mask[:, None]).astype(np.complex64)
    C = d.coils.astype(np.complex64)
    out = g.gc_sense_recon(k, C, d.mask, lr=kw["lr"], n_iter=kw["n_iter"], loss=kw["loss"],
                           lam=kw["lam"], loss_history=True)
    img, hist = sense.recon(k.astype(complex), C.astype(complex), d.mask, n_iter=kw["n_iter"],
                            lr=kw["lr"], loss=kw["loss"], lam=kw["lam"])
    err = np.abs(out["image"] - img) / np.abs(img).max()
    rel = np.abs(out["loss"] / hist - 1)
    return {"what": f"|GPU - oracle| / max|I| of the image after {kw['n_iter']} iterations "
                    f"(L1 + TV, {E} echoes x {Nc} coils, {Ny}x{Nz}); L1 residual signs at "
                    "the rounding level let FP32 and FP64 trajectories part, so the loss "
                    "histories are the sharper comparison",
            "median": float(np.median(err)), "p99": float(np.quantile(err, 0.99)),
            "max": float(err.max()), "loss_rel_max": float(rel.max()),
            "final_loss_rel": float(rel[-1])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-adam", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sense", action="store_true")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the ensemble / optimiser / regulariser legs")
    ap.add_argument("--serve-trace", default="full", choices=sorted(SERVE_TRACES),
                    help="serving trace: full (256 jobs, voxels up to 1e6) or small (64 jobs)")
    ap.add_argument("--serve-legs", default="saturated,paced",
                    help="comma list of saturated, paced")
    ap.add_argument("--bandwidth", action="store_true",
                    help="achievable HBM bandwidth of plain torch kernels (no headline line)")
    ap.add_argument("--sweep", action="store_true",
                    help="throughput against volume size per model (no headline line)")
    ap.add_argument("--profile-only", default=None,
                    help="comma list of mh (whole-brain volume), mh1 (128x128x64), adam, sense, ens, "
                         "copy: run only these legs once each (no "
                         "warm-up, no headline line) for hardware counter collection")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2511_22094_amd import lib
    g = lib()
    if args.sweep:
        sweep(g, torch)
        return
    if args.bandwidth:
        bandwidth(torch)
        return
    if args.profile_only:
        legs = [x.strip() for x in args.profile_only.split(",") if x.strip()]
        rep = {}
        for leg in legs:
            log(f"bench: profile leg {leg}")
            if leg in ("mh", "mh1"):
                r = mh_leg(g, torch, 1, 0, "cfg4" if leg == "mh" else "cfg1")
                rep[leg] = {"launches": r["launches"], "per_launch_ms": r["per_launch_ms"]}
            elif leg == "adam":
                r = adam_leg(g, torch, 1, 0)
                rep[leg] = {"per_launch_us": r["per_launch_us"], "n": r["n"]}
            elif leg == "sense":
                r = sense_leg(g, torch, 1, 0)
                rep[leg] = {k: v["launch_us"] for k, v in r["stages"].items()}
            elif leg == "ens":
                r = ens_leg(g, torch, warmup=0)
                rep[leg] = {"launch_ms": r["roofline"]["launch_ms"]}
            elif leg == "copy":
                rep[leg] = copy_leg(torch)
            else:
                raise SystemExit(f"unknown profile leg {leg!r}")
        print(json.dumps({"profile_only": rep}))
        return
    from paper_2511_22094_amd import synth
    n4 = int(synth.cfg4_mask().sum())
    threads = host_cpu()[0]
    sample = cpu_sample(n4, 64 * threads)
    log("bench: MH leg (gre3 whole-brain volume, 1,199,888 voxels, 8 chains x 10000)")
    mh = mh_leg(g, torch, args.steps, args.warmup, "cfg4", sample=sample)
    log(f"bench: MH {mh['value']:.3e} voxel-iter/s, {mh['sec']:.3f} s/step, "
        f"kernel {mh['per_launch_ms']:.2f} ms/launch")
    log("bench: MH leg (gre3 128x128x64, 4 chains x 5000)")
    mh1 = mh_leg(g, torch, max(1, min(args.steps, 5)), min(args.warmup, 1), "cfg1")
    log(f"bench: MH {mh1['value']:.3e} voxel-iter/s, {mh1['sec']:.3f} s/step, "
        f"kernel {mh1['per_launch_ms']:.2f} ms/launch")
    adam = None
    if not args.no_adam:
        log("bench: Adam+TV leg (dwi2 64^3, 500 iterations)")
        adam = adam_leg(g, torch, args.steps, args.warmup)
        log(f"bench: Adam {adam['value']:.3e} voxel-iter/s, step kernel "
            f"{adam['per_launch_us']:.1f} us")
    sense = None
    if not args.no_sense:
        log("bench: reconstruction leg (6 echoes x 32 coils, 256 x 256, 500 iterations)")
        sense = sense_leg(g, torch, args.steps, args.warmup)
        log(f"bench: reconstruction {sense['value']:.1f} iterations/s, "
            + ", ".join(f"{k} {v['launch_us']:.1f} us" for k, v in sense["stages"].items()))
    nxt = None
    if not args.no_next:
        log("bench: next-row legs (ensemble, optimisers, regularisers)")
        nxt = next_rows_leg(g, torch)
        for k, v in nxt.items():
            log(f"bench:   {k}: {v['value']:.3e} {v['unit']}, frac {v['roofline']['frac']:.3f}")
    serve = serve_small = None
    if not args.no_serve:
        serve = serve_leg(g, torch, args.serve_trace,
                          tuple(x for x in args.serve_legs.split(",") if x))
        if args.serve_trace == "full":
            serve_small = serve_leg(g, torch, "small_jobs", ("saturated",))
    cpu = oracle_err = adam_err = sense_err = None
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        cpu, oracle_err = cpu_baseline("cfg4", 64, gpu_moments=mh["moments"], sample=sample)
        log(f"bench: CPU {cpu['value']:.3e} voxel-iter/s on {cpu['cores']} threads, "
            f"{cpu['single_thread']['value']:.3e} on one")
        if adam is not None:
            log("bench: Adam+TV error against the oracle (16^3)")
            adam_err = adam_oracle_error(g, torch)
            log(f"bench:   {adam_err}")
        if nxt is not None:
            log("bench: next-row errors against the oracle")
            for k, v in next_rows_oracle_error(g, torch).items():
                nxt[k]["oracle_error"] = v
                log(f"bench:   {k}: {v}")
        if sense is not None:
            log("bench: reconstruction error against the oracle (6 x 8 x 64 x 64)")
            sense_err = sense_oracle_error(g)
            log(f"bench:   {sense_err}")
    out = {
        "metric": "voxel-iterations/sec (MCMC MH & Adam steps) at 1 GPU",
        "value": mh["value"],
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mh["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": MH_WORKLOADS["cfg4"][0], "voxels": mh["n"],
                   "chains": mh["kw"]["n_chains"], "iterations": mh["kw"]["n_iter"],
                   "burnin": mh["kw"]["burnin"], "thin": mh["kw"]["thin"]},
        "roofline": {"bound": "alu", "kernel": "mh_chunk<gre3,f32,24>",
                     "achieved": mh["achieved_tflops"], "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": mh["achieved_tflops"] / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic("mh_chunk_cfg4"),
                     "flop_per_step": FLOP_PER_MH_STEP_GRE3,
                     "mix_ceiling": MH_GRE3_MIX_CEILING,
                     "frac_of_ceiling": (mh["achieved_tflops"] / PEAK_FP32_TFLOPS /
                                         MH_GRE3_MIX_CEILING),
                     "steps_per_launch": mh["units_per_launch"],
                     "launch_ms": mh["per_launch_ms"]},
        "pack": mh["gather"],
        "cpu_baseline": cpu,
        "speedup_vs_cpu_oracle": (mh["value"] / cpu["value"]) if cpu else None,
        "paper_context": paper_context(mh, cpu, adam, adam_err),
        "oracle_error": oracle_err,
        "mh_128x128x64": {
            "value": mh1["value"], "unit": "voxel-iterations/s", "ms_per_step": mh1["sec"] * 1e3,
            "workload": MH_WORKLOADS["cfg1"][0],
            "roofline": {"bound": "alu", "kernel": "mh_chunk<gre3,f32,24>",
                         "achieved": mh1["achieved_tflops"], "peak": PEAK_FP32_TFLOPS,
                         "unit": "TFLOP/s", "frac": mh1["achieved_tflops"] / PEAK_FP32_TFLOPS,
                         "traffic": measured_traffic("mh_chunk_cfg1"),
                         "steps_per_launch": mh1["units_per_launch"],
                         "launch_ms": mh1["per_launch_ms"]}},
    }
    if adam is not None:
        out["adam"] = {"value": adam["value"], "unit": "voxel-iterations/s",
                       "ms_per_step": adam["sec"] * 1e3,
                       "workload": "dwi2 stick+ball, 64^3 voxels, 96 measurements, Adam 500 "
                                   "iterations, 3D TV lambda 1e-3 on f, Da, De",
                       "roofline": {"bound": "hbm", "kernel": "fit_step<dwi2>",
                                    "achieved": adam["achieved_gbs"], "peak": PEAK_HBM_GBS,
                                    "unit": "GB/s", "frac": adam["achieved_gbs"] / PEAK_HBM_GBS,
                                    "traffic": measured_traffic("fit_step"),
                                    "bytes_per_voxel_iter": BYTES_PER_ADAM_TV_VOXEL_ITER,
                                    "launch_us": adam["per_launch_us"]},
                       "oracle_error": adam_err}
    if sense is not None:
        dom = max(sense["stages"], key=lambda k: sense["stages"][k]["launch_us"])
        st = sense["stages"][dom]
        out["sense"] = {"value": sense["value"], "unit": "iterations/s",
                        "ms_per_step": sense["sec"] * 1e3,
                        "workload": "SENSE recon, 1 slice: 6 echoes, 32 coils, 256x256, CAIPI "
                                    "R_z=9, L1 + 2D TV lambda 0.002, Adam (rate 0.1) 500 iterations",
                        "rel_err_vs_truth": sense["rel_err"],
                        "stages_us": {k: v["launch_us"] for k, v in sense["stages"].items()},
                        "roofline": {"bound": "hbm", "kernel": dom,
                                     "achieved": st["achieved_gbs"], "peak": PEAK_HBM_GBS,
                                     "unit": "GB/s", "frac": st["achieved_gbs"] / PEAK_HBM_GBS,
                                     "traffic": measured_traffic(dom),
                                     "bytes_per_launch": st["bytes"],
                                     "launch_us": st["launch_us"]},
                        "oracle_error": sense_err}
    if nxt is not None:
        out["next_rows"] = nxt
    if serve is not None:
        out["serving"] = serve
    if serve_small is not None:
        out["serving_small_jobs"] = serve_small
    print(json.dumps(out))


if __name__ == "__main__":
    main()
