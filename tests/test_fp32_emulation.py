"""The FP32 re-run of the fit (tests/fp32_emulation.py), whose spread against
the oracle sets the GPU fits' tolerances, is the oracle's algorithm: one
plain gradient step reproduces the oracle's data + TV gradient (all three TV
forms) to FP32 accuracy, fits without TV -- where nothing amplifies
rounding -- stay within FP32 rounding of the oracle, and run in FP64 the
same code reproduces the oracle's fits, with and without TV, to FP64
rounding."""
import numpy as np
import pytest

import fp32_emulation as em
from graphs import grid_graph
from paper_2511_22094_amd import synth


def _y(orc, d):
    return synth.scatter((orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise)
                         .astype(np.float32), d.mask)


@pytest.mark.parametrize("kind", ["aniso", "iso", "graph"])
def test_one_step_gradient_matches_oracle(orc, kind):
    acq = synth.dwi_acq(np.random.default_rng(2), dirs_per_shell=10)
    d = synth.make_draw("dwi2", (4, 5, 6), 31, 0.02, acq=acq, block=2)
    y = _y(orc, d)
    rng = np.random.default_rng(32)
    x0 = (d.lb[:, None, None, None] + (d.ub - d.lb)[:, None, None, None] *
          rng.uniform(0.2, 0.8, (5,) + d.mask.shape))
    kw = dict(n_iter=1, optimizer="sgdm", lr=100.0, lam=0.05, tv_mask=0b111, tv_dim=3,
              tv_kind=kind, graph=grid_graph(d.mask, 3) if kind == "graph" else None)
    ref = orc.askadam("dwi2", d.acq, d.mask, y, d.lb, d.ub, x0=x0, **kw)
    emu, _ = em.askadam("dwi2", d.acq, d.mask, y, d.lb, d.ub, x0=x0, **kw)
    sel = d.mask.astype(bool)
    du_r = ref["maps"][:, sel] - x0[:, sel]
    du_e = emu - x0[:, sel]
    rel = np.abs(du_e - du_r).max(axis=1) / np.abs(du_r).max(axis=1)
    assert rel.max() < 1e-5, rel


@pytest.mark.parametrize("model", ["monoexp_r2s", "gre3", "dwi2", "linear3"])
def test_fit_without_tv_within_fp32_rounding(orc, model):
    acq = (synth.dwi_acq(np.random.default_rng(2), dirs_per_shell=10) if model == "dwi2"
           else synth.default_acq(model))
    d = synth.make_draw(model, (2, 5, 6), 33, 0.01, acq=acq)
    y = _y(orc, d)
    ref = orc.askadam(model, d.acq, d.mask, y, d.lb, d.ub, n_iter=100)
    emu, hist = em.askadam(model, d.acq, d.mask, y, d.lb, d.ub, n_iter=100)
    err = np.abs(emu - ref["maps"][:, d.mask.astype(bool)]) / (d.ub - d.lb)[:, None]
    assert err.max() < 3e-5, err.max()
    np.testing.assert_allclose(hist, ref["loss"], rtol=1e-4)


@pytest.mark.parametrize("tv", [None, "aniso", "graph"])
def test_fp64_run_reproduces_the_oracle(orc, tv):
    acq = synth.dwi_acq(np.random.default_rng(2), dirs_per_shell=8)
    d = synth.make_draw("dwi2", (4, 5, 6), 2, 0.02, acq=acq, block=2)
    y = _y(orc, d)
    kw = dict(n_iter=60)
    if tv:
        kw.update(lam=1e-3, tv_mask=0b111, tv_dim=3, tv_kind=tv,
                  graph=grid_graph(d.mask, 3) if tv == "graph" else None)
    ref = orc.askadam("dwi2", d.acq, d.mask, y, d.lb, d.ub, **kw)
    emu, hist = em.askadam("dwi2", d.acq, d.mask, y, d.lb, d.ub, dtype=np.float64, **kw)
    err = np.abs(emu - ref["maps"][:, d.mask.astype(bool)]) / (d.ub - d.lb)[:, None]
    assert err.max() < 1e-12, err.max()
    np.testing.assert_allclose(hist, ref["loss"], rtol=1e-12)
