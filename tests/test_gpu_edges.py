"""Edge cases of the sampling and fitting entry points against the oracle:
the largest walker count an ensemble takes, many chains per voxel, the
smallest retention a call allows, a single masked voxel, a one-iteration
fit, and parameters pinned at a bound."""
import numpy as np
import pytest

from gpu_util import G, say
from paper_2511_22094_amd import synth

pytestmark = pytest.mark.gpu


def _y(orc, d):
    y = (orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise).astype(np.float32)
    return y, synth.scatter(y, d.mask)


def _one_voxel_mask(shape, at):
    m = np.zeros(shape, np.uint8)
    m[at] = 1
    return m


def test_ensemble_largest_walker_count_fp64_bit_exact(orc):
    # 512 walkers: one voxel per block, both half-ensembles of 256 lanes
    d = synth.make_draw("monoexp_t2s", (1, 2, 3), 5, 0.02)
    y, yg = _y(orc, d)
    kw = dict(n_iter=40, burnin=10, thin=5)
    ref = orc.ensemble(d.model, d.acq, y, d.lb, d.ub, d.sigma, 9, 512, stretch=2.0, **kw)
    out = G().gc_mcmc(G().Model.from_acq(d.model, d.acq), yg, d.mask, d.lb, d.ub, 1,
                      sigma=d.sigma, seed=9, sampler="ensemble", n_walkers=512, stretch=2.0,
                      precision="fp64", final_state=True, **kw)
    assert np.array_equal(synth.gather(out["accept"], d.mask), ref["accept"])
    np.testing.assert_allclose(out["final_state"], ref["final"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(synth.gather(out["mean"], d.mask), ref["mean"], rtol=1e-11)


def test_mh_many_chains_fp64_bit_exact(orc):
    # 1,000 chains of 3 voxels: chain-major lanes span many blocks per voxel
    d = synth.make_draw("monoexp_t2s", (1, 1, 3), 6, 0.02)
    y, yg = _y(orc, d)
    kw = dict(n_chains=1000, n_iter=60, burnin=20, thin=4)
    step = synth.MH_STEP[d.model]
    ref = orc.mh(d.model, d.acq, y, d.lb, d.ub, step, d.sigma, 17, **kw)
    out = G().gc_mcmc(G().Model.from_acq(d.model, d.acq), yg, d.mask, d.lb, d.ub,
                      sigma=d.sigma, step=step, seed=17, precision="fp64", **kw)
    assert ref["margin"].min() > 1e-9
    assert np.array_equal(synth.gather(out["accept"], d.mask), ref["accept"])
    np.testing.assert_allclose(synth.gather(out["mean"], d.mask), ref["mean"], rtol=1e-11)
    np.testing.assert_allclose(synth.gather(out["std"], d.mask), ref["std"], rtol=1e-9)


def test_smallest_retention_and_single_voxel(orc):
    # n_iter = burnin + 2 thin keeps exactly two draws per chain; one voxel
    shape = (3, 4, 5)
    mask = _one_voxel_mask(shape, (2, 3, 4))
    d = synth.make_draw("gre3", shape, 7, 0.01, mask=mask)
    y, yg = _y(orc, d)
    kw = dict(n_chains=3, n_iter=30, burnin=10, thin=10)
    step = synth.MH_STEP[d.model]
    ref = orc.mh(d.model, d.acq, y, d.lb, d.ub, step, d.sigma, 3, keep_samples=True, **kw)
    out = G().gc_mcmc(G().Model.from_acq(d.model, d.acq), yg, d.mask, d.lb, d.ub,
                      sigma=d.sigma, step=step, seed=3, precision="fp64", samples=True, **kw)
    assert out["samples"].shape == (3, 2, d.n_params, 1)
    assert np.array_equal(synth.gather(out["accept"], d.mask), ref["accept"])
    np.testing.assert_allclose(out["samples"], ref["samples"].astype(np.float32), rtol=1e-6)
    np.testing.assert_allclose(synth.gather(out["std"], d.mask), ref["std"], rtol=1e-9)
    assert np.all(out["mean"][:, d.mask == 0] == 0)
    with pytest.raises(G().GcError) as e:       # one retained draw per chain: refused
        G().gc_mcmc(G().Model.from_acq(d.model, d.acq), yg, d.mask, d.lb, d.ub,
                    sigma=d.sigma, step=step, n_chains=3, n_iter=29, burnin=10, thin=10)
    assert e.value.code == -1


def test_one_iteration_fit_and_single_voxel(orc):
    shape = (2, 3, 4)
    mask = _one_voxel_mask(shape, (1, 2, 3))
    d = synth.make_draw("monoexp_r2s", shape, 8, 0.01, mask=mask)
    _, yg = _y(orc, d)
    m = G().Model.from_acq(d.model, d.acq)
    for tv in (False, True):     # the fused loop and the per-iteration step
        kw = dict(lam=1e-3, tv_params=(0, 1)) if tv else {}
        out = G().gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=1, **kw)
        ref = orc.askadam(d.model, d.acq, d.mask, yg, d.lb, d.ub, n_iter=1,
                          lam=1e-3 if tv else 0.0, tv_mask=0b11 if tv else 0, tv_dim=3)
        err = np.abs(out["maps"] - ref["maps"]).max() / (d.ub - d.lb).max()
        say("one-iteration fit, tv", tv, "max err / range", err)
        assert out["iters_run"] == 1 and err < 1e-6
        assert np.all(out["maps"][:, d.mask == 0] == 0)


def test_start_at_a_bound(orc):
    # chains started on the upper bound: proposals beyond it are rejected and
    # the chains stay inside the box, decision for decision with the oracle
    d = synth.make_draw("monoexp_t2s", (1, 4, 4), 10, 0.02)
    y, yg = _y(orc, d)
    C, kw = 2, dict(n_iter=80, burnin=20, thin=5)
    x0 = np.broadcast_to(d.ub[:, None], (d.n_params, d.n)).copy()
    step = synth.MH_STEP[d.model]
    ref = orc.mh(d.model, d.acq, y, d.lb, d.ub, step, d.sigma, 21, C,
                 x0=np.broadcast_to(x0, (C,) + x0.shape), **kw)
    out = G().gc_mcmc(G().Model.from_acq(d.model, d.acq), yg, d.mask, d.lb, d.ub, C,
                      sigma=d.sigma, step=step, seed=21, precision="fp64", final_state=True,
                      x0_map=synth.scatter(x0.astype(np.float32), d.mask), x0_mode="given",
                      **kw)
    assert ref["margin"].min() > 1e-9
    assert np.array_equal(synth.gather(out["accept"], d.mask), ref["accept"])
    fin = out["final_state"]
    assert np.all(fin <= d.ub[:, None, None]) and np.all(fin >= d.lb[:, None, None])
    np.testing.assert_allclose(fin.reshape(d.n_params, C, d.n).transpose(1, 0, 2), ref["final"],
                               rtol=1e-12, atol=1e-12)
