"""The continuous-batching server: every job's result is bit-identical to the
synchronous call (alone) whatever the mix, the admission budget, the
arrival pattern or the comparison (one-job-per-launch) mode; failures and
cancellations stay with their job."""
import ctypes
import time

import numpy as np
import pytest

from gpu_util import G, say
from paper_2511_22094_amd import synth

pytestmark = pytest.mark.gpu


def _job_specs():
    import oracle as orc
    specs = []

    def data(model, shape, seed, sigma, acq=None, block=0):
        d = synth.make_draw(model, shape, seed, sigma, acq=acq, block=block)
        y = (orc.forward(model, d.acq, d.truth) + sigma * d.noise).astype(np.float32)
        return d, synth.scatter(y, d.mask)

    d, y = data("monoexp_t2s", (10, 10, 10), 0, 0.01)
    specs.append(("mcmc", d, y, dict(n_chains=1, n_iter=600, burnin=100, thin=1,
                                     sigma=0.01, step=synth.MH_STEP[d.model], seed=0)))
    d, y = data("gre3", (4, 8, 8), 1, 0.01)
    specs.append(("mcmc", d, y, dict(n_chains=4, n_iter=800, burnin=100, thin=10,
                                     sigma=0.01, step=synth.MH_STEP[d.model], seed=1)))
    acq = synth.dwi_acq(np.random.default_rng(3), dirs_per_shell=8)
    d, y = data("dwi2", (3, 5, 6), 2, 0.02, acq=acq)
    specs.append(("mcmc", d, y, dict(n_chains=2, n_iter=300, burnin=50, thin=5, sigma=0.02,
                                     step=synth.MH_STEP[d.model], seed=2, precision="fp64")))
    d, y = data("monoexp_t2s", (2, 6, 7), 3, 0.02)
    specs.append(("mcmc", d, y, dict(n_chains=1, n_iter=300, burnin=50, thin=5, sigma=0.02,
                                     seed=3, sampler="ensemble", n_walkers=12)))
    d, y = data("monoexp_r2s", (5, 6, 7), 4, 0.01)
    specs.append(("fit", d, y, dict(n_iter=200)))
    d, y = data("dwi2", (6, 6, 6), 5, 0.02, acq=acq, block=3)
    specs.append(("fit", d, y, dict(n_iter=60, lam=1e-3, tv_params=(0, 1, 2), tv_dim=3)))
    d, y = data("gre3", (3, 5, 5), 6, 0.01)
    specs.append(("fit", d, y, dict(n_iter=300, tol=1e-6)))
    # regularisers: graph TV with the prior (step path), isotropic 2D TV, and
    # the prior alone (fused path)
    from graphs import grid_graph
    rng = np.random.default_rng(77)

    def prior_maps(d):
        P = d.lb.size
        r = (d.ub - d.lb)[:, None, None, None]
        mu = (d.lb[:, None, None, None] + r * rng.uniform(0.3, 0.7, (P,) + d.mask.shape))
        return mu.astype(np.float32), (0.2 * r * np.ones((P,) + d.mask.shape)).astype(np.float32)

    d, y = data("dwi2", (4, 5, 6), 7, 0.02, acq=acq, block=3)
    mu, sg = prior_maps(d)
    specs.append(("fit", d, y, dict(n_iter=60, lam=1e-3, tv_params=(0, 1, 2), tv_kind="graph",
                                    graph=grid_graph(d.mask, 3), prior_lam=1e-3,
                                    prior_params=(1,), prior_mu=mu, prior_sigma=sg)))
    d, y = data("dwi2", (3, 6, 6), 8, 0.02, acq=acq, block=3)
    specs.append(("fit", d, y, dict(n_iter=40, lam=1e-3, tv_params=(0,), tv_dim=2,
                                    tv_kind="iso")))
    d, y = data("monoexp_t2s", (3, 6, 6), 9, 0.02)
    mu, sg = prior_maps(d)
    specs.append(("fit", d, y, dict(n_iter=150, prior_lam=1e-3, prior_params=(0, 1),
                                    prior_mu=mu, prior_sigma=sg)))
    return specs


def _sync(g, kind, d, y, kw):
    m = g.Model.from_acq(d.model, d.acq)
    if kind == "mcmc":
        kw = dict(kw)
        C, it, b, th = kw.pop("n_chains"), kw.pop("n_iter"), kw.pop("burnin"), kw.pop("thin")
        return g.gc_mcmc(m, y, d.mask, d.lb, d.ub, C, it, b, th, **kw)
    return g.gc_fit_askadam(m, y, d.mask, d.lb, d.ub, **kw)


def _submit(srv, g, kind, d, y, kw, models):
    m = g.Model.from_acq(d.model, d.acq)
    models.append(m)
    if kind == "mcmc":
        kw = dict(kw)
        C, it, b, th = kw.pop("n_chains"), kw.pop("n_iter"), kw.pop("burnin"), kw.pop("thin")
        return srv.submit_mcmc(m, y, d.mask, d.lb, d.ub, C, it, b, th, **kw)
    return srv.submit_fit(m, y, d.mask, d.lb, d.ub, **kw)


def _same(kind, a, b):
    if kind == "mcmc":
        assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["std"], b["std"])
        assert np.array_equal(a["accept"], b["accept"])
    else:
        assert np.array_equal(a["maps"], b["maps"])
        assert a["iters_run"] == b["iters_run"] and a["stop_reason"] == b["stop_reason"]
        assert a["final_loss"] == pytest.approx(b["final_loss"], rel=1e-12)


@pytest.fixture(scope="module")
def specs_and_alone():
    g = G()
    specs = _job_specs()
    alone = [_sync(g, k, d, y, kw) for k, d, y, kw in specs]
    return specs, alone


@pytest.mark.parametrize("mode", ["batched", "baseline", "tight_budget", "staggered"])
def test_results_identical_alone_and_in_mix(specs_and_alone, mode):
    g = G()
    specs, alone = specs_and_alone
    kw = dict(baseline=(mode == "baseline"), chunk_iters=128)
    if mode == "tight_budget":
        kw["hbm_budget"] = 48 << 20     # only a few jobs resident at once
    models = []
    with g.Server(**kw) as srv:
        ids = []
        order = list(range(len(specs)))[::-1] if mode == "staggered" else range(len(specs))
        for i in order:
            k, d, y, jkw = specs[i]
            ids.append((i, _submit(srv, g, k, d, y, jkw, models)))
            if mode == "staggered":
                time.sleep(0.02)
        for i, jid in ids:
            r = srv.wait(jid)
            say(mode, i, specs[i][0], specs[i][1].model, "latency", srv.latency(jid))
            _same(specs[i][0], r, alone[i])
        st = srv.stats()
        say(mode, st)
        assert st["completed"] == len(specs) and st["failed"] == 0
        assert st["p99_latency_s"] >= st["p50_latency_s"] > 0
        assert st["voxel_iters"] > 0 and st["resident"] == 0 and st["hbm_in_use"] == 0


def test_failure_and_cancel_stay_with_their_job(specs_and_alone):
    g = G()
    specs, alone = specs_and_alone
    models = []
    with g.Server(chunk_iters=64) as srv:
        k, d, y, kw = specs[1]
        good = _submit(srv, g, k, d, y, kw, models)
        bad_y = y.copy()
        bad_y[0, 1, 2, 3] = np.nan
        bad = _submit(srv, g, k, d, bad_y, kw, models)
        long_kw = dict(kw, n_iter=200000)
        victim = _submit(srv, g, k, d, y, long_kw, models)
        srv.cancel(victim)
        r = srv.wait(good)
        _same(k, r, alone[1])
        with pytest.raises(g.GcError) as e:
            srv.wait(bad)
        assert e.value.code == -4
        with pytest.raises(g.GcError) as e:
            srv.wait(victim)
        assert e.value.code == -6
        assert srv.poll(victim) == "cancelled"
        st = srv.stats()
        assert st["failed"] == 1 and st["cancelled"] == 1 and st["completed"] == 1


def test_oversized_job_is_refused():
    g = G()
    d = synth.make_draw("monoexp_t2s", (8, 8, 8), 0, 0.01)
    y = np.zeros((12, 8, 8, 8), np.float32)
    m = g.Model.from_acq(d.model, d.acq)
    with g.Server(hbm_budget=1 << 20) as srv:
        with pytest.raises(g.GcError) as e:
            srv.submit_mcmc(m, y, None, d.lb, d.ub, 1, 100, 10, 1, sigma=0.01)
        assert e.value.code == -3


def test_jobs_outlive_their_model_handle_and_are_released(specs_and_alone):
    """A caller may destroy its model right after submitting (the server holds
    its own reference), and waited-for jobs are released on both sides."""
    import gc as pygc
    g = G()
    specs, alone = specs_and_alone
    with g.Server(chunk_iters=64) as srv:
        ids = []
        for i in (1, 5):
            k, d, y, kw = specs[i]
            tmp = []
            ids.append((i, _submit(srv, g, k, d, y, kw, tmp)))
            # drop the caller's handle at once, as a C caller may
            m = tmp.pop()
            g._L.gc_model_destroy(m.handle)
            m.handle = None
            del m, tmp
            pygc.collect()
        for i, jid in ids:
            r = srv.wait(jid)
            _same(specs[i][0], r, alone[i])
            assert srv.poll(jid) == "done" and srv.latency(jid) > 0
            assert jid not in srv._jobs
            st = ctypes.c_int()
            assert g._L.gc_poll(srv.handle, jid, ctypes.byref(st)) == -8   # released
        assert srv.stats()["completed"] == 2
