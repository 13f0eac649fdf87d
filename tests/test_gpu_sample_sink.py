"""Streaming of retained MCMC samples (gc_mcmc_hyper.sample_sink): the draws
handed to the sink, delivery by delivery, are bit for bit the samples an
in-memory call returns, for MH in both precisions (also when resuming) and
for the ensemble sampler; deliveries arrive in order and cover every draw;
a sink that declines stops the call.  The whole-brain-sized run with
samples on is in test_gpu_fullsize.py."""
import numpy as np
import pytest

from gpu_util import G, say
from paper_2511_22094_amd import synth

pytestmark = pytest.mark.gpu


def _data(orc, model, shape, seed, sigma, masked=True):
    d = synth.make_draw(model, shape, seed, sigma)
    if masked:   # a ragged mask: every third voxel out
        m = np.ones(int(np.prod(shape)), np.uint8)
        m[::3] = 0
        d = synth.make_draw(model, shape, seed, sigma, mask=m.reshape(shape))
    y = (orc.forward(model, d.acq, d.truth) + sigma * d.noise).astype(np.float32)
    return d, synth.scatter(y, d.mask)


class Collector:
    def __init__(self, C, K, P, n):
        self.buf = np.full((C, K, P, n), np.nan, np.float32)
        self.calls = []

    def __call__(self, k_first, s):
        self.calls.append((k_first, s.shape[1]))
        self.buf[:, k_first:k_first + s.shape[1]] = s
        return True


def _per_draw(C, P, n):
    return C * P * n * 4


@pytest.mark.parametrize("model,prec,kw,draws_per_delivery,chunk", [
    ("gre3", "fp32", dict(n_chains=4, n_iter=600, burnin=100, thin=5), 3, 7),
    ("gre3", "fp64", dict(n_chains=3, n_iter=400, burnin=50, thin=10), 4, 0),
    ("monoexp_t2s", "fp32", dict(n_chains=2, n_iter=500, burnin=0, thin=1), 64, 33),
    ("dwi2", "fp32", dict(n_chains=4, n_iter=300, burnin=100, thin=2), 1, 0),
])
def test_streamed_samples_equal_in_memory(orc, model, prec, kw, draws_per_delivery, chunk):
    g = G()
    sigma = 0.02
    d, y = _data(orc, model, (3, 5, 7), 11, sigma)
    m = g.Model.from_acq(model, d.acq)
    common = dict(sigma=sigma, step=synth.MH_STEP[model], seed=5, precision=prec,
                  chunk_iters=chunk, **kw)
    C, P, n = kw["n_chains"], d.lb.size, d.n
    ref = g.gc_mcmc(m, y, d.mask, d.lb, d.ub, samples=True, **common)
    K = ref["samples"].shape[1]
    col = Collector(C, K, P, n)
    out = g.gc_mcmc(m, y, d.mask, d.lb, d.ub, sample_sink=col,
                    sink_bytes=draws_per_delivery * _per_draw(C, P, n) + 5, **common)
    say(model, prec, "deliveries", len(col.calls), "K", K)
    kc = min(K, draws_per_delivery)
    assert col.calls == [(k, min(kc, K - k)) for k in range(0, K, kc)]
    assert np.array_equal(col.buf, ref["samples"])
    assert np.array_equal(out["mean"], ref["mean"]) and np.array_equal(out["std"], ref["std"])
    assert np.array_equal(out["accept"], ref["accept"])


def test_streamed_samples_when_resuming(orc):
    g = G()
    d, y = _data(orc, "monoexp_t2s", (2, 6, 6), 12, 0.01)
    m = g.Model.from_acq(d.model, d.acq)
    kw = dict(sigma=0.01, step=synth.MH_STEP[d.model], seed=9, precision="fp32")
    first = g.gc_mcmc(m, y, d.mask, d.lb, d.ub, 2, 250, 100, 5, final_state=True, **kw)
    res = dict(t_start=250, init_state=first["final_state"], init_logl=first["final_logl"])
    ref = g.gc_mcmc(m, y, d.mask, d.lb, d.ub, 2, 700, 100, 5, samples=True, **res, **kw)
    K = ref["samples"].shape[1]
    col = Collector(2, K, 2, d.n)
    g.gc_mcmc(m, y, d.mask, d.lb, d.ub, 2, 700, 100, 5, sample_sink=col,
              sink_bytes=7 * _per_draw(2, 2, d.n), **res, **kw)
    assert col.calls[0][0] == 0 and sum(c[1] for c in col.calls) == K
    assert np.array_equal(col.buf, ref["samples"])


def test_streamed_ensemble_samples(orc):
    g = G()
    d, y = _data(orc, "monoexp_t2s", (2, 4, 9), 13, 0.02)
    m = g.Model.from_acq(d.model, d.acq)
    kw = dict(sigma=0.02, seed=3, sampler="ensemble", n_walkers=12, precision="fp64")
    ref = g.gc_mcmc(m, y, d.mask, d.lb, d.ub, 1, 300, 60, 4, samples=True, **kw)
    K = ref["samples"].shape[1]
    col = Collector(12, K, 2, d.n)
    out = g.gc_mcmc(m, y, d.mask, d.lb, d.ub, 1, 300, 60, 4, sample_sink=col,
                    sink_bytes=5 * _per_draw(12, 2, d.n), **kw)
    assert np.array_equal(col.buf, ref["samples"])
    assert np.array_equal(out["mean"], ref["mean"])


def test_sink_that_declines_stops_the_call(orc):
    g = G()
    d, y = _data(orc, "gre3", (2, 4, 4), 14, 0.01, masked=False)
    m = g.Model.from_acq(d.model, d.acq)
    seen = []

    def sink(k_first, s):
        seen.append(k_first)
        return len(seen) < 3

    with pytest.raises(g.GcError) as e:
        g.gc_mcmc(m, y, None, d.lb, d.ub, 2, 2000, 0, 1, sigma=0.01,
                  step=synth.MH_STEP["gre3"], seed=1, sample_sink=sink,
                  sink_bytes=10 * _per_draw(2, 9, d.n))
    assert e.value.code == -6 and seen == [0, 10, 20]
    with pytest.raises(g.GcError) as e:   # both outputs at once is refused
        g.gc_mcmc(m, y, None, d.lb, d.ub, 2, 200, 0, 1, sigma=0.01, samples=True,
                  sample_sink=lambda k, s: True)
    assert e.value.code == -1
