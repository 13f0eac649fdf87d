"""Checkpoint / resume of the whole-volume fit (paper §2.2.1): a fit stopped
after t iterations and resumed from its optimiser state (u, m, v) gives the
iterates, losses and stopping decision of one uninterrupted fit, bit for
bit, on both kernel shapes (the fused loop without TV, the per-iteration
step with TV and a convergence window)."""
import numpy as np
import pytest

from gpu_util import G, say
from paper_2511_22094_amd import synth

pytestmark = pytest.mark.gpu


def _inputs(orc, d):
    y = (orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise).astype(np.float32)
    return synth.scatter(y, d.mask)


@pytest.mark.parametrize("optimizer", ["adam", "sgdm", "rmsprop"])
def test_fused_fit_resumes_bit_exact(orc, optimizer):
    d = synth.make_draw("gre3", (3, 7, 9), 12, 0.01)
    yg = _inputs(orc, d)
    g = G()
    m = g.Model.from_acq(d.model, d.acq)
    kw = dict(optimizer=optimizer, lr=0.01 if optimizer == "adam" else 0.002)
    full = g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=300, final_state=True, **kw)
    first = g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=120, final_state=True, **kw)
    rest = g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=300, t_start=120,
                            init_state=first["final_state"], final_state=True, **kw)
    assert rest["iters_run"] == 300
    assert np.array_equal(rest["maps"], full["maps"])
    assert np.array_equal(rest["final_state"], full["final_state"])
    assert rest["final_loss"] == full["final_loss"]
    # the state's iterate is the returned maps in normalised units
    n = int(d.mask.sum())
    assert full["final_state"].shape == (3, d.n_params, n)
    u = full["final_state"][0]
    th = (d.lb[:, None] + (d.ub - d.lb)[:, None] * u).astype(np.float32)
    np.testing.assert_allclose(full["maps"][:, d.mask.astype(bool)], th, rtol=1e-6, atol=1e-6)


def test_step_fit_with_tv_and_window_resumes_bit_exact(orc):
    acq = synth.dwi_acq(np.random.default_rng(2), dirs_per_shell=10)
    d = synth.make_draw("dwi2", (4, 6, 8), 31, 0.02, acq=acq, block=2)
    yg = _inputs(orc, d)
    g = G()
    m = g.Model.from_acq(d.model, d.acq)
    kw = dict(lam=1e-3, tv_params=(0, 1, 2), tv_dim=3, conv_window=20)
    # a window threshold that stops the fit part-way: the median |slope|
    # over the windows of an unstopped run
    free = g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=400, loss_history=True, **kw)
    L = free["loss"]
    W = kw["conv_window"]
    t = np.arange(W, dtype=np.float64)
    slopes = [abs(np.polyfit(t, L[k - W:k], 1)[0]) for k in range(W, len(L) + 1)]
    conv = float(np.median(slopes))
    full = g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=400, conv_value=conv,
                            loss_history=True, final_state=True, **kw)
    say("resume: stopped at", full["iters_run"], "reason", full["stop_reason"])
    assert full["stop_reason"] == 2 and W <= full["iters_run"] < 400
    cut = full["iters_run"] // 2 + 1          # odd or even: both iterate buffers occur
    for split in (cut, cut + 1):
        first = g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=split, conv_value=conv,
                                 loss_history=True, final_state=True, **kw)
        assert first["iters_run"] == split
        rest = g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=400, conv_value=conv,
                                t_start=split, init_state=first["final_state"],
                                loss_history=first["loss"], final_state=True, **kw)
        assert (rest["iters_run"], rest["stop_reason"]) == (full["iters_run"], 2)
        assert np.array_equal(rest["loss"], full["loss"])
        assert np.array_equal(rest["maps"], full["maps"])
        assert np.array_equal(rest["final_state"], full["final_state"])


def test_resume_with_device_tensors(orc):
    import torch
    d = synth.make_draw("monoexp_t2s", (3, 4, 5), 1, 0.01)
    yg = _inputs(orc, d)
    g = G()
    m = g.Model.from_acq(d.model, d.acq)
    yt = torch.from_numpy(yg).cuda()
    mt = torch.from_numpy(d.mask).cuda()
    full = g.gc_fit_askadam(m, yt, mt, d.lb, d.ub, n_iter=80, final_state=True)
    first = g.gc_fit_askadam(m, yt, mt, d.lb, d.ub, n_iter=30, final_state=True)
    assert first["final_state"].is_cuda
    rest = g.gc_fit_askadam(m, yt, mt, d.lb, d.ub, n_iter=80, t_start=30,
                            init_state=first["final_state"], final_state=True)
    torch.cuda.synchronize()
    assert torch.equal(rest["maps"], full["maps"])
    assert torch.equal(rest["final_state"], full["final_state"])


def test_resume_argument_checks(orc):
    d = synth.make_draw("monoexp_t2s", (2, 3, 4), 1, 0.01)
    yg = _inputs(orc, d)
    g = G()
    m = g.Model.from_acq(d.model, d.acq)
    st = g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=10, final_state=True)["final_state"]
    bad = [dict(n_iter=10, t_start=10, init_state=st),        # nothing left to run
           dict(n_iter=20, t_start=-1, init_state=st),
           dict(n_iter=20, t_start=10),                       # no state to resume from
           dict(n_iter=20, t_start=10, init_state=st, conv_value=1e-6)]   # window, no history
    for kw in bad:
        with pytest.raises(g.GcError) as e:
            g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, **kw)
        assert e.value.code == -1, kw
