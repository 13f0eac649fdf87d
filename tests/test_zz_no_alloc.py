"""The allocation-free MCMC entry point (gc_mcmc_noalloc) against gc_mcmc:
the same kernels on the same inputs give bit-identical moments, accept
counts and final states, on two calls in a row (the second smaller, so it
runs on what the first left in the shared scratch array), for FP32 and FP64
chains; a problem beyond the array's size is refused with GC_E_NOMEM."""
import numpy as np
import pytest

from gpu_util import G, say
from paper_2511_22094_amd import synth

pytestmark = pytest.mark.gpu


def _device_problem(torch, orc, model, shape, seed, sigma, masked):
    d = synth.make_draw(model, shape, seed, sigma)
    if masked:
        m = np.ones(int(np.prod(shape)), np.uint8)
        m[1::4] = 0
        d = synth.make_draw(model, shape, seed, sigma, mask=m.reshape(shape))
    y = (orc.forward(model, d.acq, d.truth) + sigma * d.noise).astype(np.float32)
    dev = torch.device("cuda:0")
    yg = torch.from_numpy(synth.scatter(y, d.mask)).to(dev)
    mask = torch.from_numpy(d.mask).to(dev)
    return d, yg, mask


def _outputs(torch, d, C):
    dev = torch.device("cuda:0")
    nz, ny, nx = d.shape
    P = d.lb.size
    mean = torch.full((P, nz, ny, nx), np.nan, dtype=torch.float64, device=dev)
    std = torch.full_like(mean, np.nan)
    return mean, std


@pytest.mark.parametrize("model,prec,C,shapes", [
    ("gre3", "fp32", 4, [(6, 16, 16), (3, 5, 7)]),
    ("dwi2", "fp64", 2, [(4, 9, 11), (2, 3, 5)]),
    ("monoexp_t2s", "fp32", 8, [(8, 20, 20), (1, 1, 33)]),
])
def test_noalloc_matches_gc_mcmc_on_two_calls(orc, model, prec, C, shapes):
    import torch
    g = G()
    for call, shape in enumerate(shapes):
        d, yg, mask = _device_problem(torch, orc, model, shape, 20 + call, 0.02, call == 0)
        m = g.Model.from_acq(model, d.acq)
        kw = dict(sigma=0.02, step=synth.MH_STEP[model], seed=7 + call, precision=prec,
                  chunk_iters=150, final_state=True)
        mean0, std0 = _outputs(torch, d, C)
        ref = g.gc_mcmc(m, yg, mask, d.lb, d.ub, C, 400, 100, 5, out_mean=mean0, out_std=std0,
                        **kw)
        mean1, std1 = _outputs(torch, d, C)
        out = g.gc_mcmc(m, yg, mask, d.lb, d.ub, C, 400, 100, 5, out_mean=mean1, out_std=std1,
                        noalloc=True, **kw)
        torch.cuda.synchronize()
        say(model, prec, shape, "voxels", d.n)
        assert torch.equal(mean1, mean0) and torch.equal(std1, std0)
        assert torch.equal(out["accept"], ref["accept"])
        assert torch.equal(out["final_state"], ref["final_state"])
        assert torch.equal(out["final_logl"], ref["final_logl"])
        # outside the mask the maps hold 0, as gc_mcmc writes them
        assert bool(torch.isfinite(mean1).all())


def test_noalloc_ensemble_matches(orc):
    import torch
    g = G()
    d, yg, mask = _device_problem(torch, orc, "monoexp_t2s", (2, 7, 9), 31, 0.02, True)
    m = g.Model.from_acq(d.model, d.acq)
    kw = dict(sigma=0.02, seed=2, sampler="ensemble", n_walkers=10, precision="fp64")
    mean0, std0 = _outputs(torch, d, 10)
    g.gc_mcmc(m, yg, mask, d.lb, d.ub, 1, 300, 50, 5, out_mean=mean0, out_std=std0, **kw)
    mean1, std1 = _outputs(torch, d, 10)
    g.gc_mcmc(m, yg, mask, d.lb, d.ub, 1, 300, 50, 5, out_mean=mean1, out_std=std1,
              noalloc=True, **kw)
    assert torch.equal(mean1, mean0) and torch.equal(std1, std0)


def test_noalloc_refuses_what_does_not_fit(orc):
    import torch
    g = G()
    cap = g.gc_noalloc_scratch_bytes()
    assert cap == 128 << 20
    # 2^18 voxels x 8 chains of gre3 FP32: chain state and moments alone are
    # 2^21 lanes x (9 x 4 + 8 + 2 x 9 x 8) B, about 396 MB
    d = synth.make_draw("gre3", (16, 128, 128), 3, 0.01, noise=False)
    dev = torch.device("cuda:0")
    yg = torch.zeros((48, 16, 128, 128), dtype=torch.float32, device=dev)
    m = g.Model.from_acq("gre3", d.acq)
    mean, std = _outputs(torch, d, 8)
    with pytest.raises(g.GcError) as e:
        g.gc_mcmc(m, yg, None, d.lb, d.ub, 8, 100, 10, 1, sigma=0.01, out_mean=mean,
                  out_std=std, noalloc=True)
    assert e.value.code == -3 and "scratch" in str(e.value)
    # host-memory arguments are refused (the entry point stages nothing)
    dsmall = synth.make_draw("gre3", (1, 2, 3), 3, 0.01)
    y = np.zeros((48, 1, 2, 3), np.float32)
    with pytest.raises(g.GcError) as e:
        g.gc_mcmc(m, y, None, dsmall.lb, dsmall.ub, 2, 100, 10, 1, sigma=0.01, noalloc=True)
    assert e.value.code == -1
    # and the entry point still works after a refusal
    d2, yg2, mask2 = _device_problem(torch, orc, "gre3", (2, 3, 4), 5, 0.01, False)
    m2 = g.Model.from_acq("gre3", d2.acq)
    mean0, std0 = _outputs(torch, d2, 2)
    g.gc_mcmc(m2, yg2, mask2, d2.lb, d2.ub, 2, 200, 20, 2, sigma=0.01, seed=1,
              out_mean=mean0, out_std=std0)
    mean1, std1 = _outputs(torch, d2, 2)
    g.gc_mcmc(m2, yg2, mask2, d2.lb, d2.ub, 2, 200, 20, 2, sigma=0.01, seed=1,
              out_mean=mean1, out_std=std1, noalloc=True)
    assert torch.equal(mean1, mean0) and torch.equal(std1, std0)
