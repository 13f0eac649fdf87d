"""The FP64 instantiation of the fits (the deterministic test path, paper
§2.2.1 Eq. 2 with the regularisers of §2.4 Eq. 4-5 and Eq. 6): the same
per-iteration kernels with the iterate, moments, bias corrections and losses
in FP64 follow the FP64 oracle to its rounding -- the maps agree after each
side's rounding to FP32, stopping rules stop at the same iteration, loss
histories agree to 1e-11.  Where FP32 rounding was amplified (TV signs of
nearly equal neighbours), FP64 rounding is not, so the bound is a few FP32
ulps; only the isotropic TV, whose subgradient divides by a norm near 0 on
flat regions, amplifies FP64 rounding too and is held to an FP64 re-run's
spread."""
import numpy as np
import pytest

from gpu_util import G, say
from graphs import grid_graph, random_graph
from paper_2511_22094_amd import synth

pytestmark = pytest.mark.gpu


def _inputs(orc, d):
    y = (orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise).astype(np.float32)
    return synth.scatter(y, d.mask)


def _ulps(a32, b64):
    """FP32 ulps between the GPU's maps and the oracle's rounded to FP32."""
    a = np.asarray(a32, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b64, np.float64).astype(np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


def _compare(out, ref, d, tag, max_ulps=4, spread=None):
    """FP32 ulps between the two after each side's rounding; where the
    iteration amplifies even FP64 rounding (spread = an FP64 re-run's
    |maps - oracle| / range), within 5x that spread instead."""
    sel = d.mask.astype(bool)
    u = _ulps(out["maps"][:, sel], ref["maps"][:, sel])
    err = np.abs(out["maps"][:, sel] - ref["maps"][:, sel]) / (d.ub - d.lb)[:, None]
    say(f"  {tag}: FP32 ulps median {np.median(u):.0f} max {u.max()}, "
        f"max err / range {err.max():.2e}")
    assert np.all(out["maps"][:, ~sel] == 0)
    if spread is None:
        assert err.max() < 1e-4
        assert u.max() <= max_ulps, (tag, u.max())
        return
    for name, f in [("median", np.median), ("p99", lambda x: np.quantile(x, 0.99)),
                    ("max", np.max)]:
        a, b = float(f(err)), float(f(spread))
        say(f"  {tag} {name}: gpu {a:.2e}  fp64 re-run {b:.2e}")
        # floor: the FP32 rounding of the returned maps (2^-24 of a value up
        # to the range is 6e-8 of it)
        assert a <= 5 * b + 1e-7, (tag, name, a, b)


ACQS = {"monoexp_r2s": synth.default_acq("monoexp_r2s"), "gre3": synth.default_acq("gre3"),
        "dwi2": synth.dwi_acq(np.random.default_rng(2), dirs_per_shell=10),
        "linear3": synth.default_acq("linear3")}


@pytest.mark.parametrize("opt", ["adam", "sgdm", "rmsprop"])
@pytest.mark.parametrize("model", ["monoexp_r2s", "gre3", "dwi2", "linear3"])
def test_fp64_fits_follow_the_oracle(orc, model, opt):
    """The FP32 tests' settings: Adam 120 iterations; SGDM and RMSProp 40
    plain (momentum / RMS-scaled) steps, the SGDM rate such that its first
    step moves u by at most 0.005.  (Over 120 iterations at rate 0.002,
    RMSProp's steps stay full-size around the minimum and amplify even FP64
    rounding: an FP64 re-run of the algorithm then parts from the oracle by
    up to 6e-3 of the range.)"""
    d = synth.make_draw(model, (3, 7, 9), 12, 0.01, acq=ACQS[model])
    yg = _inputs(orc, d)
    m = G().Model.from_acq(model, d.acq)
    kw = dict(n_iter=120, optimizer=opt, lr=0.01)
    if opt != "adam":
        mid = np.broadcast_to((0.5 * (d.lb + d.ub))[:, None], (d.n_params, d.n))
        _, gth = orc.loss_grad(model, d.acq, mid, synth.gather(yg, d.mask), p=2,
                               scale=1.0 / (d.n * m.n_meas_eff))
        gmax = np.abs((d.ub - d.lb)[:, None] * gth).max()
        kw.update(n_iter=40, lr=0.005 / gmax if opt == "sgdm" else 0.002)
    out = G().gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, precision="fp64", loss_history=True, **kw)
    ref = orc.askadam(model, d.acq, d.mask, yg, d.lb, d.ub, **kw)
    _compare(out, ref, d, f"{model} {opt}")
    np.testing.assert_allclose(out["loss"], ref["loss"], rtol=1e-11)


@pytest.mark.parametrize("kind", ["aniso", "iso", "graph", "graph_dense"])
def test_fp64_tv_fits_follow_the_oracle(orc, kind):
    """The anisotropic and graph forms agree to the FP32 rounding of the
    maps.  The isotropic form divides by the local gradient norm, which is
    near 0 on the flat blocks of these maps: there even FP64 rounding-order
    differences grow (an FP64 re-run of the algorithm parts from the oracle
    by up to ~4e-4 of the range), and the GPU is held to that spread.
    graph_dense: a random symmetric adjacency whose vertices have 3 to 12
    neighbours (a third of them more than six), so the step kernel takes both
    its first-six read and the one-by-one remainder."""
    import fp32_emulation as em
    acq = synth.dwi_acq(np.random.default_rng(2), dirs_per_shell=8)
    d = synth.make_draw("dwi2", (6, 8, 10), 2, 0.02, acq=acq, block=4)
    yg = _inputs(orc, d)
    m = G().Model.from_acq("dwi2", d.acq)
    graph = None
    if kind == "graph":
        graph = grid_graph(d.mask, 3)
    elif kind == "graph_dense":
        graph = random_graph(d.n, 3, 31)
        deg = np.diff(graph[0])
        assert deg.min() <= 6 < deg.max()
        kind = "graph"
    out = G().gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=100, lam=1e-3,
                             tv_params=(0, 1, 2), tv_dim=3, tv_kind=kind, graph=graph,
                             precision="fp64", loss_history=True)
    ref = orc.askadam("dwi2", d.acq, d.mask, yg, d.lb, d.ub, n_iter=100, lam=1e-3,
                      tv_mask=0b111, tv_dim=3, tv_kind=kind, graph=graph, n_threads=8)
    spread = None
    if kind == "iso":
        emu, _ = em.askadam("dwi2", d.acq, d.mask, yg, d.lb, d.ub, n_iter=100, lam=1e-3,
                            tv_mask=0b111, tv_dim=3, tv_kind="iso", dtype=np.float64)
        sel = d.mask.astype(bool)
        spread = np.abs(emu - ref["maps"][:, sel]) / (d.ub - d.lb)[:, None]
    _compare(out, ref, d, f"adam + {kind} TV", spread=spread)
    np.testing.assert_allclose(out["loss"], ref["loss"], rtol=1e-11 if spread is None else 1e-6)


@pytest.mark.timeout(900)
def test_fp64_adam_tv_diffusion_workload_32cubed(orc):
    """The diffusion workload's recipe (Adam 500 iterations, 3D TV 1e-3 on f,
    Da, De) on a 32^3 volume: where FP32 parts from the oracle by up to 1e-2
    of the range through flipped TV signs, FP64 does not."""
    d = synth.cfg2(shape=(32, 32, 32))
    yg = _inputs(orc, d)
    m = G().Model.from_acq("dwi2", d.acq)
    kw = synth.CFG2_ADAM
    out = G().gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=kw["n_iter"], lam=kw["lam"],
                             tv_params=(0, 1, 2), tv_dim=3, precision="fp64", loss_history=True)
    ref = orc.askadam("dwi2", d.acq, d.mask, yg, d.lb, d.ub, n_iter=kw["n_iter"], lam=kw["lam"],
                      tv_mask=0b111, tv_dim=3, n_threads=16)
    _compare(out, ref, d, "adam + TV 32^3 x 500")
    np.testing.assert_allclose(out["loss"], ref["loss"], rtol=1e-11)


def test_fp64_l1_prior_and_weights(orc):
    d = synth.make_draw("monoexp_t2s", (3, 7, 9), 24, 0.02)
    yg = _inputs(orc, d)
    rng = np.random.default_rng(25)
    P = d.lb.size
    mu = (d.lb[:, None, None, None] + (d.ub - d.lb)[:, None, None, None] *
          rng.uniform(0.3, 0.7, (P,) + d.mask.shape)).astype(np.float32)
    sg = (np.full((P,) + d.mask.shape, 0.5) * (d.ub - d.lb)[:, None, None, None]).astype(np.float32)
    w = rng.uniform(0.5, 2.0, d.mask.shape).astype(np.float32)
    m = G().Model.from_acq(d.model, d.acq)
    out = G().gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=150, loss=1, weights=w,
                             prior_lam=1e-3, prior_params=(1,), prior_mu=mu, prior_sigma=sg,
                             precision="fp64")
    ref = orc.askadam(d.model, d.acq, d.mask, yg, d.lb, d.ub, n_iter=150, loss=1, w=w,
                      prior_lam=1e-3, prior_mask=0b10, prior_mu=mu.astype(np.float64),
                      prior_sigma=sg.astype(np.float64))
    _compare(out, ref, d, "L1 + prior + weights")


def test_fp64_stopping_rules_stop_where_the_oracle_stops(orc):
    d = synth.make_draw("monoexp_t2s", (2, 6, 6), 7, 0.01)
    yg = _inputs(orc, d)
    m = G().Model.from_acq(d.model, d.acq)
    full = orc.askadam(d.model, d.acq, d.mask, yg, d.lb, d.ub, n_iter=300)
    L = np.sort(full["loss"])
    tol = float(0.5 * (L[150] + L[151]))
    for kw in (dict(tol=tol), dict(conv_value=1e-7, conv_window=20)):
        ref = orc.askadam(d.model, d.acq, d.mask, yg, d.lb, d.ub, n_iter=300, **kw)
        out = G().gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=300, precision="fp64", **kw)
        say("  fp64 stop", kw, out["iters_run"], ref["iters_run"])
        assert (out["iters_run"], out["stop_reason"]) == (ref["iters_run"], ref["stop_reason"])
        _compare(out, ref, d, f"stopped {kw}")


def test_fp64_refuses_checkpoint_fields(orc):
    d = synth.make_draw("monoexp_t2s", (1, 3, 4), 1, 0.01)
    yg = _inputs(orc, d)
    g = G()
    m = g.Model.from_acq(d.model, d.acq)
    with pytest.raises(g.GcError) as e:
        g.gc_fit_askadam(m, yg, d.mask, d.lb, d.ub, n_iter=5, precision="fp64", final_state=True)
    assert e.value.code == -1
