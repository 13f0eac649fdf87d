"""GPU parity of the image-reconstruction path (multi-coil multi-echo SENSE
with askadam, Eq. 7) against the FP64 oracle (oracle/sense.py).

The operator, its adjoint and one plain gradient step are compared element by
element; multi-step Adam runs are compared on the image and the loss history.
Shapes span the size limits (y from 2 to 1024, z from 16 to 1024, the y-pass
tile narrowing from 16 to 4 columns) and the full slice of the paper's demo
(6 echoes, 32 coils, 256 x 256, CAIPI R_z = 9)."""
import numpy as np
import pytest

from gpu_util import G, say
from oracle import sense
from paper_2511_22094_amd import synth

pytestmark = pytest.mark.gpu

# (E, Nc, Ny, Nz)
SHAPES = [(2, 3, 32, 16), (1, 2, 2, 16), (3, 4, 64, 32), (1, 2, 1024, 16), (1, 1, 16, 1024),
          (2, 2, 512, 64), (2, 20, 64, 256),   # 20 coils leave a partial last batch of coil rows
          (1, 1, 32, 256), (1, 8, 16, 256)]    # one coil: one live row per batch; 8: one full batch


def _draw(shape, seed, sigma=0.01):
    E, Nc, Ny, Nz = shape
    return synth.sense_draw(seed, E, Nc, Ny, Nz, sigma=sigma)


def _kspace(d):
    """Measurement from the oracle's operator (never from the HIP path)."""
    k = sense.forward(d.truth, d.coils) + d.sigma * d.noise
    return k * d.mask[:, None]


def _rel(a, b):
    return np.abs(np.asarray(a) - b).max() / np.abs(b).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_operator_matches_oracle(shape):
    d = _draw(shape, 1)
    out = G().gc_sense_forward(d.truth, d.coils, d.mask)
    ref = sense.forward(d.truth, d.coils) * d.mask[:, None]
    err = _rel(out, ref)
    say(shape, "forward max err / max", err)
    # FP32 radix-2 transforms: error grows like log2(N) ulps
    assert err < 2e-6 * np.log2(shape[2] * shape[3])
    assert np.all(out[np.broadcast_to(d.mask[:, None] == 0, out.shape)] == 0)


@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_operator_matches_oracle(shape):
    d = _draw(shape, 2)
    r = d.noise.copy()
    out = G().gc_sense_adjoint(r, d.coils, d.mask)
    ref = sense.adjoint(r * d.mask[:, None], d.coils)
    err = _rel(out, ref)
    say(shape, "adjoint max err / max", err)
    assert err < 2e-6 * np.log2(shape[2] * shape[3])


def test_operator_pair_is_adjoint_on_device():
    """<A x, y> = <x, A^H y> for the GPU pair itself, at the demo's full size."""
    import torch
    d = synth.sense_draw(3, 6, 32, 256, 256, noise=False)
    rng = np.random.default_rng(4)
    x = torch.from_numpy((rng.standard_normal(d.truth.shape) +
                          1j * rng.standard_normal(d.truth.shape)).astype(np.complex64)).cuda()
    y = torch.complex(torch.randn(6, 32, 256, 256, device="cuda"),
                      torch.randn(6, 32, 256, 256, device="cuda"))
    C = torch.from_numpy(d.coils.astype(np.complex64)).cuda()
    M = torch.from_numpy(d.mask).cuda()
    Ax = G().gc_sense_forward(x, C, M)
    AHy = G().gc_sense_adjoint(y, C, M)
    lhs = torch.vdot(Ax.flatten().to(torch.complex128), y.flatten().to(torch.complex128))
    rhs = torch.vdot(x.flatten().to(torch.complex128), AHy.flatten().to(torch.complex128))
    say("dot test", complex(lhs), complex(rhs))
    assert abs(complex(lhs - rhs)) < 1e-5 * abs(complex(lhs))


def test_full_slice_operators_match_oracle():
    d = synth.sense_draw(5, 6, 32, 256, 256)
    out = G().gc_sense_forward(d.truth, d.coils, d.mask)
    ref = sense.forward(d.truth, d.coils) * d.mask[:, None]
    assert _rel(out, ref) < 3e-5
    adj = G().gc_sense_adjoint(d.noise, d.coils, d.mask)
    aref = sense.adjoint(d.noise * d.mask[:, None], d.coils)
    assert _rel(adj, aref) < 3e-5


@pytest.mark.parametrize("loss,lam", [(2, 0.0), (1, 0.0), (2, 0.5), (1, 0.5)])
@pytest.mark.parametrize("shape", [(2, 3, 32, 16), (1, 2, 512, 64), (2, 20, 32, 256), (1, 3, 16, 256)])
def test_one_step_gradient_matches_oracle(loss, lam, shape):
    """SGDM with momentum 0: (init - image) / lr = dL/dRe + i dL/dIm, and the
    recorded loss is the loss at init.  The rate makes lr |g| about 100 |init|
    so that the subtraction keeps the bits of g."""
    d = _draw(shape, 6)
    k = _kspace(d).astype(np.complex64)
    C = d.coils.astype(np.complex64)
    rng = np.random.default_rng(7)
    init = (d.truth + 0.1 * (rng.standard_normal(d.truth.shape) +
                             1j * rng.standard_normal(d.truth.shape))).astype(np.complex64)
    L, gref = sense.loss_grad(init.astype(complex), C.astype(complex), d.mask, k.astype(complex),
                              loss, lam)
    lr = float(2.0 ** np.round(np.log2(100 * np.abs(init).max() / np.abs(gref).max())))
    out = G().gc_sense_recon(k, C, d.mask, init=init, optimizer="sgdm", momentum=0.0, lr=lr,
                             n_iter=1, loss=loss, lam=lam, loss_history=True)
    g = (init.astype(complex) - out["image"]) / lr
    err = _rel(g, gref)
    say(shape, loss, lam, "one-step gradient max err / max", err)
    assert err < 2e-5
    assert out["loss"][0] == pytest.approx(L, rel=2e-6)


def _start(d):
    rng = np.random.default_rng(3)
    return (0.5 * d.truth + 0.05 * (rng.standard_normal(d.truth.shape) +
                                    1j * rng.standard_normal(d.truth.shape))).astype(np.complex64)


@pytest.mark.parametrize("loss,lam,T", [(2, 0.0, 60), (2, 0.5, 60), (1, 0.0, 30), (1, 0.5, 6)])
def test_adam_recon_matches_oracle(loss, lam, T):
    """Both sides get the same FP32-rounded data and the same start image.

    The start is not 0: Adam's first step moves every component by almost
    exactly the rate, so from 0 neighbouring pixels would differ only by
    rounding and the TV signs of iteration 2 would be decided by it.  L1 runs
    are short: this problem is underdetermined (4 coils, R_z = 9), and once
    L1 residuals reach the rounding level their signs flip with the
    arithmetic and FP32 and FP64 trajectories part (an FP32 emulation of
    these steps on the CPU parts from FP64 the same way: from about
    iteration 40 without TV; with TV, one echo image from about iteration 8,
    since the L1 term couples all pixels of an echo).  TV differences also
    meet zero now and then along the way; the pixels next to such a tie take
    a different step, hence the bound on the fraction of pixels off by more
    than 1e-4 rather than on the maximum."""
    d = _draw((3, 4, 64, 32), 8)
    k = _kspace(d).astype(np.complex64)
    C = d.coils.astype(np.complex64)
    init = _start(d)
    out = G().gc_sense_recon(k, C, d.mask, init=init, lr=0.01, n_iter=T, loss=loss, lam=lam,
                             loss_history=True)
    img, hist = sense.recon(k.astype(complex), C.astype(complex), d.mask, n_iter=T, lr=0.01,
                            loss=loss, lam=lam, init=init.astype(complex))
    err = np.abs(out["image"] - img) / np.abs(img).max()
    say(loss, lam, "Adam recon |dI| median", np.median(err), "p99", np.quantile(err, 0.99),
        "max", err.max())
    assert out["iters_run"] == T
    assert np.median(err) < 1e-6
    if lam == 0:
        np.testing.assert_allclose(out["loss"], hist, rtol=1e-5)
        # Adam divides by |g|: components whose gradient is near zero take
        # steps set by the rounding of g (up to lr)
        assert err.max() < 2e-3
    else:
        np.testing.assert_allclose(out["loss"], hist, rtol=1e-4)
        assert np.mean(err > 1e-4) < 0.02 and err.max() < 0.1


@pytest.mark.parametrize("opt,kw", [("sgdm", dict(lr=1000.0, momentum=0.8)),
                                    ("rmsprop", dict(lr=0.003, rho=0.9))])
def test_sgdm_and_rmsprop_recon_match_oracle(opt, kw):
    """The other two optimisers of the parameter fits, L2, 40 iterations."""
    d = _draw((3, 4, 64, 32), 8)
    k = _kspace(d).astype(np.complex64)
    C = d.coils.astype(np.complex64)
    init = _start(d)
    out = G().gc_sense_recon(k, C, d.mask, init=init, optimizer=opt, n_iter=40, loss=2,
                             loss_history=True, **kw)
    img, hist = sense.recon(k.astype(complex), C.astype(complex), d.mask, n_iter=40, loss=2,
                            init=init.astype(complex), optimizer=opt, **kw)
    err = np.abs(out["image"] - img) / np.abs(img).max()
    say(opt, "recon |dI| median", np.median(err), "max", err.max())
    np.testing.assert_allclose(out["loss"], hist, rtol=1e-5)
    # RMSProp divides by |g| like Adam (components with g near 0 step by rounding)
    assert np.median(err) < 1e-6 and err.max() < (2e-3 if opt == "rmsprop" else 1e-5)


def test_l1_tv_recon_loss_follows_oracle():
    """L1 + TV over 30 iterations: past the point where one echo's trajectory
    parts (see above) the losses still agree to 1e-3 (the FP32 emulation on
    the CPU: within 3e-4)."""
    d = _draw((3, 4, 64, 32), 8)
    k = _kspace(d).astype(np.complex64)
    C = d.coils.astype(np.complex64)
    init = _start(d)
    out = G().gc_sense_recon(k, C, d.mask, init=init, lr=0.01, n_iter=30, loss=1, lam=0.5,
                             loss_history=True)
    _, hist = sense.recon(k.astype(complex), C.astype(complex), d.mask, n_iter=30, lr=0.01,
                          loss=1, lam=0.5, init=init.astype(complex))
    np.testing.assert_allclose(out["loss"], hist, rtol=1e-3)


def test_recon_reduces_to_least_squares_with_one_coil_full_sampling():
    """One unit coil, all of k-space measured, L2: the minimiser is the
    inverse DFT of the data, which Adam reaches."""
    rng = np.random.default_rng(9)
    E, Ny, Nz = 1, 16, 16
    truth = rng.standard_normal((E, Ny, Nz)) + 1j * rng.standard_normal((E, Ny, Nz))
    C = np.ones((1, Ny, Nz), complex)
    mask = np.ones((E, Ny, Nz), np.uint8)
    k = sense.forward(truth, C)
    out = G().gc_sense_recon(k, C, mask, lr=0.02, n_iter=3000, loss=2)
    err = np.abs(out["image"] - truth)
    say("single coil LS: max", err.max(), "median", np.median(err))
    assert err.max() < 5e-3 and np.median(err) < 5e-4


def test_recon_recovers_the_phantom():
    """Property of the method at a realistic geometry (6 echoes, 32 coils,
    R_z = 9, 64 x 64): the reconstruction error falls far below that of the
    image, and TV lowers it further at higher noise (the paper's observation
    that TV reduces noise in the reconstructed images)."""
    d = synth.sense_draw(13, 6, 32, 64, 64, sigma=0.001)
    nrm = np.linalg.norm(d.truth)
    k = _kspace(d)
    out = G().gc_sense_recon(k, d.coils, d.mask, lr=0.01, n_iter=1000, loss=2)
    e2 = np.linalg.norm(out["image"] - d.truth) / nrm
    say("L2 recon rel err", e2)
    assert e2 < 0.2
    d = synth.sense_draw(13, 6, 32, 64, 64, sigma=0.02)
    k = _kspace(d)
    e = {}
    for lam in (0.0, 0.05):
        r = G().gc_sense_recon(k, d.coils, d.mask, lr=0.01, n_iter=1000, loss=1, lam=lam)
        e[lam] = np.linalg.norm(r["image"] - d.truth) / nrm
    say("L1 recon rel err without / with TV", e)
    assert e[0.05] < e[0.0]


def test_stopping_rules_cut_the_same_computation_short():
    d = _draw((2, 3, 32, 16), 10)
    k = _kspace(d)
    full = G().gc_sense_recon(k, d.coils, d.mask, lr=0.01, n_iter=400, loss_history=True)
    tol = float(full["loss"][150])
    st = G().gc_sense_recon(k, d.coils, d.mask, lr=0.01, n_iter=400, tol=tol, loss_history=True)
    assert st["stop_reason"] == 1
    assert st["iters_run"] == int(np.argmax(full["loss"] < tol)) + 1
    # the stopped run is the same computation cut short
    cut = G().gc_sense_recon(k, d.coils, d.mask, lr=0.01, n_iter=st["iters_run"])
    np.testing.assert_array_equal(st["image"], cut["image"])
    np.testing.assert_array_equal(st["loss"], full["loss"][: st["iters_run"]])
    cv = G().gc_sense_recon(k, d.coils, d.mask, lr=0.01, n_iter=400, conv_value=1e-7,
                            conv_window=10)
    assert cv["stop_reason"] in (0, 2)


def test_device_memory_path_equals_host_path():
    import torch
    d = _draw((2, 3, 64, 32), 11)
    k = _kspace(d).astype(np.complex64)
    host = G().gc_sense_recon(k, d.coils, d.mask, lr=0.01, n_iter=20, loss=1, lam=0.2)
    dev = G().gc_sense_recon(torch.from_numpy(k).cuda(),
                             torch.from_numpy(d.coils.astype(np.complex64)).cuda(),
                             torch.from_numpy(d.mask).cuda(), lr=0.01, n_iter=20, loss=1, lam=0.2)
    np.testing.assert_array_equal(host["image"], dev["image"].cpu().numpy())
    assert host["final_loss"] == dev["final_loss"]


def test_rejects_bad_problems():
    g = G()
    d = _draw((1, 2, 32, 16), 12)
    k = _kspace(d)
    with pytest.raises(g.GcError):          # z not a power of two
        g.gc_sense_forward(d.truth[:, :, :12], d.coils[:, :, :12], d.mask[:, :, :12])
    with pytest.raises(g.GcError):          # z below the y-pass tile width
        g.gc_sense_forward(d.truth[:, :, :8], d.coils[:, :, :8], d.mask[:, :, :8])
    with pytest.raises(g.GcError):          # nothing sampled
        g.gc_sense_recon(k, d.coils, np.zeros_like(d.mask), n_iter=2)
    with pytest.raises(g.GcError):          # bad rate
        g.gc_sense_recon(k, d.coils, d.mask, n_iter=2, lr=0.0)
    with pytest.raises(ValueError):         # shape mismatch caught by the binding
        g.gc_sense_recon(k[:, :1], d.coils, d.mask, n_iter=2)
