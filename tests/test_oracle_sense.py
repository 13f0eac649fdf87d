"""CPU pins of the image-reconstruction oracle (oracle/sense.py).

Pins: the 2D DFT against a brute-force DFT matrix; the adjoint by the
dot-product test; the loss gradients by central finite differences; the TV
term against the grid TV of the C oracle (itself pinned); and convergence to
the closed-form least-squares image for one coil with full sampling.
"""
import numpy as np
import pytest

from oracle import sense


def _rand(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_forward_is_the_unitary_2d_dft():
    rng = np.random.default_rng(1)
    Ny, Nz = 4, 6
    img = _rand((1, Ny, Nz), rng)
    coils = np.ones((1, Ny, Nz), complex)
    y, z = np.arange(Ny), np.arange(Nz)
    Fy = np.exp(-2j * np.pi * np.outer(y, y) / Ny)
    Fz = np.exp(-2j * np.pi * np.outer(z, z) / Nz)
    ref = Fy @ img[0] @ Fz.T / np.sqrt(Ny * Nz)
    np.testing.assert_allclose(sense.forward(img, coils)[0, 0], ref, rtol=1e-12, atol=1e-12)


def test_adjoint_dot_product():
    rng = np.random.default_rng(2)
    E, Nc, Ny, Nz = 2, 3, 8, 4
    x = _rand((E, Ny, Nz), rng)
    y = _rand((E, Nc, Ny, Nz), rng)
    C = _rand((Nc, Ny, Nz), rng)
    lhs = np.vdot(sense.forward(x, C), y)          # <A x, y>
    rhs = np.vdot(x, sense.adjoint(y, C))          # <x, A^H y>
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_tv2_matches_grid_tv_of_the_c_oracle(orc):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 5, 7))
    R, g = sense.tv2(x)
    # grid (nz, ny, nx) = (echo, y, z) with 2D TV: differences along x and y only
    Rc, gc = orc.tv(np.ones(x.shape, np.uint8), x, dim=2)
    assert R == pytest.approx(Rc, rel=1e-14)
    np.testing.assert_allclose(g, gc, rtol=0, atol=1e-14)


@pytest.mark.parametrize("loss,lam", [(2, 0.0), (1, 0.0), (2, 0.3), (1, 0.3)])
def test_loss_gradient_finite_differences(loss, lam):
    rng = np.random.default_rng(4)
    E, Nc, Ny, Nz = 2, 2, 4, 4
    C = _rand((Nc, Ny, Nz), rng)
    mask = rng.uniform(size=(E, Ny, Nz)) < 0.6
    k = _rand((E, Nc, Ny, Nz), rng) * mask[:, None]
    img = _rand((E, Ny, Nz), rng)
    _, g = sense.loss_grad(img, C, mask, k, loss, lam)
    h = 1e-7
    for idx in [(0, 0, 0), (1, 2, 3), (0, 3, 1), (1, 1, 2)]:
        for part in (1.0, 1j):
            ip = img.copy()
            im = img.copy()
            ip[idx] += h * part
            im[idx] -= h * part
            fd = (sense.loss_grad(ip, C, mask, k, loss, lam)[0] -
                  sense.loss_grad(im, C, mask, k, loss, lam)[0]) / (2 * h)
            an = g[idx].real if part == 1.0 else g[idx].imag
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (loss, lam, idx, part)


def test_single_coil_full_sampling_converges_to_inverse_dft():
    """One unit coil, every k-space sample measured, L2: the minimiser is
    I = F2^H k, and Adam reaches it."""
    rng = np.random.default_rng(5)
    E, Ny, Nz = 1, 8, 8
    truth = _rand((E, Ny, Nz), rng)
    C = np.ones((1, Ny, Nz), complex)
    mask = np.ones((E, Ny, Nz), bool)
    k = sense.forward(truth, C)
    closed = np.fft.ifft2(k[:, 0], norm="ortho")
    np.testing.assert_allclose(closed, truth, rtol=1e-12, atol=1e-12)
    img, hist = sense.recon(k, C, mask, n_iter=3000, lr=0.02, loss=2)
    assert hist[-1] < 1e-8 * hist[0]
    # Adam with a fixed rate ends within a few of its steps of the minimiser
    np.testing.assert_allclose(img, truth, atol=2e-3)
    assert np.median(np.abs(img - truth)) < 1e-4


def _ls_problem(seed):
    """One unit coil, full sampling, L2: A^H A = 1, so the gradient is
    (2 / Nk) (I - I*) with I* = F2^H k, and every real component of the error
    follows its own scalar recurrence."""
    rng = np.random.default_rng(seed)
    E, Ny, Nz = 1, 8, 8
    truth = _rand((E, Ny, Nz), rng)
    C = np.ones((1, Ny, Nz), complex)
    mask = np.ones((E, Ny, Nz), bool)
    k = sense.forward(truth, C)
    h = 2.0 / (2.0 * mask.sum())          # curvature 2 / Nk, Nk = 2 Nc |M|
    return truth, C, mask, k, h


def test_sgdm_follows_the_heavy_ball_recurrence():
    truth, C, mask, k, h = _ls_problem(6)
    lr, mu, T = 40.0, 0.7, 25
    img, _ = sense.recon(k, C, mask, n_iter=T, lr=lr, optimizer="sgdm", momentum=mu)
    # error e = I - I*, velocity w: w <- mu w - lr h e; e <- e + w (from I = 0: e0 = -I*)
    e, w = -truth.copy(), np.zeros_like(truth)
    for _ in range(T):
        w = mu * w - lr * h * e
        e = e + w
    np.testing.assert_allclose(img - truth, e, rtol=1e-9, atol=1e-12)
    # the recurrence's characteristic roots bound the decay: |e_T| <= C rho^T
    assert np.abs(e).max() < np.abs(truth).max()


def test_rmsprop_follows_its_scalar_recurrence():
    truth, C, mask, k, h = _ls_problem(7)
    lr, rho, eps, T = 0.05, 0.9, 1e-8, 30
    img, _ = sense.recon(k, C, mask, n_iter=T, lr=lr, optimizer="rmsprop", rho=rho, eps=eps)
    for idx in [(0, 0, 0), (0, 3, 5), (0, 7, 7)]:
        for part, get in ((0, np.real), (1, np.imag)):
            e = -float(get(truth[idx]))
            v = 0.0
            for _ in range(T):
                g = h * e
                v = rho * v + (1 - rho) * g * g
                e = e - lr * g / (np.sqrt(v) + eps)
            got = float(get(img[idx] - truth[idx]))
            # RMSProp divides by |g|: the transforms' 1e-16 rounding of the
            # gradient, relative to |e| ~ 1e-4, adds up to ~1e-12 over the steps
            assert got == pytest.approx(e, rel=1e-9, abs=1e-11), (idx, part)
