"""CPU pins of the oracle's regularisers beyond the anisotropic grid TV:
isotropic grid TV, graph (surface-mesh) TV and the prior term, alone and
inside askadam.

Pins: special cases that reduce to the anisotropic TV (a line; a grid graph),
a closed form (a linear ramp), central finite differences of each
regulariser, and finite differences of the whole askadam loss against the
gradient recovered from one plain gradient step.
"""
import numpy as np
import pytest

from graphs import grid_graph, random_graph
from paper_2511_22094_amd import synth


def _fd(f, u, idx, h=1e-6):
    up = u.copy()
    dn = u.copy()
    up.flat[idx] += h
    dn.flat[idx] -= h
    return (f(up) - f(dn)) / (2 * h)


# ------------------------------------------------------------ isotropic TV
@pytest.mark.parametrize("shape", [(1, 1, 9), (1, 7, 1), (6, 1, 1)])
def test_iso_equals_aniso_on_a_line(orc, shape):
    rng = np.random.default_rng(1)
    u = rng.uniform(size=shape)
    mask = np.ones(shape, np.uint8)
    mask.flat[3] = 0
    Ra, ga = orc.tv(mask, u, 3, 0.7)
    Ri, gi = orc.tv_iso(mask, u, 3, 0.7)
    assert Ri == pytest.approx(Ra, rel=1e-15)
    np.testing.assert_allclose(gi, ga, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_iso_linear_ramp_closed_form(orc, dim):
    nz, ny, nx = 3, 4, 5
    a, b, c = 0.3, -0.7, 0.2
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = a * x + b * y + c * z
    R, _ = orc.tv_iso(np.ones((nz, ny, nx), np.uint8), u, dim)
    # per voxel: the norm of (a, b[, c]) restricted to the axes that have a
    # forward neighbour
    exp = 0.0
    for zz in range(nz):
        for yy in range(ny):
            for xx in range(nx):
                comp = []
                if xx + 1 < nx:
                    comp.append(a)
                if yy + 1 < ny:
                    comp.append(b)
                if dim == 3 and zz + 1 < nz:
                    comp.append(c)
                exp += np.sqrt(sum(t * t for t in comp))
    if dim == 2:
        # per slice: interior (nx-1)(ny-1) sqrt(a^2+b^2), last column |b|, last row |a|
        closed = nz * ((nx - 1) * (ny - 1) * np.hypot(a, b) + (ny - 1) * abs(b) +
                       (nx - 1) * abs(a))
        assert exp == pytest.approx(closed, rel=1e-14)
    assert R == pytest.approx(exp, rel=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_iso_gradient_finite_differences(orc, dim):
    rng = np.random.default_rng(2)
    shape = (3, 4, 5)
    mask = (rng.uniform(size=shape) < 0.8).astype(np.uint8)
    u = rng.uniform(size=shape)
    _, g = orc.tv_iso(mask, u, dim, 1.3)
    f = lambda uu: 1.3 * orc.tv_iso(mask, uu, dim)[0]   # noqa: E731
    for idx in range(u.size):
        if mask.flat[idx]:
            assert g.flat[idx] == pytest.approx(_fd(f, u, idx), rel=1e-6, abs=1e-8)
        else:
            assert g.flat[idx] == 0.0


def test_iso_constant_map_is_zero(orc):
    u = np.full((3, 3, 3), 0.4)
    R, g = orc.tv_iso(np.ones((3, 3, 3), np.uint8), u, 3)
    assert R == 0.0 and np.all(g == 0.0)


# ------------------------------------------------------------- graph TV
@pytest.mark.parametrize("dim", [2, 3])
def test_graph_tv_of_grid_graph_is_twice_grid_tv(orc, dim):
    rng = np.random.default_rng(3)
    shape = (3, 4, 5)
    mask = (rng.uniform(size=shape) < 0.75).astype(np.uint8)
    u = rng.uniform(size=shape)
    rowptr, col = grid_graph(mask, dim)
    uc = u[mask.astype(bool)]
    Rg, gg = orc.tv_graph(rowptr, col, uc, 0.5)
    Ra, ga = orc.tv(mask, u, dim, 0.5)
    assert Rg == pytest.approx(2 * Ra, rel=1e-14)
    np.testing.assert_allclose(gg, 2 * ga[mask.astype(bool)], rtol=1e-14, atol=1e-15)


def test_graph_tv_gradient_finite_differences(orc):
    rowptr, col = random_graph(40, 4, 4)
    u = np.random.default_rng(5).uniform(size=40)
    _, g = orc.tv_graph(rowptr, col, u, 0.9)
    f = lambda uu: 0.9 * orc.tv_graph(rowptr, col, uu)[0]   # noqa: E731
    for i in range(40):
        assert g[i] == pytest.approx(_fd(f, u, i), rel=1e-6, abs=1e-8)


# ----------------------------------------------------------------- prior
def test_prior_closed_form_and_gradient(orc):
    lb, ub = 1.0, 5.0
    u = np.array([0.0, 0.25, 0.5, 1.0])          # theta = 1, 2, 3, 5
    mu = np.array([2.0, 2.0, 2.5, 4.0])
    sg = np.array([0.5, 1.0, 2.0, 0.25])
    R, g = orc.prior(u, lb, ub, mu, sg, 2.0)
    # |(1-2)/0.5| + 0 + |0.5/2| + |1/0.25| = 2 + 0 + 0.25 + 4
    assert R == pytest.approx(6.25, rel=1e-15)
    # d/du = sign(theta - mu) (ub - lb) / sigma, times the scale; sign(0) = 0
    np.testing.assert_allclose(g, 2.0 * np.array([-1 * 4 / 0.5, 0.0, 4 / 2.0, 4 / 0.25]),
                               rtol=1e-15)


# ------------------------------------------------- regularisers in askadam
def _loss_at(orc, d, y, x0, **kw):
    r = orc.askadam(d.model, d.acq, d.mask, y, d.lb, d.ub, x0=x0, n_iter=1, **kw)
    return r["loss"][0]


@pytest.mark.parametrize("reg", ["iso", "graph", "prior"])
def test_askadam_gradient_matches_finite_differences(orc, reg):
    """One plain gradient step (SGDM, momentum 0, tiny rate, no clamping)
    reveals the full gradient dL/du, which must match central differences
    of the recorded loss with respect to the start map."""
    rng = np.random.default_rng(6)
    shape = (2, 3, 4)
    mask = (rng.uniform(size=shape) < 0.8).astype(np.uint8)
    d = synth.make_draw("dwi2", shape, 7, 0.02, mask=mask)
    y = synth.scatter((orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise)
                      .astype(np.float32), d.mask)
    P = d.lb.size
    rngp = d.ub - d.lb
    x0 = d.lb[:, None, None, None] + rngp[:, None, None, None] * rng.uniform(0.2, 0.8,
                                                                           (P,) + shape)
    kw = dict(loss=2, lam=0.05, tv_mask=0b111, tv_dim=3)
    if reg == "iso":
        kw.update(tv_kind="iso")
    elif reg == "graph":
        kw.update(tv_kind="graph", graph=grid_graph(mask, 3))
    else:
        kw.update(lam=0.0, tv_mask=0, prior_lam=0.3, prior_mask=0b11011,
                  prior_mu=(d.lb + 0.4 * rngp)[:, None, None, None] * np.ones((P,) + shape),
                  prior_sigma=(0.1 * rngp)[:, None, None, None] * np.ones((P,) + shape))
    lr = 1e-7
    r = orc.askadam(d.model, d.acq, d.mask, y, d.lb, d.ub, x0=x0, n_iter=1, optimizer="sgdm",
                    momentum=0.0, lr=lr, **kw)
    u0 = (x0 - d.lb[:, None, None, None]) / rngp[:, None, None, None]
    u1 = (r["maps"] - d.lb[:, None, None, None]) / rngp[:, None, None, None]
    g = (u0 - u1) / lr
    h = 1e-6
    flat = np.flatnonzero(mask.reshape(-1))
    for p in range(P):
        for a in flat[:: 3]:
            xp = x0.copy()
            xm = x0.copy()
            xp[p].flat[a] += h * rngp[p]
            xm[p].flat[a] -= h * rngp[p]
            fd = (_loss_at(orc, d, y, xp, **kw) - _loss_at(orc, d, y, xm, **kw)) / (2 * h)
            assert g[p].flat[a] == pytest.approx(fd, rel=2e-4, abs=1e-9), (reg, p, a)


def test_askadam_prior_alone_converges_to_mu(orc):
    """With zero data weight the minimiser of the prior term is theta = mu."""
    shape = (1, 2, 3)
    d = synth.make_draw("monoexp_t2s", shape, 8, 0.01)
    y = synth.scatter((orc.forward(d.model, d.acq, d.truth) + d.sigma * d.noise)
                      .astype(np.float32), d.mask)
    P = d.lb.size
    mu = (d.lb + np.array([0.3, 0.7]) * (d.ub - d.lb))[:, None, None, None] * np.ones((P,) + shape)
    sg = np.ones((P,) + shape)
    r = orc.askadam(d.model, d.acq, d.mask, y, d.lb, d.ub, w=np.zeros(shape, np.float32),
                    n_iter=400, lr=0.01, prior_lam=1.0, prior_mask=0b11, prior_mu=mu,
                    prior_sigma=sg)
    # Adam steps of about lr in u units keep the iterate within a few steps of mu
    err = np.abs(r["maps"] - mu) / (d.ub - d.lb)[:, None, None, None]
    assert err.max() < 0.03


@pytest.mark.parametrize("reg", ["iso", "graph", "prior"])
def test_askadam_loss_assembles_regularisers_over_n(orc, reg):
    """With zero data weight the recorded first loss is the regulariser alone,
    divided by the number N of masked voxels and times its weight."""
    rng = np.random.default_rng(9)
    shape = (2, 3, 4)
    mask = (rng.uniform(size=shape) < 0.7).astype(np.uint8)
    d = synth.make_draw("dwi2", shape, 10, 0.02, mask=mask)
    y = np.zeros((96,) + shape, np.float32)
    P = d.lb.size
    rngp = d.ub - d.lb
    u0 = rng.uniform(0.1, 0.9, (P,) + shape)
    x0 = d.lb[:, None, None, None] + rngp[:, None, None, None] * u0
    N = int(mask.sum())
    w = np.zeros(shape, np.float32)
    if reg == "iso":
        kw = dict(lam=0.2, tv_mask=0b101, tv_kind="iso", tv_dim=2)
        exp = 0.2 / N * sum(orc.tv_iso(mask, u0[p], 2)[0] for p in (0, 2))
    elif reg == "graph":
        gr = grid_graph(mask, 3)
        kw = dict(lam=0.2, tv_mask=0b10, tv_kind="graph", graph=gr)
        exp = 0.2 / N * orc.tv_graph(gr[0], gr[1], u0[1][mask.astype(bool)])[0]
    else:
        mu = rng.uniform(size=(P,) + shape)
        sg = rng.uniform(0.5, 2.0, (P,) + shape)
        kw = dict(prior_lam=0.3, prior_mask=0b10001, prior_mu=mu, prior_sigma=sg)
        m = mask.astype(bool)
        exp = 0.3 / N * sum(np.abs((x0[p][m] - mu[p][m]) / sg[p][m]).sum() for p in (0, 4))
    r = orc.askadam(d.model, d.acq, mask, y, d.lb, d.ub, x0=x0, w=w, n_iter=1, **kw)
    assert r["loss"][0] == pytest.approx(exp, rel=1e-12)
