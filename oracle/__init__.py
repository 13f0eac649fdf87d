"""ctypes wrapper of the plain FP64 CPU oracle (``gacelle_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the bench's CPU
baseline leg may use this package; the product path never does.  The
wrapper only marshals numpy arrays; every piece of arithmetic is in the C
file, which shares nothing with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gacelle_oracle.c")
# GACELLE_ORACLE_LIB names another build of the same oracle source (the tests
# rerun the oracle's pins against a build with sanitizers)
_LIB = os.environ.get("GACELLE_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

MODEL_IDS = {"monoexp_t2s": 0, "monoexp_r2s": 1, "gre3": 2, "dwi2": 3, "linear3": 4}
NPARAMS = {"monoexp_t2s": 2, "monoexp_r2s": 2, "gre3": 9, "dwi2": 5, "linear3": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over voxels only)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unknown-pragmas", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("GACELLE_ORACLE_LIB") and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u32, u64, dbl = (ctypes.c_int64, ctypes.c_int, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox_batch.argtypes = [u64, P, i64, P]
        L.orc_uniform.argtypes = [u32]
        L.orc_uniform.restype = dbl
        L.orc_box_muller.argtypes = [dbl, dbl, P, P]
        L.orc_mh_draws.argtypes = [u64, u32, u32, u32, i32, P, P]
        L.orc_init_uniform.argtypes = [u64, u32, u32, i32, P, P, P]
        L.orc_forward.argtypes = [i32, i32, P, P, P, P, i64, P]
        L.orc_jacobian.argtypes = [i32, i32, P, P, P, P, i64, P]
        L.orc_vjp.argtypes = [i32, i32, P, P, P, P, i64, P, P]
        L.orc_loss_grad.argtypes = [i32, i32, P, P, P, P, P, P, i64, i32, dbl, P, P]
        L.orc_tv.argtypes = [i32, i32, i32, P, P, i32, dbl, P]
        L.orc_tv.restype = dbl
        L.orc_tv_iso.argtypes = [i32, i32, i32, P, P, i32, dbl, P]
        L.orc_tv_iso.restype = dbl
        L.orc_tv_graph.argtypes = [i64, P, P, P, dbl, P]
        L.orc_tv_graph.restype = dbl
        L.orc_prior.argtypes = [i64, P, dbl, dbl, P, P, dbl, P]
        L.orc_prior.restype = dbl
        L.orc_askadam_reg.argtypes = ([i32, i32, P, P, P, i32, i32, i32, P, P, P, P, P, P,
                                       i32, dbl, dbl, dbl, dbl, dbl, dbl, i32, i32, dbl, u32,
                                       i32, P, dbl, dbl, i32, P, P, P, P, i32])
        L.orc_askadam.argtypes = ([i32, i32, P, P, P, i32, i32, i32, P, P, P, P, P, P,
                                   i32, dbl, dbl, dbl, dbl, dbl, dbl, i32, i32, dbl, u32,
                                   i32, dbl, dbl, i32, P, P, P, P, i32])
        L.orc_mh_nkeep.argtypes = [i32, i32, i32]
        L.orc_mh_nkeep.restype = i64
        L.orc_mh.argtypes = [i32, i32, P, P, P, i64, P, P, P, P, P, P, P, dbl, u64,
                             i32, i32, i32, i32, P, P, P, P, P, P, P, i32]
        L.orc_logl.argtypes = [i32, i32, P, P, P, P, P, P, i64, dbl, P]
        L.orc_ensemble.argtypes = [i32, i32, P, P, P, i64, P, P, P, P, P, P, i32, dbl, u64,
                                   i32, dbl, i32, i32, i32, P, P, P, P, P, i32]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


class Acq:
    """Acquisition arrays kept alive for the duration of a call."""

    def __init__(self, te=None, bval=None, bvec=None):
        self.te = _f64(te)
        self.bval = _f64(bval)
        self.bvec = _f64(bvec)
        self.M = len(self.te) if self.te is not None else len(self.bval)

    @classmethod
    def of(cls, acq):
        if isinstance(acq, Acq):
            return acq
        return cls(getattr(acq, "te", None), getattr(acq, "bval", None), getattr(acq, "bvec", None))

    def args(self):
        return (self.M, _p(self.te), _p(self.bval), _p(self.bvec))


def meas_eff(model: str, M: int) -> int:
    return 2 * M if model == "gre3" else M


# --------------------------------------------------------------------- RNG
def philox(seed: int, ctr: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(ctypes.c_uint64(seed), _p(ctr), len(ctr), _p(out))
    return out


def philox_kat(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniform(words: np.ndarray) -> np.ndarray:
    L = lib()
    w = np.asarray(words, dtype=np.uint32).ravel()
    return np.array([L.orc_uniform(int(x)) for x in w]).reshape(np.shape(words))


def box_muller(u1: float, u2: float):
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    lib().orc_box_muller(u1, u2, ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def mh_draws(seed: int, v: int, c: int, t: int, P: int):
    z = np.zeros(P)
    u = ctypes.c_double()
    lib().orc_mh_draws(ctypes.c_uint64(seed), v, c, t, P, _p(z), ctypes.byref(u))
    return z, u.value


def init_uniform(seed: int, v: int, c: int, lb, ub) -> np.ndarray:
    lb, ub = _f64(lb), _f64(ub)
    th = np.zeros(len(lb))
    lib().orc_init_uniform(ctypes.c_uint64(seed), v, c, len(lb), _p(lb), _p(ub), _p(th))
    return th


# ------------------------------------------------------------------ models
def forward(model: str, acq, theta) -> np.ndarray:
    a = Acq.of(acq)
    th = _f64(np.atleast_2d(theta))
    n = th.shape[1]
    s = np.empty((meas_eff(model, a.M), n))
    rc = lib().orc_forward(MODEL_IDS[model], *a.args(), _p(th), n, _p(s))
    assert rc == 0
    return s


def jacobian(model: str, acq, theta) -> np.ndarray:
    """[n, Meff, P]"""
    a = Acq.of(acq)
    th = _f64(np.atleast_2d(theta))
    n = th.shape[1]
    J = np.empty((n, meas_eff(model, a.M), NPARAMS[model]))
    assert lib().orc_jacobian(MODEL_IDS[model], *a.args(), _p(th), n, _p(J)) == 0
    return J


def vjp(model: str, acq, theta, ds) -> np.ndarray:
    a = Acq.of(acq)
    th = _f64(np.atleast_2d(theta))
    ds = _f64(ds)
    n = th.shape[1]
    out = np.empty((NPARAMS[model], n))
    assert lib().orc_vjp(MODEL_IDS[model], *a.args(), _p(th), n, _p(ds), _p(out)) == 0
    return out


def loss_grad(model: str, acq, theta, y, w=None, p: int = 2, scale: float = 1.0):
    a = Acq.of(acq)
    th = _f64(theta)
    y = _f32(y)
    w = _f32(w)
    n = th.shape[1]
    loss = np.empty(n)
    grad = np.empty_like(th)
    assert lib().orc_loss_grad(MODEL_IDS[model], *a.args(), _p(th), _p(y), _p(w), n, p,
                               scale, _p(loss), _p(grad)) == 0
    return loss, grad


def logl(model: str, acq, theta, y, sigma: float, w=None) -> np.ndarray:
    a = Acq.of(acq)
    th = _f64(theta)
    y = _f32(y)
    w = _f32(w)
    n = th.shape[1]
    out = np.empty(n)
    assert lib().orc_logl(MODEL_IDS[model], *a.args(), _p(th), _p(y), _p(w), n, sigma,
                          _p(out)) == 0
    return out


def tv(mask: np.ndarray, u: np.ndarray, dim: int = 3, scale: float = 1.0):
    """Returns (R, dR) for a full grid u[nz, ny, nx]."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    u = _f64(u)
    nz, ny, nx = mask.shape
    dR = np.zeros_like(u)
    R = lib().orc_tv(nx, ny, nz, _p(mask), _p(u), dim, scale, _p(dR))
    return R, dR


def tv_iso(mask: np.ndarray, u: np.ndarray, dim: int = 3, scale: float = 1.0):
    """Isotropic grid TV: returns (R, dR) for a full grid u[nz, ny, nx]."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    u = _f64(u)
    nz, ny, nx = mask.shape
    dR = np.zeros_like(u)
    R = lib().orc_tv_iso(nx, ny, nz, _p(mask), _p(u), dim, scale, _p(dR))
    return R, dR


def tv_graph(rowptr, col, u, scale: float = 1.0):
    """Graph TV over CSR adjacency (rowptr [n+1], col): returns (R, dR [n])."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    u = _f64(u)
    dR = np.zeros_like(u)
    R = lib().orc_tv_graph(u.size, _p(rowptr), _p(col), _p(u), scale, _p(dR))
    return R, dR


def prior(u, lb, ub, mu, sigma, scale: float = 1.0):
    """Prior regulariser of one map over n voxels: returns (R, dR/du [n])."""
    u = _f64(u)
    mu = _f64(np.broadcast_to(mu, u.shape))
    sigma = _f64(np.broadcast_to(sigma, u.shape))
    dR = np.zeros_like(u)
    R = lib().orc_prior(u.size, _p(u), float(lb), float(ub), _p(mu), _p(sigma), scale, _p(dR))
    return R, dR


class _Reg(ctypes.Structure):
    _fields_ = [("tv_kind", ctypes.c_int), ("graph_n", ctypes.c_int64),
                ("graph_rowptr", ctypes.c_void_p), ("graph_col", ctypes.c_void_p),
                ("prior_lambda", ctypes.c_double), ("prior_mask", ctypes.c_uint32),
                ("prior_mu", ctypes.c_void_p), ("prior_sigma", ctypes.c_void_p)]


TV_KINDS = {"aniso": 0, "iso": 1, "graph": 2}

# ---------------------------------------------------------------- askadam
OPTIMIZERS = {"adam": 0, "sgdm": 1, "rmsprop": 2}


def askadam(model: str, acq, mask, y_grid, lb, ub, *, x0=None, w=None, optimizer="adam",
            lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, momentum=0.9, rho=0.9,
            n_iter=200, loss=2, lam=0.0, tv_mask=0, tv_dim=3, tol=0.0, conv_value=0.0,
            conv_window=20, n_threads=0, tv_kind="aniso", graph=None, prior_lam=0.0,
            prior_mask=0, prior_mu=None, prior_sigma=None):
    """Returns dict(maps [P,nz,ny,nx], loss [iters_run], iters_run, stop_reason).

    tv_kind: "aniso" | "iso" (grid) | "graph" with graph = (rowptr, col) over
    the masked voxels in grid order; prior_mu / prior_sigma: [P, nz, ny, nx]."""
    a = Acq.of(acq)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = mask.shape
    P = NPARAMS[model]
    y = _f32(y_grid)
    assert y.shape == (meas_eff(model, a.M), nz, ny, nx)
    lb, ub = _f64(lb), _f64(ub)
    x0 = _f64(x0)
    w = _f32(w)
    maps = np.zeros((P, nz, ny, nx))
    hist = np.zeros(max(n_iter, 1))
    it = ctypes.c_int()
    reason = ctypes.c_int()
    reg = _Reg()
    reg.tv_kind = TV_KINDS[tv_kind]
    keep = []
    if graph is not None:
        rp = np.ascontiguousarray(graph[0], dtype=np.int64)
        cl = np.ascontiguousarray(graph[1], dtype=np.int32)
        keep += [rp, cl]
        reg.graph_n, reg.graph_rowptr, reg.graph_col = rp.size - 1, rp.ctypes.data, cl.ctypes.data
    if prior_lam:
        mu = _f64(np.broadcast_to(prior_mu, (P, nz, ny, nx)))
        sg = _f64(np.broadcast_to(prior_sigma, (P, nz, ny, nx)))
        keep += [mu, sg]
        reg.prior_lambda, reg.prior_mask = prior_lam, prior_mask
        reg.prior_mu, reg.prior_sigma = mu.ctypes.data, sg.ctypes.data
    rc = lib().orc_askadam_reg(MODEL_IDS[model], *a.args(), nx, ny, nz, _p(mask), _p(y), _p(w),
                               _p(lb), _p(ub), _p(x0), OPTIMIZERS[optimizer], lr, beta1, beta2,
                               eps, momentum, rho, n_iter, loss, lam, tv_mask, tv_dim,
                               ctypes.byref(reg), tol, conv_value, conv_window, _p(maps),
                               _p(hist), ctypes.byref(it), ctypes.byref(reason), n_threads)
    assert rc == 0, rc
    return dict(maps=maps, loss=hist[: it.value], iters_run=it.value, stop_reason=reason.value)


# ------------------------------------------------------------------- MCMC
def mh_nkeep(n_iter: int, burnin: int, thin: int) -> int:
    return int(lib().orc_mh_nkeep(n_iter, burnin, thin))


def mh(model: str, acq, y, lb, ub, step, sigma, seed, n_chains, n_iter, burnin, thin,
       x0=None, w=None, vidx=None, keep_samples=False, n_threads=0):
    """MH on compacted voxels y[Meff, n]; x0 [C, P, n] (default midpoint).

    Returns dict(mean, std [P,n], accept [C,n], final [C,P,n], logl [C,n],
    margin [n], samples [C,K,P,n] or None)."""
    a = Acq.of(acq)
    y = _f32(y)
    n = y.shape[1]
    P = NPARAMS[model]
    lb, ub, step = _f64(lb), _f64(ub), _f64(step)
    if x0 is None:
        x0 = np.broadcast_to((0.5 * (lb + ub))[None, :, None], (n_chains, P, n))
    x0 = _f64(x0)
    w = _f32(w)
    vidx = np.ascontiguousarray(np.arange(n) if vidx is None else vidx, dtype=np.uint32)
    K = mh_nkeep(n_iter, burnin, thin)
    samples = np.zeros((n_chains, K, P, n)) if keep_samples else None
    mean = np.zeros((P, n))
    sd = np.zeros((P, n))
    acc = np.zeros((n_chains, n), dtype=np.int32)
    fin = np.zeros((n_chains, P, n))
    fll = np.zeros((n_chains, n))
    marg = np.zeros(n)
    rc = lib().orc_mh(MODEL_IDS[model], *a.args(), n, _p(y), _p(w), _p(vidx), _p(lb), _p(ub),
                      _p(x0), _p(step), sigma, ctypes.c_uint64(seed), n_chains, n_iter, burnin,
                      thin, _p(samples), _p(mean), _p(sd), _p(acc), _p(fin), _p(fll), _p(marg),
                      n_threads)
    assert rc == 0, rc
    return dict(mean=mean, std=sd, accept=acc, final=fin, logl=fll, margin=marg,
                samples=samples)


def ensemble(model: str, acq, y, lb, ub, sigma, seed, n_walkers, n_iter, burnin, thin,
             stretch=2.0, x0=None, x0_mode=0, w=None, vidx=None, keep_samples=False,
             n_threads=0):
    """Affine-invariant ensemble sampler on compacted voxels y[Meff, n];
    x0 [P, n] (default midpoint) is the centre of the starting ball.

    Returns dict(mean, std [P,n], accept [K,n], final [P,K,n], samples [K,S,P,n])."""
    a = Acq.of(acq)
    y = _f32(y)
    n = y.shape[1]
    P = NPARAMS[model]
    lb, ub = _f64(lb), _f64(ub)
    if x0 is None:
        x0 = np.broadcast_to((0.5 * (lb + ub))[:, None], (P, n))
    x0 = _f64(x0)
    w = _f32(w)
    vidx = np.ascontiguousarray(np.arange(n) if vidx is None else vidx, dtype=np.uint32)
    S = mh_nkeep(n_iter, burnin, thin)
    samples = np.zeros((n_walkers, S, P, n)) if keep_samples else None
    mean = np.zeros((P, n))
    sd = np.zeros((P, n))
    acc = np.zeros((n_walkers, n), dtype=np.int32)
    fin = np.zeros((P, n_walkers, n))
    rc = lib().orc_ensemble(MODEL_IDS[model], *a.args(), n, _p(y), _p(w), _p(vidx), _p(lb),
                            _p(ub), _p(x0), x0_mode, sigma, ctypes.c_uint64(seed), n_walkers,
                            stretch, n_iter, burnin, thin, _p(samples), _p(mean), _p(sd),
                            _p(acc), _p(fin), n_threads)
    assert rc == 0, rc
    return dict(mean=mean, std=sd, accept=acc, final=fin, samples=samples)
