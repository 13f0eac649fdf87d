"""Seeded synthetic inputs shared by the HIP path, its tests and the bench.

This module only *draws* things: ground-truth parameter maps, unit-variance
noise planes, acquisition tables (echo times, b-values, gradient
directions), masks and serving traces.  It holds none of the method's
arithmetic: no forward model, likelihood, loss or update.  A caller turns a
draw into measured data by evaluating a forward model of its own
(``y = s(theta_true) + sigma * noise``) -- the tests with the CPU oracle, the
bench with the HIP forward kernel -- so neither side's arithmetic leaks into
the other's inputs.

Layouts (shared convention of the whole package):

* grids are ``[nz][ny][nx]`` with x fastest (C order);
* the compacted voxel order is the mask's C order (x fastest);
* parameter arrays are structure-of-arrays ``[P][n]``;
* measurement arrays are ``[M_eff][n]``; complex models store the M real
  planes first, then the M imaginary planes (``M_eff = 2M``).

Workload recipes follow the paper's quantitative-MRI setting (multi-echo GRE
relaxometry and multi-shell diffusion, §2.1 and §2.5) at the sizes of the
five synthetic workloads documented in the design notes; every draw is
reproducible from its seed via ``numpy.random.default_rng``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Parameter names and default bounds of the model registry (order = P index).
# ---------------------------------------------------------------------------
PARAM_NAMES: Dict[str, Tuple[str, ...]] = {
    "monoexp_t2s": ("S0", "T2star"),
    "monoexp_r2s": ("S0", "R2star"),
    "gre3": ("A1", "A2", "A3", "T2s1", "T2s2", "T2s3", "df1", "df2", "df3"),
    "dwi2": ("f", "Da", "De", "theta", "phi"),
    "linear3": ("A1", "A2", "A3"),
}

DEFAULT_BOUNDS: Dict[str, Tuple[Tuple[float, ...], Tuple[float, ...]]] = {
    # S0 (a.u.), T2* (ms)
    "monoexp_t2s": ((0.0, 1.0), (3.0, 250.0)),
    # S0 (a.u.), R2* (1/s)
    "monoexp_r2s": ((0.0, 4.0), (3.0, 1000.0)),
    # disjoint T2* ranges keep the three pools identifiable (ms); df in Hz
    "gre3": ((0.0, 0.0, 0.0, 2.0, 40.0, 20.0, -25.0, -25.0, -25.0),
             (1.0, 1.0, 1.0, 20.0, 120.0, 40.0, 25.0, 25.0, 25.0)),
    # f, Da, De (um^2/ms), polar angle in [0, pi/2] (antipodal fold), azimuth
    "dwi2": ((0.0, 0.1, 0.1, 0.0, -math.pi),
             (1.0, 3.5, 3.5, 0.5 * math.pi, math.pi)),
    "linear3": ((-10.0, -10.0, -10.0), (10.0, 10.0, 10.0)),
}

# fixed basis time constants of the linear test model (ms)
LINEAR3_TAU = (10.0, 30.0, 80.0)


@dataclasses.dataclass
class Acq:
    """Acquisition table of one model (host arrays, float64)."""
    te: Optional[np.ndarray] = None      # [M] echo times, ms
    bval: Optional[np.ndarray] = None    # [M] s/mm^2
    bvec: Optional[np.ndarray] = None    # [M, 3] unit vectors

    @property
    def n_meas(self) -> int:
        return len(self.te) if self.te is not None else len(self.bval)


@dataclasses.dataclass
class Draw:
    """One synthetic volume: truth, noise and the acquisition it belongs to."""
    model: str
    acq: Acq
    shape: Tuple[int, int, int]          # (nz, ny, nx)
    mask: np.ndarray                     # uint8 [nz, ny, nx]
    truth: np.ndarray                    # float64 [P, n] (compacted)
    noise: np.ndarray                    # float32 [M_eff, n] unit variance
    sigma: float
    lb: np.ndarray
    ub: np.ndarray
    seed: int

    @property
    def n(self) -> int:
        return self.truth.shape[1]

    @property
    def n_params(self) -> int:
        return self.truth.shape[0]


def echo_times(first: float, step: float, count: int) -> np.ndarray:
    return first + step * np.arange(count, dtype=np.float64)


def is_complex(model: str) -> bool:
    return model == "gre3"


def meas_eff(model: str, m: int) -> int:
    return 2 * m if is_complex(model) else m


def bounds(model: str) -> Tuple[np.ndarray, np.ndarray]:
    lo, hi = DEFAULT_BOUNDS[model]
    return np.array(lo, dtype=np.float64), np.array(hi, dtype=np.float64)


def midpoint(model: str) -> np.ndarray:
    lo, hi = bounds(model)
    return 0.5 * (lo + hi)


# ---------------------------------------------------------------------------
# masks and layout helpers (pure indexing, no arithmetic of the method)
# ---------------------------------------------------------------------------
def ellipsoid_mask(shape: Tuple[int, int, int], centre_zyx, semi_zyx) -> np.ndarray:
    nz, ny, nx = shape
    z, y, x = np.ogrid[:nz, :ny, :nx]
    cz, cy, cx = centre_zyx
    az, ay, ax = semi_zyx
    r = ((x - cx) / ax) ** 2 + ((y - cy) / ay) ** 2 + ((z - cz) / az) ** 2
    return (r <= 1.0).astype(np.uint8)


def scatter(compact: np.ndarray, mask: np.ndarray, fill=0) -> np.ndarray:
    """[K, n] compacted -> [K, nz, ny, nx] grid (zeros outside the mask)."""
    out = np.full((compact.shape[0],) + mask.shape, fill, dtype=compact.dtype)
    out[:, mask.astype(bool)] = compact
    return out


def gather(grid: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """[K, nz, ny, nx] grid -> [K, n] compacted in mask C order."""
    return np.ascontiguousarray(grid[:, mask.astype(bool)])


# ---------------------------------------------------------------------------
# truth draws per model
# ---------------------------------------------------------------------------
def _fold_upper(v: np.ndarray) -> np.ndarray:
    """Map unit vectors to the upper hemisphere (n and -n are the same fibre)."""
    flip = v[:, 2] < 0
    v = v.copy()
    v[flip] *= -1.0
    return v


def _angles(v: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    th = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    ph = np.arctan2(v[:, 1], v[:, 0])
    return th, ph


def truth_monoexp(rng, n: int) -> np.ndarray:
    s0 = rng.uniform(0.5, 1.5, n)
    t2 = rng.uniform(20.0, 80.0, n)
    return np.stack([s0, t2])


def truth_gre3(rng, n: int) -> np.ndarray:
    a = rng.dirichlet((2.0, 5.0, 3.0), n).T            # fractions, S0 = 1
    t2 = np.stack([rng.uniform(5.0, 15.0, n),
                   rng.uniform(40.0, 70.0, n),
                   rng.uniform(20.0, 40.0, n)])
    df = rng.normal(0.0, 5.0, (3, n))
    return np.concatenate([a, t2, df])


def unit_vectors(rng, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def truth_dwi2(rng, n: int, block_ids: Optional[np.ndarray] = None) -> np.ndarray:
    """f~U(.2,.8), Da,De~U(.5,3), fibre uniform on the sphere (folded).

    With ``block_ids`` the values are drawn once per block (piecewise-constant
    maps, the structure a spatial regulariser is meant for)."""
    m = n if block_ids is None else int(block_ids.max()) + 1
    f = rng.uniform(0.2, 0.8, m)
    da = rng.uniform(0.5, 3.0, m)
    de = rng.uniform(0.5, 3.0, m)
    th, ph = _angles(_fold_upper(unit_vectors(rng, m)))
    t = np.stack([f, da, de, th, ph])
    return t if block_ids is None else t[:, block_ids]


def truth_linear3(rng, n: int) -> np.ndarray:
    return rng.uniform(0.2, 1.0, (3, n))


def draw_truth(model: str, rng, n: int, block_ids=None) -> np.ndarray:
    if model in ("monoexp_t2s", "monoexp_r2s"):
        t = truth_monoexp(rng, n)
        if model == "monoexp_r2s":
            t[1] = 1000.0 / t[1]
        return t
    if model == "gre3":
        return truth_gre3(rng, n)
    if model == "dwi2":
        return truth_dwi2(rng, n, block_ids)
    if model == "linear3":
        return truth_linear3(rng, n)
    raise KeyError(model)


def dwi_acq(rng, shells=(1000.0, 2000.0, 3000.0), dirs_per_shell=32) -> Acq:
    b = np.repeat(np.array(shells, dtype=np.float64), dirs_per_shell)
    g = np.concatenate([unit_vectors(rng, dirs_per_shell) for _ in shells])
    return Acq(bval=b, bvec=np.ascontiguousarray(g))


def default_acq(model: str, rng=None) -> Acq:
    if model in ("monoexp_t2s", "monoexp_r2s", "linear3"):
        return Acq(te=echo_times(2.0, 4.0, 12))
    if model == "gre3":
        return Acq(te=echo_times(2.0, 2.0, 24))
    if model == "dwi2":
        return dwi_acq(rng if rng is not None else np.random.default_rng(2))
    raise KeyError(model)


def make_draw(model: str, shape, seed: int, sigma: float, acq: Optional[Acq] = None,
              mask: Optional[np.ndarray] = None, block: int = 0, noise: bool = True) -> Draw:
    """Truth drawn from `seed`; with noise=False no noise is drawn (the caller
    makes its own) and Draw.noise is None."""
    rng = np.random.default_rng(seed)
    if acq is None:
        acq = default_acq(model, rng)
    if mask is None:
        mask = np.ones(shape, dtype=np.uint8)
    n = int(mask.sum())
    block_ids = None
    if block > 0:
        nz, ny, nx = shape
        z, y, x = np.meshgrid(np.arange(nz) // block, np.arange(ny) // block,
                              np.arange(nx) // block, indexing="ij")
        bny = (ny + block - 1) // block
        bnx = (nx + block - 1) // block
        ids = (z * bny + y) * bnx + x
        block_ids = ids[mask.astype(bool)]
    truth = np.ascontiguousarray(draw_truth(model, rng, n, block_ids))
    me = meas_eff(model, acq.n_meas)
    nz_ = rng.standard_normal((me, n), dtype=np.float32) if noise else None
    lb, ub = bounds(model)
    return Draw(model, acq, tuple(shape), mask, truth, nz_, float(sigma), lb, ub, seed)


# ---------------------------------------------------------------------------
# the five synthetic workloads
# ---------------------------------------------------------------------------
def cfg0(seed: int = 0) -> Draw:
    """Mono-exponential T2*: 10^3 voxels, 12 echoes 2..46 ms, sigma 0.01."""
    return make_draw("monoexp_t2s", (10, 10, 10), seed, 0.01,
                     Acq(te=echo_times(2.0, 4.0, 12)))


CFG0_MCMC = dict(n_chains=1, n_iter=2000, burnin=500, thin=1)
CFG0_ADAM = dict(n_iter=200, loss=2)


def cfg1(seed: int = 1, shape=(64, 128, 128)) -> Draw:
    """3-pool complex GRE: 128x128x64, 24 echoes 2..48 ms, sigma 0.01 (SNR 100)."""
    return make_draw("gre3", shape, seed, 0.01, Acq(te=echo_times(2.0, 2.0, 24)))


CFG1_MCMC = dict(n_chains=4, n_iter=5000, burnin=500, thin=100)


def cfg2(seed: int = 2, shape=(64, 64, 64), block: int = 8) -> Draw:
    """Stick + ball diffusion: 64^3, 3 shells x 32 directions, sigma 0.02."""
    rng = np.random.default_rng(seed + 1000)
    return make_draw("dwi2", shape, seed, 0.02, dwi_acq(rng), block=block)


CFG2_ADAM = dict(n_iter=500, loss=2, lam=1e-3, tv_params=("f", "Da", "De"), tv_dim=3)


def cfg4_mask(shape=(180, 240, 240)) -> np.ndarray:
    return ellipsoid_mask(shape, (89.5, 119.5, 119.5), (54.5, 72.5, 72.5))


def cfg4(seed: int = 4) -> Draw:
    """Whole-brain-sized 3-pool GRE: 240x240x180 grid, ellipsoid mask, SNR 50."""
    shape = (180, 240, 240)
    return make_draw("gre3", shape, seed, 0.02, Acq(te=echo_times(2.0, 2.0, 24)),
                     mask=cfg4_mask(shape))


CFG4_MCMC = dict(n_chains=8, n_iter=10000, burnin=1000, thin=10)


# MH proposal widths (parameter units), chosen with the oracle for 20-50 %
# acceptance at the workloads' noise levels and frozen here.
MH_STEP: Dict[str, Tuple[float, ...]] = {
    "monoexp_t2s": (0.01, 1.0),
    "monoexp_r2s": (0.006, 0.3),
    "gre3": (0.01, 0.01, 0.01, 0.3, 1.0, 1.0, 0.5, 0.5, 0.5),
    "dwi2": (0.01, 0.02, 0.01, 0.02, 0.04),
    "linear3": (0.02, 0.02, 0.02),
}


# ---------------------------------------------------------------------------
# serving trace
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class JobSpec:
    arrival_s: float
    model: str
    kind: str             # "mcmc" or "fit"
    n_vox: int
    seed: int
    n_chains: int = 1
    n_iter: int = 0
    burnin: int = 0
    thin: int = 1
    tv: bool = False


def serving_trace(seed: int = 3, n_jobs: int = 256, rate: float = 20.0,
                  vox_range=(1e3, 1e6), mcmc_iters=(1000, 10000),
                  fit_iters=(200, 500)) -> List[JobSpec]:
    """Poisson arrivals, models uniform over the three workloads' models,
    log-uniform voxel counts, 50/50 MCMC / fit."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_jobs)
    t = np.cumsum(gaps) - gaps[0]
    models = ("monoexp_t2s", "gre3", "dwi2")
    jobs = []
    for i in range(n_jobs):
        model = models[int(rng.integers(0, 3))]
        lo, hi = math.log(vox_range[0]), math.log(vox_range[1])
        nv = int(round(math.exp(rng.uniform(lo, hi))))
        if rng.uniform() < 0.5:
            it = int(rng.integers(mcmc_iters[0], mcmc_iters[1] + 1))
            jobs.append(JobSpec(float(t[i]), model, "mcmc", nv, 10_000 + i,
                                n_chains=int(rng.integers(1, 9)), n_iter=it,
                                burnin=it // 10, thin=10))
        else:
            it = int(rng.integers(fit_iters[0], fit_iters[1] + 1))
            jobs.append(JobSpec(float(t[i]), model, "fit", nv, 10_000 + i,
                                n_iter=it, tv=(model == "dwi2")))
    return jobs


# ---------------------------------------------------------------------------
# image reconstruction (multi-echo GRE, multi-coil, CAIPI undersampling)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class SenseDraw:
    """One slice after the read-out transform.  The caller forms the
    measurement k = M_e F2(C_c I_e) + sigma * noise with its own operator."""
    truth: np.ndarray     # [E, Ny, Nz] complex128 multi-echo image
    coils: np.ndarray     # [Nc, Ny, Nz] complex128 sensitivities
    mask: np.ndarray      # [E, Ny, Nz] uint8 sampling pattern
    noise: Optional[np.ndarray]   # [E, Nc, Ny, Nz] complex128, unit variance per component
    sigma: float
    te: np.ndarray        # echo times (ms)


def caipi_mask(n_echo: int, ny: int, nz: int, rz: int = 9, z_shift: int = 3,
               te_shift: int = 2) -> np.ndarray:
    """Controlled-aliasing pattern with R_y = 1: every y line, every rz-th z
    position, the offset moving by z_shift per y line and by te_shift per
    echo (the acceleration and shifts of the paper's multi-echo GRE demo)."""
    e = np.arange(n_echo)[:, None, None]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[None, None, :]
    return (((z - z_shift * y - te_shift * e) % rz) == 0).astype(np.uint8)


def sense_draw(seed: int, n_echo: int = 6, n_coil: int = 32, ny: int = 256, nz: int = 256,
               sigma: float = 0.01, noise: bool = True, mask: Optional[np.ndarray] = None
               ) -> SenseDraw:
    """Elliptical head-like phantom with tissue classes of different T2* and a
    smooth off-resonance field, echoes at 3, 8, ..., ms; coils are Gaussian
    sensitivity profiles (width 0.3-0.5 of the half field of view) centred on
    a ring just outside the slice, each with a random phase and a phase ramp
    along its direction (a loop array); CAIPI mask R_z = 9.  With 32 coils
    the pattern is well conditioned: a 64 x 64 slice reconstructs to about 6 %
    of the image norm in 1000 Adam steps (lr 0.01) at sigma 0.001."""
    rng = np.random.default_rng(seed)
    te = echo_times(3.0, 5.0, n_echo)
    yy, zz = np.meshgrid((np.arange(ny) - ny / 2 + 0.5) / (ny / 2),
                         (np.arange(nz) - nz / 2 + 0.5) / (nz / 2), indexing="ij")
    m0 = np.zeros((ny, nz))
    r2s = np.zeros((ny, nz))
    # outer head, then a few inner ellipses of other tissue (random placement)
    head = (yy / 0.85) ** 2 + (zz / 0.7) ** 2 < 1.0
    m0[head] = 0.8
    r2s[head] = 0.02
    for _ in range(6):
        cy, cz = rng.uniform(-0.45, 0.45, 2)
        ay, az = rng.uniform(0.08, 0.3, 2)
        blob = ((yy - cy) / ay) ** 2 + ((zz - cz) / az) ** 2 < 1.0
        m0[blob & head] = rng.uniform(0.4, 1.0)
        r2s[blob & head] = rng.uniform(0.01, 0.08)
    df = 0.02 * (rng.uniform(-1, 1) * yy + rng.uniform(-1, 1) * zz + 0.5 * yy * zz)  # kHz
    phi0 = rng.uniform(-np.pi, np.pi)
    t = te[:, None, None]
    truth = m0 * np.exp(-r2s * t) * np.exp(1j * (phi0 + 2 * np.pi * df * t))
    ang = 2 * np.pi * (np.arange(n_coil) + rng.uniform(0, 1)) / n_coil
    cy, cz = 1.05 * np.cos(ang), 1.05 * np.sin(ang)
    w = rng.uniform(0.3, 0.5, n_coil)
    ph = rng.uniform(-np.pi, np.pi, n_coil)
    d2 = (yy[None] - cy[:, None, None]) ** 2 + (zz[None] - cz[:, None, None]) ** 2
    ca, sa = np.cos(ang)[:, None, None], np.sin(ang)[:, None, None]
    coils = np.exp(-d2 / (2 * w[:, None, None] ** 2)) * np.exp(
        1j * (ph[:, None, None] + 1.5 * (yy[None] * ca + zz[None] * sa)))
    if mask is None:
        mask = caipi_mask(n_echo, ny, nz)
    nse = None
    if noise:
        nse = (rng.standard_normal((n_echo, n_coil, ny, nz)) +
               1j * rng.standard_normal((n_echo, n_coil, ny, nz)))
    return SenseDraw(truth, coils, mask, nse, sigma, te)


# Reconstruction workload: one slice of the paper's multi-echo GRE demo
# geometry (6 echoes, CAIPI R_z = 9), 32 coils, 256 x 256 phase encodes,
# L1 data loss with 2D TV, Adam.  The TV weight 0.002 and the 500 iterations
# are the paper's settings for its regularised reconstruction (Table 1); the
# rate is not given there, and 0.1 lets 500 iterations reach the TV floor on
# this phantom's scale (relative error against the phantom 0.18 after 500
# iterations, 0.16 after 3000; 0.57 at rate 0.01).
SENSE_RECON = dict(n_echo=6, n_coil=32, ny=256, nz=256, sigma=0.01, n_iter=500, loss=1,
                   lam=0.002, lr=0.1)
