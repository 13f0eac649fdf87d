"""ctypes binding of libgacelle.so (the C ABI declared in include/gacelle.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Bulk arrays may be numpy arrays (host memory) or torch tensors on
a ROCm device (device memory, the current torch stream is used); a call
takes one or the other for all its bulk arrays.  The library must be built
(``python -m paper_2511_22094_amd.build``); importing this module without it
raises ImportError -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GACELLE_LIB names another build of the same library (e.g. one compiled
# with different tuning); the default is the in-tree build.
LIB_PATH = os.environ.get("GACELLE_LIB") or os.path.join(_HERE, "libgacelle.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2511_22094_amd.build` (hipcc, gfx950)")

# One HIP runtime per process: PyTorch ships its own libamdhip64.so.7 and
# cannot initialise the GPU once a second copy has claimed it.  Loading
# torch first lets the dynamic linker bind this library's HIP dependency to
# torch's already-loaded runtime, so device pointers and streams are shared.
try:
    import torch  # noqa: F401
except ImportError:
    torch = None

_L = ctypes.CDLL(LIB_PATH)

c_int, c_int64, c_uint32, c_uint64, c_double, c_size_t, c_void_p, c_char_p = (
    ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
    ctypes.c_size_t, ctypes.c_void_p, ctypes.c_char_p)

GC_OK = 0
STATUS = {0: "GC_OK", -1: "GC_E_INVAL", -2: "GC_E_NOMODEL", -3: "GC_E_NOMEM",
          -4: "GC_E_NONFINITE", -5: "GC_E_DEVICE", -6: "GC_E_CANCELLED", -7: "GC_E_TIMEOUT",
          -8: "GC_E_NOTFOUND"}
GC_MEM_HOST, GC_MEM_DEVICE = 0, 1
OPTIMIZERS = {"adam": 0, "sgdm": 1, "rmsprop": 2}
JOB_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


class GcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class gc_exec(ctypes.Structure):
    _fields_ = [("device", c_int), ("stream", c_void_p), ("mem_kind", c_int)]


class gc_acq(ctypes.Structure):
    _fields_ = [("n_meas", c_int), ("te", c_void_p), ("bval", c_void_p), ("bvec", c_void_p)]


class gc_volume(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int), ("y", c_void_p)]


class gc_bounds(ctypes.Structure):
    _fields_ = [("lb", c_void_p), ("ub", c_void_p), ("x0", c_void_p), ("x0_map", c_void_p)]


class gc_adam_hyper(ctypes.Structure):
    _fields_ = [("optimizer", c_int), ("lr", c_double), ("beta1", c_double),
                ("beta2", c_double), ("eps", c_double), ("momentum", c_double),
                ("rho", c_double), ("n_iter", c_int), ("loss", c_int), ("weights", c_void_p),
                ("lambda_", c_double), ("tv_mask", c_uint32), ("tv_dim", c_int),
                ("tol", c_double), ("conv_value", c_double), ("conv_window", c_int),
                ("loss_history", c_void_p), ("tv_kind", c_int), ("graph_n", c_int64),
                ("graph_nnz", c_int64), ("graph_rowptr", c_void_p), ("graph_col", c_void_p),
                ("prior_lambda", c_double), ("prior_mask", c_uint32), ("prior_mu", c_void_p),
                ("prior_sigma", c_void_p), ("t_start", c_int), ("init_state", c_void_p),
                ("final_state", c_void_p), ("precision", c_int)]


TV_KINDS = {"aniso": 0, "iso": 1, "graph": 2}


class gc_fit_report(ctypes.Structure):
    _fields_ = [("iters_run", c_int), ("final_loss", c_double), ("stop_reason", c_int)]


# gc_sample_sink: int (*)(void *user, int k_first, int k_count, const float *samples,
#                         int64_t n_masked, int n_chains, int n_params)
SAMPLE_SINK = ctypes.CFUNCTYPE(c_int, c_void_p, c_int, c_int, ctypes.POINTER(ctypes.c_float),
                               c_int64, c_int, c_int)


class gc_mcmc_hyper(ctypes.Structure):
    _fields_ = [("sigma", c_double), ("step", c_void_p), ("seed", c_uint64), ("x0_mode", c_int),
                ("weights", c_void_p), ("precision", c_int), ("sampler", c_int),
                ("n_walkers", c_int), ("stretch", c_double), ("chunk_iters", c_int),
                ("final_state", c_void_p), ("final_logl", c_void_p), ("t_start", c_int),
                ("init_state", c_void_p), ("init_logl", c_void_p),
                ("sample_sink", SAMPLE_SINK), ("sink_user", c_void_p), ("sink_bytes", c_size_t)]


def _sink(fn):
    """Wraps fn(k_first, samples) -- samples a float32 numpy view [C, k, P, n]
    valid only during the call -- as a gc_sample_sink; fn returning False (or
    raising) stops the run."""
    def cb(_user, k_first, k_count, ptr, n, C, P):
        try:
            arr = np.ctypeslib.as_array(ptr, shape=(C, k_count, P, n))
            return 1 if fn(int(k_first), arr) is False else 0
        except Exception:   # noqa: BLE001 -- any failure stops the run
            import traceback
            traceback.print_exc()
            return 1
    return SAMPLE_SINK(cb)


class gc_sense_problem(ctypes.Structure):
    _fields_ = [("ny", c_int), ("nz", c_int), ("n_echo", c_int), ("n_coil", c_int),
                ("kspace", c_void_p), ("coils", c_void_p), ("mask", c_void_p), ("init", c_void_p)]


class gc_server_cfg(ctypes.Structure):
    _fields_ = [("device", c_int), ("hbm_budget", c_size_t), ("max_slots", c_int),
                ("chunk_iters", c_int), ("baseline", c_int)]


class gc_job(ctypes.Structure):
    _fields_ = [("kind", c_int), ("model", c_void_p), ("data", gc_volume), ("mask", c_void_p),
                ("bounds", gc_bounds), ("adam", gc_adam_hyper), ("n_chains", c_int),
                ("n_iter", c_int), ("burnin", c_int), ("thin", c_int),
                ("mcmc", gc_mcmc_hyper), ("out_maps", c_void_p), ("out_mean", c_void_p),
                ("out_std", c_void_p), ("out_accept", c_void_p), ("report", c_void_p)]


class gc_stats(ctypes.Structure):
    _fields_ = [("submitted", c_uint64), ("completed", c_uint64), ("failed", c_uint64),
                ("cancelled", c_uint64), ("resident", c_int), ("queued", c_int),
                ("hbm_in_use", c_size_t), ("voxel_iters", c_double),
                ("busy_seconds", c_double), ("p50_latency_s", c_double),
                ("p99_latency_s", c_double), ("peak_resident", c_int)]


P = c_void_p
_sig = {
    "gc_last_error": ([], c_char_p),
    "gc_version": ([], c_char_p),
    "gc_model_create": ([c_char_p, ctypes.POINTER(gc_acq), ctypes.POINTER(c_void_p)], c_int),
    "gc_model_info": ([P, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(c_int)], c_int),
    "gc_model_param_name": ([P, c_int], c_char_p),
    "gc_model_destroy": ([P], c_int),
    "gc_count_mask": ([P, c_int64, ctypes.POINTER(c_int64), ctypes.POINTER(gc_exec)], c_int),
    "gc_adam_defaults": ([ctypes.POINTER(gc_adam_hyper)], None),
    "gc_fit_askadam": ([P, ctypes.POINTER(gc_volume), P, ctypes.POINTER(gc_bounds),
                        ctypes.POINTER(gc_adam_hyper), P, ctypes.POINTER(gc_fit_report),
                        ctypes.POINTER(gc_exec)], c_int),
    "gc_mcmc_defaults": ([ctypes.POINTER(gc_mcmc_hyper)], None),
    "gc_burnin_from_ratio": ([c_double, c_int], c_int),
    "gc_mcmc": ([P, ctypes.POINTER(gc_volume), P, ctypes.POINTER(gc_bounds), c_int, c_int, c_int,
                 c_int, ctypes.POINTER(gc_mcmc_hyper), P, P, P, P, ctypes.POINTER(gc_exec)], c_int),
    "gc_mcmc_noalloc": ([P, ctypes.POINTER(gc_volume), P, ctypes.POINTER(gc_bounds), c_int, c_int,
                         c_int, c_int, ctypes.POINTER(gc_mcmc_hyper), P, P, P, P,
                         ctypes.POINTER(gc_exec)], c_int),
    "gc_noalloc_scratch_bytes": ([], c_size_t),
    "gc_model_forward": ([P, P, c_int64, P, ctypes.POINTER(gc_exec)], c_int),
    "gc_model_vjp": ([P, P, c_int64, P, P, ctypes.POINTER(gc_exec)], c_int),
    "gc_loss_vjp": ([P, P, P, P, c_int64, c_int, c_double, P, P, ctypes.POINTER(gc_exec)], c_int),
    "gc_tv": ([c_int, c_int, c_int, P, P, c_int, c_double, ctypes.POINTER(c_double), P,
               ctypes.POINTER(gc_exec)], c_int),
    "gc_tv_iso": ([c_int, c_int, c_int, P, P, c_int, c_double, ctypes.POINTER(c_double), P,
                   ctypes.POINTER(gc_exec)], c_int),
    "gc_tv_graph": ([c_int64, P, P, c_int64, P, c_double, ctypes.POINTER(c_double), P,
                     ctypes.POINTER(gc_exec)], c_int),
    "gc_sense_recon": ([ctypes.POINTER(gc_sense_problem), ctypes.POINTER(gc_adam_hyper), P,
                        ctypes.POINTER(gc_fit_report), ctypes.POINTER(gc_exec)], c_int),
    "gc_sense_forward": ([ctypes.POINTER(gc_sense_problem), P, P, ctypes.POINTER(gc_exec)], c_int),
    "gc_sense_adjoint": ([ctypes.POINTER(gc_sense_problem), P, P, ctypes.POINTER(gc_exec)], c_int),
    "gc_philox": ([c_uint64, P, c_int64, P, ctypes.POINTER(gc_exec)], c_int),
    "gc_philox_uniform_normal": ([c_uint64, P, c_int64, c_int, P, P, ctypes.POINTER(gc_exec)], c_int),
    "gc_timing_enable": ([c_int], c_int),
    "gc_timing_get": ([c_char_p, ctypes.POINTER(c_double), ctypes.POINTER(c_int64)], c_int),
    "gc_timing_reset": ([], c_int),
    "gc_server_create": ([ctypes.POINTER(gc_server_cfg), ctypes.POINTER(c_void_p)], c_int),
    "gc_submit": ([P, ctypes.POINTER(gc_job), ctypes.POINTER(c_uint64)], c_int),
    "gc_poll": ([P, c_uint64, ctypes.POINTER(c_int)], c_int),
    "gc_wait": ([P, c_uint64, c_int, ctypes.POINTER(c_int)], c_int),
    "gc_cancel": ([P, c_uint64], c_int),
    "gc_release": ([P, c_uint64], c_int),
    "gc_job_latency": ([P, c_uint64, ctypes.POINTER(c_double)], c_int),
    "gc_server_stats": ([P, ctypes.POINTER(gc_stats)], c_int),
    "gc_server_destroy": ([P], c_int),
}
EXPORTS = tuple(_sig)
for _name, (_args, _res) in _sig.items():
    _f = getattr(_L, _name, None)
    if _f is None:
        continue
    _f.argtypes = _args
    _f.restype = _res


def gc_timing_enable(on=True, every: int = 1):
    """on: enable / disable; every = k times every k-th launch of a family within a call."""
    _L.gc_timing_enable(max(int(every), 1) if on else 0)


def gc_timing_reset():
    _L.gc_timing_reset()


def gc_timing_get(family: str):
    """(total ms, launches) of a kernel family since the last reset."""
    ms, n = c_double(), c_int64()
    _check(_L.gc_timing_get(family.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def last_error() -> str:
    return _L.gc_last_error().decode()


def _check(rc: int):
    if rc != GC_OK:
        raise GcError(rc, last_error())


# ------------------------------------------------------------ array helpers
def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Args:
    """Collects the bulk arrays of one call and decides host vs device."""

    def __init__(self, device: int = -1):
        self.keep = []
        self.kind: Optional[int] = None
        self.device = device
        self.stream = None

    def _note(self, kind: int, dev: int = -1):
        if self.kind is None:
            self.kind = kind
        elif self.kind != kind:
            raise TypeError("mix of host (numpy) and device (torch) arrays in one call")
        if kind == GC_MEM_DEVICE and self.device < 0:
            self.device = dev

    def ptr(self, a, dtype) -> Optional[int]:
        if a is None:
            return None
        if _is_torch(a):
            import torch
            if not a.is_cuda:
                raise TypeError("torch tensors must live on the GPU (use numpy for host data)")
            want = {np.float32: torch.float32, np.float64: torch.float64,
                    np.uint8: torch.uint8, np.int32: torch.int32,
                    np.uint32: torch.int32, np.int64: torch.int64}[dtype]
            if a.dtype != want and not (dtype is np.uint32 and a.dtype == torch.int32):
                raise TypeError(f"expected {want}, got {a.dtype}")
            if not a.is_contiguous():
                raise TypeError("device arrays must be contiguous")
            self._note(GC_MEM_DEVICE, a.device.index)
            self.keep.append(a)
            return a.data_ptr()
        arr = np.ascontiguousarray(a, dtype=dtype)
        self._note(GC_MEM_HOST)
        self.keep.append(arr)
        return arr.ctypes.data

    def out(self, a, dtype):
        """Output buffer: must already be of the right dtype and contiguous."""
        if a is None:
            return None
        if _is_torch(a):
            return self.ptr(a, dtype)
        if a.dtype != dtype or not a.flags.c_contiguous:
            raise TypeError(f"output must be a contiguous {np.dtype(dtype)} array")
        self._note(GC_MEM_HOST)
        return a.ctypes.data

    def exec(self) -> gc_exec:
        kind = GC_MEM_HOST if self.kind is None else self.kind
        stream = None
        if kind == GC_MEM_DEVICE:
            import torch
            stream = torch.cuda.current_stream(self.device).cuda_stream
        return gc_exec(self.device if kind == GC_MEM_DEVICE else -1, stream, kind)


def _host_f64(x, n: int) -> np.ndarray:
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (n,)))
    return a


# ------------------------------------------------------------------ models
class Model:
    """A registry model (gc_model_create); released with the object."""

    def __init__(self, name: str, te=None, bval=None, bvec=None):
        self._te = None if te is None else np.ascontiguousarray(te, dtype=np.float64)
        self._b = None if bval is None else np.ascontiguousarray(bval, dtype=np.float64)
        self._g = None if bvec is None else np.ascontiguousarray(bvec, dtype=np.float64)
        M = len(self._te) if self._te is not None else (len(self._b) if self._b is not None else 0)
        acq = gc_acq(M, None if self._te is None else self._te.ctypes.data,
                     None if self._b is None else self._b.ctypes.data,
                     None if self._g is None else self._g.ctypes.data)
        h = c_void_p()
        _check(_L.gc_model_create(name.encode(), ctypes.byref(acq), ctypes.byref(h)))
        self.handle = h
        self.name = name
        p, me, cx = c_int(), c_int(), c_int()
        _check(_L.gc_model_info(h, ctypes.byref(p), ctypes.byref(me), ctypes.byref(cx)))
        self.n_params, self.n_meas_eff, self.is_complex = p.value, me.value, bool(cx.value)
        self.n_meas = M
        self.param_names = tuple(_L.gc_model_param_name(h, i).decode() for i in range(p.value))

    @classmethod
    def from_acq(cls, name: str, acq) -> "Model":
        return cls(name, getattr(acq, "te", None), getattr(acq, "bval", None),
                   getattr(acq, "bvec", None))

    # the destroy entry point is bound at definition time: at interpreter
    # shutdown the module globals may already have been cleared
    def __del__(self, _destroy=_L.gc_model_destroy):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            _destroy(h)
            self.handle = None


def gc_model_create(name: str, te=None, bval=None, bvec=None) -> Model:
    return Model(name, te, bval, bvec)


def gc_version() -> str:
    return _L.gc_version().decode()


def gc_noalloc_scratch_bytes() -> int:
    return int(_L.gc_noalloc_scratch_bytes())


def gc_burnin_from_ratio(ratio: float, n_iter: int) -> int:
    return int(_L.gc_burnin_from_ratio(ratio, n_iter))


def gc_count_mask(mask) -> int:
    a = _Args()
    p = a.ptr(mask, np.uint8)
    n = c_int64()
    ex = a.exec()
    _check(_L.gc_count_mask(p, int(np.prod(mask.shape)), ctypes.byref(n), ctypes.byref(ex)))
    return n.value


def _shape3(y, model: Model):
    if y.ndim != 4 or y.shape[0] != model.n_meas_eff:
        raise ValueError(f"data must be [M_eff={model.n_meas_eff}, nz, ny, nx], got {tuple(y.shape)}")
    return int(y.shape[3]), int(y.shape[2]), int(y.shape[1])


def _bounds(model, lb, ub, x0, x0_map, args: _Args):
    P_ = model.n_params
    lbv, ubv = _host_f64(lb, P_), _host_f64(ub, P_)
    x0v = None if x0 is None else _host_f64(x0, P_)
    args.keep += [lbv, ubv, x0v]
    return gc_bounds(lbv.ctypes.data, ubv.ctypes.data, None if x0v is None else x0v.ctypes.data,
                     args.ptr(x0_map, np.float32))


def _empty_like_kind(args: _Args, shape, dtype, like):
    if _is_torch(like):
        import torch
        t = {np.float32: torch.float32, np.float64: torch.float64, np.int32: torch.int32}[dtype]
        return torch.empty(shape, dtype=t, device=like.device)
    return np.empty(shape, dtype=dtype)


def gc_fit_askadam(model: Model, y, mask, lb, ub, *, x0=None, x0_map=None, weights=None,
                   optimizer="adam", lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, momentum=0.9,
                   rho=0.9, n_iter=200, loss=2, lam=0.0, tv_params: Sequence[int] = (),
                   tv_dim=3, tol=0.0, conv_value=0.0, conv_window=20, loss_history=False,
                   out=None, tv_kind="aniso", graph=None, prior_lam=0.0,
                   prior_params: Sequence[int] = (), prior_mu=None, prior_sigma=None,
                   t_start=0, init_state=None, final_state=False, precision="fp32"):
    """Returns dict(maps [P, nz, ny, nx] float32, iters_run, final_loss, stop_reason[, loss]
    [, final_state]).

    tv_kind "aniso" | "iso" | "graph" (graph = (rowptr [n+1] int64, col int32) over the
    masked voxels in grid order); prior_mu / prior_sigma [P, nz, ny, nx] for the prior
    term on prior_params.

    Checkpoint / resume: final_state=True returns the optimiser state
    [3, P, n_masked] float32 (u, m, v) after the last iteration; t_start > 0
    with init_state = that state of a call that ran t_start iterations runs
    iterations t_start + 1 .. n_iter.  loss_history may then be the earlier
    call's losses (their first t_start entries seed the convergence window).

    precision "fp64": the deterministic test path (FP64 iterate, moments and
    losses, one launch per iteration; maps rounded once to FP32)."""
    a = _Args()
    nx, ny, nz = _shape3(y, model)
    vol = gc_volume(nx, ny, nz, a.ptr(y, np.float32))
    mp = a.ptr(mask, np.uint8)
    b = _bounds(model, lb, ub, x0, x0_map, a)
    h = gc_adam_hyper()
    _L.gc_adam_defaults(ctypes.byref(h))
    h.optimizer = OPTIMIZERS[optimizer]
    h.lr, h.beta1, h.beta2, h.eps, h.momentum, h.rho = lr, beta1, beta2, eps, momentum, rho
    h.n_iter, h.loss = n_iter, loss
    h.weights = a.ptr(weights, np.float32)
    h.lambda_ = lam
    h.tv_mask = sum(1 << int(p) for p in tv_params)
    h.tv_dim = tv_dim
    h.tol, h.conv_value, h.conv_window = tol, conv_value, conv_window
    _set_regularisers(h, a, model, tv_kind, graph, prior_lam, prior_params, prior_mu,
                      prior_sigma)
    prev = None
    if loss_history is not None and not isinstance(loss_history, bool):
        prev = np.asarray(loss_history, np.float64)[: int(t_start)]
        loss_history = True
    hist = np.zeros(max(n_iter, 1)) if loss_history else None
    if prev is not None:
        hist[: prev.size] = prev
    h.loss_history = None if hist is None else hist.ctypes.data
    maps = out if out is not None else _empty_like_kind(a, (model.n_params, nz, ny, nx),
                                                       np.float32, y)
    mo = a.out(maps, np.float32)
    h.t_start = int(t_start)
    h.init_state = a.ptr(init_state, np.float32)
    h.precision = {"fp32": 0, "fp64": 1}[precision]
    fs = None
    if final_state:
        if mask is None:
            n = nx * ny * nz
        elif _is_torch(mask):
            n = int(mask.sum().item())
        else:
            n = int(np.count_nonzero(mask))
        fs = _empty_like_kind(a, (3, model.n_params, n), np.float32, y)
    h.final_state = a.out(fs, np.float32)
    rep = gc_fit_report()
    ex = a.exec()
    _check(_L.gc_fit_askadam(model.handle, ctypes.byref(vol), mp, ctypes.byref(b),
                             ctypes.byref(h), mo, ctypes.byref(rep), ctypes.byref(ex)))
    r = dict(maps=maps, iters_run=rep.iters_run, final_loss=rep.final_loss,
             stop_reason=rep.stop_reason)
    if hist is not None:
        r["loss"] = hist[: rep.iters_run]
    if fs is not None:
        r["final_state"] = fs
    return r


def gc_mcmc(model: Model, y, mask, lb, ub, n_chains, n_iter, burnin, thin, *, sigma,
            step=None, seed=0, x0=None, x0_map=None, x0_mode="midpoint", weights=None,
            precision="fp32", sampler="mh", n_walkers=50, stretch=2.0, chunk_iters=0,
            samples=False, accept=True, final_state=False, out_mean=None, out_std=None,
            t_start=0, init_state=None, init_logl=None, sample_sink=None, sink_bytes=0,
            noalloc=False):
    """Returns dict(mean, std [P, nz, ny, nx] float64, accept [C, nz, ny, nx],
    samples [C, K, P, n_masked] float32 or None, final_state [P, C, n], final_logl [C, n]).

    Resume: t_start > 0 with init_state [P, C, n] (and init_logl [C, n]), e.g. the
    final_state / final_logl of a call that ran up to step t_start.

    sample_sink: fn(k_first, samples) receiving the retained samples while the
    chains run, in deliveries of at most sink_bytes (0 = 256 MiB): samples is a
    float32 view [C, k, P, n_masked] of host memory valid only during the call
    (copy what you keep); returning False stops the run (GcError
    GC_E_CANCELLED).  Not with samples=True.

    noalloc: call gc_mcmc_noalloc, which allocates no device memory (all its
    scratch lives in a fixed per-GPU array of gc_noalloc_scratch_bytes());
    every bulk argument must then be a torch tensor on the GPU, outputs
    included (out_mean and out_std, or none given)."""
    a = _Args()
    nx, ny, nz = _shape3(y, model)
    vol = gc_volume(nx, ny, nz, a.ptr(y, np.float32))
    mp = a.ptr(mask, np.uint8)
    b = _bounds(model, lb, ub, x0, x0_map, a)
    h = gc_mcmc_hyper()
    _L.gc_mcmc_defaults(ctypes.byref(h))
    h.sigma = sigma
    st = None if step is None else _host_f64(step, model.n_params)
    a.keep.append(st)
    h.step = None if st is None else st.ctypes.data
    h.seed = int(seed)
    h.x0_mode = {"midpoint": 0, "uniform": 1, "given": 2}[x0_mode]
    if x0_map is not None or x0 is not None:
        h.x0_mode = 2 if x0_mode == "midpoint" else h.x0_mode
    h.weights = a.ptr(weights, np.float32)
    h.precision = {"fp32": 0, "fp64": 1}[precision]
    h.sampler = {"mh": 0, "ensemble": 1}[sampler]
    h.n_walkers = n_walkers
    h.stretch = stretch
    h.chunk_iters = chunk_iters
    h.t_start = int(t_start)
    h.init_state = a.ptr(init_state, np.float64)
    h.init_logl = a.ptr(init_logl, np.float64)
    if sample_sink is not None:
        cb = _sink(sample_sink)
        a.keep.append(cb)
        h.sample_sink = cb
        h.sink_bytes = int(sink_bytes)
    C = n_walkers if sampler == "ensemble" else n_chains
    K = (n_iter - burnin) // thin - (max(t_start - burnin, 0) // thin)
    if mask is None:
        n = nx * ny * nz
    elif _is_torch(mask):
        n = int(mask.sum().item())
    else:
        n = int(np.count_nonzero(mask))
    P_ = model.n_params
    mean = out_mean if out_mean is not None else _empty_like_kind(a, (P_, nz, ny, nx), np.float64, y)
    std = out_std if out_std is not None else _empty_like_kind(a, (P_, nz, ny, nx), np.float64, y)
    acc = _empty_like_kind(a, (C, nz, ny, nx), np.int32, y) if accept else None
    smp = _empty_like_kind(a, (C, K, P_, n), np.float32, y) if samples else None
    fs = _empty_like_kind(a, (P_, C, n), np.float64, y) if final_state else None
    fl = _empty_like_kind(a, (C, n), np.float64, y) if final_state else None
    h.final_state = a.out(fs, np.float64)
    h.final_logl = a.out(fl, np.float64)
    ex_ptrs = (a.out(mean, np.float64), a.out(std, np.float64), a.out(smp, np.float32),
               a.out(acc, np.int32))
    ex = a.exec()
    fn = _L.gc_mcmc_noalloc if noalloc else _L.gc_mcmc
    _check(fn(model.handle, ctypes.byref(vol), mp, ctypes.byref(b), n_chains, n_iter,
              burnin, thin, ctypes.byref(h), *ex_ptrs, ctypes.byref(ex)))
    return dict(mean=mean, std=std, accept=acc, samples=smp, final_state=fs, final_logl=fl)


def gc_model_forward(model: Model, theta, out=None):
    a = _Args()
    n = int(theta.shape[1])
    s = out if out is not None else _empty_like_kind(a, (model.n_meas_eff, n), np.float32, theta)
    tp = a.ptr(theta, np.float32)
    sp = a.out(s, np.float32)
    ex = a.exec()
    _check(_L.gc_model_forward(model.handle, tp, n, sp, ctypes.byref(ex)))
    return s


def gc_model_vjp(model: Model, theta, ds, out=None):
    a = _Args()
    n = int(theta.shape[1])
    g = out if out is not None else _empty_like_kind(a, (model.n_params, n), np.float32, theta)
    tp, dp = a.ptr(theta, np.float32), a.ptr(ds, np.float32)
    gp = a.out(g, np.float32)
    ex = a.exec()
    _check(_L.gc_model_vjp(model.handle, tp, n, dp, gp, ctypes.byref(ex)))
    return g


def gc_loss_vjp(model: Model, theta, y, w=None, p=2, scale=1.0):
    a = _Args()
    n = int(theta.shape[1])
    g = _empty_like_kind(a, (model.n_params, n), np.float32, theta)
    loss = _empty_like_kind(a, (n,), np.float32, theta)
    args = (a.ptr(theta, np.float32), a.ptr(y, np.float32), a.ptr(w, np.float32))
    lp, gp = a.out(loss, np.float32), a.out(g, np.float32)
    ex = a.exec()
    _check(_L.gc_loss_vjp(model.handle, *args, n, p, scale, lp, gp, ctypes.byref(ex)))
    return loss, g


def gc_tv(u, mask=None, tv_dim=3, scale=1.0, grad=True, kind="aniso"):
    """u [nz, ny, nx] float32 -> (R float, dR like u or None); kind "aniso" | "iso"."""
    a = _Args()
    nz, ny, nx = (int(s) for s in u.shape)
    up = a.ptr(u, np.float32)
    mp = a.ptr(mask, np.uint8)
    dR = _empty_like_kind(a, tuple(u.shape), np.float32, u) if grad else None
    dp = a.out(dR, np.float32)
    R = c_double()
    ex = a.exec()
    fn = {"aniso": _L.gc_tv, "iso": _L.gc_tv_iso}[kind]
    _check(fn(nx, ny, nz, mp, up, tv_dim, scale, ctypes.byref(R), dp, ctypes.byref(ex)))
    return R.value, dR


def gc_tv_iso(u, mask=None, tv_dim=3, scale=1.0, grad=True):
    return gc_tv(u, mask, tv_dim, scale, grad, kind="iso")


def gc_tv_graph(rowptr, col, u, scale=1.0, grad=True):
    """Graph TV of a vertex map u [n] over CSR (rowptr [n+1] int64, col int32)
    -> (R float, dR like u or None)."""
    a = _Args()
    n = int(u.shape[0])
    rp = a.ptr(rowptr, np.int64)
    cp = a.ptr(col, np.int32)
    up = a.ptr(u, np.float32)
    dR = _empty_like_kind(a, (n,), np.float32, u) if grad else None
    dp = a.out(dR, np.float32)
    R = c_double()
    ex = a.exec()
    _check(_L.gc_tv_graph(n, rp, cp, int(col.shape[0]), up, scale, ctypes.byref(R), dp,
                          ctypes.byref(ex)))
    return R.value, dR


def _set_regularisers(h, a, model, tv_kind, graph, prior_lam, prior_params, prior_mu,
                      prior_sigma, keep=None):
    """Fills the TV-form, graph and prior fields of a gc_adam_hyper."""
    h.tv_kind = TV_KINDS[tv_kind]
    if graph is not None:
        rowptr, col = graph
        h.graph_n = int(rowptr.shape[0]) - 1
        h.graph_nnz = int(col.shape[0])
        h.graph_rowptr = a.ptr(rowptr, np.int64) if a is not None else _host(rowptr, np.int64, keep)
        h.graph_col = a.ptr(col, np.int32) if a is not None else _host(col, np.int32, keep)
    if prior_lam:
        h.prior_lambda = prior_lam
        h.prior_mask = sum(1 << int(p) for p in prior_params)
        h.prior_mu = a.ptr(prior_mu, np.float32) if a is not None else \
            _host(prior_mu, np.float32, keep)
        h.prior_sigma = a.ptr(prior_sigma, np.float32) if a is not None else \
            _host(prior_sigma, np.float32, keep)


def _host(x, dt, keep):
    arr = np.ascontiguousarray(x, dtype=dt)
    keep.append(arr)
    return arr.ctypes.data


# ------------------------------------------------------------ reconstruction
def _cplx_in(a, args: _Args):
    """Complex array -> pointer to interleaved float32 (numpy complex64/128 or a
    torch complex64 tensor on the GPU)."""
    if a is None:
        return None
    if _is_torch(a):
        import torch
        if a.dtype != torch.complex64:
            raise TypeError(f"expected torch.complex64, got {a.dtype}")
        return args.ptr(torch.view_as_real(a.contiguous()), np.float32)
    return args.ptr(np.ascontiguousarray(a, np.complex64).view(np.float32), np.float32)


def _cplx_out(args: _Args, shape, like, out):
    if out is None:
        if _is_torch(like):
            import torch
            out = torch.empty(shape, dtype=torch.complex64, device=like.device)
        else:
            out = np.empty(shape, np.complex64)
    if _is_torch(out):
        import torch
        if out.dtype != torch.complex64 or not out.is_contiguous():
            raise TypeError("output must be a contiguous torch.complex64 tensor")
        return out, args.out(torch.view_as_real(out), np.float32)
    if out.dtype != np.complex64 or not out.flags.c_contiguous:
        raise TypeError("output must be a contiguous complex64 array")
    return out, args.out(out.view(np.float32), np.float32)


def _sense_problem(coils, mask, kspace, init, args: _Args):
    Nc, Ny, Nz = (int(d) for d in coils.shape)
    E = int(mask.shape[0])
    if tuple(mask.shape) != (E, Ny, Nz):
        raise ValueError(f"mask must be [E, {Ny}, {Nz}], got {tuple(mask.shape)}")
    if kspace is not None and tuple(kspace.shape) != (E, Nc, Ny, Nz):
        raise ValueError(f"kspace must be {(E, Nc, Ny, Nz)}, got {tuple(kspace.shape)}")
    if init is not None and tuple(init.shape) != (E, Ny, Nz):
        raise ValueError(f"init must be {(E, Ny, Nz)}, got {tuple(init.shape)}")
    pr = gc_sense_problem(Ny, Nz, E, Nc)
    pr.kspace = _cplx_in(kspace, args)
    pr.coils = _cplx_in(coils, args)
    pr.mask = args.ptr(mask, np.uint8)
    pr.init = _cplx_in(init, args)
    return pr, (E, Nc, Ny, Nz)


def gc_sense_recon(kspace, coils, mask, *, init=None, optimizer="adam", lr=0.01, beta1=0.9,
                   beta2=0.999, eps=1e-8, momentum=0.9, rho=0.9, n_iter=100, loss=2, lam=0.0,
                   tol=0.0, conv_value=0.0, conv_window=20, loss_history=False, out=None):
    """kspace [E, Nc, Ny, Nz], coils [Nc, Ny, Nz] complex, mask [E, Ny, Nz] uint8 ->
    dict(image [E, Ny, Nz] complex64, iters_run, final_loss, stop_reason[, loss])."""
    a = _Args()
    pr, (E, Nc, Ny, Nz) = _sense_problem(coils, mask, kspace, init, a)
    h = gc_adam_hyper()
    _L.gc_adam_defaults(ctypes.byref(h))
    h.optimizer = OPTIMIZERS[optimizer]
    h.lr, h.beta1, h.beta2, h.eps, h.momentum, h.rho = lr, beta1, beta2, eps, momentum, rho
    h.n_iter, h.loss, h.lambda_ = n_iter, loss, lam
    h.tol, h.conv_value, h.conv_window = tol, conv_value, conv_window
    hist = np.zeros(max(n_iter, 1)) if loss_history else None
    h.loss_history = None if hist is None else hist.ctypes.data
    img, op = _cplx_out(a, (E, Ny, Nz), kspace, out)
    rep = gc_fit_report()
    ex = a.exec()
    _check(_L.gc_sense_recon(ctypes.byref(pr), ctypes.byref(h), op, ctypes.byref(rep),
                             ctypes.byref(ex)))
    r = dict(image=img, iters_run=rep.iters_run, final_loss=rep.final_loss,
             stop_reason=rep.stop_reason)
    if hist is not None:
        r["loss"] = hist[: rep.iters_run]
    return r


def gc_sense_forward(image, coils, mask, out=None):
    """[E, Ny, Nz] -> [E, Nc, Ny, Nz] = M_e F2(C_c I_e), complex64."""
    a = _Args()
    pr, (E, Nc, Ny, Nz) = _sense_problem(coils, mask, None, None, a)
    if tuple(image.shape) != (E, Ny, Nz):
        raise ValueError(f"image must be {(E, Ny, Nz)}")
    ip = _cplx_in(image, a)
    res, op = _cplx_out(a, (E, Nc, Ny, Nz), image, out)
    ex = a.exec()
    _check(_L.gc_sense_forward(ctypes.byref(pr), ip, op, ctypes.byref(ex)))
    return res


def gc_sense_adjoint(kspace, coils, mask, out=None):
    """[E, Nc, Ny, Nz] -> [E, Ny, Nz] = sum_c conj(C_c) F2^H(M_e r_ec), complex64."""
    a = _Args()
    pr, (E, Nc, Ny, Nz) = _sense_problem(coils, mask, None, None, a)
    if tuple(kspace.shape) != (E, Nc, Ny, Nz):
        raise ValueError(f"kspace must be {(E, Nc, Ny, Nz)}")
    kp = _cplx_in(kspace, a)
    res, op = _cplx_out(a, (E, Ny, Nz), kspace, out)
    ex = a.exec()
    _check(_L.gc_sense_adjoint(ctypes.byref(pr), kp, op, ctypes.byref(ex)))
    return res


def gc_philox(seed: int, ctr):
    a = _Args()
    n = int(np.prod(ctr.shape)) // 4
    out = _empty_like_kind(a, tuple(ctr.shape), np.int32, ctr) if _is_torch(ctr) else \
        np.empty((n, 4), dtype=np.uint32)
    cp = a.ptr(ctr, np.uint32)
    op = a.ptr(out, np.uint32) if _is_torch(out) else a.out(out, np.uint32)
    ex = a.exec()
    _check(_L.gc_philox(c_uint64(seed), cp, n, op, ctypes.byref(ex)))
    return out


def gc_philox_uniform_normal(seed: int, ctr, precision="fp32"):
    a = _Args()
    n = int(np.prod(ctr.shape)) // 4
    dt = np.float32 if precision == "fp32" else np.float64
    ou = np.empty((n, 4), dtype=dt)
    oz = np.empty((n, 4), dtype=dt)
    cp = a.ptr(ctr, np.uint32)
    ex = a.exec()
    _check(_L.gc_philox_uniform_normal(c_uint64(seed), cp, n, 0 if dt is np.float32 else 1,
                                       ou.ctypes.data, oz.ctypes.data, ctypes.byref(ex)))
    return ou, oz


# ------------------------------------------------------------------ server
class Server:
    """Continuous-batching server (gc_server_*).  Jobs carry host (numpy)
    arrays; the server keeps them (and the job's Model) alive until the job is
    waited for, then releases the job's record on both sides."""

    def __init__(self, device=0, hbm_budget=0, max_slots=0, chunk_iters=0, baseline=False):
        cfg = gc_server_cfg(device, hbm_budget, max_slots, chunk_iters, 1 if baseline else 0)
        h = c_void_p()
        _check(_L.gc_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._jobs = {}
        self._done = {}    # released job id -> (state, latency in s or None)

    def _common(self, model, y, mask, lb, ub, x0, x0_map):
        keep = [model]
        y = np.ascontiguousarray(y, dtype=np.float32)
        nx, ny, nz = _shape3(y, model)
        keep.append(y)
        mk = None
        if mask is not None:
            mk = np.ascontiguousarray(mask, dtype=np.uint8)
            keep.append(mk)
        P_ = model.n_params
        lbv, ubv = _host_f64(lb, P_), _host_f64(ub, P_)
        x0v = None if x0 is None else _host_f64(x0, P_)
        xm = None if x0_map is None else np.ascontiguousarray(x0_map, dtype=np.float32)
        keep += [lbv, ubv, x0v, xm]
        job = gc_job()
        job.model = model.handle
        job.data = gc_volume(nx, ny, nz, y.ctypes.data)
        job.mask = None if mk is None else mk.ctypes.data
        job.bounds = gc_bounds(lbv.ctypes.data, ubv.ctypes.data,
                               None if x0v is None else x0v.ctypes.data,
                               None if xm is None else xm.ctypes.data)
        return job, keep, (nx, ny, nz)

    def submit_mcmc(self, model, y, mask, lb, ub, n_chains, n_iter, burnin, thin, *, sigma,
                    step=None, seed=0, x0=None, x0_map=None, x0_mode="midpoint", weights=None,
                    precision="fp32", sampler="mh", n_walkers=50, stretch=2.0, accept=True):
        job, keep, (nx, ny, nz) = self._common(model, y, mask, lb, ub, x0, x0_map)
        job.kind = 1
        job.n_chains, job.n_iter, job.burnin, job.thin = n_chains, n_iter, burnin, thin
        h = gc_mcmc_hyper()
        _L.gc_mcmc_defaults(ctypes.byref(h))
        h.sigma = sigma
        st = None if step is None else _host_f64(step, model.n_params)
        h.step = None if st is None else st.ctypes.data
        h.seed = int(seed)
        h.x0_mode = {"midpoint": 0, "uniform": 1, "given": 2}[x0_mode]
        if (x0_map is not None or x0 is not None) and x0_mode == "midpoint":
            h.x0_mode = 2
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
        h.weights = None if w is None else w.ctypes.data
        h.precision = {"fp32": 0, "fp64": 1}[precision]
        h.sampler = {"mh": 0, "ensemble": 1}[sampler]
        h.n_walkers, h.stretch = n_walkers, stretch
        job.mcmc = h
        C = n_walkers if sampler == "ensemble" else n_chains
        P_ = model.n_params
        mean = np.zeros((P_, nz, ny, nx))
        std = np.zeros((P_, nz, ny, nx))
        acc = np.zeros((C, nz, ny, nx), np.int32) if accept else None
        job.out_mean, job.out_std = mean.ctypes.data, std.ctypes.data
        job.out_accept = None if acc is None else acc.ctypes.data
        keep += [st, w]
        out = dict(mean=mean, std=std, accept=acc)
        return self._submit(job, keep, out)

    def submit_fit(self, model, y, mask, lb, ub, *, x0=None, x0_map=None, weights=None,
                   optimizer="adam", lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, momentum=0.9,
                   rho=0.9, n_iter=200, loss=2, lam=0.0, tv_params=(), tv_dim=3, tol=0.0,
                   conv_value=0.0, conv_window=20, tv_kind="aniso", graph=None,
                   prior_lam=0.0, prior_params=(), prior_mu=None, prior_sigma=None):
        job, keep, (nx, ny, nz) = self._common(model, y, mask, lb, ub, x0, x0_map)
        job.kind = 0
        h = gc_adam_hyper()
        _L.gc_adam_defaults(ctypes.byref(h))
        h.optimizer = OPTIMIZERS[optimizer]
        h.lr, h.beta1, h.beta2, h.eps, h.momentum, h.rho = lr, beta1, beta2, eps, momentum, rho
        h.n_iter, h.loss = n_iter, loss
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
        h.weights = None if w is None else w.ctypes.data
        h.lambda_ = lam
        h.tv_mask = sum(1 << int(p) for p in tv_params)
        h.tv_dim = tv_dim
        h.tol, h.conv_value, h.conv_window = tol, conv_value, conv_window
        _set_regularisers(h, None, model, tv_kind, graph, prior_lam, prior_params, prior_mu,
                          prior_sigma, keep)
        job.adam = h
        maps = np.zeros((model.n_params, nz, ny, nx), np.float32)
        rep = gc_fit_report()
        job.out_maps = maps.ctypes.data
        job.report = ctypes.addressof(rep)
        keep += [w, rep]
        out = dict(maps=maps, report=rep)
        return self._submit(job, keep, out)

    def _submit(self, job, keep, out):
        jid = c_uint64()
        _check(_L.gc_submit(self.handle, ctypes.byref(job), ctypes.byref(jid)))
        self._jobs[jid.value] = (job, keep, out)
        return jid.value

    def poll(self, jid) -> str:
        if jid in self._done:
            return self._done[jid][0]
        st = c_int()
        _check(_L.gc_poll(self.handle, jid, ctypes.byref(st)))
        return JOB_STATES[st.value]

    def wait(self, jid, timeout_ms=-1):
        """Waits for a job; returns its result dict (raises GcError if it
        failed).  The job is then released: its buffers are no longer held
        and poll() / latency() answer from what was recorded here."""
        st = c_int()
        _check(_L.gc_wait(self.handle, jid, timeout_ms, ctypes.byref(st)))
        _, _, out = self._jobs[jid]
        err = None if st.value == GC_OK else GcError(st.value, last_error())
        state = c_int()
        _check(_L.gc_poll(self.handle, jid, ctypes.byref(state)))
        lat = None
        if st.value == GC_OK:
            s = c_double()
            _check(_L.gc_job_latency(self.handle, jid, ctypes.byref(s)))
            lat = s.value
        _check(_L.gc_release(self.handle, jid))
        self._done[jid] = (JOB_STATES[state.value], lat)
        del self._jobs[jid]
        if err is not None:
            raise err
        r = dict(out)
        if "report" in r:
            rep = r.pop("report")
            r.update(iters_run=rep.iters_run, final_loss=rep.final_loss,
                     stop_reason=rep.stop_reason)
        return r

    def cancel(self, jid):
        _check(_L.gc_cancel(self.handle, jid))

    def latency(self, jid) -> float:
        if jid in self._done:
            if self._done[jid][1] is None:
                raise GcError(-1, "job not finished successfully")
            return self._done[jid][1]
        s = c_double()
        _check(_L.gc_job_latency(self.handle, jid, ctypes.byref(s)))
        return s.value

    def stats(self) -> dict:
        st = gc_stats()
        _check(_L.gc_server_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in gc_stats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _L.gc_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
