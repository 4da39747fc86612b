"""Python binding of the MI355X temporal-blocked stencil library (C ABI of include/stencil.h).

Argument marshalling only: every step of the computation runs in the HIP kernels of
``libstencil_mi355.so``.  PyTorch supplies device memory (tensor data pointers) and the current
HIP stream.  If the shared library is missing, every call raises; there is no fallback.

Names follow the C ABI (``stencil_create``, ``stencil_run``, ``stencil_run_ckpt``,
``stencil_adjoint``, ``stencil_run_batched``, ...).  ``Plan``, ``run``, ``adjoint``,
``StencilFn`` and ``run_batched`` are thin conveniences over them.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstencil_mi355.so")

DIFFUSION = 0
HOTSPOT = 1
HOTSPOT_PHYS = 2   # Table 2's Hotspot 2D formula as printed (2D, forward only)

STENCIL_OK = 0
STATUS = {0: "STENCIL_OK", -1: "STENCIL_ERR_INVALID_ARG", -2: "STENCIL_ERR_UNSUPPORTED",
          -3: "STENCIL_ERR_OUT_OF_MEMORY", -4: "STENCIL_ERR_HIP", -5: "STENCIL_ERR_INTERNAL"}

EXPORTED = ("stencil_create", "stencil_run", "stencil_run_ckpt", "stencil_adjoint", "stencil_run_batched",
            "stencil_batch_destroy", "stencil_get_tuning", "stencil_destroy", "stencil_status_string",
            "stencil_last_error", "stencil_model_estimate", "stencil_plan_model", "stencil_create_star",
            "stencil_run_star", "stencil_batch_sync", "stencil_run_batched_noalloc",
            "stencil_run_slab", "stencil_get_adjoint_tuning", "stencil_run_star_hotspot", "stencil_adjoint_star")


class StencilError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class Coeffs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("cc", "cw", "ce", "cn", "cs", "cb", "ca", "cp", "c_amb", "t_amb")]


class Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("variant", "k", "vec", "bsize_x", "bsize_y", "seg_len", "nwork")]


class BatchItem(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int), ("ndim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("grid", ctypes.c_void_p), ("power", ctypes.c_void_p),
                ("coeffs", Coeffs), ("T", ctypes.c_int)]


class ModelParams(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("rad", ctypes.c_int), ("par_vec", ctypes.c_int), ("par_time", ctypes.c_int),
                ("f_max_hz", ctypes.c_double), ("size_cell", ctypes.c_int), ("num_read", ctypes.c_int),
                ("num_write", ctypes.c_int), ("bsize_x", ctypes.c_int), ("bsize_y", ctypes.c_int),
                ("dim_x", ctypes.c_long), ("dim_y", ctypes.c_long), ("dim_z", ctypes.c_long), ("iter", ctypes.c_long),
                ("th_max_gbs", ctypes.c_double)]


class ModelResult(ctypes.Structure):
    _fields_ = [("th_mem_gbs", ctypes.c_double), ("csize_x", ctypes.c_long), ("csize_y", ctypes.c_long),
                ("bnum_x", ctypes.c_long), ("bnum_y", ctypes.c_long), ("t_cell", ctypes.c_double),
                ("t_read", ctypes.c_double), ("t_write", ctypes.c_double), ("run_time_s", ctypes.c_double),
                ("throughput_gbs", ctypes.c_double)]


class PlanModel(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("mem_seconds", ctypes.c_double), ("alu_seconds", ctypes.c_double),
                ("passes", ctypes.c_long)]


_lock = threading.Lock()
_lib = None


def library_path() -> str:
    return LIB_PATH


def lib():
    """The loaded ctypes library.  Raises if libstencil_mi355.so has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libstencil_mi355.so is not built (run __graft_entry__.build() or "
                                  "python paper_1802_00438_amd/build.py)")
            L = ctypes.CDLL(LIB_PATH)
            vp, i, f = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_float)
            L.stencil_create.argtypes = [ctypes.POINTER(vp), i, i, i, i, i, ctypes.POINTER(Tuning), vp]
            L.stencil_run.argtypes = [vp, vp, vp, ctypes.POINTER(Coeffs), i]
            L.stencil_run_ckpt.argtypes = [vp, vp, vp, ctypes.POINTER(Coeffs), i, i]
            L.stencil_adjoint.argtypes = [vp, vp, vp, ctypes.POINTER(Coeffs), i, vp, vp, i]
            L.stencil_run_slab.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Coeffs), i, i, i]
            L.stencil_run_batched.argtypes = [i, ctypes.POINTER(BatchItem), vp, ctypes.POINTER(vp)]
            L.stencil_batch_sync.argtypes = [vp]
            L.stencil_run_batched_noalloc.argtypes = [i, ctypes.POINTER(BatchItem), ctypes.POINTER(vp), vp]
            L.stencil_batch_destroy.argtypes = [vp]
            L.stencil_batch_destroy.restype = None
            L.stencil_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
            L.stencil_get_adjoint_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
            L.stencil_destroy.argtypes = [vp]
            L.stencil_destroy.restype = None
            L.stencil_status_string.argtypes = [i]
            L.stencil_status_string.restype = ctypes.c_char_p
            L.stencil_last_error.argtypes = []
            L.stencil_last_error.restype = ctypes.c_char_p
            L.stencil_model_estimate.argtypes = [ctypes.POINTER(ModelParams), ctypes.POINTER(ModelResult)]
            L.stencil_plan_model.argtypes = [vp, i, ctypes.POINTER(PlanModel)]
            L.stencil_create_star.argtypes = [ctypes.POINTER(vp), i, i, i, i, i, ctypes.POINTER(Tuning), vp]
            L.stencil_run_star.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float), i]
            L.stencil_run_star_hotspot.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_float),
                                                   ctypes.POINTER(ctypes.c_float), i]
            L.stencil_adjoint_star.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                               i, vp, vp]
            for name in ("stencil_create", "stencil_run", "stencil_run_ckpt", "stencil_adjoint",
                         "stencil_run_batched", "stencil_get_tuning", "stencil_model_estimate",
                         "stencil_plan_model", "stencil_create_star", "stencil_run_star", "stencil_batch_sync",
                         "stencil_run_batched_noalloc", "stencil_run_slab", "stencil_get_adjoint_tuning",
                         "stencil_run_star_hotspot", "stencil_adjoint_star"):
                getattr(L, name).restype = i
            _lib = L
    return _lib


def _check(status: int):
    if status != STENCIL_OK:
        msg = lib().stencil_last_error().decode(errors="replace")
        raise StencilError(status, msg)


def make_coeffs(c) -> Coeffs:
    """From a 10-vector [cc, cw, ce, cn, cs, cb, ca, cp, c_amb, t_amb], a dict or a Coeffs."""
    if isinstance(c, Coeffs):
        return c
    if isinstance(c, dict):
        return Coeffs(**{k: float(v) for k, v in c.items()})
    vals = [float(v) for v in c]
    vals += [0.0] * (10 - len(vals))
    return Coeffs(*vals[:10])


def make_tuning(t) -> Tuning | None:
    if t is None:
        return None
    if isinstance(t, Tuning):
        return t
    return Tuning(**{k: int(v) for k, v in t.items()})


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


# ------------------------------------------------------------------ C ABI, same names

def stencil_create(form, ndim, nx, ny, nz, tuning=None, stream=None):
    h = ctypes.c_void_p()
    t = make_tuning(tuning)
    _check(lib().stencil_create(ctypes.byref(h), int(form), int(ndim), int(nx), int(ny), int(nz),
                                ctypes.byref(t) if t is not None else None, _stream(stream)))
    return h


def stencil_create_star(ndim, rad, nx, ny, nz, tuning=None, stream=None):
    h = ctypes.c_void_p()
    t = make_tuning(tuning)
    _check(lib().stencil_create_star(ctypes.byref(h), int(ndim), int(rad), int(nx), int(ny), int(nz),
                                     ctypes.byref(t) if t is not None else None, _stream(stream)))
    return h


def stencil_run_star(plan, grid, weights, T):
    import numpy as np
    w = np.ascontiguousarray(weights, dtype=np.float32)
    _check(lib().stencil_run_star(plan, _ptr(grid), w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(T)))


def stencil_adjoint_star(plan, cotangent, weights, src, T, grad_x0, grad_power):
    import numpy as np
    w = np.ascontiguousarray(weights, dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    sv = None if src is None else np.ascontiguousarray(src, dtype=np.float32)
    if sv is not None and sv.size != 3:
        raise ValueError("src must be (cp, c_amb, t_amb)")
    _check(lib().stencil_adjoint_star(plan, _ptr(cotangent), w.ctypes.data_as(fp),
                                      sv.ctypes.data_as(fp) if sv is not None else None, int(T), _ptr(grad_x0),
                                      _ptr(grad_power) if grad_power is not None else None))


def stencil_run_star_hotspot(plan, grid, power, weights, src, T):
    import numpy as np
    w = np.ascontiguousarray(weights, dtype=np.float32)
    sv = np.ascontiguousarray(src, dtype=np.float32)
    if sv.size != 3:
        raise ValueError("src must be (cp, c_amb, t_amb)")
    fp = ctypes.POINTER(ctypes.c_float)
    _check(lib().stencil_run_star_hotspot(plan, _ptr(grid), _ptr(power), w.ctypes.data_as(fp), sv.ctypes.data_as(fp),
                                          int(T)))


def stencil_run(plan, grid, power, coeffs, T):
    c = make_coeffs(coeffs)
    _check(lib().stencil_run(plan, _ptr(grid), _ptr(power), ctypes.byref(c), int(T)))


def stencil_run_ckpt(plan, grid, power, coeffs, T, ckpt_every=0):
    c = make_coeffs(coeffs)
    _check(lib().stencil_run_ckpt(plan, _ptr(grid), _ptr(power), ctypes.byref(c), int(T), int(ckpt_every)))


def stencil_run_slab(plan, src, dst, power, coeffs, T, ghost_lo, ghost_hi):
    c = make_coeffs(coeffs)
    _check(lib().stencil_run_slab(plan, _ptr(src), _ptr(dst), _ptr(power), ctypes.byref(c), int(T), int(ghost_lo),
                                  int(ghost_hi)))


def stencil_adjoint(plan, cotangent, power, coeffs, T, grad_x0, grad_power=None, recompute=0):
    c = make_coeffs(coeffs)
    _check(lib().stencil_adjoint(plan, _ptr(cotangent), _ptr(power), ctypes.byref(c), int(T), _ptr(grad_x0),
                                 _ptr(grad_power), int(recompute)))


def stencil_run_batched(items, stream=None, cache=None):
    """items: sequence of BatchItem.  cache: None, or a ctypes.c_void_p holder (build-and-keep /
    replay).  Returns the cache holder."""
    arr = (BatchItem * len(items))(*items)
    _check(lib().stencil_run_batched(len(items), arr, _stream(stream),
                                     ctypes.byref(cache) if cache is not None else None))
    return cache


def stencil_batch_sync(cache):
    """Wait for the latest replay of a captured batch; raises if a dependency wait failed."""
    _check(lib().stencil_batch_sync(cache))


def stencil_run_batched_noalloc(items, partners, stream=None):
    """items: sequence of BatchItem; partners: device pointers (ints), one ping-pong partner
    buffer per item, of the item's size.  Synchronous; allocates no device memory."""
    arr = (BatchItem * len(items))(*items)
    parr = (ctypes.c_void_p * len(items))(*[int(p) for p in partners])
    _check(lib().stencil_run_batched_noalloc(len(items), arr, parr, _stream(stream)))


def stencil_batch_destroy(cache):
    if cache is not None and cache.value:
        lib().stencil_batch_destroy(cache)
        cache.value = None


def stencil_get_tuning(plan) -> dict:
    t = Tuning()
    _check(lib().stencil_get_tuning(plan, ctypes.byref(t)))
    return {k: getattr(t, k) for k, _ in Tuning._fields_}


def stencil_get_adjoint_tuning(plan) -> dict:
    t = Tuning()
    _check(lib().stencil_get_adjoint_tuning(plan, ctypes.byref(t)))
    return {k: getattr(t, k) for k, _ in Tuning._fields_}


def stencil_plan_model(plan, T) -> dict:
    """The library's time model of T steps on the plan's resolved blocking."""
    m = PlanModel()
    _check(lib().stencil_plan_model(plan, int(T), ctypes.byref(m)))
    return {k: getattr(m, k) for k, _ in PlanModel._fields_}


def stencil_destroy(plan):
    lib().stencil_destroy(plan)


def stencil_status_string(status: int) -> str:
    return lib().stencil_status_string(int(status)).decode()


def stencil_last_error() -> str:
    return lib().stencil_last_error().decode(errors="replace")


def stencil_model_estimate(**kw) -> dict:
    p = ModelParams(**kw)
    r = ModelResult()
    _check(lib().stencil_model_estimate(ctypes.byref(p), ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in ModelResult._fields_}


# ------------------------------------------------------------------ conveniences

def _dims(x):
    if x.dim() == 2:
        return 2, x.shape[1], x.shape[0], 1
    if x.dim() == 3:
        return 3, x.shape[2], x.shape[1], x.shape[0]
    raise ValueError("grid must be (ny, nx) or (nz, ny, nx)")


def _check_tensor(x, name, shape=None, device=None):
    """Reject what the kernels cannot take: anything but a contiguous float32 device tensor, a
    tensor whose shape differs from the plan's (the kernels would read or write past it) and a
    tensor on another device than the plan's."""
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("%s must be a contiguous float32 CUDA/HIP tensor" % name)
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError("%s has shape %s, the plan was made for %s" % (name, tuple(x.shape), tuple(shape)))
    if device is not None and x.device.index != device:
        raise ValueError("%s is on cuda:%s, the plan on cuda:%d" % (name, x.device.index, device))


def _current_device():
    import torch
    return torch.cuda.current_device()


class Plan:
    """A plan for one grid shape: owns the ping-pong scratch and checkpoints."""

    def __init__(self, form, shape, tuning=None, stream=None):
        self.form = int(form)
        self.shape = tuple(int(s) for s in shape)
        if len(self.shape) == 2:
            ndim, nx, ny, nz = 2, self.shape[1], self.shape[0], 1
        else:
            ndim, nx, ny, nz = 3, self.shape[2], self.shape[1], self.shape[0]
        self.ndim = ndim
        self.device = _current_device()
        self.handle = None
        self.handle = stencil_create(self.form, ndim, nx, ny, nz, tuning, stream)

    def _check(self, t, name):
        _check_tensor(t, name, self.shape, self.device)

    def _check_power(self, power):
        if power is not None:
            self._check(power, "power")
        elif self.form != DIFFUSION:
            raise ValueError("the hotspot forms need a power map")

    def run(self, grid, coeffs, T, power=None):
        self._check(grid, "grid")
        self._check_power(power)
        stencil_run(self.handle, grid, power, coeffs, T)
        return grid

    def run_ckpt(self, grid, coeffs, T, ckpt_every=0, power=None):
        self._check(grid, "grid")
        self._check_power(power)
        stencil_run_ckpt(self.handle, grid, power, coeffs, T, ckpt_every)
        return grid

    def run_slab(self, src, dst, coeffs, T, ghost_lo, ghost_hi, power=None):
        """One pass of T fused steps over a slab with ghost planes (rows in 2D): reads src, writes
        the interior [ghost_lo, n - ghost_hi) of dst along the slowest axis."""
        self._check(src, "src")
        self._check(dst, "dst")
        self._check_power(power)
        stencil_run_slab(self.handle, src, dst, power, coeffs, T, ghost_lo, ghost_hi)
        return dst

    def adjoint(self, cotangent, coeffs, T, grad_x0, grad_power=None, power=None, recompute=0):
        self._check(cotangent, "cotangent")
        self._check(grad_x0, "grad_x0")
        if grad_power is not None:
            self._check(grad_power, "grad_power")
        if power is not None:
            self._check(power, "power")
        elif recompute and self.form != DIFFUSION:
            raise ValueError("recompute of a hotspot form needs the power map")
        stencil_adjoint(self.handle, cotangent, power, coeffs, T, grad_x0, grad_power, recompute)
        return grad_x0, grad_power

    @property
    def tuning(self):
        return stencil_get_tuning(self.handle)

    @property
    def adjoint_tuning(self):
        return stencil_get_adjoint_tuning(self.handle)

    def model(self, T):
        return stencil_plan_model(self.handle, T)

    def close(self):
        if self.handle is not None and self.handle.value:
            stencil_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StarPlan:
    """A plan for the radius-r star stencil of a (ny, nx) or (nz, ny, nx) grid
    (stencil_create_star)."""

    def __init__(self, rad, shape, tuning=None, stream=None):
        if len(shape) not in (2, 3):
            raise ValueError("the radius-r star stencil takes (ny, nx) or (nz, ny, nx) grids")
        self.rad = int(rad)
        self.shape = tuple(int(v) for v in shape)
        self.ndim = len(self.shape)
        self.device = _current_device()
        self.handle = None
        nz = self.shape[0] if self.ndim == 3 else 1
        self.handle = stencil_create_star(self.ndim, self.rad, self.shape[-1], self.shape[-2], nz, tuning, stream)

    @property
    def n_weights(self):
        return 1 + (6 if self.ndim == 3 else 4) * self.rad

    def adjoint(self, cotangent, weights, T, grad_x0, grad_power=None, src=None):
        """dJ/dx_0 of T steps into grad_x0 from cotangent = dJ/dx_T; with grad_power and src =
        (cp, c_amb, t_amb) (the hotspot form) also dJ/dp = cp * sum_t lambda_t into grad_power."""
        _check_tensor(cotangent, "cotangent", self.shape, self.device)
        _check_tensor(grad_x0, "grad_x0", self.shape, self.device)
        if grad_power is not None:
            _check_tensor(grad_power, "grad_power", self.shape, self.device)
            if src is None or len(src) != 3:
                raise ValueError("grad_power needs src = (cp, c_amb, t_amb)")
        if len(weights) != self.n_weights:
            raise ValueError("weights must have 1 + %d*rad entries" % (6 if self.ndim == 3 else 4))
        stencil_adjoint_star(self.handle, cotangent, weights, src, T, grad_x0, grad_power)
        return grad_x0, grad_power

    def run(self, grid, weights, T, power=None, src=None):
        """weights: cc; w_d, e_d (d = 1..rad); s_1..s_rad; n_1..n_rad; in 3D then b_1..b_rad
        (z-d) and a_1..a_rad (z+d): 1 + 4*rad values in 2D, 1 + 6*rad in 3D.  With power (a
        device tensor of the grid's shape) and src = (cp, c_amb, t_amb): the hotspot form."""
        _check_tensor(grid, "grid", self.shape, self.device)
        if len(weights) != self.n_weights:
            raise ValueError("weights must have 1 + %d*rad entries" % (6 if self.ndim == 3 else 4))
        if power is None:
            if src is not None:
                raise ValueError("src without power")
            stencil_run_star(self.handle, grid, weights, T)
        else:
            _check_tensor(power, "power", self.shape, self.device)
            if src is None or len(src) != 3:
                raise ValueError("the hotspot form needs src = (cp, c_amb, t_amb)")
            stencil_run_star_hotspot(self.handle, grid, power, weights, src, T)
        return grid

    @property
    def tuning(self):
        return stencil_get_tuning(self.handle)

    def model(self, T):
        return stencil_plan_model(self.handle, T)

    def close(self):
        if self.handle is not None and self.handle.value:
            stencil_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(x, coeffs, T, power=None, tuning=None, form=None):
    """T steps in place on x (float32 device tensor, (ny, nx) or (nz, ny, nx)).  form defaults
    to HOTSPOT when power is given, else DIFFUSION."""
    _check_tensor(x, "x")
    if form is None:
        form = HOTSPOT if power is not None else DIFFUSION
    p = Plan(form, x.shape, tuning)
    try:
        p.run(x, coeffs, T, power)
    finally:
        p.close()
    return x


class _PlanPool:
    """Plans kept for reuse by StencilFn, per (form, shape, tuning, device).  A plan is taken
    for one forward and comes back when that forward's autograd node is released, so two
    live graphs never share a plan (each plan holds the checkpoints of its own forward)."""

    def __init__(self):
        self._free = {}
        self._mu = threading.Lock()

    def take(self, form, shape, tuning):
        key = (int(form), tuple(int(s) for s in shape), None if tuning is None else tuple(sorted(tuning.items())),
               _current_device())
        with self._mu:
            lst = self._free.get(key)
            if lst:
                return key, lst.pop()
        return key, Plan(form, shape, tuning)

    def give(self, key, plan):
        with self._mu:
            self._free.setdefault(key, []).append(plan)

    def clear(self):
        with self._mu:
            plans = [p for lst in self._free.values() for p in lst]
            self._free.clear()
        for p in plans:
            p.close()


_plan_pool = _PlanPool()


class _PlanLease:
    """Holds a pooled plan for the lifetime of one autograd node."""

    def __init__(self, key, plan):
        self.key, self.plan = key, plan

    def __del__(self):
        try:
            _plan_pool.give(self.key, self.plan)
        except Exception:
            pass


def _stencil_fn():
    import torch

    class StencilFn(torch.autograd.Function):
        """x_T = T steps of the stencil applied to x0 (hotspot when power is given; form may
        name HOTSPOT_PHYS for Table 2's physical Hotspot 2D formula).

        backward returns dJ/dx0 and dJ/dpower from the library's adjoint kernels; forward keeps
        checkpoints every ckpt_every steps (0 = sqrt(T)), and recompute=1 re-runs and checks them
        during backward.  The plan (scratch and checkpoints) stays with the autograd node until
        the node is released, so backward may run more than once (retain_graph=True); plans
        are then reused by later forwards of the same shape."""

        @staticmethod
        def forward(ctx, x0, power, coeffs, T, ckpt_every=0, recompute=0, tuning=None, form=None):
            if form is None:
                form = HOTSPOT if power is not None else DIFFUSION
            key, plan = _plan_pool.take(form, x0.shape, tuning)
            lease = _PlanLease(key, plan)
            x = x0.detach().clone()
            plan.run_ckpt(x, coeffs, T, ckpt_every, power)
            ctx.lease = lease
            ctx.coeffs = coeffs
            ctx.T = T
            ctx.recompute = recompute
            ctx.has_power = power is not None
            ctx.save_for_backward(power if power is not None else torch.empty(0, device=x0.device))
            return x

        @staticmethod
        def backward(ctx, g):
            (power,) = ctx.saved_tensors
            g = g.contiguous()
            gx = torch.empty_like(g)
            gp = torch.empty_like(g) if ctx.has_power else None
            ctx.lease.plan.adjoint(g, ctx.coeffs, ctx.T, gx, gp, power if ctx.has_power else None, ctx.recompute)
            return gx, gp, None, None, None, None, None, None

    return StencilFn


_fn_cache = {}


def __getattr__(name):
    if name == "StencilFn":
        if "fn" not in _fn_cache:
            _fn_cache["fn"] = _stencil_fn()
        return _fn_cache["fn"]
    raise AttributeError(name)


def _batch_items(grids, coeffs_list, steps):
    items = []
    for x, c, T in zip(grids, coeffs_list, steps):
        _check_tensor(x, "grid")
        ndim, nx, ny, nz = _dims(x)
        items.append(BatchItem(DIFFUSION, ndim, nx, ny, nz, x.data_ptr(), None, make_coeffs(c), int(T)))
    return items


def run_batched_noalloc(grids, coeffs_list, steps, partners, stream=None):
    """As run_batched without a cache, through the entry point that allocates nothing:
    partners[i] is a device tensor of grids[i]'s shape and device (its contents are
    overwritten)."""
    if len(partners) != len(grids):
        raise ValueError("one partner buffer per grid")
    for x, q in zip(grids, partners):
        _check_tensor(q, "partner", tuple(x.shape), x.device.index)
    items = _batch_items(grids, coeffs_list, steps)
    stencil_run_batched_noalloc(items, [q.data_ptr() for q in partners], stream)


def run_batched(grids, coeffs_list, steps, stream=None, cache=None):
    """Run grids[i] (device tensors, 2D or 3D, diffusion) for steps[i] steps each, in one
    persistent launch captured in a HIP graph.  Pass the returned cache back to replay."""
    items = _batch_items(grids, coeffs_list, steps)
    if cache is None:
        cache = ctypes.c_void_p()
    return stencil_run_batched(items, stream, cache)
