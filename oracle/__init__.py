"""CPU oracle for the iterated clamped star stencils -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The HIP library never imports, links or calls it, and it shares
no code with the library.

The arithmetic lives in ``stencil_oracle.c`` (plain loops, FP64 and FP32 instantiations,
see that file's header for the paper passages it follows: Section 2.1 ping-pong
stepping, Table 2 formulas, Section 5.1 clamp-to-edge boundary).  This module only builds
that file with gcc and marshals numpy arrays into it.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py`` (dense
brute-force matrix powers, DCT-II eigenmodes, exact Green's function, conservation,
constant fields, closed-form hotspot recurrence, dimension reduction, dense transpose,
dot-product and exact central-difference checks of the adjoint).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stencil_oracle.c")
_LIB = os.path.join(_HERE, "libstencil_oracle.so")
_LIB_BASE = os.path.join(_HERE, "libstencil_oracle_base.so")
_lock = threading.Lock()
_lib = None

DIFFUSION = 0
HOTSPOT = 1
HOTSPOT_PHYS = 2   # Table 2's Hotspot 2D as printed (2D only)


def _host_has_fma() -> bool:
    """Whether this CPU runs x86-64-v3 code (AVX2 and FMA3)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("flags"):
                    flags = set(line.split(":", 1)[1].split())
                    return {"avx2", "fma"} <= flags
    except OSError:
        pass
    return False


def _lib_path() -> str:
    # Built for x86-64-v3 so that fma()/fmaf() compile to the hardware's fused multiply-add
    # instead of a library call; the result is the same correctly rounded operation either
    # way.  A host without AVX2/FMA gets a baseline build of its own.
    return _LIB if _host_has_fma() else _LIB_BASE


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no FP contraction).  Returns the .so path."""
    lib = _lib_path()
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(_SRC):
        return lib
    tmp = lib + ".tmp%d" % os.getpid()
    arch = ["-march=x86-64-v3"] if lib == _LIB else []
    cmd = ["gcc", "-O2"] + arch + ["-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared",
                                   "-fPIC", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            for suf, ct in (("f64", ctypes.c_double), ("f32", ctypes.c_float)):
                p = ctypes.POINTER(ct)
                fwd = getattr(lib, "oracle_forward_" + suf)
                fwd.restype = ctypes.c_int
                fwd.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_float), p, p, ctypes.c_int]
                adj = getattr(lib, "oracle_adjoint_" + suf)
                adj.restype = ctypes.c_int
                adj.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_float), p, ctypes.c_int, p, p]
                st = getattr(lib, "oracle_star2d_" + suf)
                st.restype = ctypes.c_int
                st.argtypes = [ctypes.c_int] * 3 + [ctypes.POINTER(ctypes.c_float), p, ctypes.c_int]
                st3 = getattr(lib, "oracle_star3d_" + suf)
                st3.restype = ctypes.c_int
                st3.argtypes = [ctypes.c_int] * 4 + [ctypes.POINTER(ctypes.c_float), p, ctypes.c_int]
                fp = ctypes.POINTER(ctypes.c_float)
                ss = getattr(lib, "oracle_star2d_src_" + suf)
                ss.restype = ctypes.c_int
                ss.argtypes = [ctypes.c_int] * 3 + [fp, fp, p, p, ctypes.c_int]
                ss3 = getattr(lib, "oracle_star3d_src_" + suf)
                ss3.restype = ctypes.c_int
                ss3.argtypes = [ctypes.c_int] * 4 + [fp, fp, p, p, ctypes.c_int]
                sa = getattr(lib, "oracle_star_adjoint_" + suf)
                sa.restype = ctypes.c_int
                sa.argtypes = [ctypes.c_int] * 5 + [fp, ctypes.c_float, p, ctypes.c_int, p]
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _dims(shape):
    if len(shape) == 2:
        return 2, shape[1], shape[0], 1
    if len(shape) == 3:
        return 3, shape[2], shape[1], shape[0]
    raise ValueError("grid must be 2D (ny, nx) or 3D (nz, ny, nx)")


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _prep(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype).copy()


def forward(x0, coeffs, T, power=None, form=None, dtype=np.float64):
    """T clamped Jacobi steps of the diffusion (power None) or hotspot stencil.

    ``x0`` has shape (ny, nx) or (nz, ny, nx); ``coeffs`` is the 10-vector
    [cc, cw, ce, cn, cs, cb, ca, cp, c_amb, t_amb] (FP32 values; the FP64 run promotes
    them exactly).  For ``form=HOTSPOT_PHYS`` (2D) the vector carries sdc in cp, Rx_1 in
    ce, Ry_1 in cs, Rz_1 in c_amb and TEMP_AMB in t_amb.  Returns a new array of
    ``dtype`` (float64 or float32).
    """
    lib = _load()
    dtype = np.dtype(dtype)
    ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
    fn = lib.oracle_forward_f64 if dtype == np.float64 else lib.oracle_forward_f32
    if form is None:
        form = HOTSPOT if power is not None else DIFFUSION
    g = _prep(x0, dtype)
    ndim, nx, ny, nz = _dims(g.shape)
    cf = np.ascontiguousarray(coeffs, dtype=np.float32)
    p = None
    if form in (HOTSPOT, HOTSPOT_PHYS):
        if power is None:
            raise ValueError("hotspot needs a power map")
        p = _prep(power, dtype)
        if p.shape != g.shape:
            raise ValueError("power must match the grid shape")
    rc = fn(form, ndim, nx, ny, nz, _ptr(cf, ctypes.c_float), _ptr(g, ct),
            _ptr(p, ct) if p is not None else None, int(T))
    if rc != 0:
        raise ValueError("oracle_forward rejected its arguments")
    return g


def adjoint(cot, coeffs, T, form=DIFFUSION, dtype=np.float64, want_grad_p=None):
    """Vector-Jacobian product of ``forward`` w.r.t. the initial field and the power map.

    ``cot`` = dJ/dx_T.  Returns (grad_x0, grad_p); grad_p is None for diffusion.
    """
    lib = _load()
    dtype = np.dtype(dtype)
    ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
    fn = lib.oracle_adjoint_f64 if dtype == np.float64 else lib.oracle_adjoint_f32
    c = _prep(cot, dtype)
    ndim, nx, ny, nz = _dims(c.shape)
    cf = np.ascontiguousarray(coeffs, dtype=np.float32)
    gx = np.empty_like(c)
    if want_grad_p is None:
        want_grad_p = form != DIFFUSION
    gp = np.empty_like(c) if want_grad_p else None
    rc = fn(form, ndim, nx, ny, nz, _ptr(cf, ctypes.c_float), _ptr(c, ct), int(T), _ptr(gx, ct),
            _ptr(gp, ct) if gp is not None else None)
    if rc != 0:
        raise ValueError("oracle_adjoint rejected its arguments")
    return gx, gp


def _star_source(power, src, shape, dtype):
    """The hotspot-form arguments of the radius-r oracles: the power map in the working
    precision and src = (cp, c_amb, t_amb) as FP32 values, or (None, None)."""
    if power is None:
        return None, None
    if src is None or len(src) != 3:
        raise ValueError("the hotspot form needs src = (cp, c_amb, t_amb)")
    pw = _prep(power, dtype)
    if pw.shape != tuple(shape):
        raise ValueError("power must have the grid's shape")
    return pw, np.ascontiguousarray(src, dtype=np.float32)


def star2d(x0, weights, T, dtype=np.float64, power=None, src=None):
    """T clamped Jacobi steps of the radius-r 2D star stencil on ``x0`` of shape (ny, nx).
    ``weights`` has 1 + 4r entries: cc, then w_d, e_d for d = 1..r, then s_1..s_r, then
    n_1..n_r (FP32 values; the FP64 run promotes them exactly).  Diffusion form by default; with
    ``power`` (same shape) and ``src`` = (cp, c_amb, t_amb) the hotspot form, whose chain starts
    from fma(cc, c, q) with q = fma(cp, p, c_amb*t_amb) as for radius 1."""
    lib = _load()
    dtype = np.dtype(dtype)
    ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
    g = _prep(x0, dtype)
    if g.ndim != 2:
        raise ValueError("the radius-r stencil is 2D: shape (ny, nx)")
    w = np.ascontiguousarray(weights, dtype=np.float32)
    if w.size < 5 or (w.size - 1) % 4:
        raise ValueError("weights must have 1 + 4r entries")
    rad = (w.size - 1) // 4
    pw, sv = _star_source(power, src, g.shape, dtype)
    if pw is None:
        fn = lib.oracle_star2d_f64 if dtype == np.float64 else lib.oracle_star2d_f32
        rc = fn(rad, g.shape[1], g.shape[0], _ptr(w, ctypes.c_float), _ptr(g, ct), int(T))
    else:
        fn = lib.oracle_star2d_src_f64 if dtype == np.float64 else lib.oracle_star2d_src_f32
        rc = fn(rad, g.shape[1], g.shape[0], _ptr(w, ctypes.c_float), _ptr(sv, ctypes.c_float), _ptr(pw, ct),
                _ptr(g, ct), int(T))
    if rc != 0:
        raise ValueError("oracle_star2d rejected its arguments")
    return g


def star3d(x0, weights, T, dtype=np.float64, power=None, src=None):
    """T clamped Jacobi steps of the radius-r 3D star stencil on ``x0`` of shape (nz, ny, nx).
    ``weights`` has 1 + 6r entries: cc, then w_d, e_d for d = 1..r, then s_1..s_r (y+d),
    n_1..n_r (y-d), b_1..b_r (z-d), a_1..a_r (z+d) (FP32 values; the FP64 run promotes them
    exactly).  ``power`` and ``src`` as for star2d."""
    lib = _load()
    dtype = np.dtype(dtype)
    ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
    g = _prep(x0, dtype)
    if g.ndim != 3:
        raise ValueError("the 3D radius-r stencil takes (nz, ny, nx) grids")
    w = np.ascontiguousarray(weights, dtype=np.float32)
    if w.size < 7 or (w.size - 1) % 6:
        raise ValueError("weights must have 1 + 6r entries")
    rad = (w.size - 1) // 6
    pw, sv = _star_source(power, src, g.shape, dtype)
    if pw is None:
        fn = lib.oracle_star3d_f64 if dtype == np.float64 else lib.oracle_star3d_f32
        rc = fn(rad, g.shape[2], g.shape[1], g.shape[0], _ptr(w, ctypes.c_float), _ptr(g, ct), int(T))
    else:
        fn = lib.oracle_star3d_src_f64 if dtype == np.float64 else lib.oracle_star3d_src_f32
        rc = fn(rad, g.shape[2], g.shape[1], g.shape[0], _ptr(w, ctypes.c_float), _ptr(sv, ctypes.c_float),
                _ptr(pw, ct), _ptr(g, ct), int(T))
    if rc != 0:
        raise ValueError("oracle_star3d rejected its arguments")
    return g


def star_adjoint(cotangent, weights, T, cp=None, dtype=np.float64):
    """Adjoint of T steps of the radius-r star stencil (2D or 3D by the cotangent's shape;
    weights as for star2d / star3d).  Returns (grad_x0, grad_p), grad_p = cp * sum_{t=1..T}
    lambda_t when cp is given (the hotspot form), else None."""
    lib = _load()
    dtype = np.dtype(dtype)
    ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
    lam = _prep(cotangent, dtype)
    ndim = lam.ndim
    if ndim not in (2, 3):
        raise ValueError("cotangent must be (ny, nx) or (nz, ny, nx)")
    w = np.ascontiguousarray(weights, dtype=np.float32)
    per = 4 if ndim == 2 else 6
    if w.size < 1 + per or (w.size - 1) % per:
        raise ValueError("weights must have 1 + %dr entries" % per)
    rad = (w.size - 1) // per
    nz, ny, nx = (1,) + lam.shape if ndim == 2 else lam.shape
    gp = np.zeros(lam.shape, dtype) if cp is not None else None
    fn = lib.oracle_star_adjoint_f64 if dtype == np.float64 else lib.oracle_star_adjoint_f32
    rc = fn(ndim, rad, nx, ny, nz, _ptr(w, ctypes.c_float), float(cp or 0.0), _ptr(lam, ct), int(T),
            _ptr(gp, ct) if gp is not None else None)
    if rc != 0:
        raise ValueError("oracle_star_adjoint rejected its arguments")
    return lam, gp


def loss(xT, target) -> float:
    """L2 misfit J = 1/2 * sum (x_T - y)^2, accumulated in FP64."""
    d = np.asarray(xT, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return 0.5 * float(np.dot(d.ravel(), d.ravel()))
