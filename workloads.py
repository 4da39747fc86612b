"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module holds no stencil arithmetic: only shapes, coefficient sets, seeds and
random draws.  Both the CPU oracle (``oracle/``) and the HIP library take their
inputs from here, so the two sides never share anything that computes the method.

Recipe (all arrays FP32, row-major, x fastest: index = (z*ny + y)*nx + x):

* A uniform draw U[a, b) is ``a + (b - a) * u`` evaluated in FP32, where ``u`` comes
  from ``numpy.random.Generator(PCG64(seed)).random(n, dtype=float32)``.
* Workload *i* (1-based, in the order listed in ``WORKLOADS``) uses seed ``1000*i``
  for the initial field, ``+1`` for the power map, ``+2`` for the target field and
  ``+3`` for the batch-size draw.

The paper's benchmarks (Section 5.1, Table 2) are Diffusion 2D/3D and Rodinia's
Hotspot 2D/3D on square/cubic grids of at least 1 GB, run for many iterations
(Section 5.2).  Rodinia's own temperature/power files are not used; the uniform
fields below stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DIFFUSION = 0
HOTSPOT = 1
HOTSPOT_PHYS = 2   # Table 2's Hotspot 2D as printed (sdc, Rx_1, Ry_1, Rz_1, TEMP_AMB)

# Coefficient vector layout used everywhere (oracle and library binding):
#   [cc, cw, ce, cn, cs, cb, ca, cp, c_amb, t_amb]
# Direction convention: w = x-1, e = x+1, n = y-1, s = y+1, b = z-1, a = z+1.
COEF_NAMES = ("cc", "cw", "ce", "cn", "cs", "cb", "ca", "cp", "c_amb", "t_amb")


def coeffs(cc, cw, ce, cn, cs, cb=0.0, ca=0.0, cp=0.0, c_amb=0.0, t_amb=0.0):
    """Pack a coefficient set as a float32 vector in the canonical layout."""
    return np.array([cc, cw, ce, cn, cs, cb, ca, cp, c_amb, t_amb], dtype=np.float32)


def phys_coeffs(sdc, rx, ry, rz, t_amb):
    """Pack the parameters of the physical Hotspot 2D form (Table 2) in the canonical layout:
    sdc in cp, Rx_1 in ce, Ry_1 in cs, Rz_1 in c_amb, TEMP_AMB in t_amb."""
    return np.array([0.0, 0.0, rx, 0.0, ry, 0.0, 0.0, sdc, rz, t_amb], dtype=np.float32)


# Coefficient sets.  D2/D3 are the diffusion weights of the workloads; the hotspot sets
# are dyadic (exact in FP32) with weights summing to exactly 1; A2/A3 are deliberately
# asymmetric so orientation and transpose mistakes show up.
SETS = {
    "D2": coeffs(0.5, 0.125, 0.125, 0.125, 0.125),
    "D3": coeffs(0.4, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1),
    "H2": coeffs(0.5 - 2.0 ** -10, 0.125, 0.125, 0.125, 0.125, cp=64.0, c_amb=2.0 ** -10, t_amb=80.0),
    "H3": coeffs(0.375 - 2.0 ** -10, 0.125, 0.125, 0.125, 0.125, 0.0625, 0.0625,
                 cp=64.0, c_amb=2.0 ** -10, t_amb=80.0),
    # Table-2-faithful hotspot 3D ambient term: ambient coupling equals c_a.
    "H3p": coeffs(0.3125, 0.125, 0.125, 0.125, 0.125, 0.0625, 0.0625, cp=64.0, c_amb=0.0625, t_amb=80.0),
    "A2": coeffs(0.375, 0.0625, 0.1875, 0.125, 0.25),
    "A3": coeffs(0.25, 0.0625, 0.1875, 0.125, 0.1875, 0.0625, 0.125),
    # asymmetric hotspot sets (for adjoint / orientation tests of the affine form)
    "AH2": coeffs(0.375, 0.0625, 0.1875, 0.125, 0.25, cp=8.0, c_amb=2.0 ** -8, t_amb=80.0),
    "AH3": coeffs(0.25, 0.0625, 0.1875, 0.125, 0.1875, 0.0625, 0.125, cp=8.0, c_amb=2.0 ** -8, t_amb=80.0),
    # physical Hotspot 2D parameters (Table 2 as printed).  HP2 is the physical reading of
    # H2: sdc*Rx_1 = sdc*Ry_1 = 1/8, sdc*Rz_1 = 2^-10, sdc = 64.  HPr is non-dyadic.
    "HP2": phys_coeffs(64.0, 2.0 ** -9, 2.0 ** -9, 2.0 ** -16, 80.0),
    "HPr": phys_coeffs(0.3, 0.8, 0.6, 0.05, 80.0),
}


def star_weights(cc, xw, xe, ys, yn):
    """Pack the weights of a radius-r 2D star stencil: cc; w_d, e_d for d = 1..r (x-d, x+d);
    s_1..s_r (y+d); n_1..n_r (y-d).  The order is also the stencil's evaluation order."""
    r = len(xw)
    out = [cc]
    for d in range(r):
        out += [xw[d], xe[d]]
    return np.array(out + list(ys) + list(yn), dtype=np.float32)


# Radius-r weights: dyadic (multiples of 1/64), asymmetric, summing to exactly 1.
STAR_SETS = {
    2: star_weights(0.28125, [0.0625, 0.03125], [0.125, 0.0625], [0.125, 0.03125], [0.1875, 0.09375]),
    3: star_weights(0.328125, [0.0625, 0.03125, 0.015625], [0.09375, 0.046875, 0.03125],
                    [0.125, 0.0625, 0.015625], [0.125, 0.046875, 0.015625]),
    4: star_weights(0.21875, [0.0625, 0.03125, 0.015625, 0.015625], [0.0625, 0.046875, 0.03125, 0.015625],
                    [0.125, 0.0625, 0.03125, 0.015625], [0.125, 0.0625, 0.046875, 0.03125]),
}


def star3_weights(cc, xw, xe, ys, yn, zb, za):
    """Pack the weights of a radius-r 3D star stencil: cc; w_d, e_d for d = 1..r (x-d, x+d);
    s_1..s_r (y+d); n_1..n_r (y-d); b_1..b_r (z-d); a_1..a_r (z+d).  The order is also the
    stencil's evaluation order."""
    r = len(xw)
    out = [cc]
    for d in range(r):
        out += [xw[d], xe[d]]
    return np.array(out + list(ys) + list(yn) + list(zb) + list(za), dtype=np.float32)


def _star3_from_ints(den, cc, xw, xe, ys, yn, zb, za):
    f = lambda v: [x / den for x in v]
    return star3_weights(cc / den, f(xw), f(xe), f(ys), f(yn), f(zb), f(za))


# Radius-r 3D weights: dyadic, asymmetric, summing to exactly 1 (r = 1 is set A3's pattern).
STAR3_SETS = {
    1: _star3_from_ints(64, 16, [4], [12], [12], [8], [4], [8]),
    2: _star3_from_ints(64, 16, [4, 2], [6, 3], [5, 2], [6, 2], [4, 3], [7, 4]),
    3: _star3_from_ints(128, 36, [6, 4, 2], [9, 5, 3], [8, 4, 2], [9, 5, 1], [7, 4, 3], [11, 6, 3]),
    4: _star3_from_ints(128, 27, [6, 4, 2, 1], [9, 5, 3, 2], [8, 4, 2, 1], [9, 5, 1, 2], [7, 4, 3, 2],
                        [11, 6, 3, 1]),
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(shape, lo: float, hi: float, seed: int) -> np.ndarray:
    """U[lo, hi) in FP32 from a PCG64 stream (see module docstring)."""
    n = int(np.prod(shape)) if len(shape) else 1
    u = rng(seed).random(n, dtype=np.float32)
    out = np.float32(lo) + np.float32(hi - lo) * u
    return out.astype(np.float32, copy=False).reshape(shape)


def grid_shape(ndim: int, nx: int, ny: int, nz: int = 1):
    """numpy shape of a grid (slowest axis first)."""
    return (ny, nx) if ndim == 2 else (nz, ny, nx)


@dataclass
class Workload:
    name: str
    form: int
    ndim: int
    nx: int
    ny: int
    nz: int
    T: int
    coef_set: str
    field_lo: float
    field_hi: float
    power_hi: float = 0.0
    seed: int = 0
    target_lo: float = 300.0
    target_hi: float = 350.0
    ckpt_every: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return grid_shape(self.ndim, self.nx, self.ny, self.nz)

    @property
    def coeffs(self) -> np.ndarray:
        return SETS[self.coef_set].copy()

    def field(self) -> np.ndarray:
        return uniform(self.shape, self.field_lo, self.field_hi, self.seed)

    def power(self):
        if self.form == DIFFUSION:
            return None
        return uniform(self.shape, 0.0, self.power_hi, self.seed + 1)

    def target(self) -> np.ndarray:
        return uniform(self.shape, self.target_lo, self.target_hi, self.seed + 2)


# The workloads, in order: small 2D diffusion, large 2D hotspot, large 3D diffusion, the
# batch of uneven grids, the 3D hotspot adjoint problem, and the large 2D hotspot problem in
# the physical form.
WORKLOADS = {
    "diffusion2d_256": Workload("diffusion2d_256", DIFFUSION, 2, 256, 256, 1, 16, "D2", 0.0, 1.0, seed=1000),
    "hotspot2d_16384": Workload("hotspot2d_16384", HOTSPOT, 2, 16384, 16384, 1, 1000, "H2", 300.0, 350.0,
                                power_hi=1e-3, seed=2000),
    "diffusion3d_512": Workload("diffusion3d_512", DIFFUSION, 3, 512, 512, 512, 200, "D3", 0.0, 1.0, seed=3000),
    "hotspot3d_256_adjoint": Workload("hotspot3d_256_adjoint", HOTSPOT, 3, 256, 256, 256, 400, "H3", 300.0, 350.0,
                                      power_hi=1e-3, seed=5000, ckpt_every=20),
    # the large 2D hotspot problem in Table 2's physical form (parameters HP2, the physical
    # reading of H2); listed sixth, so its seed is 6000
    "hotspot2d_phys_16384": Workload("hotspot2d_phys_16384", HOTSPOT_PHYS, 2, 16384, 16384, 1, 1000, "HP2",
                                     300.0, 350.0, power_hi=1e-3, seed=6000),
}
BATCH_SEED = 4000

# Radius-r star stencil workload (Eq. 1, Eq. 2 with rad = 2): 2D diffusion form, weights
# STAR_SETS[2], the large 2D grid and step count of the paper's 2D runs; listed seventh, so
# its seed is 7000.
STAR_WORKLOAD = {"name": "star2d_r2_16384", "rad": 2, "nx": 16384, "ny": 16384, "T": 1000, "seed": 7000}


def star_field(wl=STAR_WORKLOAD) -> np.ndarray:
    return uniform((wl["ny"], wl["nx"]), 0.0, 1.0, wl["seed"])


# The 3D radius-2 workload: the 512^3 grid of the 3D diffusion workload with the weights of
# STAR3_SETS[2].
STAR3_WORKLOAD = {"name": "star3d_r2_512", "rad": 2, "nx": 512, "ny": 512, "nz": 512, "T": 100, "seed": 7100}


def star3_field(wl=STAR3_WORKLOAD) -> np.ndarray:
    return uniform((wl["nz"], wl["ny"], wl["nx"]), 0.0, 1.0, wl["seed"])


@dataclass
class BatchGrid:
    ndim: int
    nx: int
    ny: int
    nz: int
    T: int
    seed: int

    @property
    def shape(self):
        return grid_shape(self.ndim, self.nx, self.ny, self.nz)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def coef_set(self) -> str:
        return "D2" if self.ndim == 2 else "D3"

    def field(self) -> np.ndarray:
        return uniform(self.shape, 0.0, 1.0, self.seed)


def batch_grids(n2d: int = 48, n3d: int = 16, lo2: int = 256, hi2: int = 4096, lo3: int = 64, hi3: int = 256,
                tlo: int = 50, thi: int = 500, seed: int = BATCH_SEED, scale: float = 1.0):
    """The batched workload: n2d square 2D grids with log-uniform side in [lo2, hi2], n3d cubic 3D
    grids with log-uniform side in [lo3, hi3], and integer step counts uniform in [tlo, thi].

    Sides are drawn first (2D then 3D), then step counts, from PCG64(seed + 3).  ``scale``
    shrinks every side (for small test versions of the same recipe).
    """
    g = rng(seed + 3)
    s2 = np.rint(np.exp(g.uniform(math.log(lo2), math.log(hi2), n2d))).astype(int)
    s3 = np.rint(np.exp(g.uniform(math.log(lo3), math.log(hi3), n3d))).astype(int)
    steps = g.integers(tlo, thi + 1, n2d + n3d)
    out = []
    for i, s in enumerate(s2):
        s = max(1, int(round(s * scale)))
        out.append(BatchGrid(2, s, s, 1, int(steps[i]), seed + 10 + i))
    for j, s in enumerate(s3):
        s = max(1, int(round(s * scale)))
        out.append(BatchGrid(3, s, s, s, int(steps[n2d + j]), seed + 10 + n2d + j))
    return out
