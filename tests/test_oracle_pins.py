"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's loop.  Each one compares it with something
independent: a hand-worked step, a dense matrix built from the definition and raised to a
power by numpy, closed-form eigenmodes, an exact rational Green's function, conservation and
fixed-point laws, a closed-form scalar recurrence, symmetry and dimension-reduction
identities, and (for the adjoint) a dense transpose, the dot-product identity, exact central
differences and an independent gather formulation.

Paper passages: Section 2.1 (Jacobi ping-pong steps), Table 2 (stencil formulas),
Section 5.1 (out-of-range neighbours fall back on the boundary cell).
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import SETS, STAR_SETS, STAR3_SETS, DIFFUSION, HOTSPOT, HOTSPOT_PHYS, phys_coeffs, uniform

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# direction -> (coefficient index in the 10-vector, offset (dz, dy, dx) of the neighbour read)
DIRS = {
    "w": (1, (0, 0, -1)), "e": (2, (0, 0, 1)), "n": (3, (0, -1, 0)), "s": (4, (0, 1, 0)),
    "b": (5, (-1, 0, 0)), "a": (6, (1, 0, 0)),
}


def dense_operator(shape, cf):
    """Dense A with (A x)_i = cc x_i + sum_d c_d x_{clamp(i + d)} (Table 2 + Section 5.1)."""
    shape3 = (1,) * (3 - len(shape)) + tuple(shape)
    nz, ny, nx = shape3
    n = nx * ny * nz
    A = np.zeros((n, n))
    dirs = ["w", "e", "n", "s"] + (["b", "a"] if len(shape) == 3 else [])
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        i = (z * ny + y) * nx + x
        A[i, i] += float(cf[0])
        for d in dirs:
            ci, (dz, dy, dx) = DIRS[d]
            zz = min(max(z + dz, 0), nz - 1)
            yy = min(max(y + dy, 0), ny - 1)
            xx = min(max(x + dx, 0), nx - 1)
            A[i, (zz * ny + yy) * nx + xx] += float(cf[ci])
    return A


def dense_forward(x0, cf, T, power=None):
    """Brute force: x_T = A^T x_0 (diffusion) or the augmented affine power (hotspot)."""
    A = dense_operator(x0.shape, cf)
    n = A.shape[0]
    x = x0.astype(np.float64).ravel()
    if power is None:
        return (np.linalg.matrix_power(A, T) @ x).reshape(x0.shape)
    q = float(cf[7]) * power.astype(np.float64).ravel() + float(cf[8]) * float(cf[9])
    Aug = np.zeros((n + 1, n + 1))
    Aug[:n, :n] = A
    Aug[:n, n] = q
    Aug[n, n] = 1.0
    xa = np.append(x, 1.0)
    return (np.linalg.matrix_power(Aug, T) @ xa)[:n].reshape(x0.shape)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- hand-worked example

def test_hand_worked_step_matches_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "hand_step_A2_3x2.txt")) if l.strip() and l[0] != "#"]
    expected = np.array(rows, dtype=np.float64)
    x0 = np.array([[1, 2, 4], [8, 16, 32]], dtype=np.float32)
    for dt in (np.float64, np.float32):
        out = oracle.forward(x0, SETS["A2"], 1, dtype=dt)
        assert np.array_equal(out.astype(np.float64), expected), dt


# ---------------------------------------------------------------- dense brute force

SMALL_2D = [(8, 8), (5, 3), (1, 7), (7, 1), (1, 1), (2, 9)]
SMALL_3D = [(6, 6, 6), (3, 4, 2), (1, 5, 4), (2, 1, 3), (1, 1, 1)]
TS = [0, 1, 2, 3, 7, 16, 33]


@pytest.mark.parametrize("shape", SMALL_2D)
@pytest.mark.parametrize("cset", ["A2", "D2", "AH2", "H2"])
def test_forward_2d_equals_dense_matrix_power(shape, cset):
    cf = SETS[cset]
    x0 = uniform(shape, 0.0, 1.0, 11)
    p = uniform(shape, 0.0, 1.0, 12) if cset.startswith(("H", "AH")) else None
    for T in TS:
        ref = dense_forward(x0, cf, T, p)
        out = oracle.forward(x0, cf, T, power=p)
        assert relerr(out, ref) < 1e-13, (shape, cset, T)
        out32 = oracle.forward(x0, cf, T, power=p, dtype=np.float32)
        assert relerr(out32, ref) < 2e-6, (shape, cset, T)


@pytest.mark.parametrize("shape", SMALL_3D)
@pytest.mark.parametrize("cset", ["A3", "D3", "AH3", "H3"])
def test_forward_3d_equals_dense_matrix_power(shape, cset):
    cf = SETS[cset]
    x0 = uniform(shape, 0.0, 1.0, 21)
    p = uniform(shape, 0.0, 1.0, 22) if cset.startswith(("H", "AH")) else None
    for T in TS:
        ref = dense_forward(x0, cf, T, p)
        out = oracle.forward(x0, cf, T, power=p)
        assert relerr(out, ref) < 1e-13, (shape, cset, T)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("shape,cset,T", [((48, 64), "D2", 16), ((37, 23), "H2", 9),
                                          ((12, 16, 20), "D3", 12), ((9, 7, 5), "H3", 7)])
def test_dct_modes_are_eigenvectors(shape, cset, T):
    """cos(pi*j*(x+1/2)/n) products are exact eigenvectors of the clamped symmetric stencil;
    the eigenvalue is cc + 2*c_x*cos(pi*jx/nx) + 2*c_y*cos(pi*jy/ny) (+ 2*c_z*cos(pi*jz/nz))."""
    cf = SETS[cset].astype(np.float64)
    axes = [np.arange(n) for n in shape]
    c_axis = {len(shape) - 1: cf[1], len(shape) - 2: cf[3]}
    if len(shape) == 3:
        c_axis[0] = cf[5]
    rng = np.random.default_rng(5)
    for _ in range(3):
        js = [int(rng.integers(0, n)) for n in shape]
        mode = np.ones(shape)
        lam = cf[0]
        for ax, (n, j) in enumerate(zip(shape, js)):
            v = np.cos(np.pi * j * (axes[ax] + 0.5) / n)
            mode = mode * v.reshape([-1 if a == ax else 1 for a in range(len(shape))])
            lam += 2.0 * c_axis[ax] * np.cos(np.pi * j / n)
        # diffusion form only: the eigen-relation is for the linear operator
        out = oracle.forward(mode, np.r_[SETS[cset][:7], 0, 0, 0].astype(np.float32), T, form=DIFFUSION)
        assert np.max(np.abs(out - lam ** T * mode)) < 1e-12, js


def _green_exact(T, cf, dirs, ndim):
    """Exact impulse response: coefficients of (cc + sum_d c_d * shift_d)^T, as Fractions.
    Reading the neighbour at offset delta moves mass by -delta."""
    terms = [((0,) * ndim, Fraction(float(cf[0])))]
    for d in dirs:
        ci, off = DIRS[d]
        off = off[3 - ndim:]
        terms.append((tuple(-o for o in off), Fraction(float(cf[ci]))))
    poly = {(0,) * ndim: Fraction(1)}
    for _ in range(T):
        nxt = {}
        for k, v in poly.items():
            for off, c in terms:
                kk = tuple(a + b for a, b in zip(k, off))
                nxt[kk] = nxt.get(kk, 0) + v * c
        poly = nxt
    return poly


@pytest.mark.parametrize("cset,shape,T", [("D2", (40, 40), 16), ("A2", (36, 41), 14), ("A3", (19, 20, 21), 8)])
def test_green_function_exact(cset, shape, T):
    """Away from the boundary the FP64 oracle reproduces the exact rational impulse response
    bit for bit (dyadic weights: every intermediate is exactly representable)."""
    cf = SETS[cset]
    ndim = len(shape)
    dirs = ["w", "e", "n", "s"] + (["b", "a"] if ndim == 3 else [])
    centre = tuple(n // 2 for n in shape)
    x0 = np.zeros(shape)
    x0[centre] = 1.0
    out = oracle.forward(x0, cf, T)
    exact = np.zeros(shape)
    for k, v in _green_exact(T, cf, dirs, ndim).items():
        exact[tuple(c + o for c, o in zip(centre, k))] = float(v)
        assert float(v) == v  # the expected value itself is exact in double
    assert np.array_equal(out, exact)


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("cset,shape", [("D2", (33, 17)), ("A2", (9, 30)), ("D3", (7, 9, 11)), ("A3", (5, 8, 6))])
def test_constant_field_preserved(cset, shape):
    cf = SETS[cset]
    x0 = np.full(shape, 0.75, dtype=np.float32)
    for dt in (np.float64, np.float32):
        out = oracle.forward(x0, cf, 40, dtype=dt)
        if cset == "D3":  # 0.4 + 6*0.1 is 1 only to FP32 rounding
            assert np.max(np.abs(out - 0.75)) < 1e-6
        else:
            assert np.all(out == 0.75)


@pytest.mark.parametrize("cset,shape", [("H2", (20, 30)), ("H3", (6, 7, 8)), ("H3p", (5, 6, 7))])
def test_hotspot_ambient_fixed_point(cset, shape):
    """With zero power, the ambient temperature is a fixed point (weights sum to exactly 1)."""
    cf = SETS[cset]
    x0 = np.full(shape, 80.0, dtype=np.float32)
    for dt in (np.float64, np.float32):
        out = oracle.forward(x0, cf, 25, power=np.zeros(shape, np.float32), dtype=dt)
        assert np.all(out == 80.0)


@pytest.mark.parametrize("cset,shape", [("H2", (6, 9)), ("H3", (4, 5, 6))])
def test_hotspot_uniform_closed_form(cset, shape):
    """Uniform X and P: x_t = x* + (X - x*)(1 - c_amb)^t, x* = t_amb + cp*P/c_amb."""
    cf = SETS[cset].astype(np.float64)
    X, P = 300.0, 1e-3
    xs = cf[9] + cf[7] * np.float64(np.float32(P)) / cf[8]
    for T in (1, 5, 50, 400):
        out = oracle.forward(np.full(shape, X), SETS[cset], T, power=np.full(shape, np.float32(P)))
        ref = xs + (X - xs) * (1.0 - cf[8]) ** T
        assert np.max(np.abs(out - ref)) / ref < 1e-13, T


@pytest.mark.parametrize("cset,shape", [("D2", (31, 47)), ("D3", (9, 13, 11))])
def test_conservation_and_maximum_principle(cset, shape):
    cf = SETS[cset]
    x0 = uniform(shape, 0.0, 1.0, 31)
    out = oracle.forward(x0, cf, 60)
    # symmetric weights summing to one: the clamped operator is symmetric and doubly stochastic
    total = float(np.sum(x0, dtype=np.float64))
    s = float(np.sum(cf[:7], dtype=np.float64))
    assert abs(float(out.sum()) - total * s ** 60) / total < 1e-12
    assert out.min() >= x0.min() - 1e-12 and out.max() <= x0.max() + 1e-12


def test_dimension_reduction_3d_single_plane():
    """3D with nz = 1 is 2D with cc' = cc + cb + ca (both z-neighbours clamp to the cell)."""
    cf3 = SETS["A3"]
    cf2 = cf3.copy()
    cf2[0] = np.float32(float(cf3[0]) + float(cf3[5]) + float(cf3[6]))
    x0 = uniform((1, 11, 14), 0.0, 1.0, 41)
    out3 = oracle.forward(x0, cf3, 9)
    out2 = oracle.forward(x0[0], cf2, 9)
    assert relerr(out3[0], out2) < 1e-14


def test_axis_swap_transposes_output():
    """Swapping x and y together with (cw, ce) <-> (cn, cs) transposes the result; catches
    index mistakes on non-square grids."""
    cf = SETS["A2"]
    sw = cf.copy()
    sw[1], sw[2], sw[3], sw[4] = cf[3], cf[4], cf[1], cf[2]
    x0 = uniform((13, 7), 0.0, 1.0, 51)
    a = oracle.forward(x0, cf, 11)
    b = oracle.forward(np.ascontiguousarray(x0.T), sw, 11)
    assert relerr(b.T, a) < 1e-14


def test_linearity():
    cf = SETS["A3"]
    x = uniform((6, 7, 8), 0.0, 1.0, 61).astype(np.float64)
    y = uniform((6, 7, 8), 0.0, 1.0, 62).astype(np.float64)
    lhs = oracle.forward(2.5 * x - 0.75 * y, cf, 10)
    rhs = 2.5 * oracle.forward(x, cf, 10) - 0.75 * oracle.forward(y, cf, 10)
    assert relerr(lhs, rhs) < 1e-13


# ---------------------------------------------------------------- adjoint

def _linear_part(cf):
    c = cf.copy()
    c[7:] = 0
    return c


@pytest.mark.parametrize("shape,cset", [((8, 8), "AH2"), ((5, 3), "A2"), ((6, 6, 6), "AH3"), ((3, 4, 2), "A3"),
                                        ((1, 6), "AH2"), ((1, 1, 4), "A3")])
def test_adjoint_equals_dense_transpose(shape, cset):
    cf = SETS[cset]
    form = HOTSPOT if cset.startswith("AH") else DIFFUSION
    A = dense_operator(shape, cf)
    g = uniform(shape, -1.0, 1.0, 71).astype(np.float64).ravel()
    for T in (0, 1, 2, 5, 13):
        gx, gp = oracle.adjoint(g.reshape(shape), cf, T, form=form)
        ref = np.linalg.matrix_power(A.T, T) @ g
        assert relerr(gx.ravel(), ref) < 1e-13, T
        if form == HOTSPOT:
            acc = np.zeros_like(g)
            lam = g.copy()
            for _ in range(T):
                acc += lam
                lam = A.T @ lam
            refp = float(cf[7]) * acc
            if T == 0:
                assert np.all(gp == 0)
            else:
                assert relerr(gp.ravel(), refp) < 1e-13, T
        # the FP32 instantiation against the same dense reference, within FP32 rounding
        gx32, gp32 = oracle.adjoint(g.reshape(shape), cf, T, form=form, dtype=np.float32)
        assert gx32.dtype == np.float32
        assert relerr(gx32.ravel(), ref) < 4e-6, T
        if form == HOTSPOT and T > 0:
            assert relerr(gp32.ravel(), refp) < 4e-6, T


def _gather_adjoint_step(lam, cf):
    """Independent gather form of A^T: mirrored weights with zero padding plus, at each
    boundary face, a self term carrying the weight of the direction that leaves the grid."""
    nd = lam.ndim
    out = float(cf[0]) * lam
    dirs = ["w", "e", "n", "s"] + (["b", "a"] if nd == 3 else [])
    for d in dirs:
        ci, off = DIRS[d]
        off = off[3 - nd:]
        c = float(cf[ci])
        ax = [i for i, o in enumerate(off) if o != 0][0]
        o = off[ax]
        n = lam.shape[ax]
        # gather lam_{j - d}: shift lam by +o along ax with zero fill
        sh = np.zeros_like(lam)
        src = [slice(None)] * nd
        dst = [slice(None)] * nd
        if n > 1:
            if o > 0:
                src[ax], dst[ax] = slice(0, n - 1), slice(1, n)
            else:
                src[ax], dst[ax] = slice(1, n), slice(0, n - 1)
            sh[tuple(dst)] = lam[tuple(src)]
        out = out + c * sh
        # self term where j + d leaves the grid
        edge = [slice(None)] * nd
        edge[ax] = slice(n - 1, n) if o > 0 else slice(0, 1)
        selfterm = np.zeros_like(lam)
        selfterm[tuple(edge)] = lam[tuple(edge)]
        out = out + c * selfterm
    return out


@pytest.mark.parametrize("shape,cset", [((9, 12), "A2"), ((5, 6, 7), "A3"), ((1, 5), "A2"), ((4, 1, 3), "A3")])
def test_adjoint_gather_form(shape, cset):
    cf = SETS[cset]
    g = uniform(shape, -1.0, 1.0, 81).astype(np.float64)
    lam = g.copy()
    for T in range(1, 8):
        lam = _gather_adjoint_step(lam, cf)
        gx, _ = oracle.adjoint(g, cf, T)
        assert relerr(gx, lam) < 1e-13, T


@pytest.mark.parametrize("shape,cset", [((23, 17), "A2"), ((7, 9, 8), "A3")])
def test_dot_product_identity(shape, cset):
    cf = SETS[cset]
    x = uniform(shape, 0.0, 1.0, 91).astype(np.float64)
    y = uniform(shape, 0.0, 1.0, 92).astype(np.float64)
    for T in (1, 6, 25):
        Ax = oracle.forward(x, cf, T)
        ATy, _ = oracle.adjoint(y, cf, T)
        a, b = float(np.vdot(ATy, x)), float(np.vdot(y, Ax))
        assert abs(a - b) / max(abs(a), abs(b)) < 1e-13


@pytest.mark.parametrize("shape,cset", [((10, 12), "AH2"), ((5, 6, 4), "AH3")])
def test_central_differences_exact_for_quadratic_loss(shape, cset):
    """J = 1/2 ||x_T - y||^2 is quadratic in (x0, p), so central differences carry no
    truncation error: they match the adjoint gradient up to rounding."""
    cf = SETS[cset]
    T = 7
    x0 = uniform(shape, 300.0, 350.0, 101).astype(np.float64)
    p = uniform(shape, 0.0, 1e-3, 102).astype(np.float64)
    y = uniform(shape, 300.0, 350.0, 103).astype(np.float64)
    xT = oracle.forward(x0, cf, T, power=p)
    gx, gp = oracle.adjoint(xT - y, cf, T, form=HOTSPOT)
    rng = np.random.default_rng(0)
    h = 0.5
    for _ in range(6):
        idx = tuple(int(rng.integers(0, n)) for n in shape)
        for which, grad in (("x", gx), ("p", gp)):
            xp, xm = x0.copy(), x0.copy()
            pp, pm = p.copy(), p.copy()
            if which == "x":
                xp[idx] += h
                xm[idx] -= h
            else:
                pp[idx] += h
                pm[idx] -= h
            jp = oracle.loss(oracle.forward(xp, cf, T, power=pp), y)
            jm = oracle.loss(oracle.forward(xm, cf, T, power=pm), y)
            fd = (jp - jm) / (2 * h)
            assert abs(fd - grad[idx]) <= 1e-7 * max(1.0, abs(grad[idx])), (which, idx, fd, grad[idx])


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((3, 3)), SETS["D2"], -1)
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((3, 3)), SETS["H2"], 1, form=HOTSPOT)


def test_fp32_vs_fp64_error_budget():
    """The FP32 oracle stays well within the 1e-5 relative budget of the FP64 one on a
    hotspot run of a thousand steps (the large 2D workload's step count)."""
    cf = SETS["H2"]
    x0 = uniform((64, 64), 300.0, 350.0, 111)
    p = uniform((64, 64), 0.0, 1e-3, 112)
    a = oracle.forward(x0, cf, 1000, power=p)
    b = oracle.forward(x0, cf, 1000, power=p, dtype=np.float32)
    assert relerr(b, a) < 1e-5


# ---------------------------------------------------------------- physical Hotspot 2D (Table 2 as printed)

def _phys_as_weights(cf):
    """The weights the physical formula expands to, in FP64 from the FP32 parameters:
    cc = 1 - sdc(2Rx_1 + 2Ry_1 + Rz_1), cw = ce = sdc Rx_1, cn = cs = sdc Ry_1, cp = sdc,
    c_amb = sdc Rz_1."""
    sdc, rx, ry, rz, ta = (float(cf[i]) for i in (7, 2, 4, 8, 9))
    return np.array([1.0 - sdc * (2 * rx + 2 * ry + rz), sdc * rx, sdc * rx, sdc * ry, sdc * ry, 0.0, 0.0,
                     sdc, sdc * rz, ta], dtype=np.float64)


def test_phys_hand_worked_step_matches_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "hand_step_HP_3x2.txt")) if l.strip() and l[0] != "#"]
    expected = np.array(rows, dtype=np.float64)
    x0 = np.array([[1, 2, 4], [8, 16, 32]], dtype=np.float32)
    p = np.array([[0, 1, 0], [2, 0, 4]], dtype=np.float32)
    cf = phys_coeffs(0.5, 0.25, 0.125, 0.0625, 16.0)
    for dt in (np.float64, np.float32):
        out = oracle.forward(x0, cf, 1, power=p, form=HOTSPOT_PHYS, dtype=dt)
        assert np.array_equal(out.astype(np.float64), expected), dt


@pytest.mark.parametrize("shape", SMALL_2D)
@pytest.mark.parametrize("cset", ["HP2", "HPr"])
def test_phys_equals_dense_affine_power(shape, cset):
    """The physical formula is the affine map of its expanded weights: brute-force matrix power."""
    cf = SETS[cset]
    x0 = uniform(shape, 300.0, 350.0, 121)
    p = uniform(shape, 0.0, 1.0, 122)
    w = _phys_as_weights(cf)
    for T in TS:
        ref = dense_forward(x0, w, T, p)
        out = oracle.forward(x0, cf, T, power=p, form=HOTSPOT_PHYS)
        assert relerr(out, ref) < 1e-13, (shape, cset, T)
        out32 = oracle.forward(x0, cf, T, power=p, form=HOTSPOT_PHYS, dtype=np.float32)
        assert relerr(out32, ref) < 2e-6, (shape, cset, T)


def test_phys_hp2_is_the_weighted_h2_set():
    """HP2 expands exactly to H2, so the two forms agree to FP64 rounding on the same inputs."""
    assert np.array_equal(_phys_as_weights(SETS["HP2"]), SETS["H2"].astype(np.float64))
    x0 = uniform((37, 29), 300.0, 350.0, 123)
    p = uniform((37, 29), 0.0, 1e-3, 124)
    a = oracle.forward(x0, SETS["HP2"], 50, power=p, form=HOTSPOT_PHYS)
    b = oracle.forward(x0, SETS["H2"], 50, power=p, form=HOTSPOT)
    assert relerr(a, b) < 1e-13


@pytest.mark.parametrize("cset", ["HP2", "HPr"])
def test_phys_ambient_is_an_exact_fixed_point(cset):
    """With zero power a field at TEMP_AMB makes every difference of the formula exactly zero,
    so it stays bit-exact in FP32 too, also with weights that are not dyadic."""
    x0 = np.full((11, 13), 80.0, dtype=np.float32)
    for dt in (np.float64, np.float32):
        out = oracle.forward(x0, SETS[cset], 60, power=np.zeros_like(x0), form=HOTSPOT_PHYS, dtype=dt)
        assert np.all(out == 80.0), dt


@pytest.mark.parametrize("cset", ["HP2", "HPr"])
def test_phys_uniform_closed_form(cset):
    """Uniform X and P: the differences vanish and x_{t+1} = x_t + sdc(P + Rz_1(TEMP_AMB - x_t)),
    so x_t = x* + (X - x*)(1 - sdc Rz_1)^t with x* = TEMP_AMB + P / Rz_1."""
    cf = SETS[cset]
    sdc, rz, ta = float(cf[7]), float(cf[8]), float(cf[9])
    X, P = 300.0, float(np.float32(1e-3))
    xs = ta + P / rz
    for T in (1, 5, 50, 400):
        out = oracle.forward(np.full((5, 7), X), cf, T, power=np.full((5, 7), np.float32(P)), form=HOTSPOT_PHYS)
        ref = xs + (X - xs) * (1.0 - sdc * rz) ** T
        assert np.max(np.abs(out - ref)) / abs(ref) < 1e-12, T


@pytest.mark.parametrize("shape", [(8, 8), (5, 3), (1, 6), (7, 1)])
def test_phys_adjoint_equals_dense_transpose(shape):
    cf = SETS["HPr"]
    A = dense_operator(shape, _phys_as_weights(cf))
    g = uniform(shape, -1.0, 1.0, 125).astype(np.float64).ravel()
    for T in (0, 1, 2, 5, 13):
        gx, gp = oracle.adjoint(g.reshape(shape), cf, T, form=HOTSPOT_PHYS)
        assert relerr(gx.ravel(), np.linalg.matrix_power(A.T, T) @ g) < 1e-13, T
        acc = np.zeros_like(g)
        lam = g.copy()
        for _ in range(T):
            acc += lam
            lam = A.T @ lam
        if T == 0:
            assert np.all(gp == 0)
        else:
            assert relerr(gp.ravel(), float(cf[7]) * acc) < 1e-13, T


def test_phys_central_differences():
    """Central differences of the quadratic loss through the physical forward match the
    physical adjoint (no truncation error)."""
    cf = SETS["HPr"]
    shape, T = (9, 11), 6
    x0 = uniform(shape, 300.0, 350.0, 126).astype(np.float64)
    p = uniform(shape, 0.0, 1e-3, 127).astype(np.float64)
    y = uniform(shape, 300.0, 350.0, 128).astype(np.float64)
    xT = oracle.forward(x0, cf, T, power=p, form=HOTSPOT_PHYS)
    gx, gp = oracle.adjoint(xT - y, cf, T, form=HOTSPOT_PHYS)
    rng = np.random.default_rng(1)
    h = 0.5
    for _ in range(6):
        idx = tuple(int(rng.integers(0, n)) for n in shape)
        for which, grad in (("x", gx), ("p", gp)):
            xp, xm, pp, pm = x0.copy(), x0.copy(), p.copy(), p.copy()
            if which == "x":
                xp[idx] += h
                xm[idx] -= h
            else:
                pp[idx] += h
                pm[idx] -= h
            jp = oracle.loss(oracle.forward(xp, cf, T, power=pp, form=HOTSPOT_PHYS), y)
            jm = oracle.loss(oracle.forward(xm, cf, T, power=pm, form=HOTSPOT_PHYS), y)
            assert abs((jp - jm) / (2 * h) - grad[idx]) <= 1e-7 * max(1.0, abs(grad[idx])), (which, idx)


def test_phys_fp32_error_budget_and_rejections():
    cf = SETS["HP2"]
    x0 = uniform((64, 64), 300.0, 350.0, 129)
    p = uniform((64, 64), 0.0, 1e-3, 130)
    a = oracle.forward(x0, cf, 1000, power=p, form=HOTSPOT_PHYS)
    b = oracle.forward(x0, cf, 1000, power=p, form=HOTSPOT_PHYS, dtype=np.float32)
    assert relerr(b, a) < 1e-5
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((2, 3, 3)), cf, 1, power=np.zeros((2, 3, 3)), form=HOTSPOT_PHYS)
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((3, 3)), cf, 1, form=HOTSPOT_PHYS)


# ---------------------------------------------------------------- radius-r star stencils (Eq. 1, Eq. 2)

STAR = STAR_SETS


def dense_star(shape, wts):
    """Dense A of the radius-r star stencil from its definition: row i gets cc at i and each
    directional weight at the clamped index of that neighbour."""
    ny, nx = shape
    r = (len(wts) - 1) // 4
    A = np.zeros((nx * ny, nx * ny))
    for y, x in itertools.product(range(ny), range(nx)):
        i = y * nx + x
        A[i, i] += float(wts[0])
        for d in range(1, r + 1):
            A[i, y * nx + max(x - d, 0)] += float(wts[2 * d - 1])
            A[i, y * nx + min(x + d, nx - 1)] += float(wts[2 * d])
            A[i, min(y + d, ny - 1) * nx + x] += float(wts[2 * r + d])
            A[i, max(y - d, 0) * nx + x] += float(wts[3 * r + d])
    return A


def test_star_radius_one_is_the_diffusion_stencil():
    cf = SETS["A2"]  # cc, cw, ce, cn, cs
    w = np.array([cf[0], cf[1], cf[2], cf[4], cf[3]], dtype=np.float32)
    x0 = uniform((37, 53), 0.0, 1.0, 141)
    for dt in (np.float64, np.float32):
        assert np.array_equal(oracle.star2d(x0, w, 19, dtype=dt), oracle.forward(x0, cf, 19, dtype=dt))


@pytest.mark.parametrize("shape", [(8, 8), (5, 3), (1, 7), (7, 1), (2, 9), (3, 3), (1, 1)])
@pytest.mark.parametrize("r", [2, 3, 4])
def test_star_equals_dense_matrix_power(shape, r):
    w = STAR[r]
    A = dense_star(shape, w)
    x0 = uniform(shape, 0.0, 1.0, 142 + r)
    for T in (0, 1, 2, 3, 7):
        ref = (np.linalg.matrix_power(A, T) @ x0.astype(np.float64).ravel()).reshape(shape)
        assert relerr(oracle.star2d(x0, w, T), ref) < 1e-13, (shape, r, T)
        assert relerr(oracle.star2d(x0, w, T, dtype=np.float32), ref) < 2e-6, (shape, r, T)


@pytest.mark.parametrize("r,T", [(2, 6), (3, 5), (4, 4)])
def test_star_green_function_exact(r, T):
    """Away from the edges the impulse response is the T-fold convolution of the stencil,
    computed here in exact integers (weights scaled by 2^6).  Its denominators fit FP64, so the
    FP64 oracle must reproduce it exactly."""
    w = STAR[r]
    scale = 64
    iw = [int(round(float(v) * scale)) for v in w]
    assert all(abs(a - float(v) * scale) == 0 for a, v in zip(iw, w))
    n = 2 * r * T + 5
    c = n // 2
    ex = {(c, c): 1}
    for _ in range(T):
        nxt = {}
        for (y, x), v in ex.items():
            # scatter: the value at (y, x) feeds (y, x) with cc, (y, x+d) with w_d (it is that
            # cell's x-d neighbour), (y, x-d) with e_d, (y-d, x) with s_d, (y+d, x) with n_d
            terms = [((y, x), iw[0])]
            for d in range(1, r + 1):
                terms += [((y, x + d), iw[2 * d - 1]), ((y, x - d), iw[2 * d]),
                          ((y - d, x), iw[2 * r + d]), ((y + d, x), iw[3 * r + d])]
            for k, wv in terms:
                nxt[k] = nxt.get(k, 0) + wv * v
        ex = nxt
    x0 = np.zeros((n, n))
    x0[c, c] = 1.0
    out = oracle.star2d(x0, w, T)
    ref = np.zeros((n, n))
    for (y, x), v in ex.items():
        ref[y, x] = Fraction(v, scale ** T)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("r", [2, 3, 4])
def test_star_constant_field_and_axis_swap(r):
    w = STAR[r]
    x0 = np.full((19, 23), 0.75, dtype=np.float32)
    assert np.all(oracle.star2d(x0, w, 30, dtype=np.float32) == 0.75)
    # swapping x and y together with (w_d, e_d) <-> (n_d, s_d) transposes the result
    sw = w.copy()
    for d in range(1, r + 1):
        sw[2 * d - 1], sw[2 * d] = w[3 * r + d], w[2 * r + d]
        sw[3 * r + d], sw[2 * r + d] = w[2 * d - 1], w[2 * d]
    x1 = uniform((13, 29), 0.0, 1.0, 150 + r)
    a = oracle.star2d(x1, w, 9)
    b = oracle.star2d(np.ascontiguousarray(x1.T), sw, 9)
    assert relerr(b.T, a) < 1e-14


def test_star_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.star2d(np.zeros((3, 3)), np.zeros(6, np.float32), 1)
    with pytest.raises(ValueError):
        oracle.star2d(np.zeros((2, 3, 3)), STAR[2], 1)
    with pytest.raises(ValueError):
        oracle.star2d(np.zeros((3, 3)), STAR[2], -1)


# ---------------------------------------------------------------- radius-r star stencil, 3D

STAR3 = STAR3_SETS


def dense_star3(shape, wts):
    """Dense operator of the radius-r 3D star stencil: row i gets every directional weight at
    the clamped index of that neighbour (Section 5.1 at every distance)."""
    nz, ny, nx = shape
    r = (len(wts) - 1) // 6
    n = nx * ny * nz
    A = np.zeros((n, n))
    idx = lambda z, y, x: (z * ny + y) * nx + x
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        i = idx(z, y, x)
        A[i, i] += float(wts[0])
        for d in range(1, r + 1):
            A[i, idx(z, y, max(x - d, 0))] += float(wts[2 * d - 1])
            A[i, idx(z, y, min(x + d, nx - 1))] += float(wts[2 * d])
            A[i, idx(z, min(y + d, ny - 1), x)] += float(wts[2 * r + d])
            A[i, idx(z, max(y - d, 0), x)] += float(wts[3 * r + d])
            A[i, idx(max(z - d, 0), y, x)] += float(wts[4 * r + d])
            A[i, idx(min(z + d, nz - 1), y, x)] += float(wts[5 * r + d])
    return A


def test_star3d_radius_one_is_the_3d_diffusion_stencil():
    w = STAR3[1]  # cc, w, e, s, n, b, a
    cf = np.array([w[0], w[1], w[2], w[4], w[3], w[5], w[6], 0, 0, 0], dtype=np.float32)
    x0 = uniform((11, 17, 23), 0.0, 1.0, 161)
    for dt in (np.float64, np.float32):
        assert np.array_equal(oracle.star3d(x0, w, 13, dtype=dt), oracle.forward(x0, cf, 13, dtype=dt))


@pytest.mark.parametrize("shape", [(6, 6, 6), (5, 4, 3), (1, 5, 7), (7, 1, 2), (2, 3, 1), (1, 1, 1), (4, 2, 6)])
@pytest.mark.parametrize("r", [2, 3, 4])
def test_star3d_equals_dense_matrix_power(shape, r):
    w = STAR3[r]
    A = dense_star3(shape, w)
    x0 = uniform(shape, 0.0, 1.0, 162 + r)
    for T in (0, 1, 2, 3, 6):
        ref = (np.linalg.matrix_power(A, T) @ x0.astype(np.float64).ravel()).reshape(shape)
        assert relerr(oracle.star3d(x0, w, T), ref) < 1e-13, (shape, r, T)
        assert relerr(oracle.star3d(x0, w, T, dtype=np.float32), ref) < 2e-6, (shape, r, T)


@pytest.mark.parametrize("r,T", [(2, 3), (3, 2), (4, 2)])
def test_star3d_green_function_exact(r, T):
    """Away from the edges the impulse response is the T-fold convolution of the stencil, here
    in exact integers (weights scaled by their common denominator); the FP64 oracle must
    reproduce it exactly."""
    w = STAR3[r]
    scale = 128
    iw = [int(round(float(v) * scale)) for v in w]
    assert all(a == float(v) * scale for a, v in zip(iw, w))
    n = 2 * r * T + 3
    c = n // 2
    ex = {(c, c, c): 1}
    for _ in range(T):
        nxt = {}
        for (z, y, x), v in ex.items():
            # scatter: the value at a cell feeds the cells that read it as a neighbour: the
            # cell at x+d reads it as its x-d neighbour (weight w_d), and so on
            terms = [((z, y, x), iw[0])]
            for d in range(1, r + 1):
                terms += [((z, y, x + d), iw[2 * d - 1]), ((z, y, x - d), iw[2 * d]),
                          ((z, y - d, x), iw[2 * r + d]), ((z, y + d, x), iw[3 * r + d]),
                          ((z + d, y, x), iw[4 * r + d]), ((z - d, y, x), iw[5 * r + d])]
            for k, wv in terms:
                nxt[k] = nxt.get(k, 0) + wv * v
        ex = nxt
    x0 = np.zeros((n, n, n))
    x0[c, c, c] = 1.0
    out = oracle.star3d(x0, w, T)
    ref = np.zeros((n, n, n))
    for k, v in ex.items():
        ref[k] = Fraction(v, scale ** T)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star3d_constant_field_and_axis_permutation(r):
    w = STAR3[r]
    x0 = np.full((9, 11, 13), 0.625, dtype=np.float32)
    assert np.all(oracle.star3d(x0, w, 20, dtype=np.float32) == 0.625)
    # exchanging the x and z axes together with (w_d, e_d) <-> (b_d, a_d) permutes the result
    sw = w.copy()
    for d in range(1, r + 1):
        sw[2 * d - 1], sw[2 * d] = w[4 * r + d], w[5 * r + d]
        sw[4 * r + d], sw[5 * r + d] = w[2 * d - 1], w[2 * d]
    x1 = uniform((7, 10, 12), 0.0, 1.0, 170 + r)
    a = oracle.star3d(x1, w, 5)
    b = oracle.star3d(np.ascontiguousarray(x1.transpose(2, 1, 0)), sw, 5)
    assert relerr(b.transpose(2, 1, 0), a) < 1e-14


def test_star3d_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.star3d(np.zeros((3, 3, 3)), np.zeros(8, np.float32), 1)
    with pytest.raises(ValueError):
        oracle.star3d(np.zeros((3, 3)), STAR3[2], 1)
    with pytest.raises(ValueError):
        oracle.star3d(np.zeros((3, 3, 3)), STAR3[2], -1)


# ---------------------------------------------------------------- radius-r hotspot form

SRC = (0.125, 0.25, 64.0)  # cp, c_amb, t_amb (dyadic, so the source q is exact in FP32)


def test_star_src_radius_one_is_the_hotspot_stencil():
    """Radius 1 with a source: the radius-1 hotspot forward (its own chain fma(cc, c, q)), bit
    for bit in FP64 and FP32, in 2D and 3D."""
    cf = SETS["AH2"]  # cc, cw, ce, cn, cs, cb, ca, cp, c_amb, t_amb
    w = np.array([cf[0], cf[1], cf[2], cf[4], cf[3]], dtype=np.float32)
    src = (cf[7], cf[8], cf[9])
    x0 = uniform((29, 41), 300.0, 350.0, 171)
    p = uniform((29, 41), 0.0, 1e-3, 172)
    for dt in (np.float64, np.float32):
        assert np.array_equal(oracle.star2d(x0, w, 15, dtype=dt, power=p, src=src),
                              oracle.forward(x0, cf, 15, power=p, dtype=dt))
    cf3 = SETS["H3"]
    w3 = np.array([cf3[0], cf3[1], cf3[2], cf3[4], cf3[3], cf3[5], cf3[6]], dtype=np.float32)
    src3 = (cf3[7], cf3[8], cf3[9])
    x3 = uniform((9, 13, 17), 300.0, 350.0, 173)
    p3 = uniform((9, 13, 17), 0.0, 1e-3, 174)
    for dt in (np.float64, np.float32):
        assert np.array_equal(oracle.star3d(x3, w3, 11, dtype=dt, power=p3, src=src3),
                              oracle.forward(x3, cf3, 11, power=p3, dtype=dt))


def affine_reference(A, x0, q, T):
    """x_T = A^T x_0 + sum_{t < T} A^t q, in FP64 from the dense operator."""
    x = x0.astype(np.float64).ravel()
    acc = np.zeros_like(x)
    Ak = np.eye(A.shape[0])
    for _ in range(T):
        acc += Ak @ q
        Ak = A @ Ak
    return Ak @ x + acc


@pytest.mark.parametrize("r", [2, 3, 4])
def test_star_src_is_the_affine_map_of_the_dense_operator(r):
    """The hotspot form is x_{t+1} = A x_t + q with A the clamped radius-r operator and
    q = cp*p + c_amb*t_amb: its T-step result is A^T x_0 + sum_{t<T} A^t q."""
    shape = (6, 5)
    w = STAR[r]
    A = dense_star(shape, w)
    x0 = uniform(shape, 0.0, 1.0, 181 + r)
    p = uniform(shape, 0.0, 1.0, 185 + r)
    q = SRC[0] * p.astype(np.float64).ravel() + SRC[1] * SRC[2]
    for T in (0, 1, 2, 5):
        ref = affine_reference(A, x0, q, T).reshape(shape)
        assert relerr(oracle.star2d(x0, w, T, power=p, src=SRC), ref) < 1e-13, (r, T)
        assert relerr(oracle.star2d(x0, w, T, dtype=np.float32, power=p, src=SRC), ref) < 2e-6, (r, T)
    shape3 = (3, 4, 5)
    w3 = STAR3[r]
    A3 = dense_star3(shape3, w3)
    x3 = uniform(shape3, 0.0, 1.0, 191 + r)
    p3 = uniform(shape3, 0.0, 1.0, 195 + r)
    q3 = SRC[0] * p3.astype(np.float64).ravel() + SRC[1] * SRC[2]
    for T in (0, 1, 3):
        ref = affine_reference(A3, x3, q3, T).reshape(shape3)
        assert relerr(oracle.star3d(x3, w3, T, power=p3, src=SRC), ref) < 1e-13, (r, T)
        assert relerr(oracle.star3d(x3, w3, T, dtype=np.float32, power=p3, src=SRC), ref) < 2e-6, (r, T)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star_src_exact_fixed_point(r):
    """Weights summing to 3/4 and q = 20 everywhere (p = 32: 0.125*32 + 0.25*64): the field 80
    is a fixed point, (3/4)*80 + 20 = 80, exactly in FP32 at every step (dyadic values)."""
    a2 = SETS["A2"]
    base2 = np.array([a2[0], a2[1], a2[2], a2[4], a2[3]], np.float32) if r == 1 else STAR[r]
    w2 = (base2.astype(np.float64) * 0.75).astype(np.float32)
    w3 = (STAR3[r].astype(np.float64) * 0.75).astype(np.float32)
    assert float(w2.astype(np.float64).sum()) == 0.75 and float(w3.astype(np.float64).sum()) == 0.75
    x2 = np.full((7, 9), 80.0, np.float32)
    x3 = np.full((4, 5, 6), 80.0, np.float32)
    for dt in (np.float32, np.float64):
        assert np.all(oracle.star2d(x2, w2, 25, dtype=dt, power=np.full(x2.shape, 32.0), src=SRC) == 80.0)
        assert np.all(oracle.star3d(x3, w3, 25, dtype=dt, power=np.full(x3.shape, 32.0), src=SRC) == 80.0)
    # one step from 0 with uniform power is q everywhere
    z = oracle.star2d(np.zeros((4, 4)), w2, 1, power=np.full((4, 4), 32.0), src=SRC)
    assert np.all(z == 20.0)


def test_star_src_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.star2d(np.zeros((3, 3)), STAR[2], 1, power=np.zeros((3, 3)))  # no src
    with pytest.raises(ValueError):
        oracle.star2d(np.zeros((3, 3)), STAR[2], 1, power=np.zeros((3, 4)), src=SRC)
    with pytest.raises(ValueError):
        oracle.star3d(np.zeros((3, 3, 3)), STAR3[2], 1, power=np.zeros((3, 3)), src=SRC)


# ---------------------------------------------------------------- radius-r adjoint

def star_weights_2d(r):
    a2 = SETS["A2"]
    return np.array([a2[0], a2[1], a2[2], a2[4], a2[3]], np.float32) if r == 1 else STAR[r]


@pytest.mark.parametrize("shape", [(6, 5), (1, 7), (5, 1), (2, 3), (1, 1), (4, 9)])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star_adjoint_is_the_dense_transpose(shape, r):
    """grad_x0 = (A^T)^T lambda_T and grad_p = cp * sum_{t=1..T} (A^T)^(T-t) lambda_T, with A the
    clamped radius-r operator built from its definition."""
    w = star_weights_2d(r)
    At = dense_star(shape, w).T
    lam = uniform(shape, -1.0, 1.0, 201 + r)
    cp = 0.375
    for T in (0, 1, 2, 5):
        g, gp = oracle.star_adjoint(lam, w, T, cp=cp)
        ref = np.linalg.matrix_power(At, T) @ lam.astype(np.float64).ravel()
        refp = cp * sum(np.linalg.matrix_power(At, T - t) @ lam.astype(np.float64).ravel() for t in range(1, T + 1)) \
            if T else np.zeros(lam.size)
        assert relerr(g, ref.reshape(shape)) < 1e-13, (shape, r, T)
        assert np.abs(gp.ravel() - refp).max() <= 1e-13 * max(1.0, np.abs(refp).max()), (shape, r, T)
        g32, _ = oracle.star_adjoint(lam, w, T, dtype=np.float32)
        assert relerr(g32, ref.reshape(shape)) < 2e-6


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 5, 3), (4, 1, 2), (2, 3, 1)])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star3d_adjoint_is_the_dense_transpose(shape, r):
    w = STAR3[r]
    At = dense_star3(shape, w).T
    lam = uniform(shape, -1.0, 1.0, 211 + r)
    for T in (1, 3):
        g, gp = oracle.star_adjoint(lam, w, T, cp=0.25)
        ref = np.linalg.matrix_power(At, T) @ lam.astype(np.float64).ravel()
        refp = 0.25 * sum(np.linalg.matrix_power(At, T - t) @ lam.astype(np.float64).ravel() for t in range(1, T + 1))
        assert relerr(g, ref.reshape(shape)) < 1e-13, (shape, r, T)
        assert np.abs(gp.ravel() - refp).max() <= 1e-13 * max(1.0, np.abs(refp).max())


@pytest.mark.parametrize("r", [2, 3, 4])
def test_star_adjoint_dot_product_identity(r):
    """<F^T(x), y> = <x, adjoint^T(y)> for the linear (diffusion) form, in 2D and 3D."""
    for shape, w, fwd in (((23, 31), STAR[r], oracle.star2d), ((7, 9, 11), STAR3[r], oracle.star3d)):
        x = uniform(shape, -1.0, 1.0, 221 + r)
        y = uniform(shape, -1.0, 1.0, 225 + r)
        for T in (1, 4, 9):
            lhs = float(np.dot(fwd(x, w, T).ravel(), y.astype(np.float64).ravel()))
            g, _ = oracle.star_adjoint(y, w, T)
            rhs = float(np.dot(x.astype(np.float64).ravel(), g.ravel()))
            assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)), (shape, r, T, lhs, rhs)


def test_star_adjoint_radius_one_is_the_radius_one_adjoint():
    """Radius 1 equals the radius-1 oracle adjoint (gradient and grad_p), 2D and 3D."""
    cf = SETS["AH2"]
    w = np.array([cf[0], cf[1], cf[2], cf[4], cf[3]], np.float32)
    lam = uniform((13, 17), -1.0, 1.0, 231)
    g, gp = oracle.star_adjoint(lam, w, 7, cp=float(cf[7]))
    g1, gp1 = oracle.adjoint(lam, cf, 7, form=HOTSPOT)
    assert relerr(g, g1) < 1e-14 and relerr(gp, gp1) < 1e-14
    cf3 = SETS["A3"]
    w3 = np.array([cf3[0], cf3[1], cf3[2], cf3[4], cf3[3], cf3[5], cf3[6]], np.float32)
    lam3 = uniform((5, 6, 7), -1.0, 1.0, 232)
    g3, _ = oracle.star_adjoint(lam3, w3, 5)
    g31, _ = oracle.adjoint(lam3, cf3, 5)
    assert relerr(g3, g31) < 1e-14


def test_star_adjoint_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.star_adjoint(np.zeros(5), STAR[2], 1)
    with pytest.raises(ValueError):
        oracle.star_adjoint(np.zeros((3, 3)), np.zeros(8, np.float32), 1)  # not 1 + 4r weights
    with pytest.raises(ValueError):
        oracle.star_adjoint(np.zeros((3, 3)), STAR[2], -1)
