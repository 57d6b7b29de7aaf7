"""CPU tests: the FP64 oracle against what the paper and mathematics fix.

No GPU.  The checks themselves live in ``pins.py``; here they are run on the
loop oracle (``oracle.forward``), on the exact table encoding
(``oracle.bruteforce``) and on mutated tables, and the adjoint and tangent
operators are pinned by exact finite differences and inner-product identities.
"""
import itertools

import numpy as np
import pytest

import oracle
import pins
from oracle import bruteforce as bf
from paper_2301_13016_amd import workloads as wl


def F_oracle(u, v, w, c):
    return oracle.forward(u, v, w, c)


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pins_hold_on_oracle(check):
    name, ok = check(F_oracle)
    assert ok, name


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pins_hold_on_exact_table(check):
    name, ok = check(pins.table_evaluator(bf.TERMS))
    assert ok, name


def test_every_plausible_table_mistake_is_caught():
    """A dropped term, flipped sign, wrong coefficient, stencil index moved by
    one in any direction, or wrong field in any operand of any of the 18 terms
    makes at least one pin fail (510 mutants)."""
    survivors = []
    n = 0
    for name, table in pins.table_mutants(bf.TERMS):
        n += 1
        if all(ok for _, ok in pins.run_all(pins.table_evaluator(table))):
            survivors.append(name)
    assert n == 510
    assert survivors == []


def test_table_structure_matches_paper_counts():
    """Per field and cell: six face sums (twelve addition operands), six
    products with one neighbour each (six multiplication operands), and the
    same coefficient/sign pattern for all three fields (paper Sec. 4); every
    operand lies inside the 27-point box of a depth-one stencil (Sec. 2.2)."""
    for o in bf.OUTPUTS:
        rows = [t for t in bf.TERMS if t[0] == o]
        assert len(rows) == 6
        assert [r[2] for r in rows] == [+1, -1, +1, -1, +1, -1]
        kinds = ["z" if r[1].startswith("tz") else r[1] for r in rows]
        assert kinds == ["tcx", "tcx", "tcy", "tcy", "z", "z"]
        operands = [x for r in rows for x in r[3:]]
        assert len(operands) == 18   # 6 multiplicands + 12 face operands
        for _, off in operands:
            assert all(abs(d) <= 1 for d in off)
        # the advected field is always the multiplicand a
        assert {r[3][0] for r in rows} == {o[1]}
        # face operands are one component per direction: u for x, v for y, w for z
        assert [r[4][0] for r in rows] == [r[5][0] for r in rows]


@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 3, 2), (1, 1, 1)])
def test_bruteforce_equals_oracle_bitwise(shape):
    """Integer winds + dyadic coefficients make every intermediate exact, so the
    rational table evaluation and the FP64 loops must agree bit for bit at every
    point (the 4^3 case covers all 64 points of a 4^3 grid)."""
    nx, ny, nz = shape
    g = wl.integer_grid(nx, ny, nz, seed=11, dtype=np.float64)
    exact = bf.forward_exact(dict(u=g.u, v=g.v, w=g.w), g.coeffs)
    got = oracle.forward(g.u, g.v, g.w, g.coeffs)
    for o, x in zip(bf.OUTPUTS, got):
        assert np.array_equal(bf.to_float_array(exact[o]), x), o


def test_magnitude_bounds_outputs():
    g = wl.make_grid(9, 7, 5, seed=12, dtype=np.float64)
    out, mag = oracle.forward(g.u, g.v, g.w, g.coeffs, magnitude=True)
    absF = oracle.forward(np.abs(g.u), np.abs(g.v), np.abs(g.w),
                          dict(g.coeffs, tcx=abs(g.tcx), tcy=abs(g.tcy)), magnitude=True)[1]
    for o, m, a in zip(out, mag, absF):
        assert np.all(np.abs(o) <= m * (1 + 1e-12))
        assert np.allclose(m, a, rtol=1e-14, atol=0)


def test_threads_do_not_change_results():
    g = wl.make_grid(17, 13, 11, seed=13, dtype=np.float64)
    a = oracle.forward(g.u, g.v, g.w, g.coeffs, nthreads=1)
    b = oracle.forward(g.u, g.v, g.w, g.coeffs, nthreads=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------- adjoint / tangent

def test_adjoint_equals_exact_rational_differences():
    """J^T r from the scatter oracle equals, bit for bit, the exact central
    differences of the rational forward operator (F is quadratic, so the
    difference quotient is exact), on a ragged 3x2x2 grid, halo included."""
    g = wl.integer_grid(3, 2, 2, seed=14, dtype=np.float64)
    rng = np.random.default_rng(15)
    r = [rng.integers(-3, 4, (2, 2, 3)).astype(np.float64) for _ in range(3)]
    exact = bf.adjoint_exact(dict(u=g.u, v=g.v, w=g.w), g.coeffs, dict(su=r[0], sv=r[1], sw=r[2]))
    got = oracle.adjoint(g.u, g.v, g.w, g.coeffs, *r)
    for f, x in zip(bf.FIELDS, got):
        assert np.array_equal(bf.to_float_array(exact[f]), x), f


def _dot(a, b):
    return float(sum(np.sum(np.asarray(x, np.float64) * np.asarray(y, np.float64)) for x, y in zip(a, b)))


def test_adjoint_finite_difference_fp64():
    """FP64 central finite differences on a 16^3 grid (eps = 1e-6, seed 40):
    <(F(x + eps d) - F(x - eps d)) / 2eps, y> = <d, J^T y>.  F is quadratic,
    so the quotient has no truncation error and only roundoff remains."""
    cfg = wl.C4_FD
    g = wl.make_grid(cfg["nx"], cfg["ny"], cfg["nz"], cfg["seed"], dtype=np.float64)
    d = wl.direction(cfg["nx"], cfg["ny"], cfg["nz"], cfg["seed"] + 1)
    y = wl.cotangents(cfg["nx"], cfg["ny"], cfg["nz"], cfg["seed"] + 2, dtype=np.float64)
    eps = cfg["eps"]
    x = (g.u, g.v, g.w)
    fp = oracle.forward(*(a + eps * b for a, b in zip(x, d)), g.coeffs)
    fm = oracle.forward(*(a - eps * b for a, b in zip(x, d)), g.coeffs)
    jd_fd = [(p - m) / (2 * eps) for p, m in zip(fp, fm)]
    jty = oracle.adjoint(*x, g.coeffs, *y)
    lhs, rhs = _dot(jd_fd, y), _dot(d, jty)
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)
    # element-wise against the tangent-linear operator
    jd = oracle.tangent(*x, *d, g.coeffs)
    for a, b in zip(jd_fd, jd):
        assert np.max(np.abs(a - b)) <= 1e-8 * np.max(np.abs(b))


def test_tangent_equals_exact_rational_differences():
    """J(x) d from the tangent oracle equals, bit for bit, the exact central
    difference (F(x + d) - F(x - d)) / 2 of the rational forward operator (F is
    quadratic, so the quotient is exact), on integer data with dyadic
    coefficients where every FP64 intermediate is exact."""
    g = wl.integer_grid(4, 3, 3, seed=24, dtype=np.float64)
    rng = np.random.default_rng(25)
    d = [rng.integers(-3, 4, g.u.shape).astype(np.float64) for _ in range(3)]
    x = dict(u=g.u, v=g.v, w=g.w)
    fp = bf.forward_exact({f: x[f] + dd for f, dd in zip(bf.FIELDS, d)}, g.coeffs)
    fm = bf.forward_exact({f: x[f] - dd for f, dd in zip(bf.FIELDS, d)}, g.coeffs)
    got = oracle.tangent(g.u, g.v, g.w, *d, g.coeffs)
    for o, a in zip(bf.OUTPUTS, got):
        exact = np.array([[[(p - m) / 2 for p, m in zip(rp, rm)] for rp, rm in zip(pp, mm)]
                          for pp, mm in zip(fp[o], fm[o])], dtype=object)
        assert np.array_equal(bf.to_float_array(exact), a), o


def test_tangent_polarisation_and_dot_product():
    """For a homogeneous quadratic F: J(x) d = F(x + d) - F(x) - F(d), and
    <J d, y> = <d, J^T y> (the dot-product test)."""
    g = wl.make_grid(12, 9, 7, seed=16, dtype=np.float64)
    d = wl.direction(12, 9, 7, seed=17)
    y = wl.cotangents(12, 9, 7, seed=18, dtype=np.float64)
    x = (g.u, g.v, g.w)
    jd = oracle.tangent(*x, *d, g.coeffs)
    pol = [a - b - c for a, b, c in zip(oracle.forward(*(p + q for p, q in zip(x, d)), g.coeffs),
                                        oracle.forward(*x, g.coeffs), oracle.forward(*d, g.coeffs))]
    for a, b in zip(jd, pol):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
    jty = oracle.adjoint(*x, g.coeffs, *y)
    assert abs(_dot(jd, y) - _dot(d, jty)) <= 1e-12 * abs(_dot(d, jty))


def test_adjoint_euler_and_symmetry_identities():
    """F(x) = B(x, x) with B symmetric bilinear, so J(x)^T y is linear in x:
    Euler <x, J^T(x) y> = 2 <F(x), y>, and symmetry <d, J^T(x) y> = <x, J^T(d) y>."""
    g = wl.make_grid(10, 8, 6, seed=19, dtype=np.float64)
    d = wl.direction(10, 8, 6, seed=20)
    y = wl.cotangents(10, 8, 6, seed=21, dtype=np.float64)
    x = (g.u, g.v, g.w)
    jx = oracle.adjoint(*x, g.coeffs, *y)
    fx = oracle.forward(*x, g.coeffs)
    assert abs(_dot(x, jx) - 2 * _dot(fx, y)) <= 1e-12 * abs(_dot(x, jx))
    jd = oracle.adjoint(*d, g.coeffs, *y)
    assert abs(_dot(d, jx) - _dot(x, jd)) <= 1e-12 * abs(_dot(d, jx))


def test_adjoint_gradient_halo_is_written():
    """The gradient covers the padded arrays: halo entries that some interior
    output reads get non-zero gradient, the 3-D corners of the halo (read by no
    output) get exactly zero."""
    g = wl.make_grid(5, 4, 3, seed=22, dtype=np.float64)
    y = wl.cotangents(5, 4, 3, seed=23, dtype=np.float64)
    gu, gv, gw = oracle.adjoint(g.u, g.v, g.w, g.coeffs, *y)
    for gr in (gu, gv, gw):
        for k, j, i in itertools.product((0, -1), (0, -1), (0, -1)):
            assert gr[k, j, i] == 0.0
        assert np.any(gr[0] != 0) or np.any(gr[-1] != 0)


# ---------------------------------------------------------------- coefficient gradients

def _unit_coeffs(nz, name, k=None):
    c = dict(tcx=0.0, tcy=0.0, tzc1=np.zeros(nz), tzc2=np.zeros(nz), tzd1=np.zeros(nz), tzd2=np.zeros(nz))
    if name in ("tcx", "tcy"):
        c[name] = 1.0
    else:
        c[name][k] = 1.0
    return c


def test_coeff_grad_is_forward_with_unit_coefficients():
    """The loss is linear in every coefficient, so dL/dc = <F(x; c = 1, all
    others 0), r> -- the forward oracle with a unit coefficient, an
    evaluation path independent of the gradient loops."""
    g = wl.make_grid(7, 5, 4, seed=26, dtype=np.float64)
    r = wl.cotangents(7, 5, 4, seed=27, dtype=np.float64)
    x = (g.u, g.v, g.w)
    got = oracle.coeff_grad(*x, *r)
    for name in ("tcx", "tcy"):
        ref = _dot(oracle.forward(*x, _unit_coeffs(4, name)), r)
        assert abs(got[name] - ref) <= 1e-13 * max(1.0, abs(ref)), name
    for name in ("tzc1", "tzc2", "tzd1", "tzd2"):
        for k in range(4):
            ref = _dot(oracle.forward(*x, _unit_coeffs(4, name, k)), r)
            assert abs(got[name][k] - ref) <= 1e-13 * max(1.0, abs(ref)), (name, k)
    assert abs(sum(got["tcx_level"]) - got["tcx"]) <= 1e-13 * abs(got["tcx"])
    assert abs(sum(got["tcy_level"]) - got["tcy"]) <= 1e-13 * abs(got["tcy"])


def test_coeff_grad_exact_on_integers():
    """Bit for bit against the exact rational forward operator with unit
    coefficients, on integer winds and cotangents (every FP64 step exact)."""
    g = wl.integer_grid(3, 3, 2, seed=28, dtype=np.float64)
    rng = np.random.default_rng(29)
    r = [rng.integers(-3, 4, (2, 3, 3)).astype(np.float64) for _ in range(3)]
    x = dict(u=g.u, v=g.v, w=g.w)
    got = oracle.coeff_grad(g.u, g.v, g.w, *r)

    def exact(c):
        f = bf.forward_exact(x, c)
        return sum(float(sum(f[o][k][j][i] * int(r[n][k, j, i]) for k in range(2) for j in range(3) for i in range(3)))
                   for n, o in enumerate(bf.OUTPUTS))
    assert got["tcx"] == exact(_unit_coeffs(2, "tcx"))
    assert got["tcy"] == exact(_unit_coeffs(2, "tcy"))
    for name in ("tzc1", "tzc2", "tzd1", "tzd2"):
        for k in range(2):
            assert got[name][k] == exact(_unit_coeffs(2, name, k)), (name, k)


def test_coeff_grad_euler_identity():
    """Summing c * dL/dc over all coefficients gives L itself (L is linear and
    homogeneous of degree one in the coefficients)."""
    g = wl.make_grid(9, 6, 5, seed=30, dtype=np.float64)
    r = wl.cotangents(9, 6, 5, seed=31, dtype=np.float64)
    got = oracle.coeff_grad(g.u, g.v, g.w, *r)
    total = g.tcx * got["tcx"] + g.tcy * got["tcy"] + sum(float(np.dot(getattr(g, n), got[n]))
                                                         for n in ("tzc1", "tzc2", "tzd1", "tzd2"))
    loss = _dot(oracle.forward(g.u, g.v, g.w, g.coeffs), r)
    assert abs(total - loss) <= 1e-12 * abs(loss)


# ---------------------------------------------------------------- halo fill

def test_halo_fill_matches_numpy_pad():
    """Periodic, copy and zero fills equal numpy's pad of the interior with
    wrap, edge and constant modes (an independent implementation of the same
    boundary rules), for halos 1 and 2, per axis and mixed."""
    from oracle import halo as H
    rng = np.random.default_rng(32)
    np_mode = dict(periodic="wrap", copy="edge", zero="constant", reflect="symmetric")
    for h in (1, 2):
        interior = rng.uniform(-1, 1, (3, 4, 5))
        a = rng.uniform(-1, 1, tuple(s + 2 * h for s in interior.shape))
        a[h:-h, h:-h, h:-h] = interior
        for modes in [("periodic",) * 3, ("copy",) * 3, ("zero",) * 3, ("reflect",) * 3,
                      ("periodic", "periodic", "copy"), ("copy", "zero", "periodic"),
                      ("periodic", "reflect", "zero")]:
            ref = interior
            for ax, m in ((2, modes[0]), (1, modes[1]), (0, modes[2])):
                pw = [(0, 0)] * 3
                pw[ax] = (h, h)
                ref = np.pad(ref, pw, mode=np_mode[m])
            got = H.fill(a, h, modes)
            assert np.array_equal(got, ref), (h, modes)


def test_halo_fill_reflect_neg_vanishes_on_the_face():
    """reflect_neg makes the mean of each mirrored pair zero: the linear
    interpolant of the field vanishes on the boundary face, for every
    halo depth (brute force over the pairs); on the other axes the cells
    equal numpy's symmetric pad."""
    from oracle import halo as H
    rng = np.random.default_rng(35)
    for h in (1, 2, 3):
        a = rng.uniform(-1, 1, (4 + 2 * h, 3 + 2 * h, 5 + 2 * h))
        got = H.fill(a, h, ("periodic", "periodic", "reflect_neg"))
        nz = 4
        for q in range(h):
            assert np.array_equal(got[h - 1 - q], -got[h + q])
            assert np.array_equal(got[nz + h + q], -got[nz + h - 1 - q])
        sym = H.fill(a, h, ("periodic", "periodic", "reflect"))
        assert np.array_equal(got[h:-h], sym[h:-h])
        assert np.array_equal(got[:h], -sym[:h]) and np.array_equal(got[-h:], -sym[-h:])
    with pytest.raises(ValueError):
        H.fill(np.zeros((7, 7, 5)), 2, ("reflect", "keep", "keep"))


def test_halo_fill_signed_zero_follows_the_axis_order():
    """Edges and corners take the sequential x, y, z fill's value, sign of
    zero included: a cell zeroed by an earlier axis and negated by a later
    one is -0, a cell negated first and zeroed later is +0 (checked cell by
    cell against the order of the two operations)."""
    from oracle import halo as H
    a = np.full((3, 4, 5), 7.0)
    got = H.fill(a, 1, ("zero", "reflect_neg", "keep"))
    corner = got[:, 0, 0]                      # x halo (zeroed), then y halo (negated)
    assert np.all(corner == 0) and np.all(np.signbit(corner))
    assert np.all(got[:, 1:-1, 0] == 0) and not np.any(np.signbit(got[:, 1:-1, 0]))
    assert np.all(got[:, 0, 1:-1] == -7.0)
    got = H.fill(a, 1, ("reflect_neg", "zero", "keep"))
    assert np.all(got[:, 0, :] == 0) and not np.any(np.signbit(got[:, 0, :]))
    got = H.fill(a, 1, ("zero", "reflect_neg", "reflect_neg"))
    assert not np.any(np.signbit(got[0, 0, 0:1]))   # negated twice after the zero: +0


def test_halo_fill_keep_and_wide_periodic():
    """keep leaves an axis' halo alone; a halo wider than the interior wraps
    more than once (brute-force index arithmetic)."""
    from oracle import halo as H
    rng = np.random.default_rng(33)
    a = rng.uniform(-1, 1, (5, 6, 7))       # h = 2: interior 1 x 2 x 3
    got = H.fill(a, 2, ("periodic", "keep", "keep"))
    assert np.array_equal(got[:, :, 2:5], a[:, :, 2:5])
    for i in (0, 1, 5, 6):
        assert np.array_equal(got[:, :, i], a[:, :, 2 + (i - 2) % 3])
    b = rng.uniform(-1, 1, (1 + 6, 1 + 6, 1 + 6))   # h = 3, n = 1: every halo cell is the one interior cell
    g2 = H.fill(b, 3, ("periodic",) * 3)
    assert np.all(g2 == b[3, 3, 3])


def test_periodic_fill_conserves_energy():
    """With halos filled periodically by the halo oracle, the forward
    operator conserves sum(u su) + ... exactly on integer winds with the
    cyclic coefficient pairing -- the same property the padded-by-numpy grids
    show, so the fill reproduces a periodic domain."""
    from oracle import halo as H
    rng = np.random.default_rng(34)
    nz, ny, nx = 4, 5, 6
    ui, vi, wi = (rng.integers(-4, 5, (nz, ny, nx)).astype(np.float64) for _ in range(3))
    pads = []
    for x in (ui, vi, wi):
        a = rng.uniform(-9, 9, (nz + 2, ny + 2, nx + 2))
        a[1:-1, 1:-1, 1:-1] = x
        pads.append(H.fill(a, 1, ("periodic",) * 3))
    tzc2 = rng.choice([0.5, 0.25, 0.125], nz)
    tzd2 = rng.choice([0.5, 0.25, 0.125], nz)
    c = dict(tcx=0.25, tcy=0.125, tzc1=np.roll(tzc2, 1), tzc2=tzc2, tzd1=np.roll(tzd2, 1), tzd2=tzd2)
    su, sv, sw = oracle.forward(*pads, c)
    assert np.sum(ui * su) + np.sum(vi * sv) + np.sum(wi * sw) == 0



def test_halo_fold_is_the_transpose_of_the_fill():
    """fold = fill^T, checked against the explicit matrix of the fill built
    column by column from unit vectors on tiny grids (exact: every entry of
    the matrix is 0 or +-1), for every mode combination."""
    from oracle import halo as H
    rng = np.random.default_rng(36)
    for h, shape in ((1, (2 + 2, 1 + 2, 3 + 2)), (2, (2 + 4, 2 + 4, 3 + 4))):
        size = int(np.prod(shape))
        for modes in itertools.product(H.MODES, repeat=3):
            if any(m.startswith("reflect") and n < h for m, n in zip(modes, (shape[2] - 2 * h, shape[1] - 2 * h,
                                                                              shape[0] - 2 * h))):
                continue
            M = np.empty((size, size))
            for c in range(size):
                e = np.zeros(size)
                e[c] = 1.0
                M[:, c] = H.fill(e.reshape(shape), h, modes).ravel()
            y = rng.integers(-5, 6, shape).astype(np.float64)
            assert np.array_equal(H.fold(y, h, modes).ravel(), M.T @ y.ravel()), (h, modes)


def test_halo_fold_dot_product_identity():
    """<fill(x), y> = <x, fold(y)> on random data, larger grids, mixed rules."""
    from oracle import halo as H
    rng = np.random.default_rng(37)
    for h, modes in ((1, ("periodic", "copy", "reflect_neg")), (2, ("reflect", "periodic", "zero")),
                     (3, ("periodic", "periodic", "periodic")), (1, ("keep", "zero", "copy"))):
        shape = (5 + 2 * h, 4 + 2 * h, 7 + 2 * h)
        x = rng.uniform(-1, 1, shape)
        y = rng.uniform(-1, 1, shape)
        lhs = float(np.sum(H.fill(x, h, modes) * y))
        rhs = float(np.sum(x * H.fold(y, h, modes)))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs)), (h, modes)
