"""Checks that pin the oracle to facts fixed by the paper and by mathematics.

Each check takes an evaluator ``F(u, v, w, coeffs) -> (su, sv, sw)`` on
halo-1 padded FP64 arrays and returns (name, ok).  They are run against the
oracle (all must hold) and, in the mutation test, against deliberately broken
copies of the brute-force term table (some check must fail for each), so the
suite demonstrably catches a dropped term, a wrong sign, a wrong coefficient,
a wrong stencil index or a wrong field.
"""
from __future__ import annotations

import itertools
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_worked_cell(path=os.path.join(GOLDEN, "worked_cell_1x1x1.txt")):
    fields = {f: np.zeros((3, 3, 3)) for f in "uvw"}
    coeffs, expect = {}, {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "coef":
                coeffs[tok[1]] = float(Fraction(tok[2]))
            elif tok[0] in fields:
                k, j, i = (int(x) for x in tok[1:4])
                fields[tok[0]][k, j, i] = float(Fraction(tok[4]))
            elif tok[0] == "expect":
                expect[tok[1]] = float(Fraction(tok[2]))
    c = dict(tcx=coeffs["tcx"], tcy=coeffs["tcy"],
             **{n: np.array([coeffs[n]]) for n in ("tzc1", "tzc2", "tzd1", "tzd2")})
    return fields, c, expect


def _coeffs(nz, rng, equal_pairs=False):
    tz = {n: rng.choice([0.5, 0.25, 0.125, 0.0625], nz) for n in ("tzc1", "tzc2", "tzd1", "tzd2")}
    if equal_pairs:
        tz["tzc2"] = tz["tzc1"].copy()
        tz["tzd2"] = tz["tzd1"].copy()
    return dict(tcx=0.25, tcy=0.125, **tz)


def _index_grids(nz, ny, nx):
    """Padded-coordinate index arrays k, j, i (FP64) for a halo-1 grid."""
    return np.meshgrid(np.arange(nz + 2.0), np.arange(ny + 2.0), np.arange(nx + 2.0), indexing="ij")


def _inner(a):
    return a[1:-1, 1:-1, 1:-1]


def check_worked_cell(F):
    f, c, e = load_worked_cell()
    su, sv, sw = F(f["u"], f["v"], f["w"], c)
    ok = su.item() == e["su"] and sv.item() == e["sv"] and sw.item() == e["sw"]
    return "worked_cell", ok


def check_zero(F):
    z = np.zeros((5, 6, 7))
    out = F(z, z, z, _coeffs(3, np.random.default_rng(1)))
    return "zero_fields", all(np.all(o == 0) for o in out)


def check_uniform(F):
    """Uniform winds U, V, W: su = 2UW(tzc1-tzc2), sv = 2VW(tzc1-tzc2),
    sw = 2W^2(tzd1-tzd2); zero when the vertical pairs are equal."""
    ok = True
    rng = np.random.default_rng(2)
    nz, ny, nx = 4, 3, 5
    for equal in (False, True):
        c = _coeffs(nz, rng, equal_pairs=equal)
        U, V, W = 3.0, -2.0, 5.0
        shp = (nz + 2, ny + 2, nx + 2)
        su, sv, sw = F(np.full(shp, U), np.full(shp, V), np.full(shp, W), c)
        dz = (c["tzc1"] - c["tzc2"])[:, None, None]
        dd = (c["tzd1"] - c["tzd2"])[:, None, None]
        ok &= np.array_equal(su, np.broadcast_to(2 * U * W * dz, su.shape))
        ok &= np.array_equal(sv, np.broadcast_to(2 * V * W * dz, sv.shape))
        ok &= np.array_equal(sw, np.broadcast_to(2 * W * W * dd, sw.shape))
    return "uniform_winds", bool(ok)


def check_ramps(F):
    """Affine winds along one axis, closed forms derived by hand (the neighbour
    differences of an affine field are constant, so each product term reduces
    to a polynomial in the centre value)."""
    nz, ny, nx = 4, 5, 6
    K, J, I = _index_grids(nz, ny, nx)
    rng = np.random.default_rng(3)
    c = _coeffs(nz, rng)
    tcx, tcy = c["tcx"], c["tcy"]
    z1 = c["tzc1"][:, None, None]
    z2 = c["tzc2"][:, None, None]
    dd = (c["tzd1"] - c["tzd2"])[:, None, None]
    zero = np.zeros_like(K)
    a, b, U, V, W = 2.0, -3.0, 1.5, -0.5, 2.5
    cases = []
    # u = a*i + b, v = w = 0:  su = -6 a tcx u
    u = a * I + b
    cases.append(((u, zero, zero, c), (-6 * a * tcx * _inner(u), 0, 0)))
    # v = a*j + b, u = w = 0:  sv = -6 a tcy v
    v = a * J + b
    cases.append(((zero, v, zero, c), (0, -6 * a * tcy * _inner(v), 0)))
    # w = a*k + b, u = v = 0, tzd1 = tzd2 = t:  sw = -6 a t w
    cc = dict(c, tzd2=c["tzd1"].copy())
    w = a * K + b
    cases.append(((zero, zero, w, cc), (0, 0, -6 * a * cc["tzd1"][:, None, None] * _inner(w))))
    # u = U, v = a*j:  su = -2 a U tcy, sv = -6 a tcy v
    v = a * J
    cases.append(((np.full_like(K, U), v, zero, c), (-2 * a * U * tcy, -6 * a * tcy * _inner(v), 0)))
    # u = U, w = a*k, tzd1 = tzd2 = t:  su = 2U (tzc1 a (k-1) - tzc2 a k), sw = -6 a t w
    w = a * K
    kin = _inner(K)
    cases.append(((np.full_like(K, U), zero, w, cc),
                  (2 * U * (z1 * a * (kin - 1) - z2 * a * kin), 0,
                   -6 * a * cc["tzd1"][:, None, None] * _inner(w))))
    # v = V, w = a*k, tzd1 = tzd2 = t:  sv = 2V (tzc1 a (k-1) - tzc2 a k)
    cases.append(((zero, np.full_like(K, V), w, cc),
                  (0, 2 * V * (z1 * a * (kin - 1) - z2 * a * kin),
                   -6 * a * cc["tzd1"][:, None, None] * _inner(w))))
    # w = W, u = a*i:  su = -6 a tcx u + 2uW(tzc1 - tzc2), sw = -2 W a tcx + 2W^2(tzd1 - tzd2)
    u = a * I
    cases.append(((u, zero, np.full_like(K, W), c),
                  (-6 * a * tcx * _inner(u) + 2 * _inner(u) * W * (z1 - z2), 0,
                   -2 * W * a * tcx + 2 * W * W * dd)))
    # w = W, v = a*j:  sv = -6 a tcy v + 2vW(tzc1 - tzc2), sw = -2 W a tcy + 2W^2(tzd1 - tzd2)
    v = a * J
    cases.append(((zero, v, np.full_like(K, W), c),
                  (0, -6 * a * tcy * _inner(v) + 2 * _inner(v) * W * (z1 - z2),
                   -2 * W * a * tcy + 2 * W * W * dd)))
    # v = V, u = a*i:  su = -6 a tcx u, sv = -2 a V tcx
    u = a * I
    cases.append(((u, np.full_like(K, V), zero, c), (-6 * a * tcx * _inner(u), -2 * a * V * tcx, 0)))
    # u = a*j, v = V:  su = -4 a V tcy, sv = 0
    u = a * J
    cases.append(((u, np.full_like(K, V), zero, c), (-4 * a * V * tcy, 0, 0)))
    # u = a*k + b (vertical shear), w = W:  su = 2W (tzc1 u(k-1) - tzc2 u(k+1)),
    # sw = 2W^2(tzd1 - tzd2)
    u = a * K + b
    uin = _inner(u)
    cases.append(((u, zero, np.full_like(K, W), c),
                  (2 * W * (z1 * (uin - a) - z2 * (uin + a)), 0, 2 * W * W * dd)))
    # v = a*k + b (vertical shear), w = W:  sv = 2W (tzc1 v(k-1) - tzc2 v(k+1)),
    # sw = 2W^2(tzd1 - tzd2)
    v = a * K + b
    vin = _inner(v)
    cases.append(((zero, v, np.full_like(K, W), c),
                  (0, 2 * W * (z1 * (vin - a) - z2 * (vin + a)), 2 * W * W * dd)))
    ok = True
    for (uu, vv, ww, cf), expect in cases:
        out = F(uu, vv, ww, cf)
        for o, e in zip(out, expect):
            ok &= np.array_equal(o, np.broadcast_to(np.asarray(e, dtype=np.float64), o.shape))
    return "affine_closed_forms", bool(ok)


def _periodic(x):
    return np.pad(x, 1, mode="wrap")


def check_energy(F):
    """Quadratic (kinetic-energy) conservation, the defining property of the PW
    form: on a fully periodic grid with tzc1[k] = tzc2[k-1] and
    tzd1[k] = tzd2[k-1] (cyclically), every flux telescopes, so
    sum(u*su) = sum(v*sv) = sum(w*sw) = 0 -- exactly, for integer winds and
    dyadic coefficients.  Checked separately for each direction's term group."""
    rng = np.random.default_rng(4)
    nz, ny, nx = 4, 5, 6
    ok = True
    for trial in range(3):
        ui, vi, wi = (rng.integers(-4, 5, (nz, ny, nx)).astype(np.float64) for _ in range(3))
        u, v, w = _periodic(ui), _periodic(vi), _periodic(wi)
        tzc2 = rng.choice([0.5, 0.25, 0.125], nz)
        tzd2 = rng.choice([0.5, 0.25, 0.125], nz)
        full = dict(tcx=0.25, tcy=0.125, tzc1=np.roll(tzc2, 1), tzc2=tzc2,
                    tzd1=np.roll(tzd2, 1), tzd2=tzd2)
        zt = np.zeros(nz)
        only_x = dict(full, tcy=0.0, tzc1=zt, tzc2=zt, tzd1=zt, tzd2=zt)
        only_y = dict(full, tcx=0.0, tzc1=zt, tzc2=zt, tzd1=zt, tzd2=zt)
        only_z = dict(full, tcx=0.0, tcy=0.0)
        for c in (full, only_x, only_y, only_z):
            su, sv, sw = F(u, v, w, c)
            ok &= np.sum(ui * su) == 0 and np.sum(vi * sv) == 0 and np.sum(wi * sw) == 0
    return "energy_conservation", bool(ok)


def check_homogeneity(F):
    """F(2x) = 4 F(x) bit for bit (scaling by powers of two is exact)."""
    rng = np.random.default_rng(5)
    u, v, w = (rng.uniform(-10, 10, (5, 6, 7)) for _ in range(3))
    c = dict(tcx=0.0025, tcy=0.0025, **{n: rng.uniform(0.5, 1.5, 3) * 0.005
                                         for n in ("tzc1", "tzc2", "tzd1", "tzd2")})
    a = F(u, v, w, c)
    b = F(2 * u, 2 * v, 2 * w, c)
    return "quadratic_homogeneity", all(np.array_equal(4 * x, y) for x, y in zip(a, b))


def check_translation(F):
    """Shifting the periodic winds by one cell in x or y shifts the outputs."""
    rng = np.random.default_rng(6)
    nz, ny, nx = 3, 4, 5
    ui, vi, wi = (rng.integers(-4, 5, (nz, ny, nx)).astype(np.float64) for _ in range(3))
    c = _coeffs(nz, rng)
    base = F(_periodic(ui), _periodic(vi), _periodic(wi), c)
    ok = True
    for axis in (1, 2):
        sh = F(*(_periodic(np.roll(x, 1, axis=axis)) for x in (ui, vi, wi)), c)
        ok &= all(np.array_equal(np.roll(b, 1, axis=axis), s) for b, s in zip(base, sh))
    return "translation_invariance", bool(ok)


ALL_CHECKS = (check_worked_cell, check_zero, check_uniform, check_ramps, check_energy,
              check_homogeneity, check_translation)


def run_all(F):
    return [chk(F) for chk in ALL_CHECKS]


def table_evaluator(table):
    """Vectorised FP64 evaluation of a brute-force style term table (used to run
    the checks on mutated tables)."""
    def F(u, v, w, coeffs):
        fields = dict(u=np.asarray(u, np.float64), v=np.asarray(v, np.float64),
                      w=np.asarray(w, np.float64))
        pz, py, px = fields["u"].shape
        nz, ny, nx = pz - 2, py - 2, px - 2
        out = {o: np.zeros((nz, ny, nx)) for o in ("su", "sv", "sw")}

        def sl(f, off):
            return fields[f][1 + off[0]:1 + off[0] + nz, 1 + off[1]:1 + off[1] + ny,
                             1 + off[2]:1 + off[2] + nx]

        for (o, cname, s, (fa, oa), (fb, ob), (fd, od)) in table:
            cv = coeffs[cname]
            cv = float(cv) if np.ndim(cv) == 0 else np.asarray(cv, np.float64)[:, None, None]
            out[o] = out[o] + s * (cv * (sl(fa, oa) * (sl(fb, ob) + sl(fd, od))))
        return out["su"], out["sv"], out["sw"]
    return F


def table_mutants(table):
    """Every single-row mistake in a term table: a dropped row, a flipped sign,
    another coefficient, an operand offset moved by one (staying inside the
    27-point box) or another field in an operand; yields (name, table)."""
    coefs = ("tcx", "tcy", "tzc1", "tzc2", "tzd1", "tzd2")
    T = list(table)
    for r, (o, c, s, A, B, D) in enumerate(T):
        yield "drop%d" % r, T[:r] + T[r + 1:]
        yield "sign%d" % r, T[:r] + [(o, c, -s, A, B, D)] + T[r + 1:]
        for c2 in coefs:
            if c2 != c:
                yield "coef%d:%s" % (r, c2), T[:r] + [(o, c2, s, A, B, D)] + T[r + 1:]
        for role in range(3):
            f, off = (A, B, D)[role]
            for dim, dd in itertools.product(range(3), (-1, 1)):
                no = list(off)
                no[dim] += dd
                if abs(no[dim]) > 1:
                    continue
                new = [A, B, D]
                new[role] = (f, tuple(no))
                yield "off%d%s%d%+d" % (r, "abd"[role], dim, dd), T[:r] + [(o, c, s, *new)] + T[r + 1:]
            for f2 in "uvw":
                if f2 != f:
                    new = [A, B, D]
                    new[role] = (f2, off)
                    yield "field%d%s:%s" % (r, "abd"[role], f2), T[:r] + [(o, c, s, *new)] + T[r + 1:]
