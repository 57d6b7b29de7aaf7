"""CPU tests: the error scales that every GPU parity gate divides by.

A GPU result is compared with the oracle as |GPU - oracle| / scale, so a scale
that is too large (a doubled term, a term counted at the wrong cell) would
loosen every gate without any test failing.  Here each scale is pinned to
something other than its own code:

* A(p), the forward scale the oracle returns (``magnitude=True``), is
  compared bit for bit with its definition -- the sum over the point's six
  products of |coefficient| * |a| * (|b| + |d|) (paper, Sec. 4 and Fig. 2:
  six face sums, six products per field) -- evaluated on the brute-force term
  table, which is itself pinned by ``test_oracle_pins.py``; with closed forms
  for uniform winds and for single non-zero cells; and every plausible
  mistake in the oracle's C expressions for A (a dropped or doubled term, a
  wrong coefficient, field or offset, a missing absolute value) is compiled
  and shown to fail these pins.
* The adjoint scale is the exact gradient of sum_p |r_p| A_p(x) on the
  positive orthant (central differences of the pinned A, exact for a
  quadratic with integer data), and every table mistake fails that pin.
* The tangent scale is the exact directional derivative of A, and pairs with
  the adjoint scale in a dot-product identity.
* The coefficient-gradient scale satisfies Euler's identity for A, which is
  linear in |c|, and is the exact difference of A under a unit coefficient.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import pins
import scales
from oracle import bruteforce as bf

COEFS = ("tcx", "tcy", "tzc1", "tzc2", "tzd1", "tzd2")
DYADIC = np.array([0.5, 0.25, 0.125, 0.0625, 0.03125])


def signed_grid(nx, ny, nz, seed, halo=1, lo=-4, hi=4):
    """Integer winds of both signs and dyadic coefficients of both signs,
    distinct per level: every FP64 operation on them is exact."""
    rng = np.random.default_rng(seed)
    shp = (nz + 2 * halo, ny + 2 * halo, nx + 2 * halo)
    u, v, w = (rng.integers(lo, hi + 1, shp).astype(np.float64) for _ in range(3))
    sgn = lambda n: rng.choice([-1.0, 1.0], n)  # noqa: E731
    c = dict(tcx=0.25, tcy=-0.125, **{n: sgn(nz) * rng.choice(DYADIC, nz) for n in COEFS[2:]})
    return (u, v, w), c


def table_scale(u, v, w, coeffs, halo=1, terms=bf.TERMS):
    """A(p) from its definition on a term table: for every output the sum over
    its rows of |c| * |a| * (|b| + |d|)."""
    f = dict(u=np.abs(u), v=np.abs(v), w=np.abs(w))
    pz, py, px = u.shape
    nz, ny, nx = pz - 2 * halo, py - 2 * halo, px - 2 * halo
    out = {o: np.zeros((nz, ny, nx)) for o in bf.OUTPUTS}

    def sl(name, off):
        return f[name][halo + off[0]:halo + off[0] + nz, halo + off[1]:halo + off[1] + ny,
                       halo + off[2]:halo + off[2] + nx]

    for (o, cname, _s, (fa, oa), (fb, ob), (fd, od)) in terms:
        c = coeffs[cname]
        c = abs(float(c)) if np.ndim(c) == 0 else np.abs(np.asarray(c, np.float64))[:, None, None]
        out[o] = out[o] + c * (sl(fa, oa) * (sl(fb, ob) + sl(fd, od)))
    return out["su"], out["sv"], out["sw"]


def oracle_scale(u, v, w, c, halo=1):
    return oracle.forward(u, v, w, c, halo=halo, magnitude=True)[1]


# ---------------------------------------------------------------- pins of A(p)

def pin_table_bitwise(scale_fn):
    """A equals its definition on the pinned term table, bit for bit, on
    signed integer grids (ragged, halo 1)."""
    for shape, seed in (((5, 4, 3), 61), ((4, 4, 4), 62), ((1, 1, 1), 63), ((7, 2, 3), 64)):
        (u, v, w), c = signed_grid(*shape, seed)
        got = scale_fn(u, v, w, c)
        for a, b in zip(got, table_scale(u, v, w, c)):
            if not np.array_equal(a, b):
                return False
    return True


def pin_uniform_closed_form(scale_fn):
    """Uniform winds U, V, W: every face sum is 2x a wind, so (by hand)
    A_u = |U| (4|tcx||U| + 4|tcy||V| + 2|W|(|tzc1| + |tzc2|)),
    A_v = |V| (4|tcx||U| + 4|tcy||V| + 2|W|(|tzc1| + |tzc2|)),
    A_w = |W| (4|tcx||U| + 4|tcy||V| + 2|W|(|tzd1| + |tzd2|))."""
    rng = np.random.default_rng(65)
    nz, ny, nx = 3, 4, 5
    for U, V, W in ((3.0, -2.0, 5.0), (-1.0, 4.0, -3.0)):
        c = dict(tcx=-0.25, tcy=0.125, **{n: rng.choice([-1.0, 1.0], nz) * rng.choice(DYADIC, nz)
                                           for n in COEFS[2:]})
        shp = (nz + 2, ny + 2, nx + 2)
        au, av, aw = scale_fn(np.full(shp, U), np.full(shp, V), np.full(shp, W), c)
        t = lambda n: np.abs(c[n])[:, None, None]  # noqa: E731
        horiz = 4 * abs(c["tcx"]) * abs(U) + 4 * abs(c["tcy"]) * abs(V)
        eu = abs(U) * (horiz + 2 * abs(W) * (t("tzc1") + t("tzc2")))
        ev = abs(V) * (horiz + 2 * abs(W) * (t("tzc1") + t("tzc2")))
        ew = abs(W) * (horiz + 2 * abs(W) * (t("tzd1") + t("tzd2")))
        for a, e in ((au, eu), (av, ev), (aw, ew)):
            if not np.array_equal(a, np.broadcast_to(e, a.shape)):
                return False
    return True


def pin_single_cells(scale_fn):
    """One non-zero value x at cell q of a single field, all else zero: a
    product a (b + d) is non-zero only where a and one of b, d are that cell.
    So (by hand) u at q gives A_u = |tcx| x^2 at q -+ one cell in x; v at q
    gives A_v = |tcy| x^2 at q -+ one cell in y; w at q gives A_w =
    |tzd1[k]| x^2 at q + one level and |tzd2[k]| x^2 at q - one level;
    every other entry is zero."""
    nz, ny, nx = 4, 5, 6
    rng = np.random.default_rng(66)
    c = dict(tcx=0.25, tcy=-0.125, **{n: rng.choice([-1.0, 1.0], nz) * rng.choice(DYADIC, nz)
                                       for n in COEFS[2:]})
    x = -3.0
    q = (2, 3, 3)                      # padded coordinates, well inside
    shp = (nz + 2, ny + 2, nx + 2)
    for field in range(3):
        fields = [np.zeros(shp) for _ in range(3)]
        fields[field][q] = x
        got = scale_fn(*fields, c)
        want = [np.zeros((nz, ny, nx)) for _ in range(3)]
        k, j, i = q[0] - 1, q[1] - 1, q[2] - 1          # interior coordinates of q
        if field == 0:
            want[0][k, j, i + 1] = want[0][k, j, i - 1] = abs(c["tcx"]) * x * x
        elif field == 1:
            want[1][k, j + 1, i] = want[1][k, j - 1, i] = abs(c["tcy"]) * x * x
        else:
            want[2][k + 1, j, i] = abs(c["tzd1"][k + 1]) * x * x
            want[2][k - 1, j, i] = abs(c["tzd2"][k - 1]) * x * x
        if not all(np.array_equal(a, b) for a, b in zip(got, want)):
            return False
    return True


SCALE_PINS = (pin_table_bitwise, pin_uniform_closed_form, pin_single_cells)


@pytest.mark.parametrize("pin", SCALE_PINS, ids=lambda p: p.__name__)
def test_oracle_scale_holds_pin(pin):
    assert pin(oracle_scale)


def test_oracle_scale_wider_halo_and_threads():
    """Halo 2 (the stencil still reads one cell) and several threads give the
    definition's values bit for bit."""
    (u, v, w), c = signed_grid(6, 3, 4, seed=67, halo=2)
    for n in (1, 3):
        got = oracle.forward(u, v, w, c, halo=2, magnitude=True, nthreads=n)[1]
        for a, b in zip(got, table_scale(u, v, w, c, halo=2)):
            assert np.array_equal(a, b)


# ------------------------------------------- mutation sweep over the oracle's C code

_TERM = re.compile(
    r"^(?P<lead>\s*(?:(?P<out>mag_[uvw])\[o\] =|\+))\s*"
    r"fabs\((?P<c>[a-z0-9]+(?:\[kk\])?)\) \* fabs\((?P<fa>[UVW])\((?P<ia>[^)]*)\)\) \* "
    r"\(fabs\((?P<fb>[UVW])\((?P<ib>[^)]*)\)\) \+ fabs\((?P<fd>[UVW])\((?P<id>[^)]*)\)\)\)"
    r"(?P<end>;?)\s*$")
_CNAMES = ("tcx", "tcy", "tzc1[kk]", "tzc2[kk]", "tzd1[kk]", "tzd2[kk]")


def _parse_index(txt):
    offs = []
    for comp, var in zip(txt.split(","), "kji"):
        m = re.fullmatch(r"\s*%s(?:\s*([+-])\s*1)?\s*" % var, comp)
        assert m, txt
        offs.append(0 if m.group(1) is None else (1 if m.group(1) == "+" else -1))
    return offs


def _fmt_index(offs):
    return ", ".join(var + ("" if o == 0 else " %s %d" % ("+" if o > 0 else "-", abs(o)))
                     for var, o in zip("kji", offs))


def oracle_scale_terms():
    """The 18 terms of the oracle's C expressions for A, parsed from the
    source: (output, coefficient, [(field, offsets)] for a, b, d)."""
    src = open(os.path.join(os.path.dirname(oracle.__file__), "pw_oracle.c")).read()
    terms, out = [], None
    for line in src.splitlines():
        m = _TERM.match(line)
        if not m:
            continue
        out = m.group("out") or out
        terms.append((out, m.group("c"), [(m.group("f" + r), _parse_index(m.group("i" + r))) for r in "abd"]))
        # the parse reproduces the line exactly
        assert _term_text(terms[-1][1], terms[-1][2]) in line
    assert len(terms) == 18
    return terms


def _term_text(c, ops, abs_c=True, abs_ops=(True, True, True), plus=True):
    def op(k):
        f, offs = ops[k]
        t = "%s(%s)" % (f, _fmt_index(offs))
        return "fabs(%s)" % t if abs_ops[k] else "(%s)" % t
    cc = "fabs(%s)" % c if abs_c else "(%s)" % c
    return "%s * %s * (%s %s %s)" % (cc, op(0), op(1), "+" if plus else "-", op(2))


def scale_mutants(terms):
    """(name, list of 18 term texts or None for a dropped term, output
    permutation) for every single mistake in one term, plus whole-expression
    mistakes."""
    base = [_term_text(c, ops) for (_, c, ops) in terms]
    ident = {"mag_u": "mag_u", "mag_v": "mag_v", "mag_w": "mag_w"}
    yield "none", base, ident
    for t, (_, c, ops) in enumerate(terms):
        def put(txt):
            return base[:t] + [txt] + base[t + 1:]
        yield "drop%d" % t, put("0.0"), ident
        yield "double%d" % t, put("2.0 * (%s)" % base[t]), ident
        yield "minus%d" % t, put(_term_text(c, ops, plus=False)), ident
        yield "nofabs_c%d" % t, put(_term_text(c, ops, abs_c=False)), ident
        for r in range(3):
            yield "nofabs%d%s" % (t, "abd"[r]), put(_term_text(c, ops, abs_ops=tuple(q != r for q in range(3)))), ident
        for c2 in _CNAMES:
            if c2 != c:
                yield "coef%d:%s" % (t, c2), put(_term_text(c2, ops)), ident
        for r in range(3):
            f, offs = ops[r]
            for f2 in "UVW":
                if f2 != f:
                    new = list(ops)
                    new[r] = (f2, offs)
                    yield "field%d%s:%s" % (t, "abd"[r], f2), put(_term_text(c, new)), ident
            for dim in range(3):
                for dd in (-1, 1):
                    o2 = list(offs)
                    o2[dim] += dd
                    if abs(o2[dim]) > 1:
                        continue
                    new = list(ops)
                    new[r] = (f, o2)
                    yield "off%d%s%d%+d" % (t, "abd"[r], dim, dd), put(_term_text(c, new)), ident
    for out in ("mag_u", "mag_v", "mag_w"):
        yield "whole_double:" + out, [("2.0 * (%s)" % x if terms[t][0] == out else x) for t, x in enumerate(base)], ident
    yield "swap_uv", base, {"mag_u": "mag_v", "mag_v": "mag_u", "mag_w": "mag_w"}


_PRELUDE = r"""
#include <math.h>
#include <stdint.h>
#define IDX(k, j, i) ((((int64_t)(k)) * py + (int64_t)(j)) * px + (int64_t)(i))
#define U(k, j, i) u[IDX(k, j, i)]
#define V(k, j, i) v[IDX(k, j, i)]
#define W(k, j, i) w[IDX(k, j, i)]
"""


def _mutant_function(n, texts, terms, outmap):
    stmts = {}
    for (out, _, _), txt in zip(terms, texts):
        stmts.setdefault(outmap[out], []).append(txt)
    body = "\n".join("            %s[o] = %s;" % (out, "\n                + ".join(t)) for out, t in sorted(stmts.items()))
    return r"""
void mag_mut_%d(int64_t nx, int64_t ny, int64_t nz, int64_t h,
                const double *u, const double *v, const double *w, double tcx, double tcy,
                const double *tzc1, const double *tzc2, const double *tzd1, const double *tzd2,
                double *mag_u, double *mag_v, double *mag_w)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    (void)tcx; (void)tcy; (void)tzc1; (void)tzc2; (void)tzd1; (void)tzd2;
    for (int64_t k = h; k < h + nz; ++k)
      for (int64_t j = h; j < h + ny; ++j)
        for (int64_t i = h; i < h + nx; ++i) {
            const int64_t kk = k - h;
            const int64_t o = (kk * ny + (j - h)) * nx + (i - h);
%s
        }
}
""" % (n, body)


@pytest.fixture(scope="module")
def mutant_library(tmp_path_factory):
    terms = oracle_scale_terms()
    muts = list(scale_mutants(terms))
    src = _PRELUDE + "".join(_mutant_function(n, texts, terms, om) for n, (_, texts, om) in enumerate(muts))
    d = tmp_path_factory.mktemp("scale_mutants")
    c_path, so_path = d / "mutants.c", d / "libmutants.so"
    c_path.write_text(src)
    subprocess.run(["gcc", "-O0", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                    "-o", str(so_path), str(c_path), "-lm"], check=True)
    lib = ctypes.CDLL(str(so_path))
    return lib, muts


def _mutant_scale(lib, n):
    fn = getattr(lib, "mag_mut_%d" % n)
    i64, dbl, p = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    fn.argtypes = [i64] * 4 + [p] * 3 + [dbl, dbl] + [p] * 4 + [p] * 3
    fn.restype = None

    def scale(u, v, w, c, halo=1):
        u, v, w = (np.ascontiguousarray(x, np.float64) for x in (u, v, w))
        pz, py, px = u.shape
        nz, ny, nx = pz - 2 * halo, py - 2 * halo, px - 2 * halo
        tz = [np.ascontiguousarray(c[n], np.float64) for n in COEFS[2:]]
        out = [np.zeros((nz, ny, nx)) for _ in range(3)]
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        fn(nx, ny, nz, halo, ptr(u), ptr(v), ptr(w), float(c["tcx"]), float(c["tcy"]),
           *[ptr(t) for t in tz], *[ptr(o) for o in out])
        return tuple(out)
    return scale


def test_unmutated_copy_is_the_oracle(mutant_library):
    """The sweep's scaffolding is faithful: the unmutated copy of the oracle's
    expressions gives the oracle's A bit for bit and passes every pin."""
    lib, muts = mutant_library
    assert muts[0][0] == "none"
    s0 = _mutant_scale(lib, 0)
    (u, v, w), c = signed_grid(9, 5, 4, seed=68)
    for a, b in zip(s0(u, v, w, c), oracle_scale(u, v, w, c)):
        assert np.array_equal(a, b)
    assert all(pin(s0) for pin in SCALE_PINS)


def test_every_mistake_in_the_oracle_scale_is_caught(mutant_library):
    """Each single mistake in the oracle's C expressions for A -- a dropped,
    doubled or sign-flipped term, a missing absolute value, another
    coefficient, another field, any operand offset moved by one, a doubled
    whole expression or swapped outputs -- fails at least one pin."""
    lib, muts = mutant_library
    assert len(muts) > 500
    survivors = [name for n, (name, _, _) in enumerate(muts) if n > 0
                 and all(pin(_mutant_scale(lib, n)) for pin in SCALE_PINS)]
    assert survivors == []


# ---------------------------------------------------------------- adjoint scale

def _positive_grid(nx, ny, nz, seed):
    """Winds in [2, 6] (x -+ 1 stays positive, where A is a polynomial) and
    signed dyadic coefficients."""
    (u, v, w), c = signed_grid(nx, ny, nz, seed)
    rng = np.random.default_rng(seed + 1000)
    u, v, w = (rng.integers(2, 7, u.shape).astype(np.float64) for _ in range(3))
    return [u, v, w], c


def _weighted_scale(x, c, ar):
    return sum(float(np.sum(a * m)) for a, m in zip(ar, oracle_scale(*x, c)))


def exact_adjoint_scale(x, c, r):
    """Gradient of L(x) = sum_p |r_p| A_p(x) by central differences with unit
    steps: on the positive orthant A is a quadratic polynomial, so the
    quotient is exact, and with integer data every FP64 step is exact."""
    ar = [np.abs(a) for a in r]
    g = [np.zeros_like(a) for a in x]
    for f in range(3):
        for q in np.ndindex(*x[f].shape):
            x0 = x[f][q]
            x[f][q] = x0 + 1
            lp = _weighted_scale(x, c, ar)
            x[f][q] = x0 - 1
            lm = _weighted_scale(x, c, ar)
            x[f][q] = x0
            g[f][q] = (lp - lm) / 2
    return g


@pytest.fixture(scope="module")
def adjoint_case():
    x, c = _positive_grid(3, 2, 2, seed=69)
    rng = np.random.default_rng(70)
    r = [rng.integers(-3, 4, (2, 2, 3)).astype(np.float64) for _ in range(3)]
    return x, c, r, exact_adjoint_scale(x, c, r)


def test_adjoint_scale_is_gradient_of_weighted_A(adjoint_case):
    x, c, r, exact = adjoint_case
    got = scales.adjoint_scale(*x, c, r)
    for a, b in zip(got, exact):
        assert np.array_equal(a, b)
    # signs of the winds do not enter
    rng = np.random.default_rng(71)
    flipped = [a * rng.choice([-1.0, 1.0], a.shape) for a in x]
    for a, b in zip(scales.adjoint_scale(*flipped, c, r), exact):
        assert np.array_equal(a, b)


def test_adjoint_scale_euler_identity():
    """A is homogeneous of degree two in |x|, so
    sum_q |x_q| S_q = 2 sum_p |r_p| A_p (random real data)."""
    rng = np.random.default_rng(72)
    (u, v, w), c = signed_grid(8, 6, 5, seed=73)
    x = [rng.uniform(-10, 10, u.shape) for _ in range(3)]
    r = [rng.uniform(-1, 1, (5, 6, 8)) for _ in range(3)]
    s = scales.adjoint_scale(*x, c, r)
    lhs = sum(float(np.sum(np.abs(a) * b)) for a, b in zip(x, s))
    rhs = 2 * _weighted_scale(x, c, [np.abs(a) for a in r])
    assert abs(lhs - rhs) <= 1e-13 * rhs


def test_every_table_mistake_in_the_adjoint_scale_is_caught(adjoint_case):
    """Every table mutant except a flipped sign (the scale takes absolute
    values, so the sign does not enter it) changes the adjoint scale away
    from the exact gradient."""
    x, c, r, exact = adjoint_case
    survivors = []
    n = 0
    for name, table in pins.table_mutants(bf.TERMS):
        if name.startswith("sign"):
            continue
        n += 1
        got = scales.adjoint_scale(*x, c, r, terms=table)
        if all(np.array_equal(a, b) for a, b in zip(got, exact)):
            survivors.append(name)
    assert n == 510 - 18
    assert survivors == []


# ---------------------------------------------------------------- tangent scale

def test_tangent_scale_is_directional_derivative_of_A():
    """With 0 <= |d| < |x| elementwise, (A(|x| + |d|) - A(|x| - |d|)) / 2 is
    the exact derivative of the quadratic A along |d| (integer data), and
    the tangent scale must equal it; it also equals the definition
    sum |c| (|da| (|b| + |d_|) + |a| (|db| + |dd|)) on the term table."""
    x, c = _positive_grid(5, 4, 3, seed=74)
    rng = np.random.default_rng(75)
    d = [rng.integers(-1, 2, a.shape).astype(np.float64) for a in x]   # |d| <= 1 < 2 <= x
    got = scales.tangent_scale(*x, d, c)
    ad = [np.abs(a) for a in d]
    plus = oracle_scale(*(a + b for a, b in zip(x, ad)), c)
    minus = oracle_scale(*(a - b for a, b in zip(x, ad)), c)
    for g_, p, m in zip(got, plus, minus):
        assert np.array_equal(g_, (p - m) / 2)
    # the definition, term by term on the table
    f = dict(u=np.abs(x[0]), v=np.abs(x[1]), w=np.abs(x[2]))
    df = dict(u=ad[0], v=ad[1], w=ad[2])
    nz, ny, nx = 3, 4, 5
    want = {o: np.zeros((nz, ny, nx)) for o in bf.OUTPUTS}

    def sl(a, off):
        return a[1 + off[0]:1 + off[0] + nz, 1 + off[1]:1 + off[1] + ny, 1 + off[2]:1 + off[2] + nx]
    for (o, cn, _s, (fa, oa), (fb, ob), (fd, od)) in bf.TERMS:
        cc = c[cn]
        cc = abs(float(cc)) if np.ndim(cc) == 0 else np.abs(cc)[:, None, None]
        want[o] = want[o] + cc * (sl(df[fa], oa) * (sl(f[fb], ob) + sl(f[fd], od))
                                  + sl(f[fa], oa) * (sl(df[fb], ob) + sl(df[fd], od)))
    for g_, o in zip(got, bf.OUTPUTS):
        assert np.array_equal(g_, want[o])


def test_tangent_and_adjoint_scales_are_transposes():
    """Both are linear in their second argument with the same |partials|:
    sum_p |r_p| T(x, d)_p = sum_q |d_q| S(x, r)_q, exactly on integers."""
    (u, v, w), c = signed_grid(6, 5, 4, seed=76)
    rng = np.random.default_rng(77)
    d = [rng.integers(-3, 4, u.shape).astype(np.float64) for _ in range(3)]
    r = [rng.integers(-3, 4, (4, 5, 6)).astype(np.float64) for _ in range(3)]
    t = scales.tangent_scale(u, v, w, d, c)
    s = scales.adjoint_scale(u, v, w, c, r)
    lhs = sum(float(np.sum(np.abs(a) * b)) for a, b in zip(r, t))
    rhs = sum(float(np.sum(np.abs(a) * b)) for a, b in zip(d, s))
    assert lhs == rhs
    # Euler: T(x, x) = 2 A(x)
    for a, b in zip(scales.tangent_scale(u, v, w, (u, v, w), c), oracle_scale(u, v, w, c)):
        assert np.array_equal(a, 2 * b)


# ---------------------------------------------------------------- coefficient-gradient scale

def test_coeff_grad_scale_euler_and_unit_differences():
    """A is linear in |c|: sum over coefficients of |c| * scale_c equals
    sum_p |r_p| A_p at the actual coefficients (Euler), and each per-level
    entry is the exact difference L(c + e_k) - L(c) of L(c) = sum |r| A(c)
    at non-negative c (integer data, exact)."""
    (u, v, w), c = signed_grid(5, 4, 3, seed=78)
    rng = np.random.default_rng(79)
    r = [rng.integers(-3, 4, (3, 4, 5)).astype(np.float64) for _ in range(3)]
    ar = [np.abs(a) for a in r]
    s = scales.coeff_grad_scale(u, v, w, r, nz=3)
    total = abs(c["tcx"]) * s["tcx"] + abs(c["tcy"]) * s["tcy"] + \
        sum(float(np.dot(np.abs(c[n]), s[n])) for n in COEFS[2:])
    assert total == _weighted_scale((u, v, w), c, ar)
    cpos = {n: (abs(c[n]) if np.ndim(c[n]) == 0 else np.abs(c[n])) for n in COEFS}
    base = _weighted_scale((u, v, w), cpos, ar)
    for n in COEFS:
        if n in ("tcx", "tcy"):
            assert s[n] == _weighted_scale((u, v, w), dict(cpos, **{n: cpos[n] + 1}), ar) - base, n
        else:
            for k in range(3):
                bumped = cpos[n].copy()
                bumped[k] += 1
                assert s[n][k] == _weighted_scale((u, v, w), dict(cpos, **{n: bumped}), ar) - base, (n, k)
