"""Exact, table-driven Piacsek-Williams advection for tiny grids.

TEST INFRASTRUCTURE ONLY (part of the oracle).  A second, independent encoding
of the operator that ``pw_oracle.c`` implements with loops: here every output is
a signed sum of six product terms  s * c * a * (b + d)  listed in a table, and
the arithmetic is done in exact rationals (``fractions.Fraction``), so with
integer fields and dyadic coefficients the FP64 loops must agree bit for bit.

Table rows follow the paper's per-cell decomposition (Sec. 4, Fig. 2): per
output field six face sums (b + d, twelve operands), six products with a
neighbouring value a (six operands), then differences and a reduction; the
three fields use the same arithmetic and differ only in stencil locations
(Sec. 4, discussion of Table 1).  Offsets are (dk, dj, di) relative to the
output point in padded coordinates.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

# (output, coefficient, sign, (field, offset) of a, of b, of d)
TERMS = (
    ("su", "tcx", +1, ("u", (0, 0, -1)), ("u", (0, 0, 0)), ("u", (0, 0, -1))),
    ("su", "tcx", -1, ("u", (0, 0, +1)), ("u", (0, 0, 0)), ("u", (0, 0, +1))),
    ("su", "tcy", +1, ("u", (0, -1, 0)), ("v", (0, -1, 0)), ("v", (0, -1, +1))),
    ("su", "tcy", -1, ("u", (0, +1, 0)), ("v", (0, 0, 0)), ("v", (0, 0, +1))),
    ("su", "tzc1", +1, ("u", (-1, 0, 0)), ("w", (-1, 0, 0)), ("w", (-1, 0, +1))),
    ("su", "tzc2", -1, ("u", (+1, 0, 0)), ("w", (0, 0, 0)), ("w", (0, 0, +1))),

    ("sv", "tcx", +1, ("v", (0, 0, -1)), ("u", (0, 0, -1)), ("u", (0, +1, -1))),
    ("sv", "tcx", -1, ("v", (0, 0, +1)), ("u", (0, 0, 0)), ("u", (0, +1, 0))),
    ("sv", "tcy", +1, ("v", (0, -1, 0)), ("v", (0, 0, 0)), ("v", (0, -1, 0))),
    ("sv", "tcy", -1, ("v", (0, +1, 0)), ("v", (0, 0, 0)), ("v", (0, +1, 0))),
    ("sv", "tzc1", +1, ("v", (-1, 0, 0)), ("w", (-1, 0, 0)), ("w", (-1, +1, 0))),
    ("sv", "tzc2", -1, ("v", (+1, 0, 0)), ("w", (0, 0, 0)), ("w", (0, +1, 0))),

    ("sw", "tcx", +1, ("w", (0, 0, -1)), ("u", (0, 0, -1)), ("u", (+1, 0, -1))),
    ("sw", "tcx", -1, ("w", (0, 0, +1)), ("u", (0, 0, 0)), ("u", (+1, 0, 0))),
    ("sw", "tcy", +1, ("w", (0, -1, 0)), ("v", (0, -1, 0)), ("v", (+1, -1, 0))),
    ("sw", "tcy", -1, ("w", (0, +1, 0)), ("v", (0, 0, 0)), ("v", (+1, 0, 0))),
    ("sw", "tzd1", +1, ("w", (-1, 0, 0)), ("w", (0, 0, 0)), ("w", (-1, 0, 0))),
    ("sw", "tzd2", -1, ("w", (+1, 0, 0)), ("w", (0, 0, 0)), ("w", (+1, 0, 0))),
)

OUTPUTS = ("su", "sv", "sw")
FIELDS = ("u", "v", "w")


def _exact(x):
    return Fraction(x) if not isinstance(x, Fraction) else x


def _coef(coeffs, name, kk):
    c = coeffs[name]
    if np.ndim(c) == 0 and not isinstance(c, (list, tuple)):
        return _exact(float(c)) if not isinstance(c, Fraction) else c
    return _exact(c[kk]) if isinstance(c[kk], Fraction) else _exact(float(c[kk]))


def forward_exact(fields, coeffs, halo=1):
    """Exact F at every interior point.  ``fields`` maps u/v/w to padded arrays
    (numbers or Fractions); returns a dict su/sv/sw -> nested lists of Fractions
    indexed [k][j][i] over the interior."""
    pz, py, px = np.shape(fields["u"])
    h = halo
    nz, ny, nx = pz - 2 * h, py - 2 * h, px - 2 * h
    val = {f: np.asarray(fields[f], dtype=object) for f in FIELDS}
    out = {o: [[[Fraction(0)] * nx for _ in range(ny)] for _ in range(nz)] for o in OUTPUTS}
    for k in range(h, h + nz):
        kk = k - h
        for j in range(h, h + ny):
            for i in range(h, h + nx):
                for (o, cname, s, (fa, oa), (fb, ob), (fd, od)) in TERMS:
                    c = _coef(coeffs, cname, kk)
                    a = _exact(val[fa][k + oa[0], j + oa[1], i + oa[2]])
                    b = _exact(val[fb][k + ob[0], j + ob[1], i + ob[2]])
                    d = _exact(val[fd][k + od[0], j + od[1], i + od[2]])
                    out[o][kk][j - h][i - h] += s * c * a * (b + d)
    return out


def adjoint_exact(fields, coeffs, cotangents, halo=1):
    """Exact J^T r by central differences of ``forward_exact``.

    F is a homogeneous quadratic, so for a unit perturbation e_q of one padded
    input entry (F(x + e_q) - F(x - e_q)) / 2 = J(x) e_q holds exactly in
    rational arithmetic, and (J^T r)_q = <J e_q, r>.  Independent of any
    hand-derived partial derivative.  Returns dict u/v/w -> padded arrays of
    Fractions (dtype object)."""
    shape = np.shape(fields["u"])
    base = {f: np.asarray(fields[f], dtype=object).copy() for f in FIELDS}
    r = {o: np.asarray(cotangents[o], dtype=object) for o in OUTPUTS}
    grads = {f: np.empty(shape, dtype=object) for f in FIELDS}
    for f in FIELDS:
        for q in np.ndindex(*shape):
            x0 = base[f][q]
            base[f][q] = _exact(x0) + 1
            fp = forward_exact(base, coeffs, halo)
            base[f][q] = _exact(x0) - 1
            fm = forward_exact(base, coeffs, halo)
            base[f][q] = x0
            acc = Fraction(0)
            for o in OUTPUTS:
                fpo, fmo, ro = fp[o], fm[o], r[o]
                for kk in range(len(fpo)):
                    for jj in range(len(fpo[0])):
                        for ii in range(len(fpo[0][0])):
                            dif = fpo[kk][jj][ii] - fmo[kk][jj][ii]
                            if dif:
                                acc += dif / 2 * _exact(ro[kk, jj, ii])
            grads[f][q] = acc
    return grads


def to_float_array(nested):
    """Nested lists (or object array) of Fractions -> float64 array (exact when
    the values are representable)."""
    return np.vectorize(float, otypes=[np.float64])(np.asarray(nested, dtype=object))
