"""Halo fill of padded arrays, written as the plain per-axis definition
(TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``).

The stencil (Sec. 2.2) reads one layer of neighbours around the interior, so
before each call a model fills the halo: periodic or neighbour values in the
horizontal and a boundary condition at the surface and the lid (Sec. 2.1, the
host model's setting).  The paper does not fix these rules; this module
defines the ones the library offers.

A padded array has shape (nz+2h, ny+2h, nx+2h).  Each axis is filled in turn
-- x, then y (whole rows, x-halo included), then z (whole planes) -- so edge
and corner cells get what a sequential exchange gives.  Per axis with n
interior cells, halo cell p (padded index, p < h or p >= n+h) takes:
  periodic     the interior cell h + ((p - h) mod n)
  copy         the nearest interior cell (zero normal gradient)
  zero         0
  reflect      the mirror image across the boundary face: 2h-1-p below,
               2(n+h)-1-p above (needs n >= h)
  reflect_neg  minus that mirror image (the field vanishes on the face)
  keep         its own value (the axis is left alone)

fold() is the adjoint (transpose) of fill(): the fill is linear, fill = Fz Fy
Fx with one map per axis, so its transpose applies the per-axis transposes
in the reverse order z, y, x.  Each adds every halo cell of its axis, times
the sign of its rule, into the cell it was copied from and clears the halo
cell (zero: the halo value is dropped; keep: the axis is left alone).  It
turns gradients with respect to filled arrays into gradients with respect to
the arrays before the fill.
"""
from __future__ import annotations

import numpy as np

MODES = ("keep", "periodic", "copy", "zero", "reflect", "reflect_neg")


def _source_index(p, n, h, mode):
    if mode == "periodic":
        return h + (p - h) % n
    if mode == "copy":
        return min(max(p, h), h + n - 1)
    if mode in ("reflect", "reflect_neg"):
        return 2 * h - 1 - p if p < h else 2 * (n + h) - 1 - p
    raise ValueError(mode)


def fill(a, halo, modes):
    """A copy of padded array ``a`` with its halo filled; ``modes`` is
    (mode_x, mode_y, mode_z)."""
    out = np.array(a, copy=True)
    h = halo
    for ax, mode in zip((2, 1, 0), modes):
        if mode not in MODES:
            raise ValueError("unknown halo mode %r" % mode)
        if mode == "keep":
            continue
        size = out.shape[ax]
        n = size - 2 * h
        if mode in ("reflect", "reflect_neg") and n < h:
            raise ValueError("reflect needs at least as many interior cells as the halo is wide")
        for p in list(range(h)) + list(range(n + h, size)):
            dst = [slice(None)] * 3
            dst[ax] = p
            if mode == "zero":
                out[tuple(dst)] = 0
                continue
            src = [slice(None)] * 3
            src[ax] = _source_index(p, n, h, mode)
            out[tuple(dst)] = -out[tuple(src)] if mode == "reflect_neg" else out[tuple(src)]
    return out


def fold(g, halo, modes):
    """The adjoint of fill(., halo, modes) applied to padded array ``g``."""
    out = np.array(g, dtype=np.float64, copy=True)
    h = halo
    for ax, mode in reversed(list(zip((2, 1, 0), modes))):
        if mode not in MODES:
            raise ValueError("unknown halo mode %r" % mode)
        if mode == "keep":
            continue
        size = out.shape[ax]
        n = size - 2 * h
        if mode in ("reflect", "reflect_neg") and n < h:
            raise ValueError("reflect needs at least as many interior cells as the halo is wide")
        for p in list(range(h)) + list(range(n + h, size)):
            dst = [slice(None)] * 3
            dst[ax] = p
            if mode != "zero":
                src = [slice(None)] * 3
                src[ax] = _source_index(p, n, h, mode)
                sign = -1.0 if mode == "reflect_neg" else 1.0
                out[tuple(src)] += sign * out[tuple(dst)]
            out[tuple(dst)] = 0.0
    return out
