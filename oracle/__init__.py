"""FP64 CPU oracle for Piacsek-Williams advection.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this package to check the GPU library.  The library never
imports it, and it imports nothing from the library.

* ``pw_oracle.c`` -- plain FP64 loops of the forward operator, its adjoint
  (scatter form of J^T r), its tangent-linear operator (J dx) and the
  gradients with respect to the coefficients; built with gcc into
  ``liboracle.so`` and called through ctypes.
* ``bruteforce.py`` -- an independent, table-driven evaluation of the same
  operator in exact rational arithmetic, for tiny grids.

Every function takes numpy arrays: padded inputs of shape (nz+2h, ny+2h, nx+2h)
(x fastest) and returns interior outputs of shape (nz, ny, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``pw_oracle.c`` into ``liboracle.so`` (gcc, FP64, no FMA contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, dbl, p, c_int = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        lib.pwo_forward.argtypes = [i64] * 4 + [p] * 3 + [dbl, dbl] + [p] * 4 + [p] * 3 + [p] * 3 + [c_int]
        lib.pwo_forward.restype = None
        lib.pwo_adjoint.argtypes = [i64] * 4 + [p] * 3 + [dbl, dbl] + [p] * 4 + [p] * 3 + [p] * 3
        lib.pwo_adjoint.restype = None
        lib.pwo_tangent.argtypes = [i64] * 4 + [p] * 3 + [p] * 3 + [dbl, dbl] + [p] * 4 + [p] * 3
        lib.pwo_tangent.restype = None
        lib.pwo_coeff_grad.argtypes = [i64] * 4 + [p] * 3 + [p] * 3 + [p] * 8
        lib.pwo_coeff_grad.restype = None
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dims(u, h):
    pz, py, px = u.shape
    nz, ny, nx = pz - 2 * h, py - 2 * h, px - 2 * h
    if min(nx, ny, nz) < 1 or h < 1:
        raise ValueError("padded shape %r too small for halo %d" % (u.shape, h))
    return nx, ny, nz


def _coeffs(c, nz):
    tz = [_f64(c[name]) for name in ("tzc1", "tzc2", "tzd1", "tzd2")]
    for t in tz:
        if t.shape != (nz,):
            raise ValueError("vertical coefficient arrays must have length nz=%d" % nz)
    return float(c["tcx"]), float(c["tcy"]), tz


def forward(u, v, w, coeffs, halo=1, magnitude=False, nthreads=1):
    """su, sv, sw = F(u, v, w) in FP64.  ``coeffs`` is a mapping with tcx, tcy,
    tzc1, tzc2, tzd1, tzd2.  With ``magnitude`` also returns the error scales
    A_u, A_v, A_w (sum of |c||a|(|b|+|d|) over each output's products)."""
    lib = _load()
    u, v, w = _f64(u), _f64(v), _f64(w)
    if not (u.shape == v.shape == w.shape):
        raise ValueError("u, v, w must share one padded shape")
    nx, ny, nz = _dims(u, halo)
    tcx, tcy, tz = _coeffs(coeffs, nz)
    out = [np.empty((nz, ny, nx)) for _ in range(3)]
    mag = [np.empty((nz, ny, nx)) for _ in range(3)] if magnitude else [None] * 3
    lib.pwo_forward(nx, ny, nz, halo, _ptr(u), _ptr(v), _ptr(w), tcx, tcy,
                    *[_ptr(t) for t in tz], *[_ptr(o) for o in out],
                    *[_ptr(m) for m in mag], int(nthreads))
    if magnitude:
        return tuple(out), tuple(mag)
    return tuple(out)


def adjoint(u, v, w, coeffs, ru, rv, rw, halo=1):
    """gu, gv, gw = J(u, v, w)^T (ru, rv, rw): padded-shaped gradients (halo
    included) of <F(u, v, w), r> for interior-shaped cotangents r."""
    lib = _load()
    u, v, w = _f64(u), _f64(v), _f64(w)
    nx, ny, nz = _dims(u, halo)
    tcx, tcy, tz = _coeffs(coeffs, nz)
    r = [_f64(x) for x in (ru, rv, rw)]
    for x in r:
        if x.shape != (nz, ny, nx):
            raise ValueError("cotangents must be interior-shaped")
    g = [np.empty(u.shape) for _ in range(3)]
    lib.pwo_adjoint(nx, ny, nz, halo, _ptr(u), _ptr(v), _ptr(w), tcx, tcy,
                    *[_ptr(t) for t in tz], *[_ptr(x) for x in r], *[_ptr(x) for x in g])
    return tuple(g)


def tangent(u, v, w, du, dv, dw, coeffs, halo=1):
    """tu, tv, tw = J(u, v, w) (du, dv, dw): the directional derivative of the
    outputs along a padded-shaped direction."""
    lib = _load()
    u, v, w = _f64(u), _f64(v), _f64(w)
    d = [_f64(x) for x in (du, dv, dw)]
    nx, ny, nz = _dims(u, halo)
    for x in d:
        if x.shape != u.shape:
            raise ValueError("direction must be padded-shaped")
    tcx, tcy, tz = _coeffs(coeffs, nz)
    out = [np.empty((nz, ny, nx)) for _ in range(3)]
    lib.pwo_tangent(nx, ny, nz, halo, _ptr(u), _ptr(v), _ptr(w),
                    *[_ptr(x) for x in d], tcx, tcy, *[_ptr(t) for t in tz],
                    *[_ptr(o) for o in out])
    return tuple(out)


def coeff_grad(u, v, w, ru, rv, rw, halo=1):
    """Gradients of <F(u, v, w), r> with respect to the coefficients (the
    loss is linear in them, so the coefficients' values do not enter):
    a dict with tcx, tcy (floats), tzc1, tzc2, tzd1, tzd2 (length nz) and
    tcx_level, tcy_level (each level's share of tcx, tcy)."""
    lib = _load()
    u, v, w = _f64(u), _f64(v), _f64(w)
    nx, ny, nz = _dims(u, halo)
    r = [_f64(x) for x in (ru, rv, rw)]
    for x in r:
        if x.shape != (nz, ny, nx):
            raise ValueError("cotangents must be interior-shaped")
    arrs = [np.empty(nz) for _ in range(6)]
    sx, sy = np.empty(1), np.empty(1)
    lib.pwo_coeff_grad(nx, ny, nz, halo, _ptr(u), _ptr(v), _ptr(w), *[_ptr(x) for x in r],
                       *[_ptr(a) for a in arrs], _ptr(sx), _ptr(sy))
    names = ("tzc1", "tzc2", "tzd1", "tzd2", "tcx_level", "tcy_level")
    out = dict(zip(names, arrs))
    out["tcx"], out["tcy"] = float(sx[0]), float(sy[0])
    return out
