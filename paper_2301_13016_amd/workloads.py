"""Seeded synthetic workloads for Piacsek-Williams advection.

This module only draws random inputs; it holds none of the scheme's arithmetic.
It is the one piece shared by the GPU library's tests and benchmark and by the
FP64 oracle's checks, so both sides always see the same numbers.

Recipe (the paper measures one unnamed FP32 problem of about 67 million grid
points, Sec. 3 and Tables 1-2; these synthetic grids stand in for it):

* Generator: ``numpy.random.default_rng(seed)`` (PCG64).  Draw order: u, v, w
  over the whole halo-padded array in C order (x fastest), then tzc1, tzc2,
  tzd1, tzd2.
* Winds: i.i.d. uniform in [-10, 10], drawn in FP64 and stored in the storage
  dtype (FP32 rounding by RNE; BF16/FP16 copies are made from the FP32 values
  by RNE).
* Coefficients: tcx = tcy = 0.25/100 (0.25 / grid spacing, 100 m);
  tz* = U[0.5, 1.5] * 0.25/50 per level (50 m levels with density-like
  weights), drawn in FP64.  For FP32-family paths they are rounded once to
  FP32, and the oracle is fed those rounded values.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TCX = 0.25 / 100.0
TCY = 0.25 / 100.0
TZ_SCALE = 0.25 / 50.0
WIND_LO, WIND_HI = -10.0, 10.0
_CHUNK = 1 << 22


def _uniform(rng, n, lo, hi, dtype):
    """n uniform draws in [lo, hi), drawn in FP64 in chunks (same stream as one
    big draw) and stored in ``dtype``."""
    out = np.empty(n, dtype=dtype)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        out[s:e] = rng.uniform(lo, hi, e - s)
    return out


def padded_shape(nx, ny, nz, halo=1):
    return (nz + 2 * halo, ny + 2 * halo, nx + 2 * halo)


@dataclass
class Grid:
    """One halo-padded subdomain: winds (numpy, storage dtype) and coefficients."""
    nx: int
    ny: int
    nz: int
    halo: int
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    tcx: float
    tcy: float
    tzc1: np.ndarray
    tzc2: np.ndarray
    tzd1: np.ndarray
    tzd2: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def coeffs(self):
        return dict(tcx=self.tcx, tcy=self.tcy, tzc1=self.tzc1, tzc2=self.tzc2,
                    tzd1=self.tzd1, tzd2=self.tzd2)

    @property
    def points(self):
        return self.nx * self.ny * self.nz


def make_grid(nx, ny, nz, seed, halo=1, dtype=np.float32, rng=None):
    """Seeded grid: u, v, w ~ U[-10, 10] over the padded array, then the four
    vertical arrays ~ U[0.5, 1.5] * 0.25/50.  ``dtype`` float32 or float64;
    coefficients are rounded to FP32 for float32 storage."""
    rng = np.random.default_rng(seed) if rng is None else rng
    shp = padded_shape(nx, ny, nz, halo)
    n = int(np.prod(shp))
    u = _uniform(rng, n, WIND_LO, WIND_HI, dtype).reshape(shp)
    v = _uniform(rng, n, WIND_LO, WIND_HI, dtype).reshape(shp)
    w = _uniform(rng, n, WIND_LO, WIND_HI, dtype).reshape(shp)
    tz = [rng.uniform(0.5, 1.5, nz) * TZ_SCALE for _ in range(4)]
    tcx, tcy = TCX, TCY
    if dtype != np.float64:
        tz = [t.astype(np.float32).astype(np.float64) for t in tz]
        tcx = float(np.float32(tcx))
        tcy = float(np.float32(tcy))
    return Grid(nx, ny, nz, halo, u, v, w, tcx, tcy, *tz, meta=dict(seed=seed))


def cotangents(nx, ny, nz, seed, dtype=np.float32):
    """Interior-shaped output cotangents ru, rv, rw ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    return tuple(_uniform(rng, n, -1.0, 1.0, dtype).reshape(nz, ny, nx) for _ in range(3))


def direction(nx, ny, nz, seed, halo=1, dtype=np.float64):
    """Padded-shaped perturbation direction du, dv, dw ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    shp = padded_shape(nx, ny, nz, halo)
    n = int(np.prod(shp))
    return tuple(_uniform(rng, n, -1.0, 1.0, dtype).reshape(shp) for _ in range(3))


def integer_grid(nx, ny, nz, seed, halo=1, lo=-4, hi=4, dtype=np.float32):
    """Small-integer winds and dyadic coefficients: every intermediate of the
    scheme is then exact in FP64, FP32 and FP32-from-BF16/FP16, so all
    evaluation orders agree bit for bit."""
    rng = np.random.default_rng(seed)
    shp = padded_shape(nx, ny, nz, halo)
    u, v, w = (rng.integers(lo, hi + 1, shp).astype(dtype) for _ in range(3))
    tz = [np.asarray(rng.choice([0.25, 0.125, 0.0625], nz), dtype=np.float64) for _ in range(4)]
    return Grid(nx, ny, nz, halo, u, v, w, 0.25, 0.125, *tz, meta=dict(seed=seed, integer=True))


# --- the five workload configurations -------------------------------------------------

#: c0: FP64 forward, 64^3 interior, 1-cell halo, seed 0 (oracle-sized).
C0 = dict(name="pw-fwd-f64-64x64x64", nx=64, ny=64, nz=64, seed=0, dtype=np.float64)
#: c1: FP32 forward, 512x512x64 (16.8 M points), seed 1: the headline launch.
C1 = dict(name="pw-fwd-f32-512x512x64", nx=512, ny=512, nz=64, seed=1, dtype=np.float32)
#: c2: precision form, 1024x1024x256 (268 M points), seed 2; BF16/FP16 copies of FP32 draws.
C2 = dict(name="pw-fwd-lowp-1024x1024x256", nx=1024, ny=1024, nz=256, seed=2, dtype=np.float32)
#: c4: differentiation form, 256x256x128, seed 4; cotangents seed 44.
C4 = dict(name="pw-adj-f32-256x256x128", nx=256, ny=256, nz=128, seed=4, dtype=np.float32,
          cot_seed=44)
#: c4 finite-difference check: 16^3 FP64, seed 40, eps 1e-6.
C4_FD = dict(nx=16, ny=16, nz=16, seed=40, eps=1e-6)


def config_grid(cfg, dtype=None):
    return make_grid(cfg["nx"], cfg["ny"], cfg["nz"], cfg["seed"],
                     dtype=cfg["dtype"] if dtype is None else dtype)


def batch_shapes(n=64, seed=3):
    """c3: shapes of the 64 uneven subdomains, nx, ny ~ U{32..256}, nz ~ U{64..256};
    subdomain b is drawn from ``default_rng((seed, b))``."""
    shapes = []
    for b in range(n):
        rng = np.random.default_rng((seed, b))
        nx, ny = (int(x) for x in rng.integers(32, 257, 2))
        nz = int(rng.integers(64, 257))
        shapes.append((nx, ny, nz))
    return shapes


def batch_grids(n=64, seed=3, shapes=None):
    """c3: the subdomains themselves, FP32, each with its own fields and vertical
    arrays, drawn from ``default_rng((seed, b))`` after its shape."""
    out = []
    for b in range(n):
        rng = np.random.default_rng((seed, b))
        nx, ny = (int(x) for x in rng.integers(32, 257, 2))
        nz = int(rng.integers(64, 257))
        if shapes is not None:
            nx, ny, nz = shapes[b]
        out.append(make_grid(nx, ny, nz, seed=None, rng=rng, dtype=np.float32))
    return out


def to_bf16_bits(x32):
    """FP32 -> BF16 by round-to-nearest-even, returned as uint16 bit patterns
    (finite inputs)."""
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def from_bf16_bits(bits):
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)
