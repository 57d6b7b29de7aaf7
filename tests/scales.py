"""Error scales of the differentiated operators, used by the GPU parity gates.

Each parity gate divides |GPU - oracle| by a per-entry scale: the sum, over
the product terms that feed the entry, of the absolute values of what the
term contributes.  The forward scale A(p) comes from the oracle itself
(``oracle.forward(..., magnitude=True)``); the three scales here extend it to
the adjoint (J^T r), the tangent-linear operator (J d) and the coefficient
gradients (dL/dc).  They are pinned on the CPU by ``test_scale_pins.py``
against exact finite differences of A and against the term table.

Every term of the scheme has the form s * c * a * (b + d) (paper, Sec. 4 and
Fig. 2: six face sums, six products, differences and a reduction per field);
its partial derivatives are s*c*(b+d) with respect to a and s*c*a with
respect to b and d.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle.bruteforce import TERMS

NAMES = ("tzc1", "tzc2", "tzd1", "tzd2")


def adjoint_scale(u, v, w, coeffs, r, halo=1, terms=TERMS):
    """Per padded gradient entry q: sum over the terms that read q of
    |partial derivative of the term with respect to q| * |cotangent|."""
    f = dict(u=np.abs(np.asarray(u, np.float64)), v=np.abs(np.asarray(v, np.float64)),
             w=np.abs(np.asarray(w, np.float64)))
    rr = dict(su=np.abs(np.asarray(r[0], np.float64)), sv=np.abs(np.asarray(r[1], np.float64)),
              sw=np.abs(np.asarray(r[2], np.float64)))
    pz, py, px = f["u"].shape
    nz, ny, nx = pz - 2 * halo, py - 2 * halo, px - 2 * halo
    g = {k: np.zeros((pz, py, px)) for k in "uvw"}

    def sl(off):
        return (slice(halo + off[0], halo + off[0] + nz), slice(halo + off[1], halo + off[1] + ny),
                slice(halo + off[2], halo + off[2] + nx))

    for (o, cname, s, (fa, oa), (fb, ob), (fd, od)) in terms:
        c = coeffs[cname]
        c = abs(float(c)) if np.ndim(c) == 0 else np.abs(np.asarray(c, np.float64))[:, None, None]
        g[fa][sl(oa)] += c * rr[o] * (f[fb][sl(ob)] + f[fd][sl(od)])
        g[fb][sl(ob)] += c * rr[o] * f[fa][sl(oa)]
        g[fd][sl(od)] += c * rr[o] * f[fa][sl(oa)]
    return g["u"], g["v"], g["w"]


def tangent_scale(u, v, w, d, coeffs, halo=1):
    """Per interior output: sum over its terms of
    |c| * (|da| (|b| + |d_|) + |a| (|db| + |dd|)), the magnitude of each
    term's derivative along the direction d.  A(|x|) is a quadratic form with
    non-negative coefficients, so this is A(|x| + |d|) - A(|x|) - A(|d|)."""
    ax = [np.abs(np.asarray(a, np.float64)) for a in (u, v, w)]
    ad = [np.abs(np.asarray(a, np.float64)) for a in d]
    both = [a + b for a, b in zip(ax, ad)]
    _, m_both = oracle.forward(*both, coeffs, halo=halo, magnitude=True)
    _, m_x = oracle.forward(*ax, coeffs, halo=halo, magnitude=True)
    _, m_d = oracle.forward(*ad, coeffs, halo=halo, magnitude=True)
    return [np.maximum(p - q - s, 0.0) for p, q, s in zip(m_both, m_x, m_d)]


def coeff_grad_scale(u, v, w, r, nz, halo=1):
    """Per coefficient gradient: sum over the products that the coefficient
    multiplies of |cotangent| * |coefficient-free product|, i.e. the forward
    scale A with that coefficient set to one and all others to zero, weighted
    by |r|.  tcx and tcy are totals over the grid; tz* are per level."""
    ar = [np.abs(np.asarray(x, np.float64)) for x in r]
    zero = dict(tcx=0.0, tcy=0.0, **{n: np.zeros(nz) for n in NAMES})
    out = {}
    for name in ("tcx", "tcy") + NAMES:
        c = dict(zero)
        c[name] = 1.0 if name in ("tcx", "tcy") else np.ones(nz)
        _, mag = oracle.forward(u, v, w, c, halo=halo, magnitude=True)
        per_level = sum(np.sum(a * m, axis=(1, 2)) for a, m in zip(ar, mag))
        out[name] = float(per_level.sum()) if name in ("tcx", "tcy") else per_level
    return out
