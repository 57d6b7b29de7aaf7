"""Helpers for the GPU parity tests: moving seeded grids to the device and
comparing GPU outputs with the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle


def dev_grid(g, device="cuda", storage=None):
    """Torch copies of a workloads.Grid's winds (optionally re-stored as
    torch.bfloat16/float16 from the FP32 values, RNE) and coefficients."""
    import torch
    from paper_2301_13016_amd import binding as B
    f = [torch.from_numpy(np.ascontiguousarray(x)).to(device) for x in (g.u, g.v, g.w)]
    if storage is not None:
        f = [x.to(storage) for x in f]
    cdt = torch.float64 if g.u.dtype == np.float64 else torch.float32
    return f, B.Coeffs.from_host(g.coeffs, device=device, dtype=cdt)


def a_scaled_error(got, ref, mag):
    """max |got - ref| / A over all points (A = the oracle's error scale)."""
    got = np.asarray(got, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        e = np.abs(got - ref) / np.where(mag > 0, mag, 1.0)
    return float(np.max(e)) if e.size else 0.0


def normwise_error(got, ref):
    d = np.max(np.abs(np.asarray(got, np.float64) - ref))
    s = np.max(np.abs(ref))
    return float(d / s) if s > 0 else float(d)


def oracle_errors(outs, u, v, w, coeffs, halo=1):
    """A-scaled and normwise errors of GPU outputs (host arrays) per field."""
    ref, mag = oracle.forward(u, v, w, coeffs, halo=halo, magnitude=True)
    return [(a_scaled_error(o, r, m), normwise_error(o, r)) for o, r, m in zip(outs, ref, mag)]


def subbox_errors(outs_dev, g, boxes, halo=1, inputs=None, normwise=None):
    """Worst A-scaled error per field of device outputs on interior sub-boxes
    (k0, k1, j0, j1, i0, i1): the oracle is run on each box with its halo cut
    out of the padded inputs.  If ``normwise`` is a list, the worst
    max|got - ref| / max|ref| per field (over the boxes) is appended to it."""
    u, v, w = (g.u, g.v, g.w) if inputs is None else inputs
    worst = [0.0, 0.0, 0.0]
    dmax, rmax = [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]
    for (k0, k1, j0, j1, i0, i1) in boxes:
        sl = (slice(k0, k1 + 2 * halo), slice(j0, j1 + 2 * halo), slice(i0, i1 + 2 * halo))
        c = dict(tcx=g.tcx, tcy=g.tcy, **{n: getattr(g, n)[k0:k1] for n in ("tzc1", "tzc2", "tzd1", "tzd2")})
        ref, mag = oracle.forward(u[sl], v[sl], w[sl], c, halo=halo, magnitude=True)
        for f in range(3):
            got = outs_dev[f][k0:k1, j0:j1, i0:i1].cpu().numpy()
            worst[f] = max(worst[f], a_scaled_error(got, ref[f], mag[f]))
            dmax[f] = max(dmax[f], float(np.max(np.abs(got.astype(np.float64) - ref[f]))))
            rmax[f] = max(rmax[f], float(np.max(np.abs(ref[f]))))
    if normwise is not None:
        normwise.extend(d / r if r > 0 else d for d, r in zip(dmax, rmax))
    return worst


def sample_boxes(nx, ny, nz, n_random=6, size=(8, 16, 70), seed=0):
    """Corner, edge and random interior boxes of the interior grid."""
    rng = np.random.default_rng(seed)
    bz, by, bx = (min(s, n) for s, n in zip(size, (nz, ny, nx)))
    boxes = []
    for k0 in (0, nz - bz):
        for j0 in (0, ny - by):
            for i0 in (0, nx - bx):
                boxes.append((k0, k0 + bz, j0, j0 + by, i0, i0 + bx))
    for _ in range(n_random):
        k0 = int(rng.integers(0, nz - bz + 1))
        j0 = int(rng.integers(0, ny - by + 1))
        i0 = int(rng.integers(0, nx - bx + 1))
        boxes.append((k0, k0 + bz, j0, j0 + by, i0, i0 + bx))
    return sorted(set(boxes))


def adjoint_magnitude(u, v, w, coeffs, r, halo=1):
    """Error scale of J^T r: for every gradient entry the sum of |partial
    derivative of a term| * |cotangent| over the terms that read it (the
    brute-force term table, scattered with absolute values)."""
    from oracle.bruteforce import TERMS
    f = dict(u=np.abs(np.asarray(u, np.float64)), v=np.abs(np.asarray(v, np.float64)),
             w=np.abs(np.asarray(w, np.float64)))
    rr = dict(su=np.abs(r[0]), sv=np.abs(r[1]), sw=np.abs(r[2]))
    pz, py, px = f["u"].shape
    nz, ny, nx = pz - 2 * halo, py - 2 * halo, px - 2 * halo
    g = {k: np.zeros((pz, py, px)) for k in "uvw"}

    def sl(off):
        return (slice(halo + off[0], halo + off[0] + nz), slice(halo + off[1], halo + off[1] + ny),
                slice(halo + off[2], halo + off[2] + nx))

    for (o, cname, s, (fa, oa), (fb, ob), (fd, od)) in TERMS:
        c = coeffs[cname]
        c = abs(float(c)) if np.ndim(c) == 0 else np.abs(np.asarray(c, np.float64))[:, None, None]
        g[fa][sl(oa)] += c * rr[o] * (f[fb][sl(ob)] + f[fd][sl(od)])
        g[fb][sl(ob)] += c * rr[o] * f[fa][sl(oa)]
        g[fd][sl(od)] += c * rr[o] * f[fa][sl(oa)]
    return g["u"], g["v"], g["w"]
