"""Helpers for the GPU parity tests: moving seeded grids to the device and
comparing GPU outputs with the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle
from scales import adjoint_scale


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


def host_threads():
    """Host threads the oracle may use: the usable cores, at most 16."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def full_grid_errors(outs, g, slab=32, halo=1):
    """Worst A-scaled and normwise error per field, over EVERY interior point,
    of several device results for one grid: ``outs`` maps a name to the
    (su, sv, sw) device tensors.  The oracle runs once per z-slab of ``slab``
    levels (with its halo planes) on the grid's own values, multithreaded, and
    every result is compared with the same reference.  Returns
    {name: (a_scaled[3], normwise[3])}."""
    nz = g.nz
    worst = {n: [0.0, 0.0, 0.0] for n in outs}
    dmax = {n: [0.0, 0.0, 0.0] for n in outs}
    rmax = [0.0, 0.0, 0.0]
    nt = host_threads()
    for k0 in range(0, nz, slab):
        k1 = min(nz, k0 + slab)
        sl = slice(k0, k1 + 2 * halo)
        c = dict(tcx=g.tcx, tcy=g.tcy, **{n: getattr(g, n)[k0:k1] for n in ("tzc1", "tzc2", "tzd1", "tzd2")})
        ref, mag = oracle.forward(g.u[sl], g.v[sl], g.w[sl], c, halo=halo, magnitude=True, nthreads=nt)
        for f in range(3):
            rmax[f] = max(rmax[f], float(np.max(np.abs(ref[f]))))
            inv = 1.0 / np.where(mag[f] > 0, mag[f], 1.0)
            for name, o in outs.items():
                got = o[f][k0:k1].cpu().numpy().astype(np.float64)
                got -= ref[f]
                np.abs(got, out=got)
                dmax[name][f] = max(dmax[name][f], float(np.max(got)))
                got *= inv
                worst[name][f] = max(worst[name][f], float(np.max(got)))
    return {n: (worst[n], [d / r if r > 0 else d for d, r in zip(dmax[n], rmax)]) for n in outs}


def adjoint_magnitude(u, v, w, coeffs, r, halo=1):
    """Error scale of J^T r (see scales.adjoint_scale)."""
    return adjoint_scale(u, v, w, coeffs, r, halo=halo)


def unread_cells(shape, halo):
    """Per field (u, v, w), a boolean mask of the padded cells that no interior
    output reads: the complement of every term operand's offset applied over
    the interior (from the brute-force term table)."""
    from oracle.bruteforce import TERMS
    pz, py, px = shape
    nz, ny, nx = pz - 2 * halo, py - 2 * halo, px - 2 * halo
    read = {f: np.zeros(shape, bool) for f in "uvw"}
    for t in TERMS:
        for f, off in t[3:]:
            read[f][halo + off[0]:halo + off[0] + nz, halo + off[1]:halo + off[1] + ny,
                    halo + off[2]:halo + off[2] + nx] = True
    return [~read[f] for f in "uvw"]


def poison_unread(g):
    """Write NaN, +Inf and -Inf (in turn) into every cell of g's winds that no
    output reads; returns the masks."""
    unread = unread_cells(g.u.shape, g.halo)
    poison = np.array([np.nan, np.inf, -np.inf])
    for x, m in zip((g.u, g.v, g.w), unread):
        x[m] = poison[np.arange(int(m.sum())) % 3].astype(x.dtype)
    return unread
