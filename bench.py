"""Benchmark of PW advection on one MI355X.

One step = one forward launch of the PW stencil (face sums, products,
differences, reduction, store: the whole hot path) over the FP32 grid
512 x 512 x 64 (16.8 M interior points, 1-cell halo), with inputs resident in
HBM.  K steps are timed between two device synchronisations; consecutive steps
use different buffer sets (4 x 410 MB) so the 256 MB MALL cannot serve a
repeat.  The dominant kernel's average duration comes from two HIP events
around the timed launches on the launch stream (no event between launches).
Launch shapes are the library's choice (its built-in tuning table); the
batched form is tuned in the run.

Also measured in the same run ("forms"):
  * BF16 / FP16 storage vs FP32 on 1024 x 1024 x 256 (268 M points);
  * the adjoint (J^T r), the tangent (J dx) and the coefficient gradients vs the
    forward on 256 x 256 x 128 FP32;
  * 64 uneven subdomains (FP32) in one persistent launch replayed from a HIP
    graph vs 64 plain launches;
  * a plain copy kernel and a three-stream copy (the stencil's pattern of three
    arrays read and three written), and a probe kernel swept over loads in
    flight per lane, cache policy and workgroup count for copy, read-only and
    write-only streams: reachable-bandwidth references;
  * the FP64 oracle on the host cores ("cpu_baseline", the only use of the
    oracle here).
Their errors against the oracle are measured by the GPU test suite.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algo_bytes(nx, ny, nz, halo, in_bytes, out_bytes=4):
    """Algorithmic HBM bytes of one forward launch: every padded input element
    read once, every interior output written once."""
    padded = (nx + 2 * halo) * (ny + 2 * halo) * (nz + 2 * halo)
    return 3 * padded * in_bytes + 3 * nx * ny * nz * out_bytes


def adjoint_bytes(nx, ny, nz, halo, es=4):
    """Algorithmic bytes of one adjoint launch: u, v, w and the three
    cotangents read once, the three padded gradients written once."""
    padded = (nx + 2 * halo) * (ny + 2 * halo) * (nz + 2 * halo)
    return 3 * padded * es + 3 * nx * ny * nz * es + 3 * padded * es


def kernel_fingerprint():
    """sha256[:16] of the FP32 forward kernel's sources plus the tuning-table
    row that picks its launch shape for 512 x 512 x 64.  Any change to either
    makes stored HBM-counter readings stale."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2301_13016_amd", "csrc")
    hsh = hashlib.sha256()
    for name in ("pw_stencil.h", "pw_forward_impl.h", "pw_forward_f32.hip", "pw_forward_lds_f32.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            hsh.update(f.read())
    with open(os.path.join(csrc, "pw_tune_defaults.inc")) as f:
        rows = [ln.split("//")[0].strip() for ln in f if ln.startswith("{0, 0, 9, 9, 6,")]
    hsh.update("\n".join(rows).encode())
    return hsh.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE
    readings (already scaled by the copy-kernel calibration), or None when
    there are none or the kernel has changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            ent = json.load(f)[key]
    except (OSError, KeyError, ValueError):
        return None
    if ent.get("source_sha256_16") != kernel_fingerprint():
        return None
    return int(ent["traffic_bytes"])


def tangent_bytes(nx, ny, nz, halo, es=4):
    """Algorithmic bytes of one tangent launch: u, v, w and du, dv, dw read
    once (padded), tu, tv, tw written once (interior)."""
    padded = (nx + 2 * halo) * (ny + 2 * halo) * (nz + 2 * halo)
    return 6 * padded * es + 3 * nx * ny * nz * es


def time_launches(torch, launch, nsets, steps, warmup, stream):
    """Run ``launch(i)`` for warmup + steps iterations (i = buffer set) and
    time the steps back to back: a wall clock between two device
    synchronisations, and two HIP events on ``stream`` around the same
    region.  Returns (wall ms per step, event ms per launch).  No event sits
    between launches: an event with timing makes the next kernel wait until
    the previous one has drained, which costs several microseconds per step
    and is not part of the kernel."""
    for i in range(warmup):
        launch(i % nsets)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for i in range(steps):
        launch(i % nsets)
    b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return wall / steps, a.elapsed_time(b) / steps


def prewarm(torch, launch, nsets, min_ms):
    """Launch ``launch(i)`` in batches of 50 until at least ``min_ms`` of wall
    time has passed (the GPU clocks ramp up over the first ~100 launches);
    untimed, before the counted warm-up.  Returns (launches, wall ms)."""
    n, t0 = 0, time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < min_ms:
        for _ in range(50):
            launch(n % nsets)
            n += 1
        torch.cuda.synchronize()
    return n, (time.perf_counter() - t0) * 1e3


def time_blocks(torch, launch, nsets, steps, warmup, stream, blocks=5):
    """Like time_launches, with HIP events also at the boundaries of
    ``blocks`` equal runs of back-to-back launches inside the timed region
    (the paper reports the mean of five runs).  Returns (wall ms per step,
    event ms per launch over all steps, [event ms per launch of each
    block])."""
    for i in range(warmup):
        launch(i % nsets)
    torch.cuda.synchronize()
    bounds = [round(b * steps / blocks) for b in range(blocks + 1)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in bounds]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for b in range(blocks):
        for i in range(bounds[b], bounds[b + 1]):
            launch(i % nsets)
        ev[b + 1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    per_block = [ev[b].elapsed_time(ev[b + 1]) / max(1, bounds[b + 1] - bounds[b]) for b in range(blocks)]
    return wall / steps, ev[0].elapsed_time(ev[-1]) / steps, per_block


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_oracle(oracle, fields, coeffs, nthreads, seconds, max_reps=1000):
    """Repeat the FP64 oracle on the full grid for about ``seconds``;
    returns the list of per-repetition times (s)."""
    times = []
    while sum(times) < seconds and len(times) < max_reps:
        t0 = time.perf_counter()
        oracle.forward(*fields, coeffs, nthreads=nthreads)
        times.append(time.perf_counter() - t0)
    return times


def prebuilt_forward(B, ins, outs, coeffs, stream, tile=None):
    """ctypes arguments of one pw_advect_ex call, built once (the timed loop
    then only crosses the C ABI)."""
    from paper_2301_13016_amd.binding import _dtype_code, _grid_from, _layout_from
    u, v, w = ins
    su, sv, sw = outs
    keep = (_grid_from(u, 1), _layout_from(u, su), coeffs.c_struct(),
            B.pw_tile(*tile) if tile else None)
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u),
            u.data_ptr(), v.data_ptr(), w.data_ptr(), ctypes.byref(keep[2]),
            su.data_ptr(), sv.data_ptr(), sw.data_ptr(),
            ctypes.byref(keep[3]) if tile else None, ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_advect_ex

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_advect_ex")
    call.keep = keep
    return call


def prebuilt_epilogue(B, ins, outs, coeffs, alpha, stream):
    """ctypes arguments of one pw_advect_epilogue call accumulating into
    ``outs`` (out += alpha * F), built once."""
    from paper_2301_13016_amd.binding import _dtype_code, _grid_from, _layout_from
    u, v, w = ins
    keep = (_grid_from(u, 1), _layout_from(u, outs[0]), coeffs.c_struct(),
            B.pw_epilogue(float(alpha), *(x.data_ptr() for x in outs)))
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u),
            u.data_ptr(), v.data_ptr(), w.data_ptr(), ctypes.byref(keep[2]), ctypes.byref(keep[3]),
            *(x.data_ptr() for x in outs), None, ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_advect_epilogue

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_advect_epilogue")
    call.keep = keep
    return call


def prebuilt_zfast(B, ins, outs, coeffs, stream, accumulate=False):
    """ctypes arguments of one pw_advect_zfast call (arrays stored z-fastest,
    indexed [i, j, k]), built once; with ``accumulate`` the fused epilogue
    out += F (pw_advect_zfast_epilogue)."""
    from paper_2301_13016_amd.binding import _dtype_code
    u, v, w = ins
    pi, pj, pk = u.shape
    keep = (B.pw_grid(pi - 2, pj - 2, pk - 2, 1),
            B.pw_layout_zfast(u.stride(1), u.stride(0), outs[0].stride(1), outs[0].stride(0)), coeffs.c_struct(),
            B.pw_epilogue(1.0, *(o.data_ptr() for o in outs)))
    ep = (ctypes.byref(keep[3]),) if accumulate else ()
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(),
            ctypes.byref(keep[2]), *ep, *(o.data_ptr() for o in outs), None, ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_advect_zfast_epilogue if accumulate else B.lib().pw_advect_zfast

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_advect_zfast")
    call.keep = keep
    return call


def prebuilt_bc(B, ins, outs, coeffs, bc, stream):
    """ctypes arguments of one pw_advect_bc call (boundary rules by
    addressing, one (x, y, z) triple per field, no epilogue), built once."""
    from paper_2301_13016_amd.binding import _dtype_code, _grid_from, _layout_from
    u, v, w = ins
    rules = (B.pw_halo_modes * 3)(*(B.pw_halo_modes(*m) for m in bc))
    keep = (_grid_from(u, 1), _layout_from(u, outs[0]), coeffs.c_struct(), rules)
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(),
            ctypes.byref(keep[2]), keep[3], None, *(o.data_ptr() for o in outs), None,
            ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_advect_bc

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_advect_bc")
    call.keep = keep
    return call


def prebuilt_halo(B, fields, modes, stream):
    """ctypes arguments of one pw_halo_fill call over ``fields``, built once."""
    from paper_2301_13016_amd.binding import _dtype_code, _grid_from
    u = fields[0]
    g = _grid_from(u, 1)
    keep = (g, B.pw_layout(u.stride(1), u.stride(0), g.nx, g.nx * g.ny),
            (ctypes.c_void_p * len(fields))(*(f.data_ptr() for f in fields)),
            (B.pw_halo_modes * len(fields))(*(B.pw_halo_modes(*m) for m in modes)))
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u), keep[2], keep[3], len(fields),
            ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_halo_fill

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_halo_fill")
    call.keep = keep
    return call


B_HALO_ZERO = 3   # PW_HALO_ZERO


def halo_bytes(nx, ny, nz, h, es, modes):
    """Algorithmic bytes of one halo fill: every written cell once, and its
    source once unless the cell is zeroed."""
    px, py = nx + 2 * h, ny + 2 * h
    total = 0
    for mx, my, mz in modes:
        zc = 2 * h * py * px
        cells = zc + nz * 2 * h * px + nz * ny * 2 * h
        zero = zc if mz == B_HALO_ZERO else 0
        total += (2 * cells - zero) * es
    return total


def prebuilt_tangent(B, ins, dirs, outs, coeffs, stream):
    """ctypes arguments of one pw_advect_tangent_ex call, built once."""
    from paper_2301_13016_amd.binding import _dtype_code, _grid_from, _layout_from
    u, v, w = ins
    keep = (_grid_from(u, 1), _layout_from(u, outs[0]), coeffs.c_struct())
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u),
            u.data_ptr(), v.data_ptr(), w.data_ptr(), ctypes.byref(keep[2]),
            *(x.data_ptr() for x in dirs), *(x.data_ptr() for x in outs),
            None, ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_advect_tangent_ex

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_advect_tangent_ex")
    call.keep = keep
    return call


def prebuilt_coeff_grad(B, ins, cots, stream, torch):
    """ctypes arguments of one pw_advect_coeff_grad call (output and
    workspace allocated here, once)."""
    from paper_2301_13016_amd.binding import _dtype_code, _grid_from, _layout_from
    u, v, w = ins
    grid = _grid_from(u, 1)
    need = ctypes.c_int64()
    B.lib().pw_advect_coeff_grad_workspace(ctypes.byref(grid), _dtype_code(u), ctypes.byref(need))
    out = torch.empty(6 * int(grid.nz) + 2, dtype=torch.float64, device=u.device)
    ws = torch.empty(max(1, need.value // 8), dtype=torch.float64, device=u.device)
    keep = (grid, _layout_from(u, cots[0]), out, ws)
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(),
            *(x.data_ptr() for x in cots), out.data_ptr(), ws.data_ptr(), need.value,
            ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_advect_coeff_grad

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_advect_coeff_grad")
    call.keep = keep
    return call


def prebuilt_fused_backward(B, ins, cots, grads, coeffs, stream, torch):
    """ctypes arguments of one pw_advect_adjoint_coeff_grad call (wind and
    coefficient gradients in one pass; output and workspace allocated here)."""
    from paper_2301_13016_amd.binding import _dtype_code, _grid_from, _layout_from
    u, v, w = ins
    grid = _grid_from(u, 1)
    need = ctypes.c_int64()
    B.lib().pw_advect_coeff_grad_workspace(ctypes.byref(grid), _dtype_code(u), ctypes.byref(need))
    out = torch.empty(6 * int(grid.nz) + 2, dtype=torch.float64, device=u.device)
    ws = torch.empty(max(1, need.value // 8), dtype=torch.float64, device=u.device)
    keep = (grid, _layout_from(u, cots[0]), coeffs.c_struct(), out, ws)
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(),
            ctypes.byref(keep[2]), *(x.data_ptr() for x in cots), *(x.data_ptr() for x in grads), out.data_ptr(),
            ws.data_ptr(), need.value, ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_advect_adjoint_coeff_grad

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_advect_adjoint_coeff_grad")
    call.keep = keep
    return call


def prebuilt_adjoint(B, ins, cots, grads, coeffs, stream):
    """ctypes arguments of one pw_advect_adjoint_ex call, built once."""
    from paper_2301_13016_amd.binding import _dtype_code, _grid_from, _layout_from
    u, v, w = ins
    keep = (_grid_from(u, 1), _layout_from(u, cots[0]), coeffs.c_struct())
    args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), _dtype_code(u),
            u.data_ptr(), v.data_ptr(), w.data_ptr(), ctypes.byref(keep[2]),
            *(x.data_ptr() for x in cots), *(x.data_ptr() for x in grads),
            None, ctypes.c_void_p(stream.cuda_stream))
    fn = B.lib().pw_advect_adjoint_ex

    def call():
        st = fn(*args)
        if st != B.PW_OK:
            raise B.PWError(st, B.pw_last_error(), "pw_advect_adjoint_ex")
    call.keep = keep
    return call


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps first (about 16 ms: the clocks settle within the first ~100)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate host time spent timing the oracle on all cores (half of it again on 1)")
    ap.add_argument("--prewarm-ms", type=float, default=150.0,
                    help="wall time of untimed headline launches before the counted warm-up")
    ap.add_argument("--forms", default="all",
                    help="comma-separated forms to time besides the headline step, the bandwidth probe and the "
                         "CPU baseline (which always run): c1 (more forms on the headline grid: halo fill, "
                         "boundaries by addressing, z-fastest layout), precision (1024x1024x256 FP32, "
                         "BF16, FP16, FP64), differentiation (256x256x128 adjoint, tangent, coefficient "
                         "gradients, fused backward), batched (64 subdomains); default all")
    args = ap.parse_args()
    known = ("c1", "precision", "differentiation", "batched")
    forms_sel = set(known) if args.forms == "all" else {f.strip() for f in args.forms.split(",") if f.strip()}
    if not forms_sel <= set(known):
        ap.error("--forms: unknown %s (choose from all, %s)" % (", ".join(sorted(forms_sel - set(known))),
                                                                 ", ".join(known)))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: libpwadv runs on one GPU (the stencil's multi-GPU halo exchange is a "
              "design, not an implementation); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_2301_13016_amd import binding as B
    from paper_2301_13016_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    log("device:", torch.cuda.get_device_name(dev), "lib:", B.pw_version())

    # ------------------------------------------------------------ headline: c1 FP32
    cfg = wl.C1
    nx, ny, nz, h = cfg["nx"], cfg["ny"], cfg["nz"], 1
    tiles = {}
    g = wl.config_grid(cfg)
    coeffs = B.Coeffs.from_host(g.coeffs, device=dev)
    nsets = 4
    host = [torch.from_numpy(x) for x in (g.u, g.v, g.w)]
    calls = []
    keep = []
    for _ in range(nsets):
        ins = [x.to(dev) for x in host]
        outs = tuple(torch.empty((nz, ny, nx), device=dev) for _ in range(3))
        keep.append((ins, outs))
        calls.append(prebuilt_forward(B, ins, outs, coeffs, stream))

    forms = {}
    pre_n, pre_ms = prewarm(torch, lambda i: calls[i](), nsets, args.prewarm_ms)
    log("pre-warm: %d launches in %.0f ms" % (pre_n, pre_ms))
    ms_step, k_ms, k_blocks = time_blocks(torch, lambda i: calls[i](), nsets, args.steps, args.warmup, stream)
    k_median = float(np.median(k_blocks))
    # fused accumulation on the same grid and buffers: out += F (reads the outputs too)
    acc_calls = [prebuilt_epilogue(B, kp[0], kp[1], coeffs, 1.0, stream) for kp in keep]
    _, acc_ms = time_launches(torch, lambda i: acc_calls[i](), nsets, 100, 10, stream)
    del acc_calls
    pts = nx * ny * nz
    gpts = pts / (ms_step * 1e-3) / 1e9
    nbytes = algo_bytes(nx, ny, nz, h, 4)
    achieved = nbytes / (k_ms * 1e-3) / 1e9
    log("c1 fp32: %.4f ms/step, kernel %.4f ms (median of 5 blocks %.4f), %.1f Gpt/s, %.0f GB/s algorithmic"
        % (ms_step, k_ms, k_median, gpts, achieved))

    # plain copy kernel of the same byte count (reachable-bandwidth reference)
    cbytes = (nbytes // 2) // 16 * 16
    srcs = [torch.empty(cbytes // 4, device=dev) for _ in range(4)]
    dsts = [torch.empty_like(s) for s in srcs]
    _, copy_ms = time_launches(torch, lambda i: B.stream_copy(srcs[i], dsts[i]), 4, 200, 10, stream)
    copy_gbs = 2 * cbytes / (copy_ms * 1e-3) / 1e9
    log("copy %d MB each way: %.4f ms, %.0f GB/s" % (cbytes >> 20, copy_ms, copy_gbs))
    del srcs, dsts
    # three-stream copy: the stencil's pattern (three arrays read, three
    # written), each the size of one output array
    obytes = nx * ny * nz * 4
    sets3 = [([torch.empty(obytes // 4, device=dev) for _ in range(3)],
              [torch.empty(obytes // 4, device=dev) for _ in range(3)]) for _ in range(4)]
    _, c3_ms = time_launches(torch, lambda i: B.stream_copy3(*sets3[i]), 4, 200, 10, stream)
    copy3_gbs = 6 * obytes / (c3_ms * 1e-3) / 1e9
    log("three-stream copy 3 x %d MB each way: %.4f ms, %.0f GB/s" % (obytes >> 20, c3_ms, copy3_gbs))
    # reachable bandwidth: the probe kernel (copy, read-only, write-only) swept
    # over loads in flight per lane, cache policy and workgroup count, on
    # 512 MiB buffers (twice the MALL), four sets in rotation
    pb = 512 << 20
    psrc = [torch.empty(pb // 4, device=dev) for _ in range(4)]
    pdst = [torch.empty(pb // 4, device=dev) for _ in range(4)]
    for x in psrc:
        x.fill_(1.0)
    sink = torch.zeros(1024, dtype=torch.int32, device=dev)
    reach = {}
    for mode, name, loads_list, flag_list in ((0, "copy", (1, 2, 4, 8), (0, 1, 2, 3)), (1, "read", (1, 4, 8), (0, 1)),
                                              (2, "write", (1, 4), (0, 2))):
        best = None
        for loads in loads_list:
            for flags in flag_list:
                for blocks in (512, 1024, 2048, 4096, 8192, 16384, 32768):
                    def probe(i, mode=mode, loads=loads, flags=flags, blocks=blocks):
                        if mode == 1:
                            B.stream_probe(1, loads, flags, psrc[i], sink, blocks)
                        else:
                            B.stream_probe(mode, loads, flags, psrc[i], pdst[i], blocks)
                    _, pms = time_launches(torch, probe, 4, 20, 3, stream)
                    gbs = (2 if mode == 0 else 1) * pb / (pms * 1e-3) / 1e9
                    if best is None or gbs > best["gbs"]:
                        best = dict(gbs=round(gbs, 1), loads_per_lane=loads, nt_loads=bool(flags & 1),
                                    nt_stores=bool(flags & 2), blocks=blocks)
        reach[name] = best
    log("reachable bandwidth (best of the probe sweep): copy %.0f GB/s, read %.0f GB/s, write %.0f GB/s"
        % (reach["copy"]["gbs"], reach["read"]["gbs"], reach["write"]["gbs"]))
    forms["reachable_bandwidth"] = reach
    del psrc, pdst, sink
    nbytes_acc = nbytes + 3 * nx * ny * nz * 4
    forms["fused_accumulate_512x512x64"] = dict(
        kernel_ms=round(acc_ms, 4), over_plain=round(acc_ms / k_ms, 3),
        ideal_ratio_from_bytes=round(nbytes_acc / nbytes, 3), hbm_gbs=round(nbytes_acc / (acc_ms * 1e-3) / 1e9, 1))
    log("c1 fused accumulate (out += F): %.4f ms, %.3f x the plain step" % (acc_ms, acc_ms / k_ms))
    if "c1" in forms_sel:
        # the step before: halo fill of u, v, w (periodic x, y; free-slip lid:
        # u, v zero-gradient, w zero), on the same buffers
        hmodes = [(1, 1, 2), (1, 1, 2), (1, 1, B_HALO_ZERO)]
        halo_calls = [prebuilt_halo(B, kp[0], hmodes, stream) for kp in keep]
        _, halo_ms = time_launches(torch, lambda i: halo_calls[i](), nsets, 200, 20, stream)
        del halo_calls
        hb = halo_bytes(nx, ny, nz, h, 4, hmodes)
        forms["halo_fill_512x512x64"] = dict(kernel_ms=round(halo_ms, 4), over_plain=round(halo_ms / k_ms, 3),
                                             bytes=hb, hbm_gbs=round(hb / (halo_ms * 1e-3) / 1e9, 1))
        log("c1 halo fill (u, v, w): %.4f ms, %.3f x the plain step" % (halo_ms, halo_ms / k_ms))
        # boundaries applied by addressing inside the forward, no fill step:
        # remapped reads only (periodic x, y; zero-gradient z for all three
        # fields), and the free-slip lid above, whose w = 0 is a value rule
        addressed = {}
        for name, rules in (("periodic_copy", [(1, 1, 2)] * 3), ("free_slip_lid", hmodes)):
            fill_calls = [prebuilt_halo(B, kp[0], rules, stream) for kp in keep]
            _, fill_ms = time_launches(torch, lambda i: fill_calls[i](), nsets, 200, 20, stream)
            bc_calls = [prebuilt_bc(B, kp[0], kp[1], coeffs, rules, stream) for kp in keep]
            _, bc_ms = time_launches(torch, lambda i: bc_calls[i](), nsets, 500, 100, stream)
            del fill_calls, bc_calls
            addressed[name] = dict(rules=rules, kernel_ms=round(bc_ms, 4), over_plain=round(bc_ms / k_ms, 3),
                                   fill_ms=round(fill_ms, 4), fill_then_forward_ms=round(fill_ms + k_ms, 4),
                                   saved=round(1 - bc_ms / (fill_ms + k_ms), 3))
            log("c1 forward with %s boundaries by addressing: %.4f ms (fill + forward %.4f ms)"
                % (name.replace("_", " "), bc_ms, fill_ms + k_ms))
        forms["boundaries_by_addressing_512x512x64"] = addressed
        # the same grid stored z-fastest (column-major, [i, j, k])
        zsets = [(tuple(x.permute(2, 1, 0).contiguous() for x in kp[0]),
                  tuple(torch.empty((nx, ny, nz), device=dev) for _ in range(3))) for kp in keep]
        zf_calls = [prebuilt_zfast(B, zi, zo, coeffs, stream) for zi, zo in zsets]
        _, zf_ms = time_launches(torch, lambda i: zf_calls[i](), nsets, 500, 100, stream)
        # the x-fastest step again, under the same conditions
        _, xf_ms = time_launches(torch, lambda i: calls[i](), nsets, 500, 100, stream)
        zacc_calls = [prebuilt_zfast(B, zi, zo, coeffs, stream, accumulate=True) for zi, zo in zsets]
        _, zacc_ms = time_launches(torch, lambda i: zacc_calls[i](), nsets, 200, 20, stream)
        zshape = B.launch_shape("zfast", nx, ny, nz, torch.float32)
        del zf_calls, zacc_calls, zsets
        forms["zfast_512x512x64"] = dict(kernel_ms=round(zf_ms, 4), over_xfast=round(zf_ms / xf_ms, 3),
                                         accumulate_ms=round(zacc_ms, 4),
                                         gpts=round(pts / (zf_ms * 1e-3) / 1e9, 2),
                                         hbm_gbs=round(nbytes / (zf_ms * 1e-3) / 1e9, 1), tile=list(zshape))
        log("c1 z-fastest layout: %.4f ms, %.3f x the x-fastest step timed after it (%.4f ms; tile %s)"
            % (zf_ms, zf_ms / xf_ms, xf_ms, zshape))
    del keep, calls, sets3
    torch.cuda.empty_cache()

    # ------------------------------------------------------------ CPU baseline (oracle)
    ncpu = len(os.sched_getaffinity(0))
    f64 = [x.astype(np.float64) for x in (g.u, g.v, g.w)]
    t_all = time_oracle(oracle, f64, g.coeffs, ncpu, args.cpu_seconds)
    t_one = time_oracle(oracle, f64, g.coeffs, 1, args.cpu_seconds / 2)
    cpu_gpts = len(t_all) * pts / sum(t_all) / 1e9
    cpu_gpts_median = pts / float(np.median(t_all)) / 1e9
    cpu1_gpts = len(t_one) * pts / sum(t_one) / 1e9
    log("oracle on %d host threads: %.3f Gpt/s (median %.3f; %d reps of the full grid); on 1 thread %.4f Gpt/s"
        % (ncpu, cpu_gpts, cpu_gpts_median, len(t_all), cpu1_gpts))
    del f64

    # ------------------------------------------------------------ precision form: c2
    if "precision" in forms_sel:
        c2 = wl.C2
        n2 = (c2["nx"], c2["ny"], c2["nz"])
        log("generating the 1024x1024x256 grid ...")
        g2 = wl.config_grid(c2)
        co2 = B.Coeffs.from_host(g2.coeffs, device=dev)
        co2_64 = B.Coeffs.from_host(g2.coeffs, device=dev, dtype=torch.float64)
        f32 = [torch.from_numpy(x).to(dev) for x in (g2.u, g2.v, g2.w)]
        del g2
        outs2 = tuple(torch.empty((n2[2], n2[1], n2[0]), device=dev) for _ in range(3))
        pts2 = n2[0] * n2[1] * n2[2]
        res2 = {}
        for name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16), ("fp16", torch.float16)):
            ins = f32 if dt == torch.float32 else [x.to(dt) for x in f32]
            call = prebuilt_forward(B, ins, outs2, co2, stream)
            _, kms2 = time_launches(torch, lambda i: call(), 1, 30, 3, stream)
            eb = 2 if dt != torch.float32 else 4
            res2[name] = dict(gpts=round(pts2 / (kms2 * 1e-3) / 1e9, 2), kernel_ms=round(kms2, 4),
                              hbm_gbs=round(algo_bytes(*n2, 1, eb) / (kms2 * 1e-3) / 1e9, 1))
            log("c2 %s: kernel %.4f ms, %.1f Gpt/s" % (name, kms2, res2[name]["gpts"]))
            if dt != torch.float32:
                del ins
        # FP64 storage and arithmetic (the FP32 values widened exactly)
        del outs2
        outs64 = tuple(torch.empty((n2[2], n2[1], n2[0]), device=dev, dtype=torch.float64) for _ in range(3))
        ins64 = [x.double() for x in f32]
        call = prebuilt_forward(B, ins64, outs64, co2_64, stream)
        _, kms64 = time_launches(torch, lambda i: call(), 1, 30, 3, stream)
        res2["fp64"] = dict(gpts=round(pts2 / (kms64 * 1e-3) / 1e9, 2), kernel_ms=round(kms64, 4),
                            hbm_gbs=round(algo_bytes(*n2, 1, 8, 8) / (kms64 * 1e-3) / 1e9, 1))
        log("c2 fp64: kernel %.4f ms, %.1f Gpt/s" % (kms64, res2["fp64"]["gpts"]))
        del call, ins64, outs64
        for name in ("bf16", "fp16", "fp64"):
            res2[name]["speed_vs_fp32"] = round(res2["fp32"]["kernel_ms"] / res2[name]["kernel_ms"], 3)
        forms["precision_1024x1024x256"] = res2
        del f32
        torch.cuda.empty_cache()

    # ------------------------------------------------------------ differentiation form: c4
    if "differentiation" in forms_sel:
        c4 = wl.C4
        n4 = (c4["nx"], c4["ny"], c4["nz"])
        g4 = wl.config_grid(c4)
        co4 = B.Coeffs.from_host(g4.coeffs, device=dev)
        # 4 buffer sets (about 4 x 540 MB) so that the MALL cannot serve repeats
        host4 = [torch.from_numpy(x) for x in (g4.u, g4.v, g4.w)]
        hcot4 = [torch.from_numpy(x) for x in wl.cotangents(*n4, c4["cot_seed"])]
        hdir4 = [torch.from_numpy(x.astype(np.float32)) for x in wl.direction(*n4, seed=46)]
        fcalls, acalls, tcalls, ccalls, bcalls, keep4 = [], [], [], [], [], []
        for _ in range(4):
            ins4 = [x.to(dev) for x in host4]
            cot4 = [x.to(dev) for x in hcot4]
            dir4 = [x.to(dev) for x in hdir4]
            o4 = tuple(torch.empty((n4[2], n4[1], n4[0]), device=dev) for _ in range(3))
            t4 = tuple(torch.empty((n4[2], n4[1], n4[0]), device=dev) for _ in range(3))
            gr4 = tuple(torch.empty_like(x) for x in ins4)
            keep4.append((ins4, cot4, dir4, o4, t4, gr4))
            fcalls.append(prebuilt_forward(B, ins4, o4, co4, stream))
            acalls.append(prebuilt_adjoint(B, ins4, cot4, gr4, co4, stream))
            tcalls.append(prebuilt_tangent(B, ins4, dir4, t4, co4, stream))
            ccalls.append(prebuilt_coeff_grad(B, ins4, cot4, stream, torch))
            bcalls.append(prebuilt_fused_backward(B, ins4, cot4, gr4, co4, stream, torch))
        _, fms = time_launches(torch, lambda i: fcalls[i](), 4, 100, 5, stream)
        _, ams = time_launches(torch, lambda i: acalls[i](), 4, 100, 5, stream)
        _, tms = time_launches(torch, lambda i: tcalls[i](), 4, 100, 5, stream)
        _, cms = time_launches(torch, lambda i: ccalls[i](), 4, 100, 5, stream)
        _, bms = time_launches(torch, lambda i: bcalls[i](), 4, 100, 5, stream)
        pts4 = n4[0] * n4[1] * n4[2]
        forms["adjoint_256x256x128"] = dict(
            forward_ms=round(fms, 4), adjoint_ms=round(ams, 4), adjoint_over_forward=round(ams / fms, 3),
            ideal_ratio_from_bytes=round(adjoint_bytes(*n4, 1) / algo_bytes(*n4, 1, 4), 3),
            adjoint_gpts=round(pts4 / (ams * 1e-3) / 1e9, 2),
            adjoint_hbm_gbs=round(adjoint_bytes(*n4, 1) / (ams * 1e-3) / 1e9, 1))
        tbytes = tangent_bytes(*n4, 1)
        forms["tangent_256x256x128"] = dict(
            tangent_ms=round(tms, 4), tangent_over_forward=round(tms / fms, 3),
            ideal_ratio_from_bytes=round(tbytes / algo_bytes(*n4, 1, 4), 3),
            tangent_gpts=round(pts4 / (tms * 1e-3) / 1e9, 2), tangent_hbm_gbs=round(tbytes / (tms * 1e-3) / 1e9, 1))
        cbytes4 = adjoint_bytes(*n4, 1) - 3 * (n4[0] + 2) * (n4[1] + 2) * (n4[2] + 2) * 4   # its reads only
        forms["coeff_grad_256x256x128"] = dict(
            coeff_grad_ms=round(cms, 4), coeff_grad_over_forward=round(cms / fms, 3),
            ideal_ratio_from_bytes=round(cbytes4 / algo_bytes(*n4, 1, 4), 3),
            coeff_grad_hbm_gbs=round(cbytes4 / (cms * 1e-3) / 1e9, 1))
        forms["fused_backward_256x256x128"] = dict(
            backward_ms=round(bms, 4), over_adjoint=round(bms / ams, 3), separate_ms=round(ams + cms, 4),
            backward_over_forward=round(bms / fms, 3))
        log("c4: forward %.4f ms, adjoint %.4f ms (ratio %.3f), tangent %.4f ms (ratio %.3f), "
            "coefficient gradients %.4f ms (ratio %.3f)" % (fms, ams, ams / fms, tms, tms / fms, cms, cms / fms))
        log("c4: wind and coefficient gradients in one pass %.4f ms (%.3f x the adjoint; separately %.4f ms)"
            % (bms, bms / ams, ams + cms))
        del keep4, fcalls, acalls, tcalls, ccalls, bcalls
        torch.cuda.empty_cache()

    # ------------------------------------------------------------ batched form: c3
    if "batched" in forms_sel:
        log("generating the 64 subdomains ...")
        grids3 = wl.batch_grids()
        subs, plain = [], []
        for gg in grids3:
            ins = [torch.from_numpy(x).to(dev) for x in (gg.u, gg.v, gg.w)]
            cc = B.Coeffs.from_host(gg.coeffs, device=dev)
            outs = tuple(torch.empty((gg.nz, gg.ny, gg.nx), device=dev) for _ in range(3))
            subs.append((*ins, cc, outs))
            plain.append(prebuilt_forward(B, ins, outs, cc, stream))
        pts3 = sum(gg.points for gg in grids3)
        bytes3 = sum(algo_bytes(gg.nx, gg.ny, gg.nz, 1, 4) for gg in grids3)
        del grids3
        batch = B.Batch(subs)
        btile = batch.tune()
        gstream = torch.cuda.Stream()
        batch.capture(gstream)
        torch.cuda.synchronize()

        def all_plain(i):
            for c in plain:
                c()
        pms_step, _ = time_launches(torch, all_plain, 1, 20, 2, stream)
        gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
        for _ in range(2):
            batch.replay(gstream)
        torch.cuda.synchronize()
        for a_, b_ in gev:
            a_.record(gstream)
            batch.replay(gstream)
            b_.record(gstream)
        torch.cuda.synchronize()
        bms = float(np.mean([a_.elapsed_time(b_) for a_, b_ in gev]))
        tile3, items3, groups3 = batch.info()
        forms["batched_64_subdomains"] = dict(
            points=pts3, graph_replay_ms=round(bms, 4), plain_64_launches_ms=round(pms_step, 4),
            speedup_vs_plain=round(pms_step / bms, 3), gpts=round(pts3 / (bms * 1e-3) / 1e9, 2),
            hbm_gbs=round(bytes3 / (bms * 1e-3) / 1e9, 1), tile=tile3, work_items=items3, workgroups=groups3)
        log("c3: graph replay %.4f ms vs 64 plain launches %.4f ms (tile %s)" % (bms, pms_step, btile))
        batch.close()
        del subs, plain

    line = {
        "metric": "PW advection Gpoints/s + % HBM roofline; FP32 vs BF16-store vs adjoint",
        "value": round(gpts, 3),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "prewarm": {"launches": pre_n, "ms": round(pre_ms, 1)},
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded uniform winds in [-10,10], per-level coefficients)",
        "config": {"workload": cfg["name"], "nx": nx, "ny": ny, "nz": nz, "halo": h,
                   "points": pts, "buffer_sets": nsets},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("pw_forward_f32_512x512x64"),
                     "algorithmic_bytes_per_launch": nbytes, "kernel_ms": round(k_ms, 6),
                     "kernel_ms_median_of_blocks": round(k_median, 6),
                     "kernel_ms_blocks": [round(x, 6) for x in k_blocks],
                     "copy_kernel_gbs": round(copy_gbs, 1), "copy3_kernel_gbs": round(copy3_gbs, 1),
                     "reachable_copy_gbs": forms["reachable_bandwidth"]["copy"]["gbs"],
                     "frac_of_reachable_copy": round(achieved / forms["reachable_bandwidth"]["copy"]["gbs"], 4)},
        "cpu_baseline": {"value": round(cpu_gpts, 4), "unit": "Gpoints/s", "cores": ncpu, "kind": "oracle",
                         "sample": "FP64 oracle on the full 512x512x64 grid, %d repetitions (%.1f s) on %d "
                                   "threads; %d repetitions (%.1f s) on 1 thread"
                                   % (len(t_all), sum(t_all), ncpu, len(t_one), sum(t_one)),
                         "median": round(cpu_gpts_median, 4), "value_1_thread": round(cpu1_gpts, 5),
                         "cpu_model": cpu_model(),
                         "useful_gflops": round(cpu_gpts * 63, 2)},
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
