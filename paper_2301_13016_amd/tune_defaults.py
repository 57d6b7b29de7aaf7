"""Regenerate the built-in tuning table (csrc/pw_tune_defaults.inc) on the GPU.

Runs the library's autotuner (pw_tune) for the shape classes the library is
benchmarked and tested on and writes the chosen launch shapes as C
initialisers.  Each forward pick is then re-timed against the shapes next to
it (1, 2 or 4 rows per strip, 1-8 z-chunks, its other choices kept) on
separately allocated fields, as callers hold them -- the tuner times one packed
allocation, and the two orders of memory can rank close shapes differently --
in interleaved rounds, and a neighbour replaces the pick when its median is
at least 0.5 % lower.  Rebuild the library afterwards.  Usage (on an MI355X):

    python paper_2301_13016_amd/tune_defaults.py [output.inc]
"""
import ctypes
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

# (nx, ny, nz, dtype name, flags): forward for all storage types, adjoint and
# tangent for FP32/FP64, the z-fastest forward for the FP32 / FP64 classes
SHAPES = [
    (512, 512, 64, "float32", 15),
    (1024, 1024, 256, "float32", 9),
    (1024, 1024, 256, "bfloat16", 1),
    (1024, 1024, 256, "float16", 1),
    (256, 256, 128, "float32", 15),
    (64, 64, 64, "float64", 15),
    (16, 16, 16, "float64", 7),
    (128, 128, 128, "float32", 15),
    (256, 256, 256, "float32", 9),
    (512, 512, 128, "float32", 9),
    (1024, 1024, 256, "float64", 1),
    (512, 512, 64, "float64", 1),
]


def ceil_log2(x):
    return (int(x) - 1).bit_length()


def neighbours(tile, nz):
    """The forward shape ``tile`` and the shapes next to it: the same columns
    per lane, waves per group, prefetch and row sharing, with 1, 2 or 4 rows
    per strip and the tuner's z-chunk counts (1, 2, 3, 4, 6, 8)."""
    px, _, _, wpb, depth, share = tile
    out = [tuple(tile)]
    for ry in (1, 2, 4):
        for nzc in (1, 2, 3, 4, 6, 8):
            t = (px, ry, -(-nz // nzc), wpb, depth, share)
            if t not in out:
                out.append(t)
    return out


def confirm_forward(B, torch, nx, ny, nz, dtype, pick, rounds=5, sets=2):
    """Re-time ``pick`` and its neighbours on separately allocated fields
    (winds uniform in [-10, 10), coefficients of the workloads' scale),
    rotating over ``sets`` buffer sets, in ``rounds`` interleaved rounds of
    about 20 ms per shape (forward, backward, ... order).  Returns the shape
    with the lowest median if that is at least 0.5 % below the pick's, else
    the pick, and the medians in microseconds."""
    gen = torch.Generator(device="cuda").manual_seed(7)
    cdt = torch.float64 if dtype == torch.float64 else torch.float32
    padded = (nz + 2, ny + 2, nx + 2)
    fields = [[(torch.rand(padded, device="cuda", generator=gen, dtype=cdt) * 20 - 10).to(dtype) for _ in range(3)]
              for _ in range(sets)]
    outs = [[torch.empty((nz, ny, nx), device="cuda", dtype=cdt) for _ in range(3)] for _ in range(sets)]
    coeffs = B.Coeffs(0.0025, 0.0025, *[(torch.rand(nz, device="cuda", generator=gen, dtype=cdt) + 0.5) * 0.005
                                        for _ in range(4)])
    stream = torch.cuda.current_stream()
    fn = B.lib().pw_advect_ex

    def prebuilt(tile, i):   # ctypes arguments built once: the timed loop only crosses the C ABI
        u, v, w = fields[i]
        keep = (B._grid_from(u, 1), B._layout_from(u, outs[i][0]), coeffs.c_struct(), B.pw_tile(*tile))
        args = (ctypes.byref(keep[0]), ctypes.byref(keep[1]), B._dtype_code(u), u.data_ptr(), v.data_ptr(),
                w.data_ptr(), ctypes.byref(keep[2]), *(o.data_ptr() for o in outs[i]), ctypes.byref(keep[3]),
                ctypes.c_void_p(stream.cuda_stream))

        def call():
            st = fn(*args)
            if st != B.PW_OK:
                raise B.PWError(st, B.pw_last_error(), "pw_advect_ex")
        call.keep = keep
        return call

    calls = {}
    for t in neighbours(pick, nz):
        try:
            c = [prebuilt(t, i) for i in range(sets)]
            c[0]()
        except B.PWError:
            continue
        calls[t] = c
    torch.cuda.synchronize()

    def timed(t, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(n):
            calls[t][i % sets]()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / n * 1e3

    for _ in range(100):                       # clocks settle
        calls[tuple(pick)][0]()
    reps = {t: max(10, min(500, int(20e3 / timed(t, 10)))) for t in calls}
    med = {t: [] for t in calls}
    order = list(calls)
    for r in range(rounds):
        for t in (order if r % 2 == 0 else order[::-1]):
            med[t].append(timed(t, reps[t]))
    med = {t: statistics.median(v) for t, v in med.items()}
    best = min(med, key=med.get)
    del fields, outs
    torch.cuda.empty_cache()
    return (best if med[best] < 0.995 * med[tuple(pick)] else tuple(pick)), med


def main(out_path):
    import torch
    from paper_2301_13016_amd import binding as B
    code = {"float32": B.PW_F32, "float64": B.PW_F64, "bfloat16": B.PW_BF16, "float16": B.PW_F16}
    tdt = {"float32": torch.float32, "float64": torch.float64, "bfloat16": torch.bfloat16, "float16": torch.float16}
    lines = ["// kind, dtype, log2 nx, log2 ny, log2 nz, cols/lane, rows/strip, z-chunks, waves/group, prefetch, "
             "share_rows",
             "// (kind 3, z-fastest: levels/lane, rows/strip, x-chunks, waves/group, prefetch, 0)",
             "// generated on %s by paper_2301_13016_amd/tune_defaults.py, unedited (forward rows: pw_tune's "
             "pick re-timed" % torch.cuda.get_device_name(0),
             "// against its neighbours on separately allocated fields)"]
    B.pw_tune_reset()
    for nx, ny, nz, dt, flags in SHAPES:
        B._check(B.pw_tune(B.pw_grid(nx, ny, nz, 1), code[dt], flags, None, None), "pw_tune")
        key = (ceil_log2(nx), ceil_log2(ny), ceil_log2(nz))
        for kind, name, bit, zext in ((0, "forward", 1, nz), (1, "adjoint", 2, nz + 2), (2, "tangent", 4, nz),
                                      (3, "zfast", 8, nx)):
            if not flags & bit:
                continue
            t = B.launch_shape(name, nx, ny, nz, tdt[dt])
            if kind == 0:
                pick = t
                t, med = confirm_forward(B, torch, nx, ny, nz, tdt[dt], pick)
                print("# %dx%dx%d %s forward: pw_tune %s %.2f us; kept %s %.2f us" % (
                    nx, ny, nz, dt, pick, med[tuple(pick)], t, med[tuple(t)]), flush=True)
            nzc = -(-zext // t[2])
            lines.append("{%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d},  // %dx%dx%d %s %s" % (
                kind, code[dt], *key, t[0], t[1], nzc, t[3], t[4], t[5], nx, ny, nz, dt, name))
            print(lines[-1], flush=True)
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "csrc", "pw_tune_defaults.inc"))
