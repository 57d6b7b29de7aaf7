"""CPU tests of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching HIP.

No GPU and no compute call: the pointers passed below are fake addresses that
the library only inspects arithmetically (null, alignment, overlap), so every
call returns from argument validation or from the device check.
"""
import ctypes

import pytest

from paper_2301_13016_amd import binding as B


@pytest.fixture(scope="module")
def lib():
    try:
        return B.lib()
    except B.PWLibraryMissing:
        import __graft_entry__
        __graft_entry__.build()
        return B.lib()


def test_exports_every_declared_symbol(lib):
    declared = B.header_functions()
    assert "pw_advect" in declared and "pw_advect_adjoint" in declared
    missing = [n for n in declared if not hasattr(lib, n)]
    assert missing == []


def test_version(lib):
    assert "libpwadv" in B.pw_version()


A = 0x10000000   # fake, 256-byte aligned "device" addresses, never dereferenced
MB = 1 << 20


def _args(nx=8, ny=8, nz=8, halo=1, dtype=B.PW_F32):
    g = B.pw_grid(nx, ny, nz, halo)
    c = B.pw_coeffs(0.0025, 0.0025, A + 10 * MB, A + 11 * MB, A + 12 * MB, A + 13 * MB)
    ptrs = [A + i * MB for i in range(6)]   # u v w su sv sw, 1 MiB apart
    return g, c, ptrs


def _call(g, layout, dtype, c, ptrs, tile=None):
    u, v, w, su, sv, sw = ptrs
    return B.pw_advect_ex(g, layout, dtype, u, v, w, c, su, sv, sw, tile, None)


def _no_gpu_status():
    # valid arguments: PW_ERR_NO_DEVICE without a GPU; on a GPU machine the
    # fake addresses are caught by the device-pointer check instead
    return (B.PW_ERR_NO_DEVICE, B.PW_ERR_INVALID_ARG)


def test_valid_arguments_reach_device_check(lib):
    g, c, p = _args()
    assert _call(g, None, B.PW_F32, c, p) in _no_gpu_status()


@pytest.mark.parametrize("field,value", [("nx", 0), ("ny", -1), ("nz", 0), ("halo", 0), ("halo", -2)])
def test_bad_grid(lib, field, value):
    g, c, p = _args()
    setattr(g, field, value)
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG
    assert B.pw_last_error() != ""


def test_null_grid_and_coeffs(lib):
    g, c, p = _args()
    u, v, w, su, sv, sw = p
    st = lib.pw_advect(None, None, B.PW_F32, u, v, w, ctypes.byref(c), su, sv, sw, None)
    assert st == B.PW_ERR_INVALID_ARG
    st = lib.pw_advect(ctypes.byref(g), None, B.PW_F32, u, v, w, None, su, sv, sw, None)
    assert st == B.PW_ERR_INVALID_ARG


@pytest.mark.parametrize("which", range(6))
def test_null_array(lib, which):
    g, c, p = _args()
    p[which] = None
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG


def test_null_coefficient_array(lib):
    g, c, p = _args()
    c.tzd2 = None
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG


def test_misaligned_pointer(lib):
    g, c, p = _args()
    p[1] += 2
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG
    # 2-byte alignment is enough for 16-bit storage
    assert _call(g, None, B.PW_BF16, c, p) in _no_gpu_status()


def test_bad_dtype(lib):
    g, c, p = _args()
    assert _call(g, None, 7, c, p) == B.PW_ERR_INVALID_ARG


@pytest.mark.parametrize("bad", [dict(in_sy=9), dict(in_sz=10 * 10 - 1), dict(out_sy=7), dict(out_sz=63)])
def test_strides_too_small(lib, bad):
    g, c, p = _args()
    L = B.pw_layout(10, 100, 8, 64)
    for k, val in bad.items():
        setattr(L, k, val)
    assert _call(g, L, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG


def test_pitched_layout_accepted(lib):
    g, c, p = _args()
    L = B.pw_layout(16, 16 * 12, 8, 80)
    assert _call(g, L, B.PW_F32, c, p) in _no_gpu_status()


def test_output_overlapping_input_rejected(lib):
    g, c, p = _args()
    p[3] = p[0] + 4 * 100   # su inside u's padded extent
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG
    assert "overlap" in B.pw_last_error()


def test_outputs_overlapping_each_other_rejected(lib):
    g, c, p = _args()
    p[4] = p[3] + 4 * 8
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG


def test_output_overlapping_coefficients_rejected(lib):
    # coefficient arrays are read through the scalar cache, so no output may
    # overlap them; inputs may (they are only read)
    g, c, p = _args()
    p[5] = A + 13 * MB + 4 * 7   # sw starts on tzd2[7], the last level
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG
    assert "tzd2" in B.pw_last_error()
    p[5] = A + 13 * MB + 4 * 8   # just past tzd2: fine
    assert _call(g, None, B.PW_F32, c, p) in _no_gpu_status()
    g, c, p = _args()
    c.tzc1 = p[0]                # coefficients inside an input: fine
    assert _call(g, None, B.PW_F32, c, p) in _no_gpu_status()
    q = [A + i * MB for i in range(9)]
    c.tzc1 = q[7] + 4 * 100      # inside gradient gv
    st = B.pw_advect_adjoint(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9])
    assert st == B.PW_ERR_INVALID_ARG and "tzc1" in B.pw_last_error()


def test_huge_plane_unsupported(lib):
    g, c, p = _args(nx=40000, ny=20000, nz=1)
    p = [A + i * (1 << 34) for i in range(6)]
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_UNSUPPORTED


@pytest.mark.parametrize("tile", [(1, 3, 8, 4), (1, 4, 0, 4), (1, 4, 8, 0), (1, 4, 8, 9), (3, 1, 8, 4),
                                  (4, 8, 8, 4), (8, 1, 8, 1), (0, 1, 8, 1)])
def test_bad_tile(lib, tile):
    g, c, p = _args()
    assert _call(g, None, B.PW_F32, c, p, B.pw_tile(*tile)) == B.PW_ERR_INVALID_ARG


@pytest.mark.parametrize("tile", [(1, 1, 1, 1), (1, 4, 8, 8), (2, 4, 3, 4), (4, 1, 16, 1), (4, 2, 64, 2),
                                  (4, 4, 8, 4)])
def test_good_tile(lib, tile):
    g, c, p = _args()
    assert _call(g, None, B.PW_F32, c, p, B.pw_tile(*tile)) in _no_gpu_status()


def test_shared_row_tile_rules(lib):
    """share_rows: 1 or 2 with 2 or 4 wavefronts per group, prefetch 1 and
    the instantiated column / row counts per dtype; 0 is independent strips.
    Only the forward takes it."""
    g, c, p = _args()
    ok = [(B.PW_F32, (4, 1, 8, 4, 1, 1)), (B.PW_F32, (4, 2, 8, 2, 1, 2)), (B.PW_F32, (4, 4, 8, 4, 0, 1)),
          (B.PW_BF16, (8, 2, 8, 4, 1, 1)), (B.PW_F16, (4, 4, 8, 2, 1, 2)), (B.PW_F64, (2, 4, 8, 4, 1, 1))]
    bad = [(B.PW_F32, (4, 2, 8, 1, 1, 1)), (B.PW_F32, (4, 2, 8, 8, 1, 1)), (B.PW_F32, (4, 2, 8, 4, 2, 1)),
           (B.PW_F32, (2, 2, 8, 4, 1, 1)), (B.PW_F32, (4, 2, 8, 4, 1, 3)), (B.PW_F32, (4, 2, 8, 4, 1, -1)),
           (B.PW_BF16, (8, 4, 8, 4, 1, 1)), (B.PW_F64, (4, 2, 8, 4, 1, 1)), (B.PW_F64, (2, 1, 8, 4, 1, 1))]
    for dt, t in ok:
        assert _call(g, None, dt, c, p, B.pw_tile(*t)) in _no_gpu_status(), (dt, t)
    for dt, t in bad:
        assert _call(g, None, dt, c, p, B.pw_tile(*t)) == B.PW_ERR_INVALID_ARG, (dt, t)
    q = [A + i * MB for i in range(9)]
    st = B.pw_advect_adjoint_ex(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9], B.pw_tile(1, 2, 8, 4, 1, 1))
    assert st == B.PW_ERR_INVALID_ARG
    st = B.pw_advect_tangent_ex(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9], B.pw_tile(2, 2, 8, 4, 1, 1))
    assert st == B.PW_ERR_INVALID_ARG


def test_f64_tile_limits(lib):
    g, c, p = _args(dtype=B.PW_F64)
    for bad in [(4, 1, 8, 4), (1, 8, 8, 4), (2, 8, 8, 4)]:
        assert _call(g, None, B.PW_F64, c, p, B.pw_tile(*bad)) == B.PW_ERR_INVALID_ARG
    for good in [(2, 2, 8, 4), (1, 4, 8, 4), (2, 4, 8, 1)]:
        assert _call(g, None, B.PW_F64, c, p, B.pw_tile(*good)) in _no_gpu_status()


def test_adjoint_tile_limits(lib):
    g, c, p = _args()
    q = [A + i * MB for i in range(9)]
    for bad, ok in [((2, 1, 8, 4), False), ((1, 8, 8, 4), False), ((1, 4, 8, 4), True)]:
        st = B.pw_advect_adjoint_ex(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9], B.pw_tile(*bad))
        assert (st in _no_gpu_status()) if ok else st == B.PW_ERR_INVALID_ARG


def test_adjoint_rejects_16bit(lib):
    g, c, p = _args()
    q = [A + i * MB for i in range(9)]
    st = B.pw_advect_adjoint(g, None, B.PW_BF16, *q[:3], c, *q[3:6], *q[6:9])
    assert st == B.PW_ERR_UNSUPPORTED


def test_adjoint_gradient_overlap_rejected(lib):
    g, c, p = _args()
    q = [A + i * MB for i in range(9)]
    q[6] = q[0]
    st = B.pw_advect_adjoint(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9])
    assert st == B.PW_ERR_INVALID_ARG


def test_prefetch_depth_validation(lib):
    """prefetch: 0 (= 1), 1 or 2 for the forward, the adjoint, the tangent
    and the batched form."""
    g, c, p = _args()
    for pf, ok in [(0, True), (1, True), (2, True), (3, False), (-1, False)]:
        st = _call(g, None, B.PW_F32, c, p, B.pw_tile(4, 2, 8, 1, pf))
        assert (st in _no_gpu_status()) if ok else st == B.PW_ERR_INVALID_ARG, pf
    q = [A + i * MB for i in range(9)]
    st = B.pw_advect_adjoint_ex(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9], B.pw_tile(1, 2, 8, 1, 2))
    assert st in _no_gpu_status()
    st = B.pw_advect_adjoint_ex(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9], B.pw_tile(1, 2, 8, 1, 3))
    assert st == B.PW_ERR_INVALID_ARG
    st = B.pw_advect_tangent_ex(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9], B.pw_tile(1, 2, 8, 1, 2))
    assert st in _no_gpu_status()
    st = B.pw_advect_tangent_ex(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9], B.pw_tile(1, 2, 8, 1, 3))
    assert st == B.PW_ERR_INVALID_ARG
    assert B.pw_advect_tangent_ex(g, None, B.PW_F32, *q[:3], c, *q[3:6], *q[6:9],
                                  B.pw_tile(1, 2, 8, 1, 1)) in _no_gpu_status()
    h = ctypes.c_void_p()
    assert B.pw_batch_create(_items(2), 2, B.PW_F32, B.pw_tile(1, 2, 8, 4, 3), h) == B.PW_ERR_INVALID_ARG


def test_tangent_validation(lib):
    g, c, p = _args()
    q = [A + i * MB for i in range(9)]   # u v w du dv dw tu tv tw
    call = lambda dt, qq, tile=None: B.pw_advect_tangent_ex(g, None, dt, *qq[:3], c, *qq[3:6], *qq[6:9],  # noqa: E731
                                                             tile)
    assert call(B.PW_F32, q) in _no_gpu_status()
    assert call(B.PW_F64, q) in _no_gpu_status()
    assert call(B.PW_BF16, q) == B.PW_ERR_UNSUPPORTED
    assert call(9, q) == B.PW_ERR_INVALID_ARG
    bad = list(q)
    bad[6] = q[4] + 4 * 10                 # tu inside dv
    assert call(B.PW_F32, bad) == B.PW_ERR_INVALID_ARG and "overlaps" in B.pw_last_error()
    bad = list(q)
    bad[7] = q[1]                          # tv on v
    assert call(B.PW_F32, bad) == B.PW_ERR_INVALID_ARG
    bad = list(q)
    bad[3] = 0                             # du NULL
    assert call(B.PW_F32, bad) == B.PW_ERR_INVALID_ARG
    for t, ok in [((1, 1, 8, 4), True), ((2, 2, 8, 8), True), ((4, 1, 8, 4), False), ((1, 4, 8, 4), False),
                  ((1, 1, 0, 4), False), ((1, 1, 8, 9), False)]:
        st = call(B.PW_F32, q, B.pw_tile(*t))
        assert (st in _no_gpu_status()) if ok else st == B.PW_ERR_INVALID_ARG, t
    assert call(B.PW_F64, q, B.pw_tile(2, 1, 8, 4)) == B.PW_ERR_INVALID_ARG


def _table_row(kind, dt, nx, ny, nz):
    """The built-in tuning table's row for a shape class, or None."""
    import os
    import re
    path = os.path.join(os.path.dirname(B.__file__), "csrc", "pw_tune_defaults.inc")
    key = (kind, dt) + tuple((n - 1).bit_length() for n in (nx, ny, nz))
    for line in open(path):
        m = re.match(r"\{([^}]*)\}", line.strip())
        if m:
            row = tuple(int(x) for x in m.group(1).split(","))
            if row[:5] == key:
                return row[5:] + (0,) * (11 - len(row))   # rows without share_rows: 0
    return None


def test_launch_shape_query(lib):
    """pw_launch_shape needs no device: the built-in table's entry, or the
    default shape for a class the table does not hold."""
    torch = pytest.importorskip("torch")
    row = _table_row(0, B.PW_F32, 512, 512, 64)
    assert row is not None
    px, ry, nzc, wpb, depth, share = row
    assert B.launch_shape("forward", 512, 512, 64, torch.float32) == (px, ry, -(-64 // nzc), wpb, depth, share)
    row = _table_row(1, B.PW_F32, 256, 256, 128)
    px, ry, nzc, wpb, depth, share = row
    assert share == 0
    assert B.launch_shape("adjoint", 256, 256, 128, torch.float32) == (px, ry, -(-130 // nzc), wpb, depth, 0)
    shape = B.launch_shape("tangent", 100, 3, 5, torch.float64)   # no table entry: the default
    assert shape[0] == 1 and shape[1] in (1, 2) and 1 <= shape[2] <= 5 and 1 <= shape[3] <= 8 and shape[4] == 1
    assert shape[5] == 0
    t = B.pw_tile()
    assert lib.pw_launch_shape(1, ctypes.byref(B.pw_grid(8, 8, 8, 1)), B.PW_BF16, ctypes.byref(t)) \
        == B.PW_ERR_UNSUPPORTED
    assert lib.pw_launch_shape(7, ctypes.byref(B.pw_grid(8, 8, 8, 1)), B.PW_F32, ctypes.byref(t)) \
        == B.PW_ERR_INVALID_ARG
    assert lib.pw_launch_shape(0, None, B.PW_F32, ctypes.byref(t)) == B.PW_ERR_INVALID_ARG
    assert lib.pw_launch_shape(0, ctypes.byref(B.pw_grid(0, 8, 8, 1)), B.PW_F32, ctypes.byref(t)) \
        == B.PW_ERR_INVALID_ARG


def test_pwadv_tile_override(lib, monkeypatch):
    """PWADV_TILE sets the forward's shape for calls without a tile and what
    pw_launch_shape reports; a malformed or unsupported value fails those
    calls before any device work, naming the variable; an explicit tile and
    the other kernels ignore it."""
    torch = pytest.importorskip("torch")
    g, c, p = _args()
    ep = B.pw_epilogue(1.0, A + 20 * MB, A + 21 * MB, A + 22 * MB)
    bc = (B.pw_halo_modes * 3)(*[B.pw_halo_modes(1, 1, 2)] * 3)
    calls = {
        "pw_advect": lambda: _call(g, None, B.PW_F32, c, p),
        "pw_advect_epilogue": lambda: lib.pw_advect_epilogue(ctypes.byref(g), None, B.PW_F32, *p[:3], ctypes.byref(c),
                                                             ctypes.byref(ep), *p[3:], None, None),
        "pw_advect_bc": lambda: lib.pw_advect_bc(ctypes.byref(g), None, B.PW_F32, *p[:3], ctypes.byref(c), bc,
                                                 None, *p[3:], None, None),
    }
    for bad in ("garbage", "4x2", "4x2x", "4x2x32x4x1x2x9", "4;2;32", "3x1x8", "4x1x0", "8x2x16"):
        monkeypatch.setenv("PWADV_TILE", bad)
        for name, call in calls.items():
            assert call() == B.PW_ERR_INVALID_ARG, (bad, name)
            assert "PWADV_TILE" in B.pw_last_error(), (bad, name)
        t = B.pw_tile()
        assert lib.pw_launch_shape(0, ctypes.byref(B.pw_grid(8, 8, 8, 1)), B.PW_F32, ctypes.byref(t)) \
            == B.PW_ERR_INVALID_ARG, bad
        # an explicit tile and the adjoint's shape query do not read it
        assert _call(g, None, B.PW_F32, c, p, tile=B.pw_tile(1, 2, 8, 4)) in _no_gpu_status()
        assert "PWADV_TILE" not in B.pw_last_error()
        assert lib.pw_launch_shape(1, ctypes.byref(B.pw_grid(8, 8, 8, 1)), B.PW_F32, ctypes.byref(t)) == B.PW_OK
    for val, want in (("4x2x32x4x1x2", (4, 2, 32, 4, 1, 2)), ("4,2,32", (4, 2, 32, 4, 1, 0)),
                      ("2x4x5x2x2", (2, 4, 5, 2, 2, 0)), ("1x1x1x1x0", (1, 1, 1, 1, 1, 0))):
        monkeypatch.setenv("PWADV_TILE", val)
        assert B.launch_shape("forward", 512, 512, 64, torch.float32) == want, val
        for name, call in calls.items():
            assert call() in _no_gpu_status(), (val, name)
            assert "PWADV_TILE" not in B.pw_last_error(), (val, name)
    monkeypatch.setenv("PWADV_TILE", "8x2x16")      # a 16-bit shape: fine for BF16, not for FP32
    assert B.launch_shape("forward", 64, 64, 64, torch.bfloat16) == (8, 2, 16, 4, 1, 0)
    assert _call(g, None, B.PW_BF16, c, p) in _no_gpu_status() and "PWADV_TILE" not in B.pw_last_error()
    monkeypatch.setenv("PWADV_TILE", "")             # empty: as if unset
    row = _table_row(0, B.PW_F32, 512, 512, 64)
    assert B.launch_shape("forward", 512, 512, 64, torch.float32)[:2] == row[:2]


def test_tune_cache_file_read_without_device(tmp_path):
    """The cache file is read on first use, with no device: v3 lines carry
    share_rows, v2 lines the prefetch depth (share_rows 0), v1 lines mean
    depth 1, malformed lines are ignored, and a file entry overrides the
    built-in table."""
    import os
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    # classes: 512x512x64 forward (also in the built-in table), 100x100x10 adjoint and tangent
    cache.write_text("pwadv-tune-v2 0 0 9 9 6 2 2 4 1 2\n"
                     "pwadv-tune-v1 1 0 7 7 4 1 4 2 1\n"
                     "garbage line\n"
                     "pwadv-tune-v2 2 0 7 7 4 2 1 2 8 3\n"    # depth 3 is invalid: ignored
                     "pwadv-tune-v3 0 0 10 10 8 4 4 1 2 1 1\n"
                     "pwadv-tune-v3 0 0 7 7 7 4 2 1 4 1 3\n")   # share_rows 3 is invalid: ignored
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, torch; sys.path.insert(0, %r)\n"
            "from paper_2301_13016_amd import binding as B\n"
            "print(B.launch_shape('forward', 512, 512, 64, torch.float32))\n"
            "print(B.launch_shape('adjoint', 100, 100, 10, torch.float32))\n"
            "print(B.launch_shape('tangent', 100, 100, 10, torch.float32))\n"
            "print(B.launch_shape('forward', 1024, 1024, 256, torch.float32))\n"
            "print(B.launch_shape('forward', 128, 128, 128, torch.float32))\n" % root)
    r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, PWADV_TUNE_CACHE=str(cache)),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    fwd, adj, tan, big, mid = r.stdout.strip().splitlines()
    assert fwd == str((2, 2, 16, 1, 2, 0))
    assert adj == str((1, 4, 6, 1, 1, 0))       # 12 padded levels in 2 chunks
    assert tan != str((2, 1, 5, 8, 3, 0))       # the invalid line did not take effect
    assert big == str((4, 4, 256, 2, 1, 1))
    assert mid != str((4, 2, 128, 4, 1, 3))
    assert cache.read_text().count("\n") == 6   # reading never rewrites the file


def test_stream_copy_validation(lib):
    assert B.pw_stream_copy(None, A, 16) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_copy(A, A + MB, 15) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_copy(A + 4, A + MB, 16) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_copy(A, A + 8, 64) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_copy(A, A + MB, 64) in _no_gpu_status()


def test_stream_probe_validation(lib):
    ok = [(0, 1, 0), (0, 8, 3), (1, 4, 1), (2, 2, 2)]
    for mode, loads, flags in ok:
        assert B.pw_stream_probe(mode, loads, flags, A, A + MB, 4096, 64) in _no_gpu_status()
    assert B.pw_stream_probe(2, 1, 0, None, A, 4096, 64) in _no_gpu_status()      # writes need no source
    assert B.pw_stream_probe(3, 1, 0, A, A + MB, 4096, 64) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_probe(0, 3, 0, A, A + MB, 4096, 64) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_probe(0, 1, 4, A, A + MB, 4096, 64) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_probe(0, 1, 0, A, A + MB, 4096, 0) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_probe(0, 1, 0, A, A + MB, 4100, 64) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_probe(0, 1, 0, A, A + 64, 4096, 64) == B.PW_ERR_INVALID_ARG     # overlap
    assert B.pw_stream_probe(1, 1, 0, A, A + 8192, 1 << 20, 64) == B.PW_ERR_INVALID_ARG   # sink inside src
    assert B.pw_stream_probe(0, 1, 0, A + 8, A + MB, 4096, 64) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_probe(0, 1, 0, None, A + MB, 4096, 64) == B.PW_ERR_INVALID_ARG


def test_epilogue_validation(lib):
    g, c, p = _args()
    call = lambda ep, pp=p, tile=None: lib.pw_advect_epilogue(  # noqa: E731
        ctypes.byref(g), None, B.PW_F32, *pp[:3], ctypes.byref(c), ep, *pp[3:6], tile, None)
    addends = [A + (20 + i) * MB for i in range(3)]
    ok = B.pw_epilogue(1.0, *addends)
    assert call(ctypes.byref(ok)) in _no_gpu_status()
    assert call(None) == B.PW_ERR_INVALID_ARG
    inplace = B.pw_epilogue(1.0, *p[3:6])                      # accumulate into the outputs
    assert call(ctypes.byref(inplace)) in _no_gpu_status()
    crossed = B.pw_epilogue(1.0, p[4], p[4], p[5])             # cu is sv
    assert call(ctypes.byref(crossed)) == B.PW_ERR_INVALID_ARG and "overlaps" in B.pw_last_error()
    partial = B.pw_epilogue(1.0, p[3] + 4 * 16, p[4], p[5])    # cu half inside su
    assert call(ctypes.byref(partial)) == B.PW_ERR_INVALID_ARG
    on_input = B.pw_epilogue(0.5, p[0], p[1], p[2])           # addends inside the inputs: read-only, fine
    assert call(ctypes.byref(on_input)) in _no_gpu_status()
    misaligned = B.pw_epilogue(1.0, addends[0] + 2, addends[1], addends[2])
    assert call(ctypes.byref(misaligned)) == B.PW_ERR_INVALID_ARG
    nan = B.pw_epilogue(float("nan"), *addends)
    assert call(ctypes.byref(nan)) == B.PW_ERR_INVALID_ARG
    assert call(ctypes.byref(ok), tile=ctypes.byref(B.pw_tile(3, 1, 8, 4))) == B.PW_ERR_INVALID_ARG


def test_coeff_grad_validation(lib):
    g, c, p = _args()
    need = ctypes.c_int64()
    assert lib.pw_advect_coeff_grad_workspace(ctypes.byref(g), B.PW_F32, ctypes.byref(need)) == B.PW_OK
    # the adjoint's strips of 62 padded columns, for one-row strips (the most
    # strips): 10 padded columns -> 1 x 10 strips; 6 quantities x 8 levels
    assert need.value == 6 * 8 * 10 * 8
    assert lib.pw_advect_coeff_grad_workspace(ctypes.byref(g), B.PW_F64, ctypes.byref(need)) == B.PW_OK
    assert need.value == 6 * 8 * 10 * 8
    g2 = B.pw_grid(123, 5, 3, 2)              # 127 padded columns -> 3 strips of 62; 9 padded rows
    assert lib.pw_advect_coeff_grad_workspace(ctypes.byref(g2), B.PW_F32, ctypes.byref(need)) == B.PW_OK
    assert need.value == 6 * 3 * 3 * 9 * 8
    assert lib.pw_advect_coeff_grad_workspace(ctypes.byref(g), B.PW_BF16, ctypes.byref(need)) == B.PW_ERR_UNSUPPORTED
    assert lib.pw_advect_coeff_grad_workspace(ctypes.byref(g), B.PW_F32, None) == B.PW_ERR_INVALID_ARG
    q = [A + i * MB for i in range(8)]   # u v w gsu gsv gsw grad workspace
    call = lambda qq, nbytes=4096: lib.pw_advect_coeff_grad(ctypes.byref(g), None, B.PW_F32, *qq[:6], qq[6],  # noqa
                                                              qq[7], nbytes, None)
    assert call(q) in _no_gpu_status()
    assert call(q, 100) == B.PW_ERR_INVALID_ARG and "workspace" in B.pw_last_error()
    bad = list(q); bad[6] = q[0] + 8          # grad inside u
    assert call(bad) == B.PW_ERR_INVALID_ARG
    bad = list(q); bad[7] = q[6] + 16         # workspace overlapping grad
    assert call(bad) == B.PW_ERR_INVALID_ARG
    bad = list(q); bad[6] = q[6] + 4          # grad not 8-byte aligned
    assert call(bad) == B.PW_ERR_INVALID_ARG


def test_fused_backward_validation(lib):
    """pw_advect_adjoint_coeff_grad: the adjoint's checks and the coefficient
    gradients' checks, and grad / workspace apart from the wind gradients."""
    g, c, p = _args()
    need = ctypes.c_int64()
    assert lib.pw_advect_coeff_grad_workspace(ctypes.byref(g), B.PW_F32, ctypes.byref(need)) == B.PW_OK
    q = [A + i * MB for i in range(11)]   # u v w gsu gsv gsw gu gv gw grad workspace
    call = lambda qq, nbytes=need.value, dt=B.PW_F32: lib.pw_advect_adjoint_coeff_grad(  # noqa: E731
        ctypes.byref(g), None, dt, *qq[:3], ctypes.byref(c), *qq[3:9], qq[9], qq[10], nbytes, None)
    assert call(q) in _no_gpu_status()
    assert call(q, dt=B.PW_F64) in _no_gpu_status() or "coefficient" in B.pw_last_error()
    assert call(q, dt=B.PW_BF16) == B.PW_ERR_UNSUPPORTED
    assert call(q, need.value - 8) == B.PW_ERR_INVALID_ARG and "workspace" in B.pw_last_error()
    bad = list(q); bad[10] = 0                # workspace NULL
    assert call(bad) == B.PW_ERR_INVALID_ARG
    bad = list(q); bad[9] = q[6] + 64         # grad inside gu
    assert call(bad) == B.PW_ERR_INVALID_ARG and "overlaps" in B.pw_last_error()
    bad = list(q); bad[10] = q[8] + 256       # workspace inside gw
    assert call(bad) == B.PW_ERR_INVALID_ARG and "overlaps" in B.pw_last_error()
    bad = list(q); bad[6] = q[0]              # gu on u
    assert call(bad) == B.PW_ERR_INVALID_ARG
    bad = list(q); bad[9] = q[9] + 4          # grad misaligned
    assert call(bad) == B.PW_ERR_INVALID_ARG


def test_coeff_grad_static_validation(lib):
    """The allocation-free coefficient-gradient entry point: the same checks
    as with a workspace, and grids whose partials exceed its static scratch
    are refused (PW_ERR_UNSUPPORTED) before any HIP call."""
    g, c, p = _args()
    q = [A + i * MB for i in range(7)]   # u v w gsu gsv gsw grad
    call = lambda gg, qq, dt=B.PW_F32: lib.pw_advect_coeff_grad_static(ctypes.byref(gg), None, dt,  # noqa: E731
                                                                        *qq[:6], qq[6], None)
    assert call(g, q) in _no_gpu_status()
    bad = list(q); bad[6] = q[3] + 8          # grad inside gsu
    assert call(g, bad) == B.PW_ERR_INVALID_ARG
    bad = list(q); bad[6] = q[6] + 4          # grad not 8-byte aligned
    assert call(g, bad) == B.PW_ERR_INVALID_ARG
    assert call(g, q, B.PW_BF16) == B.PW_ERR_UNSUPPORTED
    # 2048 x 2048 x 256 FP32: 34 x 2050 strips x 6 x 256 levels x 8 B = 816 MiB of partials
    big = B.pw_grid(2048, 2048, 256, 1)
    need = ctypes.c_int64()
    assert lib.pw_advect_coeff_grad_workspace(ctypes.byref(big), B.PW_F32, ctypes.byref(need)) == B.PW_OK
    assert need.value > 16 << 20
    assert call(big, q) == B.PW_ERR_UNSUPPORTED and "static scratch" in B.pw_last_error()
    # a grid that fits: 16 MiB / (6 * 8 B) partials per level and strip
    edge = B.pw_grid(256, 256, 128 * 2, 1)    # 5 x 258 strips x 256 levels x 48 B = 15.1 MiB
    far = [A + i * (1 << 30) for i in range(7)]   # 1 GiB apart: no array overlaps another
    st = call(edge, far)
    assert st in _no_gpu_status() and "static scratch" not in B.pw_last_error()
    if st == B.PW_ERR_INVALID_ARG:            # on a GPU machine: the device-pointer check, nothing else
        assert "device" in B.pw_last_error()


def test_stream_copy3_validation(lib):
    s = [A + i * MB for i in range(3)]
    d = [A + (3 + i) * MB for i in range(3)]
    assert B.pw_stream_copy3(s, d, 64) in _no_gpu_status()
    assert B.pw_stream_copy3(s, d, 0) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_copy3(s, d, 24) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_copy3([s[0], 0, s[2]], d, 64) == B.PW_ERR_INVALID_ARG
    assert B.pw_stream_copy3(s, [d[0], d[1], d[2] + 8], 64) == B.PW_ERR_INVALID_ARG     # misaligned
    assert B.pw_stream_copy3(s, [d[0], s[1] + 32, d[2]], 64) == B.PW_ERR_INVALID_ARG   # dst on a src
    assert "overlap" in B.pw_last_error()
    assert B.pw_stream_copy3(s, [d[0], d[0] + 16, d[2]], 64) == B.PW_ERR_INVALID_ARG   # two dsts overlap
    assert lib.pw_stream_copy3(None, None, 64, None) == B.PW_ERR_INVALID_ARG


def test_last_error_is_per_thread(lib):
    import threading
    g, c, p = _args()
    g.halo = 0
    assert _call(g, None, B.PW_F32, c, p) == B.PW_ERR_INVALID_ARG
    seen = []
    t = threading.Thread(target=lambda: seen.append(B.pw_last_error()))
    t.start()
    t.join()
    assert seen == [""]
    assert "halo" in B.pw_last_error()


# ------------------------------------------------------------------ batched form / tuner

def _items(n, overlap=False):
    items = (B.pw_batch_item * n)()
    for i in range(n):
        base = A + i * 16 * MB
        items[i].grid = B.pw_grid(8, 8, 8, 1)
        items[i].u, items[i].v, items[i].w = base, base + MB, base + 2 * MB
        items[i].coeffs = B.pw_coeffs(0.0025, 0.0025, base + 10 * MB, base + 11 * MB, base + 12 * MB, base + 13 * MB)
        items[i].su, items[i].sv, items[i].sw = base + 3 * MB, base + 4 * MB, base + 5 * MB
    if overlap:
        items[1].su = items[0].u   # an output of item 1 on an input of item 0
    return items


def test_batch_argument_errors(lib):
    h = ctypes.c_void_p()
    assert B.pw_batch_create(_items(2), 0, B.PW_F32, None, h) == B.PW_ERR_INVALID_ARG
    assert lib.pw_batch_create(_items(2), 2, B.PW_F32, None, None) == B.PW_ERR_INVALID_ARG
    assert B.pw_batch_create(_items(2), 2, B.PW_BF16, None, h) == B.PW_ERR_UNSUPPORTED
    assert B.pw_batch_create(_items(2), 2, B.PW_F32, B.pw_tile(4, 4, 8, 4), h) == B.PW_ERR_INVALID_ARG
    # the batch runs independent wavefronts only (share_rows 0)
    for bad in [(4, 2, 8, 4, 1, 1), (0, 2, 8, 4, 1, 2)]:
        assert B.pw_batch_create(_items(2), 2, B.PW_F32, B.pw_tile(*bad), h) == B.PW_ERR_INVALID_ARG, bad
    # columns per lane 0 (chosen per subdomain): rows per strip as for 1 and 2 columns
    assert B.pw_batch_create(_items(2), 2, B.PW_F32, B.pw_tile(0, 8, 8, 4), h) == B.PW_ERR_INVALID_ARG
    assert B.pw_batch_create(_items(2), 2, B.PW_F32, B.pw_tile(0, 4, 8, 4, 3), h) == B.PW_ERR_INVALID_ARG
    bad = _items(3)
    bad[2].grid.halo = 0
    assert B.pw_batch_create(bad, 3, B.PW_F32, None, h) == B.PW_ERR_INVALID_ARG
    assert "item 2" in B.pw_last_error()
    assert B.pw_batch_create(_items(2, overlap=True), 2, B.PW_F32, None, h) == B.PW_ERR_INVALID_ARG
    assert "overlaps" in B.pw_last_error()
    bad = _items(3)
    bad[2].sv = bad[0].coeffs.tzc2   # an output of item 2 on a coefficient array of item 0
    assert B.pw_batch_create(bad, 3, B.PW_F32, None, h) == B.PW_ERR_INVALID_ARG
    assert "item 2" in B.pw_last_error() and "item 0" in B.pw_last_error()
    ok = _items(3)
    ok[2].u = ok[0].coeffs.tzc2      # an input sharing memory with coefficients: fine
    assert B.pw_batch_create(ok, 3, B.PW_F32, None, h) in _no_gpu_status()
    assert h.value is None


def test_batch_valid_items_reach_device_check(lib):
    h = ctypes.c_void_p()
    assert B.pw_batch_create(_items(4), 4, B.PW_F32, None, h) in _no_gpu_status()
    assert h.value is None


def test_batch_null_handle(lib):
    for fn in (lib.pw_batch_run, lib.pw_batch_replay):
        assert fn(None, None) == B.PW_ERR_INVALID_ARG
    assert lib.pw_batch_capture(None, None) == B.PW_ERR_INVALID_ARG
    assert lib.pw_batch_tune(None, None, None) == B.PW_ERR_INVALID_ARG
    assert lib.pw_batch_destroy(None) == B.PW_OK


def test_tune_argument_errors(lib):
    assert lib.pw_tune(None, B.PW_F32, 0, None, None) == B.PW_ERR_INVALID_ARG
    g = B.pw_grid(0, 8, 8, 1)
    assert B.pw_tune(g, B.PW_F32) == B.PW_ERR_INVALID_ARG
    g = B.pw_grid(8, 8, 8, 1)
    assert B.pw_tune(g, 9) == B.PW_ERR_INVALID_ARG
    assert B.pw_tune(g, B.PW_F32, flags=16) == B.PW_ERR_INVALID_ARG
    assert B.pw_tune(g, B.PW_F32) in (B.PW_ERR_NO_DEVICE, B.PW_OK)   # OK where a GPU is present
    assert B.pw_tune_reset() == B.PW_OK


def test_halo_fill_validation(lib):
    g = B.pw_grid(8, 8, 8, 1)
    f = [A + i * MB for i in range(3)]
    per = [(1, 1, 2), (1, 1, 2), (1, 1, 3)]
    assert B.pw_halo_fill(g, None, B.PW_F32, f, per) in _no_gpu_status()
    assert B.pw_halo_fill(g, None, B.PW_F32, f, [(0, 0, 0)] * 3) in _no_gpu_status()
    assert B.pw_halo_fill(g, None, B.PW_F32, [], []) == B.PW_ERR_INVALID_ARG
    assert B.pw_halo_fill(g, None, B.PW_F32, [A + i * MB for i in range(9)], [(1, 1, 1)] * 9) == B.PW_ERR_INVALID_ARG
    assert B.pw_halo_fill(g, None, B.PW_F32, f, [(1, 1, 6)] * 3) == B.PW_ERR_INVALID_ARG
    assert "mode" in B.pw_last_error()
    assert B.pw_halo_fill(g, None, B.PW_F32, f, [(1, 1, -1)] * 3) == B.PW_ERR_INVALID_ARG
    assert B.pw_halo_fill(g, None, B.PW_F32, [f[0], 0, f[2]], per) == B.PW_ERR_INVALID_ARG
    assert B.pw_halo_fill(g, None, B.PW_F32, [f[0], f[1] + 2, f[2]], per) == B.PW_ERR_INVALID_ARG  # misaligned
    assert B.pw_halo_fill(g, None, B.PW_F32, [f[0], f[0] + 3996, f[2]], per) == B.PW_ERR_INVALID_ARG
    assert "overlap" in B.pw_last_error()
    assert B.pw_halo_fill(g, None, 9, f, per) == B.PW_ERR_INVALID_ARG
    # reflect needs n >= h on that axis; periodic, copy and zero do not
    g2 = B.pw_grid(8, 8, 2, 3)
    assert B.pw_halo_fill(g2, None, B.PW_F32, f, [(1, 1, 4)] * 3) == B.PW_ERR_INVALID_ARG
    assert "reflect" in B.pw_last_error()
    assert B.pw_halo_fill(g2, None, B.PW_F32, f, [(4, 5, 1)] * 3) in _no_gpu_status()
    # input strides: in_sy < nx + 2h is rejected; the output strides are ignored
    assert B.pw_halo_fill(g, B.pw_layout(9, 100, 0, 0), B.PW_F32, f, per) == B.PW_ERR_INVALID_ARG
    assert B.pw_halo_fill(g, B.pw_layout(16, 160, 0, 0), B.PW_F32, f, per) in _no_gpu_status()
    assert lib.pw_halo_fill(ctypes.byref(g), None, B.PW_F32, None, None, 1, None) == B.PW_ERR_INVALID_ARG


def test_zfast_validation(lib):
    """z-fastest forward: dense default strides, stride checks, overlap,
    tile rules; valid arguments reach the device check."""
    g, c, p = _args(nx=8, ny=6, nz=5)
    call = lambda layout=None, tile=None, ptrs=p, dt=B.PW_F32: B.pw_advect_zfast(  # noqa: E731
        g, layout, dt, *ptrs[:3], c, *ptrs[3:], tile, None)
    assert call() in _no_gpu_status()
    assert call(B.pw_layout_zfast(7, 7 * 8, 5, 30)) in _no_gpu_status()      # exact dense strides
    assert call(B.pw_layout_zfast(6, 6 * 8, 5, 30)) == B.PW_ERR_INVALID_ARG  # in_sj < nz + 2h
    assert "in_sj" in B.pw_last_error()
    assert call(B.pw_layout_zfast(7, 7 * 8 - 1, 5, 30)) == B.PW_ERR_INVALID_ARG
    assert call(B.pw_layout_zfast(7, 56, 4, 30)) == B.PW_ERR_INVALID_ARG     # out_sj < nz
    assert call(B.pw_layout_zfast(7, 56, 5, 29)) == B.PW_ERR_INVALID_ARG     # out_si < ny * out_sj
    assert call(B.pw_layout_zfast(7, 1 << 30, 5, 30)) == B.PW_ERR_UNSUPPORTED   # x-plane over 2 GiB
    # the dense input spans 10 * 8 * 7 floats = 2240 B: an output 2236 B after u overlaps it
    bad = list(p); bad[3] = p[0] + 2236
    assert call(ptrs=bad) == B.PW_ERR_INVALID_ARG and "overlaps" in B.pw_last_error()
    bad = list(p); bad[3] = p[0] + 2240
    assert call(ptrs=bad) in _no_gpu_status()
    assert call(tile=B.pw_tile(4, 2, 8, 1, 1)) in _no_gpu_status()
    assert call(tile=B.pw_tile(4, 4, 8, 1, 1)) == B.PW_ERR_INVALID_ARG   # 4 rows need <= 2 levels per lane
    assert call(tile=B.pw_tile(4, 1, 8, 1, 1), dt=B.PW_F64) == B.PW_ERR_INVALID_ARG
    assert call(tile=B.pw_tile(1, 2, 8, 1, 3)) == B.PW_ERR_INVALID_ARG   # prefetch 1 or 2
    assert call(tile=B.pw_tile(1, 8, 8, 1, 2)) in _no_gpu_status()
    assert call(tile=B.pw_tile(2, 8, 8, 1, 1)) == B.PW_ERR_INVALID_ARG
    assert call(tile=B.pw_tile(1, 2, 0, 1, 1)) == B.PW_ERR_INVALID_ARG
    assert call(tile=B.pw_tile(1, 3, 8, 1, 1)) == B.PW_ERR_INVALID_ARG


def test_zfast_launch_shape(lib):
    torch = pytest.importorskip("torch")
    row = _table_row(3, B.PW_F32, 512, 512, 64)
    assert row is not None
    pz, rj, nxc, wpb, depth, _ = row
    assert B.launch_shape("zfast", 512, 512, 64, torch.float32) == (pz, rj, -(-512 // nxc), wpb, depth, 0)
    shape = B.launch_shape("zfast", 10, 3, 200, torch.bfloat16)
    assert shape[0] in (1, 2, 4) and 1 <= shape[2] <= 10


def test_zfast_epilogue_validation(lib):
    g, c, p = _args(nx=8, ny=6, nz=5)
    q = [A + (20 + i) * MB for i in range(3)]   # addends
    call = lambda ep, ptrs=p: lib.pw_advect_zfast_epilogue(  # noqa: E731
        ctypes.byref(g), None, B.PW_F32, *ptrs[:3], ctypes.byref(c), ep, *ptrs[3:], None, None)
    assert call(ctypes.byref(B.pw_epilogue(1.0, *q))) in _no_gpu_status()
    assert call(ctypes.byref(B.pw_epilogue(1.0, *p[3:]))) in _no_gpu_status()        # in place
    assert call(None) == B.PW_ERR_INVALID_ARG
    assert call(ctypes.byref(B.pw_epilogue(1.0, p[4], p[4], p[5]))) == B.PW_ERR_INVALID_ARG   # cu is sv
    assert "overlaps output" in B.pw_last_error()
    assert call(ctypes.byref(B.pw_epilogue(float("inf"), *q))) == B.PW_ERR_INVALID_ARG
    assert call(ctypes.byref(B.pw_epilogue(1.0, q[0] + 2, q[1], q[2]))) == B.PW_ERR_INVALID_ARG   # misaligned


def test_advect_bc_validation(lib):
    g, c, p = _args()
    call = lambda bc, ep=None: lib.pw_advect_bc(ctypes.byref(g), None, B.PW_F32, *p[:3], ctypes.byref(c),  # noqa
                                                bc, ep, *p[3:], None, None)

    def rules(*triples):   # one triple for all three fields, or three
        if len(triples) == 1:
            triples = triples * 3
        return (B.pw_halo_modes * 3)(*(B.pw_halo_modes(*t) for t in triples))
    assert call(rules((1, 1, 2))) in _no_gpu_status()
    assert call(rules((0, 0, 0))) in _no_gpu_status()
    assert call(None) == B.PW_ERR_INVALID_ARG
    # value rules: free-slip lid, no-slip wall, zero / mirrored walls in x and y
    assert call(rules((1, 1, 2), (1, 1, 2), (1, 1, 3))) in _no_gpu_status()
    assert call(rules((1, 1, 5), (1, 1, 5), (1, 1, 3))) in _no_gpu_status()
    assert call(rules((3, 5, 1), (4, 2, 1), (5, 3, 1))) in _no_gpu_status()
    # the read remapping must agree across fields on each axis
    assert call(rules((1, 1, 2), (1, 1, 2), (1, 1, 1))) == B.PW_ERR_UNSUPPORTED   # nearest vs periodic
    assert "all keep" in B.pw_last_error()
    assert call(rules((0, 1, 2), (2, 1, 2), (2, 1, 2))) == B.PW_ERR_UNSUPPORTED   # keep vs nearest
    assert call(rules((1, 1, 9))) == B.PW_ERR_INVALID_ARG                          # unknown rule
    assert call(rules((1, 1, 2), (1, 1, 2), (1, 1, -1))) == B.PW_ERR_INVALID_ARG
    # mirror rules need n >= h, as for the fill
    g3 = B.pw_grid(8, 8, 2, 3)
    st = lib.pw_advect_bc(ctypes.byref(g3), None, B.PW_F32, *p[:3], ctypes.byref(c), rules((1, 1, 4)), None,
                          *p[3:], None, None)
    assert st == B.PW_ERR_INVALID_ARG and "reflect" in B.pw_last_error()
    q = [A + (20 + i) * MB for i in range(3)]
    assert call(rules((1, 1, 1)), ctypes.byref(B.pw_epilogue(0.5, *q))) in _no_gpu_status()
    assert call(rules((1, 1, 5)), ctypes.byref(B.pw_epilogue(0.5, *q))) in _no_gpu_status()
    assert call(rules((1, 1, 1)), ctypes.byref(B.pw_epilogue(float("nan"), *q))) == B.PW_ERR_INVALID_ARG


def test_halo_fold_validation(lib):
    g = B.pw_grid(8, 8, 8, 1)
    f = [A + i * MB for i in range(3)]
    per = [(1, 1, 2), (1, 1, 2), (1, 1, 3)]
    assert B.pw_halo_fold(g, None, B.PW_F32, f, per) in _no_gpu_status()
    assert B.pw_halo_fold(g, None, B.PW_F64, f, per) in _no_gpu_status()
    assert B.pw_halo_fold(g, None, B.PW_BF16, f, per) == B.PW_ERR_UNSUPPORTED
    assert B.pw_halo_fold(g, None, B.PW_F32, f, [(1, 1, 7)] * 3) == B.PW_ERR_INVALID_ARG
    assert B.pw_halo_fold(g, None, B.PW_F32, [f[0], f[0] + 100, f[2]], per) == B.PW_ERR_INVALID_ARG
    assert B.pw_halo_fold(B.pw_grid(8, 8, 2, 3), None, B.PW_F32, f, [(1, 1, 4)] * 3) == B.PW_ERR_INVALID_ARG
