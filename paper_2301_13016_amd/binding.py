"""ctypes binding of libpwadv (include/pwadv.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libpwadv.so``.  Loading fails loudly (``PWLibraryMissing``) if the
library has not been built; there is no CPU fallback.

Two layers:
* ``pw_advect``, ``pw_advect_ex``, ``pw_advect_adjoint``, ... -- the C entry
  points with the same names and arguments (pointers as Python ints).
* ``advect``, ``advect_adjoint``, ``PWAdvect`` -- the same calls on torch
  tensors (torch supplies device memory and the stream).
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpwadv.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pwadv.h")

PW_OK, PW_ERR_INVALID_ARG, PW_ERR_UNSUPPORTED, PW_ERR_NO_DEVICE, PW_ERR_HIP, PW_ERR_ALLOC = range(6)
PW_F32, PW_F64, PW_BF16, PW_F16 = range(4)
STATUS_NAMES = {0: "PW_OK", 1: "PW_ERR_INVALID_ARG", 2: "PW_ERR_UNSUPPORTED", 3: "PW_ERR_NO_DEVICE",
                4: "PW_ERR_HIP", 5: "PW_ERR_ALLOC"}


class PWLibraryMissing(RuntimeError):
    pass


class PWError(RuntimeError):
    def __init__(self, status, message, call=""):
        self.status = status
        self.message = message
        super().__init__("%s: %s (%s)" % (call, STATUS_NAMES.get(status, status), message))


class pw_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("halo", ctypes.c_int32)]


class pw_layout(ctypes.Structure):
    _fields_ = [("in_sy", ctypes.c_int64), ("in_sz", ctypes.c_int64),
                ("out_sy", ctypes.c_int64), ("out_sz", ctypes.c_int64)]


class pw_coeffs(ctypes.Structure):
    _fields_ = [("tcx", ctypes.c_double), ("tcy", ctypes.c_double),
                ("tzc1", ctypes.c_void_p), ("tzc2", ctypes.c_void_p),
                ("tzd1", ctypes.c_void_p), ("tzd2", ctypes.c_void_p)]


class pw_tile(ctypes.Structure):
    _fields_ = [("cols_per_lane", ctypes.c_int32), ("rows_per_strip", ctypes.c_int32),
                ("zlen", ctypes.c_int32), ("waves_per_group", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("share_rows", ctypes.c_int32)]


def _tile_tuple(t):
    """(cols_per_lane, rows_per_strip, zlen, waves_per_group, prefetch, share_rows)."""
    return (t.cols_per_lane, t.rows_per_strip, t.zlen, t.waves_per_group, t.prefetch, t.share_rows)


class pw_epilogue(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("cu", ctypes.c_void_p), ("cv", ctypes.c_void_p), ("cw", ctypes.c_void_p)]


class pw_layout_zfast(ctypes.Structure):
    _fields_ = [("in_sj", ctypes.c_int64), ("in_si", ctypes.c_int64),
                ("out_sj", ctypes.c_int64), ("out_si", ctypes.c_int64)]


class pw_halo_modes(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32), ("z", ctypes.c_int32)]


HALO_MODES = {"keep": 0, "periodic": 1, "copy": 2, "zero": 3, "reflect": 4, "reflect_neg": 5}


class pw_batch_item(ctypes.Structure):
    _fields_ = [("grid", pw_grid), ("layout", pw_layout), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("coeffs", pw_coeffs), ("su", ctypes.c_void_p), ("sv", ctypes.c_void_p),
                ("sw", ctypes.c_void_p)]


PW_TUNE_FORWARD, PW_TUNE_ADJOINT, PW_TUNE_TANGENT, PW_TUNE_ZFAST = 1, 2, 4, 8
PW_KERNEL_FORWARD, PW_KERNEL_ADJOINT, PW_KERNEL_TANGENT, PW_KERNEL_ZFAST = 0, 1, 2, 3

_P = ctypes.c_void_p
_SIGNATURES = {
    "pw_advect": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                  _P, _P, _P, ctypes.POINTER(pw_coeffs), _P, _P, _P, _P],
    "pw_advect_ex": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                     _P, _P, _P, ctypes.POINTER(pw_coeffs), _P, _P, _P, ctypes.POINTER(pw_tile), _P],
    "pw_advect_epilogue": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                           _P, _P, _P, ctypes.POINTER(pw_coeffs), ctypes.POINTER(pw_epilogue), _P, _P, _P,
                           ctypes.POINTER(pw_tile), _P],
    "pw_advect_adjoint": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                          _P, _P, _P, ctypes.POINTER(pw_coeffs), _P, _P, _P, _P, _P, _P, _P],
    "pw_advect_adjoint_ex": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                             _P, _P, _P, ctypes.POINTER(pw_coeffs), _P, _P, _P, _P, _P, _P,
                             ctypes.POINTER(pw_tile), _P],
    "pw_advect_tangent": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                          _P, _P, _P, ctypes.POINTER(pw_coeffs), _P, _P, _P, _P, _P, _P, _P],
    "pw_advect_tangent_ex": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                             _P, _P, _P, ctypes.POINTER(pw_coeffs), _P, _P, _P, _P, _P, _P,
                             ctypes.POINTER(pw_tile), _P],
    "pw_advect_coeff_grad_workspace": [ctypes.POINTER(pw_grid), ctypes.c_int, ctypes.POINTER(ctypes.c_int64)],
    "pw_advect_coeff_grad": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                             _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int64, _P],
    "pw_advect_coeff_grad_static": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                                    _P, _P, _P, _P, _P, _P, _P, _P],
    "pw_advect_adjoint_coeff_grad": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int,
                                     _P, _P, _P, ctypes.POINTER(pw_coeffs), _P, _P, _P, _P, _P, _P, _P, _P,
                                     ctypes.c_int64, _P],
    "pw_advect_zfast": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout_zfast), ctypes.c_int,
                        _P, _P, _P, ctypes.POINTER(pw_coeffs), _P, _P, _P, ctypes.POINTER(pw_tile), _P],
    "pw_advect_zfast_epilogue": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout_zfast), ctypes.c_int,
                                 _P, _P, _P, ctypes.POINTER(pw_coeffs), ctypes.POINTER(pw_epilogue), _P, _P, _P,
                                 ctypes.POINTER(pw_tile), _P],
    "pw_advect_bc": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int, _P, _P, _P,
                     ctypes.POINTER(pw_coeffs), ctypes.POINTER(pw_halo_modes), ctypes.POINTER(pw_epilogue),
                     _P, _P, _P, ctypes.POINTER(pw_tile), _P],
    "pw_halo_fill": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int, ctypes.POINTER(_P),
                     ctypes.POINTER(pw_halo_modes), ctypes.c_int32, _P],
    "pw_halo_fold": [ctypes.POINTER(pw_grid), ctypes.POINTER(pw_layout), ctypes.c_int, ctypes.POINTER(_P),
                     ctypes.POINTER(pw_halo_modes), ctypes.c_int32, _P],
    "pw_stream_copy": [_P, _P, ctypes.c_int64, _P],
    "pw_stream_probe": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_int32, _P],
    "pw_stream_copy3": [ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_int64, _P],
    "pw_tune": [ctypes.POINTER(pw_grid), ctypes.c_int, ctypes.c_int32, ctypes.POINTER(pw_tile),
                ctypes.POINTER(pw_tile)],
    "pw_tune_reset": [],
    "pw_launch_shape": [ctypes.c_int, ctypes.POINTER(pw_grid), ctypes.c_int, ctypes.POINTER(pw_tile)],
    "pw_batch_create": [ctypes.POINTER(pw_batch_item), ctypes.c_int32, ctypes.c_int, ctypes.POINTER(pw_tile),
                        ctypes.POINTER(ctypes.c_void_p)],
    "pw_batch_run": [_P, _P],
    "pw_batch_capture": [_P, _P],
    "pw_batch_replay": [_P, _P],
    "pw_batch_tune": [_P, _P, ctypes.POINTER(pw_tile)],
    "pw_batch_info": [_P, ctypes.POINTER(pw_tile), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)],
    "pw_batch_destroy": [_P],
    "pw_version": [],
    "pw_last_error": [],
}

_lib = None


def header_functions(path=HEADER):
    """Names of the functions declared in include/pwadv.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pw_[a-z_0-9]+)\s*\(", text)))


def lib():
    """The loaded libpwadv.so (raises PWLibraryMissing if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PWLibraryMissing("libpwadv.so not built: run __graft_entry__.build() "
                                   "(or python paper_2301_13016_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, argtypes in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = argtypes
            fn.restype = ctypes.c_char_p if name in ("pw_version", "pw_last_error") else ctypes.c_int
        _lib = L
    return _lib


def _check(status, call):
    if status != PW_OK:
        raise PWError(status, lib().pw_last_error().decode(), call)
    return status


# ------------------------------------------------------------------ raw C calls

def pw_version():
    return lib().pw_version().decode()


def pw_last_error():
    return lib().pw_last_error().decode()


def pw_advect(grid, layout, dtype, u, v, w, coeffs, su, sv, sw, stream=None):
    """Raw call: returns the pw_status (does not raise)."""
    return lib().pw_advect(ctypes.byref(grid), ctypes.byref(layout) if layout is not None else None,
                           int(dtype), u, v, w, ctypes.byref(coeffs), su, sv, sw, stream)


def pw_advect_ex(grid, layout, dtype, u, v, w, coeffs, su, sv, sw, tile=None, stream=None):
    return lib().pw_advect_ex(ctypes.byref(grid), ctypes.byref(layout) if layout is not None else None,
                              int(dtype), u, v, w, ctypes.byref(coeffs), su, sv, sw,
                              ctypes.byref(tile) if tile is not None else None, stream)


def pw_advect_adjoint(grid, layout, dtype, u, v, w, coeffs, gsu, gsv, gsw, gu, gv, gw, stream=None):
    return lib().pw_advect_adjoint(ctypes.byref(grid), ctypes.byref(layout) if layout is not None else None,
                                   int(dtype), u, v, w, ctypes.byref(coeffs), gsu, gsv, gsw,
                                   gu, gv, gw, stream)


def pw_advect_adjoint_ex(grid, layout, dtype, u, v, w, coeffs, gsu, gsv, gsw, gu, gv, gw, tile=None,
                         stream=None):
    return lib().pw_advect_adjoint_ex(ctypes.byref(grid), ctypes.byref(layout) if layout is not None else None,
                                      int(dtype), u, v, w, ctypes.byref(coeffs), gsu, gsv, gsw, gu, gv, gw,
                                      ctypes.byref(tile) if tile is not None else None, stream)


def pw_advect_tangent(grid, layout, dtype, u, v, w, coeffs, du, dv, dw, tu, tv, tw, stream=None):
    return lib().pw_advect_tangent(ctypes.byref(grid), ctypes.byref(layout) if layout is not None else None,
                                   int(dtype), u, v, w, ctypes.byref(coeffs), du, dv, dw, tu, tv, tw, stream)


def pw_advect_tangent_ex(grid, layout, dtype, u, v, w, coeffs, du, dv, dw, tu, tv, tw, tile=None,
                         stream=None):
    return lib().pw_advect_tangent_ex(ctypes.byref(grid), ctypes.byref(layout) if layout is not None else None,
                                      int(dtype), u, v, w, ctypes.byref(coeffs), du, dv, dw, tu, tv, tw,
                                      ctypes.byref(tile) if tile is not None else None, stream)


def pw_advect_zfast(grid, layout, dtype, u, v, w, coeffs, su, sv, sw, tile=None, stream=None):
    return lib().pw_advect_zfast(grid, layout, dtype, u, v, w, coeffs, su, sv, sw, tile, stream)


def pw_halo_fill(grid, layout, dtype, fields, modes, stream=None):
    """fields: device addresses; modes: (x, y, z) mode codes per field."""
    n = len(fields)
    f = (_P * max(n, 1))(*fields)
    m = (pw_halo_modes * max(n, 1))(*[pw_halo_modes(*mm) for mm in modes])
    return lib().pw_halo_fill(grid, layout, dtype, f, m, n, stream)


def pw_halo_fold(grid, layout, dtype, fields, modes, stream=None):
    """fields: device addresses; modes: (x, y, z) mode codes per field."""
    n = len(fields)
    f = (_P * max(n, 1))(*fields)
    m = (pw_halo_modes * max(n, 1))(*[pw_halo_modes(*mm) for mm in modes])
    return lib().pw_halo_fold(grid, layout, dtype, f, m, n, stream)


def pw_stream_copy(src, dst, nbytes, stream=None):
    return lib().pw_stream_copy(src, dst, int(nbytes), stream)


def pw_tune(grid, dtype, flags=0, fwd_best=None, adj_best=None):
    return lib().pw_tune(ctypes.byref(grid), int(dtype), int(flags),
                         ctypes.byref(fwd_best) if fwd_best is not None else None,
                         ctypes.byref(adj_best) if adj_best is not None else None)


def pw_tune_reset():
    return lib().pw_tune_reset()


def pw_batch_create(items, n, dtype, tile, out_handle):
    """items: ctypes array of pw_batch_item; out_handle: ctypes.c_void_p."""
    return lib().pw_batch_create(items, int(n), int(dtype), ctypes.byref(tile) if tile is not None else None,
                                 ctypes.byref(out_handle))


def pw_batch_run(handle, stream=None):
    return lib().pw_batch_run(handle, stream)


def pw_batch_capture(handle, stream):
    return lib().pw_batch_capture(handle, stream)


def pw_batch_replay(handle, stream=None):
    return lib().pw_batch_replay(handle, stream)


def pw_batch_tune(handle, stream=None, chosen=None):
    return lib().pw_batch_tune(handle, stream, ctypes.byref(chosen) if chosen is not None else None)


def pw_batch_info(handle, tile, items, groups):
    return lib().pw_batch_info(handle, ctypes.byref(tile), ctypes.byref(items), ctypes.byref(groups))


def pw_batch_destroy(handle):
    return lib().pw_batch_destroy(handle)


# ------------------------------------------------------------------ torch layer

@dataclass
class Coeffs:
    """Scheme coefficients on the device: tcx, tcy scalars and the four vertical
    arrays (torch tensors of length nz, float32 -- float64 for FP64 grids)."""
    tcx: float
    tcy: float
    tzc1: "object"
    tzc2: "object"
    tzd1: "object"
    tzd2: "object"

    def c_struct(self):
        return pw_coeffs(float(self.tcx), float(self.tcy), self.tzc1.data_ptr(), self.tzc2.data_ptr(),
                         self.tzd1.data_ptr(), self.tzd2.data_ptr())

    @classmethod
    def from_host(cls, c, device="cuda", dtype=None):
        import torch
        dt = torch.float32 if dtype is None else dtype
        mk = lambda a: torch.as_tensor(a, dtype=dt).to(device).contiguous()  # noqa: E731
        return cls(float(c["tcx"]), float(c["tcy"]), mk(c["tzc1"]), mk(c["tzc2"]), mk(c["tzd1"]), mk(c["tzd2"]))


def _dtype_code(t):
    import torch
    m = {torch.float32: PW_F32, torch.float64: PW_F64, torch.bfloat16: PW_BF16, torch.float16: PW_F16}
    if t.dtype not in m:
        raise TypeError("unsupported input dtype %s" % t.dtype)
    return m[t.dtype]


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _grid_from(u, halo):
    pz, py, px = u.shape
    return pw_grid(px - 2 * halo, py - 2 * halo, pz - 2 * halo, halo)


def _layout_from(inp, out):
    if inp.stride(-1) != 1 or out.stride(-1) != 1:
        raise ValueError("x (last) dimension must be contiguous")
    return pw_layout(inp.stride(1), inp.stride(0), out.stride(1), out.stride(0))


def _check_inputs(u, v, w):
    """u, v, w: one shape, one set of strides, one dtype, one device."""
    if not (u.shape == v.shape == w.shape and u.stride() == v.stride() == w.stride()
            and u.dtype == v.dtype == w.dtype and u.device == v.device == w.device):
        raise ValueError("u, v, w must share shape, strides, dtype and device")
    if u.dim() != 3:
        raise ValueError("u, v, w must be 3-D padded arrays")


def _check_group(ts, what, shape, dtype, device):
    """Every tensor in ``ts`` has ``shape``, ``dtype`` and ``device``, and all
    share one set of strides (the library sizes every buffer of a group from
    one layout)."""
    ts = list(ts)
    for t in ts:
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s must have shape %s (got %s)" % (what, tuple(shape), tuple(t.shape)))
        if t.dtype != dtype:
            raise ValueError("%s must be %s (got %s)" % (what, dtype, t.dtype))
        if t.device != device:
            raise ValueError("%s must be on %s (got %s)" % (what, device, t.device))
    if any(t.stride() != ts[0].stride() for t in ts):
        raise ValueError("%s must share one set of strides" % what)


def _compute_dtype(t):
    import torch
    return torch.float64 if t.dtype == torch.float64 else torch.float32


def _check_coeffs(coeffs, nz, dtype, device):
    """The vertical arrays: ``dtype`` (float64 for FP64 grids, else float32),
    contiguous, on ``device``, at least nz elements each."""
    for n in ("tzc1", "tzc2", "tzd1", "tzd2"):
        t = getattr(coeffs, n)
        if t.dtype != dtype:
            raise ValueError("coefficient %s must be %s for this grid (got %s)" % (n, dtype, t.dtype))
        if t.device != device:
            raise ValueError("coefficient %s must be on %s (got %s)" % (n, device, t.device))
        if not t.is_contiguous() or t.numel() < nz:
            raise ValueError("coefficient %s must be contiguous with at least nz=%d elements" % (n, nz))


def advect(u, v, w, coeffs: Coeffs, halo=1, out=None, tile=None, stream=None):
    """su, sv, sw = PW source terms of padded winds u, v, w (torch tensors on the
    GPU; float32, float64, bfloat16 or float16; identical shapes and strides)."""
    import torch
    _check_inputs(u, v, w)
    grid = _grid_from(u, halo)
    odt = _compute_dtype(u)
    _check_coeffs(coeffs, grid.nz, odt, u.device)
    if out is None:
        out = tuple(torch.empty((grid.nz, grid.ny, grid.nx), dtype=odt, device=u.device) for _ in range(3))
    su, sv, sw = out
    _check_group(out, "outputs", (grid.nz, grid.ny, grid.nx), odt, u.device)
    layout = _layout_from(u, su)
    c = coeffs.c_struct()
    tl = None if tile is None else pw_tile(*tile)
    st = pw_advect_ex(grid, layout, _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(), c,
                      su.data_ptr(), sv.data_ptr(), sw.data_ptr(), tl, _stream_handle(stream))
    _check(st, "pw_advect")
    return su, sv, sw


def advect_zfast(u, v, w, coeffs: Coeffs, halo=1, out=None, tile=None, stream=None):
    """su, sv, sw of winds stored z-fastest: u, v, w have shape
    (nx+2h, ny+2h, nz+2h) indexed [i, j, k] with k contiguous; the outputs
    (nx, ny, nz) likewise.  Bit-identical to advect() on the transposed
    arrays."""
    import torch
    _check_inputs(u, v, w)
    pi, pj, pk = u.shape
    grid = pw_grid(pi - 2 * halo, pj - 2 * halo, pk - 2 * halo, halo)
    odt = _compute_dtype(u)
    _check_coeffs(coeffs, grid.nz, odt, u.device)
    if out is None:
        out = tuple(torch.empty((grid.nx, grid.ny, grid.nz), dtype=odt, device=u.device) for _ in range(3))
    su, sv, sw = out
    _check_group(out, "outputs", (grid.nx, grid.ny, grid.nz), odt, u.device)
    if u.stride(-1) != 1 or su.stride(-1) != 1:
        raise ValueError("z (last) dimension must be contiguous")
    layout = pw_layout_zfast(u.stride(1), u.stride(0), su.stride(1), su.stride(0))
    c = coeffs.c_struct()
    tl = None if tile is None else pw_tile(*tile)
    st = pw_advect_zfast(grid, layout, _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(), c,
                         su.data_ptr(), sv.data_ptr(), sw.data_ptr(), tl, _stream_handle(stream))
    _check(st, "pw_advect_zfast")
    return su, sv, sw


def advect_bc(u, v, w, coeffs: Coeffs, bc, halo=1, out=None, addends=None, alpha=1.0, tile=None, stream=None):
    """The forward (with ``addends``: out = addends + alpha * F) with boundary
    rules applied by addressing: ``bc`` is one (x, y, z) triple of rules for
    all three fields or a list of three triples (u, v, w), each entry a name
    from HALO_MODES or its code.  Equals halo_fill with the same rules
    followed by advect / advect_epilogue, without touching the halo.  On each
    axis the three fields must all keep, all be periodic or all use
    nearest-cell rules (copy, zero, reflect, reflect_neg)."""
    import torch
    _check_inputs(u, v, w)
    grid = _grid_from(u, halo)
    odt = _compute_dtype(u)
    _check_coeffs(coeffs, grid.nz, odt, u.device)
    if out is None:
        out = tuple(torch.empty((grid.nz, grid.ny, grid.nx), dtype=odt, device=u.device) for _ in range(3))
    su, sv, sw = out
    _check_group(out, "outputs", (grid.nz, grid.ny, grid.nx), odt, u.device)
    layout = _layout_from(u, su)
    modes = (pw_halo_modes * 3)(*(pw_halo_modes(*(_halo_code(m) for m in t)) for t in _per_field_modes(bc, 3)))
    ep = None
    if addends is not None:
        _check_group(list(addends) + list(out), "addends and outputs", (grid.nz, grid.ny, grid.nx), odt, u.device)
        ep = pw_epilogue(float(alpha), *(c.data_ptr() for c in addends))
    tl = None if tile is None else pw_tile(*tile)
    st = lib().pw_advect_bc(grid, layout, _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(), coeffs.c_struct(),
                            modes, ep, su.data_ptr(), sv.data_ptr(), sw.data_ptr(), tl, _stream_handle(stream))
    _check(st, "pw_advect_bc")
    return su, sv, sw


def advect_zfast_epilogue(u, v, w, coeffs: Coeffs, addends, alpha=1.0, halo=1, out=None, tile=None, stream=None):
    """out = addends + alpha * F(u, v, w) on z-fastest arrays (see
    advect_zfast); ``addends`` are (nx, ny, nz)-indexed tensors in the output
    dtype, each either its output (accumulation in place) or disjoint from
    the outputs."""
    import torch
    _check_inputs(u, v, w)
    pi, pj, pk = u.shape
    grid = pw_grid(pi - 2 * halo, pj - 2 * halo, pk - 2 * halo, halo)
    odt = _compute_dtype(u)
    _check_coeffs(coeffs, grid.nz, odt, u.device)
    cu, cv, cw = addends
    _check_group(addends, "addends", (grid.nx, grid.ny, grid.nz), odt, u.device)
    if out is None:
        out = tuple(torch.empty((grid.nx, grid.ny, grid.nz), dtype=odt, device=u.device) for _ in range(3))
    su, sv, sw = out
    _check_group(out, "outputs", (grid.nx, grid.ny, grid.nz), odt, u.device)
    if u.stride(-1) != 1 or su.stride(-1) != 1:
        raise ValueError("z (last) dimension must be contiguous")
    if su.stride() != cu.stride():
        raise ValueError("addends and outputs must share strides")
    layout = pw_layout_zfast(u.stride(1), u.stride(0), su.stride(1), su.stride(0))
    c = coeffs.c_struct()
    ep = pw_epilogue(float(alpha), cu.data_ptr(), cv.data_ptr(), cw.data_ptr())
    tl = None if tile is None else pw_tile(*tile)
    st = lib().pw_advect_zfast_epilogue(grid, layout, _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(),
                                        c, ep, su.data_ptr(), sv.data_ptr(), sw.data_ptr(), tl,
                                        _stream_handle(stream))
    _check(st, "pw_advect_zfast_epilogue")
    return su, sv, sw


def advect_epilogue(u, v, w, coeffs: Coeffs, addends, alpha=1.0, halo=1, out=None, tile=None, stream=None):
    """out = addends + alpha * F(u, v, w) with one rounding per element.
    ``addends`` is (cu, cv, cw) in the outputs' layout and compute dtype;
    pass the outputs themselves to accumulate in place (``out=addends``)."""
    import torch
    _check_inputs(u, v, w)
    grid = _grid_from(u, halo)
    odt = _compute_dtype(u)
    _check_coeffs(coeffs, grid.nz, odt, u.device)
    cu, cv, cw = addends
    if out is None:
        out = tuple(torch.empty_like(x) for x in (cu, cv, cw))
    su, sv, sw = out
    _check_group(list(out) + list(addends), "outputs and addends", (grid.nz, grid.ny, grid.nx), odt, u.device)
    layout = _layout_from(u, su)
    tl = None if tile is None else pw_tile(*tile)
    ep = pw_epilogue(float(alpha), cu.data_ptr(), cv.data_ptr(), cw.data_ptr())
    st = lib().pw_advect_epilogue(ctypes.byref(grid), ctypes.byref(layout), _dtype_code(u), u.data_ptr(),
                                  v.data_ptr(), w.data_ptr(), ctypes.byref(coeffs.c_struct()), ctypes.byref(ep),
                                  su.data_ptr(), sv.data_ptr(), sw.data_ptr(),
                                  ctypes.byref(tl) if tl is not None else None, _stream_handle(stream))
    _check(st, "pw_advect_epilogue")
    return su, sv, sw


def advect_adjoint(u, v, w, coeffs: Coeffs, gsu, gsv, gsw, halo=1, out=None, tile=None, stream=None):
    """gu, gv, gw = J(u, v, w)^T (gsu, gsv, gsw), padded-shaped (halo included)."""
    import torch
    _check_inputs(u, v, w)
    grid = _grid_from(u, halo)
    _check_coeffs(coeffs, grid.nz, _compute_dtype(u), u.device)
    if out is None:
        out = tuple(torch.empty_like(u) for _ in range(3))
    gu, gv, gw = out
    for g in (gsu, gsv, gsw):
        _check_group([g], "cotangents", (grid.nz, grid.ny, grid.nx), u.dtype, u.device)
    gsu, gsv, gsw = (g.contiguous() if g.stride(-1) != 1 else g for g in (gsu, gsv, gsw))
    if not (gsu.stride() == gsv.stride() == gsw.stride()):
        gsu, gsv, gsw = (g.contiguous() for g in (gsu, gsv, gsw))
    layout = _layout_from(u, gsu)
    _check_group(out, "gradients", tuple(u.shape), u.dtype, u.device)
    if gu.stride() != u.stride():
        raise ValueError("gradients must share the inputs' strides")
    tl = None if tile is None else pw_tile(*tile)
    st = pw_advect_adjoint_ex(grid, layout, _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(),
                              coeffs.c_struct(), gsu.data_ptr(), gsv.data_ptr(), gsw.data_ptr(),
                              gu.data_ptr(), gv.data_ptr(), gw.data_ptr(), tl, _stream_handle(stream))
    _check(st, "pw_advect_adjoint")
    return gu, gv, gw


def advect_tangent(u, v, w, coeffs: Coeffs, du, dv, dw, halo=1, out=None, tile=None, stream=None):
    """tu, tv, tw = J(u, v, w) (du, dv, dw), interior-shaped; du, dv, dw are
    padded like u (the halo is read)."""
    import torch
    _check_inputs(u, v, w)
    grid = _grid_from(u, halo)
    _check_coeffs(coeffs, grid.nz, _compute_dtype(u), u.device)
    for d in (du, dv, dw):
        if d.shape != u.shape or d.dtype != u.dtype or d.device != u.device:
            raise ValueError("the direction must match u in shape, dtype and device")
    if not (du.stride() == dv.stride() == dw.stride() == u.stride()):
        du, dv, dw = (d.contiguous() for d in (du, dv, dw))
        if du.stride() != u.stride():
            raise ValueError("the direction must share the inputs' strides")
    if out is None:
        nz, ny, nx = (s - 2 * halo for s in u.shape)
        out = tuple(torch.empty((nz, ny, nx), dtype=u.dtype, device=u.device) for _ in range(3))
    tu, tv, tw = out
    _check_group(out, "outputs", (grid.nz, grid.ny, grid.nx), u.dtype, u.device)
    layout = _layout_from(u, tu)
    tl = None if tile is None else pw_tile(*tile)
    st = pw_advect_tangent_ex(grid, layout, _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(),
                              coeffs.c_struct(), du.data_ptr(), dv.data_ptr(), dw.data_ptr(),
                              tu.data_ptr(), tv.data_ptr(), tw.data_ptr(), tl, _stream_handle(stream))
    _check(st, "pw_advect_tangent")
    return tu, tv, tw


def pw_advect_coeff_grad_static(grid, layout, dtype, u, v, w, gsu, gsv, gsw, grad, stream=None):
    """Raw call of the allocation-free entry point; returns the pw_status."""
    return lib().pw_advect_coeff_grad_static(ctypes.byref(grid), ctypes.byref(layout) if layout is not None else None,
                                             int(dtype), u, v, w, gsu, gsv, gsw, grad, stream)


def advect_coeff_grad(u, v, w, gsu, gsv, gsw, halo=1, stream=None, out=None, static_scratch=False):
    """Gradients of <su, gsu> + <sv, gsv> + <sw, gsw> with respect to the
    coefficients (their values do not enter: the loss is linear in them).
    Returns a dict of float64 device tensors: tcx, tcy (0-d), tzc1, tzc2,
    tzd1, tzd2 (length nz), tcx_level, tcy_level (each level's share), views
    of one (6 nz + 2)-element buffer (``out`` if given).  With
    ``static_scratch`` the library's own scratch replaces the workspace
    (pw_advect_coeff_grad_static: nothing is allocated when ``out`` is
    given)."""
    import torch
    _check_inputs(u, v, w)
    grid = _grid_from(u, halo)
    for g in (gsu, gsv, gsw):
        _check_group([g], "cotangents", (grid.nz, grid.ny, grid.nx), u.dtype, u.device)
    gs = [g.contiguous() if g.stride(-1) != 1 else g for g in (gsu, gsv, gsw)]
    if not (gs[0].stride() == gs[1].stride() == gs[2].stride()):
        gs = [g.contiguous() for g in gs]
    layout = _layout_from(u, gs[0])
    nz = int(grid.nz)
    if out is None:
        out = torch.empty(6 * nz + 2, dtype=torch.float64, device=u.device)
    _check_group([out], "out", (6 * nz + 2,), torch.float64, u.device)
    if static_scratch:
        st = pw_advect_coeff_grad_static(grid, layout, _dtype_code(u), u.data_ptr(), v.data_ptr(), w.data_ptr(),
                                         *(g.data_ptr() for g in gs), out.data_ptr(), _stream_handle(stream))
        _check(st, "pw_advect_coeff_grad_static")
    else:
        need = ctypes.c_int64()
        _check(lib().pw_advect_coeff_grad_workspace(ctypes.byref(grid), _dtype_code(u), ctypes.byref(need)),
               "pw_advect_coeff_grad_workspace")
        ws = torch.empty(max(1, need.value // 8), dtype=torch.float64, device=u.device)
        st = lib().pw_advect_coeff_grad(ctypes.byref(grid), ctypes.byref(layout), _dtype_code(u), u.data_ptr(),
                                        v.data_ptr(), w.data_ptr(), *(g.data_ptr() for g in gs), out.data_ptr(),
                                        ws.data_ptr(), need.value, _stream_handle(stream))
        _check(st, "pw_advect_coeff_grad")
    return _coeff_grad_dict(out, nz)


def _coeff_grad_dict(out, nz):
    names = ("tzc1", "tzc2", "tzd1", "tzd2", "tcx_level", "tcy_level")
    res = {n: out[i * nz:(i + 1) * nz] for i, n in enumerate(names)}
    res["tcx"], res["tcy"] = out[6 * nz], out[6 * nz + 1]
    return res


def advect_adjoint_coeff_grad(u, v, w, coeffs: Coeffs, gsu, gsv, gsw, halo=1, out=None, grad_out=None,
                              stream=None):
    """The whole backward in one pass (pw_advect_adjoint_coeff_grad): the wind
    gradients (gu, gv, gw) as advect_adjoint and the coefficient gradients as
    advect_coeff_grad (a dict of views of ``grad_out``), bit for bit."""
    import torch
    _check_inputs(u, v, w)
    grid = _grid_from(u, halo)
    _check_coeffs(coeffs, grid.nz, _compute_dtype(u), u.device)
    if out is None:
        out = tuple(torch.empty_like(u) for _ in range(3))
    gu, gv, gw = out
    for g in (gsu, gsv, gsw):
        _check_group([g], "cotangents", (grid.nz, grid.ny, grid.nx), u.dtype, u.device)
    gsu, gsv, gsw = (g.contiguous() if g.stride(-1) != 1 else g for g in (gsu, gsv, gsw))
    if not (gsu.stride() == gsv.stride() == gsw.stride()):
        gsu, gsv, gsw = (g.contiguous() for g in (gsu, gsv, gsw))
    layout = _layout_from(u, gsu)
    _check_group(out, "gradients", tuple(u.shape), u.dtype, u.device)
    if gu.stride() != u.stride():
        raise ValueError("gradients must share the inputs' strides")
    nz = int(grid.nz)
    if grad_out is None:
        grad_out = torch.empty(6 * nz + 2, dtype=torch.float64, device=u.device)
    _check_group([grad_out], "grad_out", (6 * nz + 2,), torch.float64, u.device)
    need = ctypes.c_int64()
    _check(lib().pw_advect_coeff_grad_workspace(ctypes.byref(grid), _dtype_code(u), ctypes.byref(need)),
           "pw_advect_coeff_grad_workspace")
    ws = torch.empty(max(1, need.value // 8), dtype=torch.float64, device=u.device)
    st = lib().pw_advect_adjoint_coeff_grad(ctypes.byref(grid), ctypes.byref(layout), _dtype_code(u), u.data_ptr(),
                                            v.data_ptr(), w.data_ptr(), ctypes.byref(coeffs.c_struct()),
                                            gsu.data_ptr(), gsv.data_ptr(), gsw.data_ptr(), gu.data_ptr(),
                                            gv.data_ptr(), gw.data_ptr(), grad_out.data_ptr(), ws.data_ptr(),
                                            need.value, _stream_handle(stream))
    _check(st, "pw_advect_adjoint_coeff_grad")
    return (gu, gv, gw), _coeff_grad_dict(grad_out, nz)


def tune(nx, ny, nz, dtype, halo=1, flags=0):
    """Run the autotuner for this grid class; returns (forward tile, adjoint
    tile) as (cols_per_lane, rows_per_strip, zlen, waves_per_group, prefetch,
    share_rows) tuples (the adjoint entry is None when not tuned)."""
    import torch
    code = {torch.float32: PW_F32, torch.float64: PW_F64, torch.bfloat16: PW_BF16, torch.float16: PW_F16}[dtype]
    f, a = pw_tile(), pw_tile()
    _check(pw_tune(pw_grid(nx, ny, nz, halo), code, flags, f, a), "pw_tune")
    return _tile_tuple(f), (_tile_tuple(a) if a.rows_per_strip else None)


def launch_shape(kind, nx, ny, nz, dtype, halo=1):
    """The launch shape ``kind`` ("forward", "adjoint", "tangent" or "zfast")
    takes for this grid when called without a tile, as (cols_per_lane,
    rows_per_strip, zlen, waves_per_group, prefetch, share_rows)."""
    import torch
    code = {torch.float32: PW_F32, torch.float64: PW_F64, torch.bfloat16: PW_BF16, torch.float16: PW_F16}[dtype]
    k = {"forward": PW_KERNEL_FORWARD, "adjoint": PW_KERNEL_ADJOINT, "tangent": PW_KERNEL_TANGENT,
         "zfast": PW_KERNEL_ZFAST}[kind]
    t = pw_tile()
    _check(lib().pw_launch_shape(k, ctypes.byref(pw_grid(nx, ny, nz, halo)), code, ctypes.byref(t)),
           "pw_launch_shape")
    return _tile_tuple(t)


class Batch:
    """Many subdomains in one persistent launch (FP32).  ``subdomains`` is a
    list of (u, v, w, coeffs, (su, sv, sw)) with padded inputs and interior
    outputs as torch tensors on the current device."""

    def __init__(self, subdomains, halo=1, tile=None):
        n = len(subdomains)
        items = (pw_batch_item * n)()
        self._keep = []
        import torch
        for i, (u, v, w, c, outs) in enumerate(subdomains):
            su, sv, sw = outs
            _check_inputs(u, v, w)
            if u.dtype != torch.float32:
                raise ValueError("batched subdomains are float32")
            g = _grid_from(u, halo)
            _check_coeffs(c, g.nz, torch.float32, u.device)
            _check_group(outs, "outputs of subdomain %d" % i, (g.nz, g.ny, g.nx), torch.float32, u.device)
            items[i].grid = _grid_from(u, halo)
            items[i].layout = _layout_from(u, su)
            items[i].u, items[i].v, items[i].w = u.data_ptr(), v.data_ptr(), w.data_ptr()
            items[i].coeffs = c.c_struct()
            items[i].su, items[i].sv, items[i].sw = su.data_ptr(), sv.data_ptr(), sw.data_ptr()
            self._keep.append((u, v, w, c, outs))
        self.handle = ctypes.c_void_p()
        tl = None if tile is None else pw_tile(*tile)
        _check(pw_batch_create(items, n, PW_F32, tl, self.handle), "pw_batch_create")

    def run(self, stream=None):
        _check(pw_batch_run(self.handle, _stream_handle(stream)), "pw_batch_run")

    def capture(self, stream):
        _check(pw_batch_capture(self.handle, _stream_handle(stream)), "pw_batch_capture")

    def replay(self, stream=None):
        _check(pw_batch_replay(self.handle, _stream_handle(stream)), "pw_batch_replay")

    def tune(self, stream=None):
        t = pw_tile()
        _check(pw_batch_tune(self.handle, _stream_handle(stream), t), "pw_batch_tune")
        return _tile_tuple(t)

    def info(self):
        t, it, g = pw_tile(), ctypes.c_int64(), ctypes.c_int32()
        _check(pw_batch_info(self.handle, t, it, g), "pw_batch_info")
        return _tile_tuple(t), it.value, g.value

    def close(self):
        if self.handle:
            pw_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _halo_code(m):
    if isinstance(m, str):
        if m not in HALO_MODES:
            raise ValueError("unknown halo mode %r (one of %s)" % (m, ", ".join(HALO_MODES)))
        return HALO_MODES[m]
    return int(m)


def _per_field_modes(modes, n):
    """One (x, y, z) rule triple for each of n fields: ``modes`` is one triple
    for all of them or a list of n triples."""
    modes = list(modes)
    if len(modes) == 3 and all(isinstance(m, (str, int)) for m in modes):
        return [tuple(modes)] * n
    if len(modes) != n or any(len(m) != 3 for m in modes):
        raise ValueError("one (x, y, z) mode triple for all fields or one per field")
    return [tuple(m) for m in modes]


def _halo_call(fn, name, fields, modes, halo, stream):
    fields = list(fields)
    if not fields:
        return fields
    u = fields[0]
    if any(f.shape != u.shape or f.stride() != u.stride() or f.dtype != u.dtype or f.device != u.device
           for f in fields):
        raise ValueError("fields must share shape, strides, dtype and device")
    if u.dim() != 3:
        raise ValueError("fields must be 3-D padded arrays")
    codes = [tuple(_halo_code(m) for m in mm) for mm in _per_field_modes(modes, len(fields))]
    grid = _grid_from(u, halo)
    if u.stride(-1) != 1:
        raise ValueError("x (last) dimension must be contiguous")
    layout = pw_layout(u.stride(1), u.stride(0), grid.nx, grid.nx * grid.ny)
    _check(fn(grid, layout, _dtype_code(u), [f.data_ptr() for f in fields], codes, _stream_handle(stream)), name)
    return fields


def halo_fold(fields, modes, halo=1, stream=None):
    """The adjoint of halo_fill with the same rules, in place on float32 /
    float64 gradient tensors shaped like the padded fields.  Returns
    ``fields``."""
    return _halo_call(pw_halo_fold, "pw_halo_fold", fields, modes, halo, stream)


def advect_bc_adjoint(u, v, w, coeffs: Coeffs, bc, gsu, gsv, gsw, halo=1, stream=None):
    """Gradients of <advect_bc(u, v, w, bc), (gsu, gsv, gsw)> with respect to
    the padded u, v, w as given (before the boundary rules): the adjoint
    kernel at the filled state, then the fold.  Halo entries on axes whose
    rule is not keep come out zero."""
    filled = [x.clone() for x in (u, v, w)]
    halo_fill(filled, bc, halo=halo, stream=stream)
    grads = advect_adjoint(*filled, coeffs, gsu, gsv, gsw, halo=halo, stream=stream)
    return tuple(halo_fold(list(grads), bc, halo=halo, stream=stream))


def halo_fill(fields, modes, halo=1, stream=None):
    """Fill the halo of padded tensors in place (same shape, strides and dtype,
    on the GPU).  ``modes`` is one (x, y, z) triple for every field or a list
    of triples, one per field; each entry is a name from HALO_MODES or its
    code.  Returns ``fields``."""
    return _halo_call(pw_halo_fill, "pw_halo_fill", fields, modes, halo, stream)


def pw_stream_probe(mode, loads_per_lane, flags, src, dst, nbytes, blocks, stream=None):
    return lib().pw_stream_probe(int(mode), int(loads_per_lane), int(flags), src, dst, int(nbytes), int(blocks),
                                 stream)


def stream_probe(mode, loads_per_lane, flags, src, dst, blocks, stream=None):
    """One launch of the bandwidth probe (mode 0 copy, 1 read, 2 write; see
    pw_stream_probe) over ``src`` (or ``dst`` for writes) of torch tensors."""
    buf = dst if mode == 2 else src
    n = buf.numel() * buf.element_size()
    _check(pw_stream_probe(mode, loads_per_lane, flags, 0 if src is None else src.data_ptr(), dst.data_ptr(), n,
                           blocks, _stream_handle(stream)), "pw_stream_probe")


def stream_copy(src, dst, stream=None):
    _check(pw_stream_copy(src.data_ptr(), dst.data_ptr(), src.numel() * src.element_size(),
                          _stream_handle(stream)), "pw_stream_copy")
    return dst


def pw_stream_copy3(srcs, dsts, nbytes, stream=None):
    s = (_P * 3)(*srcs)
    d = (_P * 3)(*dsts)
    return lib().pw_stream_copy3(s, d, int(nbytes), stream)


def stream_copy3(srcs, dsts, stream=None):
    """dsts[i] <- srcs[i] for three equal-sized tensors, in one kernel."""
    n = srcs[0].numel() * srcs[0].element_size()
    if any(t.numel() * t.element_size() != n for t in list(srcs) + list(dsts)):
        raise ValueError("all six tensors must have the same size in bytes")
    _check(pw_stream_copy3([t.data_ptr() for t in srcs], [t.data_ptr() for t in dsts], n, _stream_handle(stream)),
           "pw_stream_copy3")
    return dsts


def _autograd_function():
    import torch

    class PWAdvect(torch.autograd.Function):
        """Differentiable PW advection: forward = ``advect``; reverse mode
        (backward) = the hand-written adjoint kernel, forward mode (jvp) = the
        hand-written tangent-linear kernel.  Derivatives are w.r.t. u, v, w;
        the coefficients are treated as constants."""

        @staticmethod
        def forward(ctx, u, v, w, coeffs, halo=1):
            ctx.save_for_backward(u, v, w)
            ctx.save_for_forward(u, v, w)
            ctx.coeffs = coeffs
            ctx.halo = halo
            return advect(u, v, w, coeffs, halo)

        @staticmethod
        def jvp(ctx, du, dv, dw, _dcoeffs=None, _dhalo=None):
            u, v, w = ctx.saved_tensors
            du, dv, dw = (torch.zeros_like(u) if d is None else d for d in (du, dv, dw))
            return advect_tangent(u, v, w, ctx.coeffs, du, dv, dw, ctx.halo)

        @staticmethod
        def backward(ctx, gsu, gsv, gsw):
            u, v, w = ctx.saved_tensors
            gu, gv, gw = advect_adjoint(u, v, w, ctx.coeffs, gsu, gsv, gsw, ctx.halo)
            return gu, gv, gw, None, None

    return PWAdvect


_PWAdvect = None
_PWAdvectCoeffs = None
_PWAdvectBC = None


def _autograd_function_bc():
    import torch

    class PWAdvectBC(torch.autograd.Function):
        """PW advection with boundary rules applied by addressing:
        apply(u, v, w, coeffs, bc, halo=1) = advect_bc.  Reverse mode = the
        adjoint kernel at the filled state followed by the halo fold, so the
        gradients are with respect to u, v, w as given (zero in the halo on
        axes whose rule is not keep); forward mode = the tangent kernel on the
        filled state and direction."""

        @staticmethod
        def forward(ctx, u, v, w, coeffs, bc, halo=1):
            ctx.save_for_backward(u, v, w)
            ctx.save_for_forward(u, v, w)
            ctx.coeffs, ctx.bc, ctx.halo = coeffs, bc, halo
            return advect_bc(u, v, w, coeffs, bc, halo=halo)

        @staticmethod
        def jvp(ctx, du, dv, dw, _dcoeffs=None, _dbc=None, _dhalo=None):
            u, v, w = ctx.saved_tensors
            d = [torch.zeros_like(u) if x is None else x.clone() for x in (du, dv, dw)]
            xf = [x.clone() for x in (u, v, w)]
            halo_fill(xf, ctx.bc, halo=ctx.halo)
            halo_fill(d, ctx.bc, halo=ctx.halo)
            return advect_tangent(*xf, ctx.coeffs, *d, halo=ctx.halo)

        @staticmethod
        def backward(ctx, gsu, gsv, gsw):
            u, v, w = ctx.saved_tensors
            gu, gv, gw = advect_bc_adjoint(u, v, w, ctx.coeffs, ctx.bc, gsu.contiguous(), gsv.contiguous(),
                                           gsw.contiguous(), halo=ctx.halo)
            return gu, gv, gw, None, None, None

    return PWAdvectBC


def PWAdvectBC():
    """The autograd Function of advect_bc (created on first use)."""
    global _PWAdvectBC
    if _PWAdvectBC is None:
        _PWAdvectBC = _autograd_function_bc()
    return _PWAdvectBC


def _autograd_function_coeffs():
    import torch

    class PWAdvectCoeffs(torch.autograd.Function):
        """PW advection differentiable in the winds and in the coefficients:
        apply(u, v, w, tcx, tcy, tzc1, tzc2, tzd1, tzd2, halo=1) with tcx, tcy
        0-d tensors and tz* device tensors of length nz.  Backward runs one
        adjoint march for both the winds and the coefficients when both are
        needed (advect_adjoint_coeff_grad), else only the one needed."""

        @staticmethod
        def forward(ctx, u, v, w, tcx, tcy, tzc1, tzc2, tzd1, tzd2, halo=1):
            c = Coeffs(float(tcx), float(tcy), tzc1, tzc2, tzd1, tzd2)
            ctx.save_for_backward(u, v, w)
            ctx.coeffs, ctx.halo = c, halo
            ctx.cdtypes = [(t.dtype, t.device) for t in (tcx, tcy)]
            return advect(u, v, w, c, halo)

        @staticmethod
        def backward(ctx, gsu, gsv, gsw):
            u, v, w = ctx.saved_tensors
            need = ctx.needs_input_grad
            gu = gv = gw = None
            g = None
            if any(need[:3]) and any(need[3:9]):   # one pass over the winds and cotangents
                (gu, gv, gw), g = advect_adjoint_coeff_grad(u, v, w, ctx.coeffs, gsu, gsv, gsw, ctx.halo)
            elif any(need[:3]):
                gu, gv, gw = advect_adjoint(u, v, w, ctx.coeffs, gsu, gsv, gsw, ctx.halo)
            elif any(need[3:9]):
                g = advect_coeff_grad(u, v, w, gsu, gsv, gsw, ctx.halo)
            cg = [None] * 6
            if g is not None:
                c = ctx.coeffs
                (d0, v0), (d1, v1) = ctx.cdtypes
                cg = [g["tcx"].to(device=v0, dtype=d0), g["tcy"].to(device=v1, dtype=d1)] + \
                     [g[n].to(getattr(c, n).dtype) for n in ("tzc1", "tzc2", "tzd1", "tzd2")]
            return (gu, gv, gw, *cg, None)

    return PWAdvectCoeffs


def PWAdvectCoeffs():
    """The autograd Function differentiable in the coefficients too (created
    on first use)."""
    global _PWAdvectCoeffs
    if _PWAdvectCoeffs is None:
        _PWAdvectCoeffs = _autograd_function_coeffs()
    return _PWAdvectCoeffs


def PWAdvect():
    """The torch.autograd.Function class (created on first use, so importing
    this module does not import torch)."""
    global _PWAdvect
    if _PWAdvect is None:
        _PWAdvect = _autograd_function()
    return _PWAdvect
