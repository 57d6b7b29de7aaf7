"""GPU tests of the hand-written tangent-linear kernel (J(x) dx, Jacobian-
vector product) against the FP64 oracle's tangent, plus the identities that
tie it to the forward and adjoint kernels.

Tolerances: A-scaled with A_TL = sum over terms of |c| (|da| (|b|+|d|) +
|a| (|db|+|dd|)) (scales.tangent_scale, pinned on the CPU); 1e-6 in FP32
(about a dozen roundings of 2^-24 = 6e-8 along a point's sum, so at most
about 7e-7), 1e-13 in FP64, and bit for bit on integer data with dyadic
coefficients.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import a_scaled_error, dev_grid
from scales import tangent_scale
from paper_2301_13016_amd import binding as B
from paper_2301_13016_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture(autouse=True)
def _announce(request):
    sys.__stderr__.write("\n[gpu-test] %s\n" % request.node.nodeid)
    sys.__stderr__.flush()
    yield


def _dev(arrs):
    return [torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in arrs]


def gpu_tangent(g, d, tile=None, halo=1):
    (u, v, w), c = dev_grid(g)
    dd = [x.to(u.dtype) for x in _dev(d)]
    out = B.advect_tangent(u, v, w, c, *dd, halo=halo, tile=tile)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def tl_magnitude(g, d, halo=1):
    return tangent_scale(g.u, g.v, g.w, d, g.coeffs, halo=halo)


def tl_errors(got, g, d, halo=1):
    dq = [np.asarray(x, g.u.dtype).astype(np.float64) for x in d]   # the direction as the kernel saw it
    ref = oracle.tangent(g.u, g.v, g.w, *dq, g.coeffs, halo=halo)
    mag = tl_magnitude(g, dq, halo=halo)
    return [a_scaled_error(x, y, m) for x, y, m in zip(got, ref, mag)], ref


SHAPES = [(130, 70, 20), (64, 64, 64), (1, 1, 1), (65, 3, 1), (1, 200, 5), (61, 9, 17), (128, 4, 3),
          (129, 5, 2), (257, 3, 4), (300, 7, 9)]


@pytest.mark.parametrize("tile", [None, (1, 1, 5, 4), (1, 2, 9, 1), (2, 1, 7, 8), (2, 2, 64, 2), (1, 2, 6, 4, 2),
                                  (2, 2, 9, 1, 2), (2, 1, 64, 8, 2)])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_f32_tangent_matches_oracle(shape, tile):
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=400 + nx + ny + nz)
    d = wl.direction(nx, ny, nz, seed=500 + nx)
    errs, _ = tl_errors(gpu_tangent(g, d, tile=tile), g, d)
    assert max(errs) <= 1e-6, errs


@pytest.mark.parametrize("tile", [None, (1, 1, 3, 1), (1, 2, 64, 8), (1, 2, 5, 4, 2)])
def test_f64_tangent_matches_oracle(tile):
    g = wl.make_grid(70, 33, 21, seed=401, dtype=np.float64)
    d = wl.direction(70, 33, 21, seed=501)
    errs, _ = tl_errors(gpu_tangent(g, d, tile=tile), g, d)
    assert max(errs) <= 1e-13, errs


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_integer_tangent_bitwise(dtype):
    g = wl.integer_grid(130, 11, 7, seed=402, dtype=dtype)
    rng = np.random.default_rng(502)
    d = [rng.integers(-3, 4, g.u.shape).astype(dtype) for _ in range(3)]
    got = gpu_tangent(g, d)
    ref = oracle.tangent(g.u, g.v, g.w, *d, g.coeffs)
    for a, b in zip(got, ref):
        assert np.array_equal(a.astype(np.float64), b)


def test_tangent_strided_layout_bitwise():
    """Values, direction and outputs as views into larger buffers (extra
    columns and rows per plane): the dense result bit for bit, nothing outside
    the output views written."""
    g = wl.make_grid(150, 37, 23, seed=404)
    d = wl.direction(150, 37, 23, seed=504)
    dense = gpu_tangent(g, d)
    (u, v, w), c = dev_grid(g)
    dd = [x.to(u.dtype) for x in _dev(d)]

    def view(src, extra_rows, extra_cols, fill):
        big = torch.full((src.shape[0], src.shape[1] + extra_rows, src.shape[2] + extra_cols), fill,
                         dtype=src.dtype, device=src.device)
        big[:, :src.shape[1], :src.shape[2]] = src
        return big, big[:, :src.shape[1], :src.shape[2]]

    xs = [view(x, 2, 5, 3.0)[1] for x in (u, v, w)]
    ds = [view(x, 2, 5, 3.0)[1] for x in dd]
    outs = [view(torch.full((23, 37, 150), float("nan"), device="cuda"), 1, 4, -2.0) for _ in range(3)]
    got = B.advect_tangent(*xs, c, *ds, out=tuple(vw for _, vw in outs))
    torch.cuda.synchronize()
    for a, (b, vw) in zip(dense, outs):
        assert np.array_equal(a, vw.cpu().numpy())
        outside = b.clone()
        outside[:, :37, :150] = -2.0
        assert bool((outside == -2.0).all())
    assert all(x is vw for x, (_, vw) in zip(got, outs))


def test_tangent_tile_invariance_bitwise():
    g = wl.make_grid(150, 37, 23, seed=403)
    d = wl.direction(150, 37, 23, seed=503)
    base = gpu_tangent(g, d, tile=(1, 2, 16, 4))
    for t in [(1, 1, 1, 1), (1, 1, 9, 4), (1, 2, 5, 8), (2, 1, 64, 4), (2, 2, 3, 2), (2, 2, 23, 1), (1, 1, 2, 4, 2),
              (2, 2, 23, 1, 2), (2, 1, 7, 8, 2)]:
        got = gpu_tangent(g, d, tile=t)
        for a, b in zip(base, got):
            assert np.array_equal(a, b), t


@pytest.mark.parametrize("halo", [2, 3])
def test_tangent_wider_halo(halo):
    g = wl.make_grid(70, 20, 9, seed=404, halo=halo)
    d = wl.direction(70, 20, 9, seed=504, halo=halo)
    errs, _ = tl_errors(gpu_tangent(g, d, halo=halo), g, d, halo=halo)
    assert max(errs) <= 1e-6, errs


def _dot(a, b):
    return float(sum(np.sum(np.asarray(x, np.float64) * np.asarray(y, np.float64)) for x, y in zip(a, b)))


def test_tangent_central_difference_fp64():
    """F is quadratic, so (F(x+d) - F(x-d)) / 2 = J(x) d exactly in exact
    arithmetic: GPU FP64 forward against GPU FP64 tangent, A-scaled."""
    g = wl.make_grid(90, 20, 12, seed=405, dtype=np.float64)
    d = wl.direction(90, 20, 12, seed=505)
    (u, v, w), c = dev_grid(g)
    dd = _dev(d)
    fp = B.advect(*(a + b for a, b in zip((u, v, w), dd)), c)
    fm = B.advect(*(a - b for a, b in zip((u, v, w), dd)), c)
    cd = [((p - m) / 2).cpu().numpy() for p, m in zip(fp, fm)]
    tl = gpu_tangent(g, d)
    mag = tl_magnitude(g, d)
    _, m_x = oracle.forward(*(np.abs(a) for a in (g.u, g.v, g.w)), g.coeffs, magnitude=True)
    _, m_d = oracle.forward(*(np.abs(a) for a in d), g.coeffs, magnitude=True)
    for a, b, m, mx, md in zip(cd, tl, mag, m_x, m_d):
        # the difference of the two forward results carries the rounding of A(x) + A(d)
        assert a_scaled_error(a, b, m + mx + md) <= 1e-14


def test_dot_product_with_adjoint(report):
    """<J dx, y> = <dx, J^T y> with both sides from the GPU kernels, in
    FP64 (1e-11) and in FP32 (1e-5) (256 x 256 x 128, the differentiation workload)."""
    g = wl.make_grid(64, 40, 24, seed=406, dtype=np.float64)
    d = wl.direction(64, 40, 24, seed=506)
    y = wl.cotangents(64, 40, 24, seed=606, dtype=np.float64)
    (u, v, w), c = dev_grid(g)
    jd = gpu_tangent(g, d)
    jty = [x.cpu().numpy() for x in B.advect_adjoint(u, v, w, c, *_dev(y))]
    lhs, rhs = _dot(jd, y), _dot(d, jty)
    assert abs(lhs - rhs) <= 1e-11 * abs(rhs)
    cfg = wl.C4
    g4 = wl.config_grid(cfg)
    y4 = wl.cotangents(cfg["nx"], cfg["ny"], cfg["nz"], cfg["cot_seed"])
    d4 = [x.astype(np.float32) for x in wl.direction(cfg["nx"], cfg["ny"], cfg["nz"], seed=45)]
    (u4, v4, w4), c4 = dev_grid(g4)
    jd4 = gpu_tangent(g4, d4)
    jty4 = [x.cpu().numpy() for x in B.advect_adjoint(u4, v4, w4, c4, *_dev(y4))]
    rel = abs(_dot(jd4, y4) - _dot(d4, jty4)) / abs(_dot(d4, jty4))
    report["tangent_adjoint_dot_f32_256x256x128"] = dict(rel=rel)
    assert rel <= 1e-5, rel


def test_c4_tangent_full_grid_parity(report):
    """The 256 x 256 x 128 FP32 tangent in the library's launch shape, every
    output against the oracle."""
    cfg = wl.C4
    g = wl.config_grid(cfg)
    d = wl.direction(cfg["nx"], cfg["ny"], cfg["nz"], seed=46)
    errs, _ = tl_errors(gpu_tangent(g, d), g, d)
    report["tangent_f32_256x256x128"] = dict(zip(("tu", "tv", "tw"), errs))
    assert max(errs) <= 1e-6, errs


def test_forward_mode_autograd():
    """torch forward-mode AD through PWAdvect (jvp = the tangent kernel)."""
    import torch.autograd.forward_ad as fwAD
    PW = B.PWAdvect()
    g = wl.make_grid(33, 9, 6, seed=407, dtype=np.float64)
    d = wl.direction(33, 9, 6, seed=507)
    (u, v, w), c = dev_grid(g)
    dd = _dev(d)
    with fwAD.dual_level():
        duals = [fwAD.make_dual(x, t) for x, t in zip((u, v, w), dd)]
        outs = PW.apply(*duals, c)
        tang = [fwAD.unpack_dual(o).tangent.cpu().numpy() for o in outs]
    ref = oracle.tangent(g.u, g.v, g.w, *d, g.coeffs)
    for a, b in zip(tang, ref):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    # only some inputs carry a tangent: the others count as zero
    with fwAD.dual_level():
        outs = PW.apply(fwAD.make_dual(u, dd[0]), v, w, c)
        tang = [fwAD.unpack_dual(o).tangent for o in outs]
    ref = oracle.tangent(g.u, g.v, g.w, d[0], np.zeros_like(d[1]), np.zeros_like(d[2]), g.coeffs)
    for a, b in zip(tang, ref):
        assert np.allclose(a.cpu().numpy(), b, rtol=1e-12, atol=1e-12)


def test_tangent_argument_errors():
    g = wl.make_grid(20, 8, 4, seed=408)
    (u, v, w), c = dev_grid(g)
    d = [torch.zeros_like(u) for _ in range(3)]
    with pytest.raises(B.PWError):
        B.advect_tangent(u.to(torch.bfloat16), v.to(torch.bfloat16), w.to(torch.bfloat16), c,
                         *(x.to(torch.bfloat16) for x in d))
    out = [torch.empty((4, 8, 20), device="cuda") for _ in range(3)]
    tu_bad = d[1].view(-1)[:4 * 8 * 20].view(4, 8, 20)   # an output inside a direction array
    with pytest.raises(B.PWError):
        B.advect_tangent(u, v, w, c, *d, out=(tu_bad, out[1], out[2]))
    with pytest.raises(B.PWError):
        B.advect_tangent(u, v, w, c, *d, tile=(4, 1, 8, 4))
