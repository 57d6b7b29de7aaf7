"""GPU tests of the hand-written adjoint kernel (J^T r, gather form) against
the FP64 oracle's scatter-form adjoint, plus the finite-difference and
dot-product checks of the differentiation form.

Tolerances: A-scaled (A = sum over the terms reading an entry of |partial| *
|cotangent|, scales.adjoint_scale, pinned on the CPU) 1e-6 in FP32 (at most
~12 roundings of 2^-24 = 6e-8 along any gradient sum, so about 7e-7) and
1e-13 in FP64; bit for bit on integer data with dyadic coefficients.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import a_scaled_error, adjoint_magnitude, dev_grid, poison_unread
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


def gpu_adjoint(g, r, tile=None, halo=1):
    (u, v, w), c = dev_grid(g)
    rd = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in r]
    # NaN-filled outputs: every padded entry must be written
    pre = tuple(torch.full_like(u, float("nan")) for _ in range(3))
    out = B.advect_adjoint(u, v, w, c, *rd, halo=halo, tile=tile, out=pre)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def adj_errors(got, g, r, halo=1):
    ref = oracle.adjoint(g.u, g.v, g.w, g.coeffs, *r, halo=halo)
    mag = adjoint_magnitude(g.u, g.v, g.w, g.coeffs, [np.asarray(x, np.float64) for x in r], halo=halo)
    return [a_scaled_error(x, y, m) for x, y, m in zip(got, ref, mag)], ref


SHAPES = [(130, 70, 20), (64, 64, 64), (1, 1, 1), (65, 3, 1), (1, 200, 5), (61, 9, 17), (60, 7, 3),
          (128, 4, 3), (129, 5, 2), (257, 3, 4)]


@pytest.mark.parametrize("tile", [None, (1, 1, 5, 4), (1, 2, 9, 1), (1, 4, 64, 8), (1, 2, 7, 4, 2), (1, 4, 3, 1, 2)])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_f32_adjoint_matches_oracle(shape, tile):
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=200 + nx + ny + nz)
    r = wl.cotangents(nx, ny, nz, seed=300 + nx)
    errs, ref = adj_errors(gpu_adjoint(g, r, tile=tile), g, r)
    assert max(errs) <= 1e-6, errs


@pytest.mark.parametrize("tile", [None, (1, 2, 4, 4, 2)])
def test_f64_adjoint_matches_oracle(tile):
    g = wl.make_grid(70, 33, 21, seed=201, dtype=np.float64)
    r = wl.cotangents(70, 33, 21, seed=301, dtype=np.float64)
    errs, _ = adj_errors(gpu_adjoint(g, r, tile=tile), g, r)
    assert max(errs) <= 1e-13, errs


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_integer_adjoint_bitwise(dtype):
    g = wl.integer_grid(130, 11, 7, seed=202, dtype=dtype)
    rng = np.random.default_rng(302)
    r = [rng.integers(-3, 4, (7, 11, 130)).astype(dtype) for _ in range(3)]
    got = gpu_adjoint(g, r)
    ref = oracle.adjoint(g.u, g.v, g.w, g.coeffs, *r)
    for a, b in zip(got, ref):
        assert np.array_equal(a.astype(np.float64), b)


def test_adjoint_tile_invariance_bitwise():
    g = wl.make_grid(150, 37, 23, seed=203)
    r = wl.cotangents(150, 37, 23, seed=303)
    base = gpu_adjoint(g, r, tile=(1, 2, 16, 4))
    for t in [(1, 1, 1, 1), (1, 1, 9, 4), (1, 2, 5, 8), (1, 4, 64, 4), (1, 4, 3, 2), (1, 1, 7, 8), (1, 2, 130, 1),
              (1, 1, 1, 1, 2), (1, 2, 6, 4, 2), (1, 4, 130, 8, 2)]:
        got = gpu_adjoint(g, r, tile=t)
        for a, b in zip(base, got):
            assert np.array_equal(a, b), t


@pytest.mark.parametrize("tile", [None, (1, 1, 4, 4), (1, 4, 5, 1, 2)])
@pytest.mark.parametrize("halo", [2, 3])
def test_adjoint_wider_halo(halo, tile):
    """x-halo columns beyond the first get no contribution and are written as
    zeros (the gradient buffers start as garbage)."""
    g = wl.make_grid(70, 20, 9, seed=204, halo=halo)
    r = wl.cotangents(70, 20, 9, seed=304)
    errs, ref = adj_errors(gpu_adjoint(g, r, halo=halo, tile=tile), g, r, halo=halo)
    assert max(errs) <= 1e-6, errs


def test_adjoint_strided_layout_bitwise():
    """Inputs, cotangents and gradients as views into larger buffers (extra
    columns and rows per plane): the same result bit for bit as dense arrays,
    and nothing outside the views is written."""
    nx, ny, nz = 70, 13, 9
    g = wl.make_grid(nx, ny, nz, seed=206)
    r = wl.cotangents(nx, ny, nz, seed=306)
    dense = gpu_adjoint(g, r)
    (u0, v0, w0), c = dev_grid(g)
    pz, py, px = u0.shape

    def view(src, extra_rows, extra_cols, fill):
        big = torch.full((src.shape[0], src.shape[1] + extra_rows, src.shape[2] + extra_cols), fill,
                         dtype=src.dtype, device=src.device)
        big[:, :src.shape[1], :src.shape[2]] = src
        return big, big[:, :src.shape[1], :src.shape[2]]

    ins = [view(x, 2, 5, 7.0) for x in (u0, v0, w0)]
    cots = [view(torch.from_numpy(np.ascontiguousarray(x)).to("cuda"), 1, 3, 9.0) for x in r]
    outs = [view(torch.empty_like(u0), 2, 5, float("nan")) for _ in range(3)]
    bigs = [b for b, _ in outs]
    for b, vw in outs:
        b.fill_(-3.0)
        vw.fill_(float("nan"))
    assert ins[0][1].stride() == (py * (px + 5) + 2 * (px + 5), px + 5, 1)
    got = B.advect_adjoint(*(vw for _, vw in ins), c, *(vw for _, vw in cots), out=tuple(vw for _, vw in outs))
    torch.cuda.synchronize()
    for a, b in zip(dense, got):
        assert np.array_equal(a, b.cpu().numpy())
    for b in bigs:
        outside = b.clone()
        outside[:, :py, :px] = -3.0
        assert bool((outside == -3.0).all())


def _dot(a, b):
    return float(sum(np.sum(np.asarray(x, np.float64) * np.asarray(y, np.float64)) for x, y in zip(a, b)))


def test_fd_check_fp64_16cubed(report):
    """FP64 central finite differences of the forward operator (eps = 1e-6,
    16^3, seed 40) against the GPU FP64 adjoint through the inner-product
    identity; F is quadratic, so only roundoff separates them."""
    cfg = wl.C4_FD
    n = (cfg["nx"], cfg["ny"], cfg["nz"])
    g = wl.make_grid(*n, cfg["seed"], dtype=np.float64)
    d = wl.direction(*n, cfg["seed"] + 1)
    y = wl.cotangents(*n, cfg["seed"] + 2, dtype=np.float64)
    eps = cfg["eps"]
    (u, v, w), c = dev_grid(g)
    dd = [torch.from_numpy(x).cuda() for x in d]
    fp = B.advect(*(a + eps * b for a, b in zip((u, v, w), dd)), c)
    fm = B.advect(*(a - eps * b for a, b in zip((u, v, w), dd)), c)
    jd = [((p - m) / (2 * eps)).cpu().numpy() for p, m in zip(fp, fm)]
    yd = [torch.from_numpy(x).cuda() for x in y]
    jty = [x.cpu().numpy() for x in B.advect_adjoint(u, v, w, c, *yd)]
    lhs, rhs = _dot(jd, y), _dot(d, jty)
    rel = abs(lhs - rhs) / abs(rhs)
    report["adjoint_fd_fp64_16cubed"] = dict(rel=rel, eps=eps)
    assert rel <= 1e-8, rel


@pytest.fixture(scope="module")
def grid_c4():
    cfg = wl.C4
    g = wl.config_grid(cfg)
    r = wl.cotangents(cfg["nx"], cfg["ny"], cfg["nz"], cfg["cot_seed"])
    return g, r


def test_c4_adjoint_full_grid_parity(grid_c4, report):
    """The 256 x 256 x 128 FP32 adjoint in the benchmark's launch shape,
    every gradient entry against the oracle."""
    g, r = grid_c4
    errs, _ = adj_errors(gpu_adjoint(g, r), g, r)
    report["adjoint_f32_256x256x128"] = dict(zip(("gu", "gv", "gw"), errs))
    assert max(errs) <= 1e-6, errs


def test_c4_dot_product_fp32(grid_c4, report):
    """<J dx, y> = <dx, J^T y> to 1e-5 relative: J dx from the FP64 tangent
    oracle and, GPU-only, by polarisation F(x+dx) - F(x) - F(dx); J^T y from
    the FP32 adjoint kernel."""
    g, y = grid_c4
    cfg = wl.C4
    d = wl.direction(cfg["nx"], cfg["ny"], cfg["nz"], seed=45)
    (u, v, w), c = dev_grid(g)
    yd = [torch.from_numpy(x).cuda() for x in y]
    jty = [x.cpu().numpy() for x in B.advect_adjoint(u, v, w, c, *yd)]
    rhs = _dot(d, jty)
    jd = oracle.tangent(g.u, g.v, g.w, *d, g.coeffs)
    rel_oracle = abs(_dot(jd, y) - rhs) / abs(rhs)
    dd = [torch.from_numpy(x.astype(np.float32)).cuda() for x in d]
    fxd = B.advect(*(a + b for a, b in zip((u, v, w), dd)), c)
    fx = B.advect(u, v, w, c)
    fd_ = B.advect(*dd, c)
    pol = [(a.double() - b.double() - e.double()).cpu().numpy() for a, b, e in zip(fxd, fx, fd_)]
    rel_pol = abs(_dot(pol, y) - rhs) / abs(rhs)
    report["dot_product_f32_256x256x128"] = dict(vs_tangent_oracle=rel_oracle, vs_polarisation=rel_pol)
    assert rel_oracle <= 1e-5, rel_oracle
    assert rel_pol <= 1e-5, rel_pol


def test_euler_identity_fp64():
    """<x, J^T(x) y> = 2 <F(x), y> on the GPU (FP64 kernels)."""
    g = wl.make_grid(90, 20, 12, seed=205, dtype=np.float64)
    y = wl.cotangents(90, 20, 12, seed=305, dtype=np.float64)
    (u, v, w), c = dev_grid(g)
    yd = [torch.from_numpy(x).cuda() for x in y]
    jty = [x.cpu().numpy() for x in B.advect_adjoint(u, v, w, c, *yd)]
    fx = [x.cpu().numpy() for x in B.advect(u, v, w, c)]
    lhs = _dot((g.u, g.v, g.w), jty)
    assert abs(lhs - 2 * _dot(fx, y)) <= 1e-12 * abs(lhs)


def test_autograd_function_and_gradcheck():
    PW = B.PWAdvect()
    g = wl.make_grid(9, 7, 5, seed=206, dtype=np.float64)
    (u, v, w), c = dev_grid(g)
    xs = [x.clone().requires_grad_(True) for x in (u, v, w)]
    su, sv, sw = PW.apply(*xs, c)
    y = wl.cotangents(9, 7, 5, seed=306, dtype=np.float64)
    loss = sum((o * torch.from_numpy(t).cuda()).sum() for o, t in zip((su, sv, sw), y))
    loss.backward()
    ref = oracle.adjoint(g.u, g.v, g.w, g.coeffs, *y)
    for x, r in zip(xs, ref):
        assert np.allclose(x.grad.cpu().numpy(), r, rtol=1e-12, atol=1e-12)
    small = wl.make_grid(4, 3, 3, seed=207, dtype=np.float64)
    (a, b, e), c2 = dev_grid(small)
    inp = tuple(x.clone().requires_grad_(True) for x in (a, b, e))
    assert torch.autograd.gradcheck(lambda p, q, s: PW.apply(p, q, s, c2), inp, fast_mode=True)


@pytest.mark.parametrize("tile", [None, (1, 1, 5, 4), (1, 4, 3, 1, 2)])
@pytest.mark.parametrize("shape,halo", [((70, 13, 9), 1), ((130, 5, 3), 1), ((61, 9, 17), 2), ((3, 2, 2), 1)],
                         ids=lambda x: "x".join(map(str, x)) if isinstance(x, tuple) else "h%d" % x)
def test_unread_cells_do_not_reach_the_gradient(shape, halo, tile):
    """NaN and +-Inf in every padded cell that no output reads (halo corners
    and edges, the outer halo layers) change nothing: the gradient is finite,
    matches the oracle, and is exactly zero in those cells."""
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=207 + nx, halo=halo)
    r = wl.cotangents(nx, ny, nz, seed=307 + nx)
    unread = poison_unread(g)
    got = gpu_adjoint(g, r, tile=tile, halo=halo)
    for a, m in zip(got, unread):
        assert np.all(np.isfinite(a))
        assert np.all(a[m] == 0)
    errs, ref = adj_errors(got, g, r, halo=halo)
    assert all(np.all(np.isfinite(x)) for x in ref)
    assert max(errs) <= 1e-6, errs
