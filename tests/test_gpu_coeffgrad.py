"""GPU tests of the coefficient-gradient kernel (dL/d(tcx, tcy, tz*) for
L = <F(x), r>) against the FP64 oracle, plus reproducibility and autograd.

Tolerance: the error of each gradient entry is scaled by the sum, over the
terms it collects, of |cotangent| * |coefficient-free product| (the oracle's
forward magnitude with that coefficient set to one); 1e-6 in FP32 (each
product is formed in FP32 with a few roundings and summed in FP64), 1e-13 in
FP64.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import dev_grid
from scales import coeff_grad_scale
from paper_2301_13016_amd import binding as B
from paper_2301_13016_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

NAMES = ("tzc1", "tzc2", "tzd1", "tzd2")


@pytest.fixture(autouse=True)
def _announce(request):
    sys.__stderr__.write("\n[gpu-test] %s\n" % request.node.nodeid)
    sys.__stderr__.flush()
    yield


def _dev(arrs, dtype=None):
    out = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in arrs]
    return [o.to(dtype) for o in out] if dtype is not None else out


def magnitudes(g, r):
    """Per gradient entry: sum over its terms of |r| * |product|."""
    return coeff_grad_scale(g.u, g.v, g.w, r, g.nz, halo=g.halo)


def check(g, r, tol, halo=1):
    (u, v, w), _ = dev_grid(g)
    rd = _dev(r, u.dtype)
    got = B.advect_coeff_grad(u, v, w, *rd, halo=halo)
    torch.cuda.synchronize()
    rq = [np.asarray(x, g.u.dtype).astype(np.float64) for x in r]   # cotangents as the kernel saw them
    ref = oracle.coeff_grad(g.u, g.v, g.w, *rq, halo=halo)
    mag = magnitudes(g, rq)
    worst = 0.0
    for name in ("tcx", "tcy") + NAMES:
        e = np.abs(got[name].cpu().numpy() - ref[name]) / np.maximum(mag[name], 1e-300)
        worst = max(worst, float(np.max(e)))
    lev = got["tcx_level"].cpu().numpy()
    assert np.max(np.abs(lev - ref["tcx_level"])) <= tol * mag["tcx"]
    assert worst <= tol, worst
    return got, worst


@pytest.mark.parametrize("shape", [(130, 70, 20), (1, 1, 1), (65, 3, 1), (129, 5, 2), (257, 3, 4), (61, 9, 17)],
                         ids=lambda s: "x".join(map(str, s)))
def test_f32_coeff_grad_matches_oracle(shape):
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=700 + nx)
    r = wl.cotangents(nx, ny, nz, seed=800 + nx)
    check(g, r, 1e-6)


def test_f64_coeff_grad_matches_oracle():
    g = wl.make_grid(70, 33, 21, seed=701, dtype=np.float64)
    r = wl.cotangents(70, 33, 21, seed=801, dtype=np.float64)
    check(g, r, 1e-13)


@pytest.mark.parametrize("halo", [2, 3])
def test_coeff_grad_wider_halo(halo):
    g = wl.make_grid(70, 20, 9, seed=702, halo=halo)
    r = wl.cotangents(70, 20, 9, seed=802)
    check(g, r, 1e-6, halo=halo)


def test_coeff_grad_reproducible_bitwise():
    g = wl.make_grid(150, 37, 23, seed=703)
    r = wl.cotangents(150, 37, 23, seed=803)
    (u, v, w), _ = dev_grid(g)
    rd = _dev(r)
    a = B.advect_coeff_grad(u, v, w, *rd)
    b = B.advect_coeff_grad(u, v, w, *rd)
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_coeff_grad_strided_layout_bitwise():
    """Values and cotangents as views into larger buffers (extra columns and
    rows per plane): the same gradients bit for bit as dense arrays."""
    g = wl.make_grid(150, 37, 23, seed=704)
    r = wl.cotangents(150, 37, 23, seed=804)
    (u, v, w), _ = dev_grid(g)
    rd = _dev(r)
    dense = B.advect_coeff_grad(u, v, w, *rd)

    def view(src, extra_rows, extra_cols):
        big = torch.full((src.shape[0], src.shape[1] + extra_rows, src.shape[2] + extra_cols), 5.0,
                         dtype=src.dtype, device=src.device)
        big[:, :src.shape[1], :src.shape[2]] = src
        return big[:, :src.shape[1], :src.shape[2]]

    vs = [view(x, 3, 7) for x in (u, v, w)]
    cs = [view(x, 1, 2) for x in rd]
    assert vs[0].stride(1) == u.shape[2] + 7 and cs[0].stride(1) == rd[0].shape[2] + 2
    got = B.advect_coeff_grad(*vs, *cs)
    for k in dense:
        assert torch.equal(dense[k], got[k]), k


def test_c4_coeff_grad_parity(report):
    """256 x 256 x 128 FP32, every coefficient gradient against the oracle."""
    cfg = wl.C4
    g = wl.config_grid(cfg)
    r = wl.cotangents(cfg["nx"], cfg["ny"], cfg["nz"], cfg["cot_seed"])
    _, worst = check(g, r, 1e-6)
    report["coeff_grad_f32_256x256x128"] = dict(worst_scaled=worst)


def test_euler_identity_on_gpu():
    """sum of c * dL/dc over all coefficients = L (L is linear in them)."""
    g = wl.make_grid(90, 20, 12, seed=704, dtype=np.float64)
    r = wl.cotangents(90, 20, 12, seed=804, dtype=np.float64)
    (u, v, w), c = dev_grid(g)
    rd = _dev(r)
    got = B.advect_coeff_grad(u, v, w, *rd)
    f = B.advect(u, v, w, c)
    loss = float(sum((a * b).sum() for a, b in zip(f, rd)))
    total = g.tcx * float(got["tcx"]) + g.tcy * float(got["tcy"]) + \
        sum(float((getattr(c, n) * got[n]).sum()) for n in NAMES)
    assert abs(total - loss) <= 1e-12 * abs(loss)


def test_autograd_with_coefficients_gradcheck():
    PW = B.PWAdvectCoeffs()
    g = wl.make_grid(5, 4, 3, seed=705, dtype=np.float64)
    (u, v, w), c = dev_grid(g)
    dd = torch.float64
    args = [x.clone().requires_grad_(True) for x in (u, v, w)]
    args += [torch.tensor(g.tcx, dtype=dd, requires_grad=True), torch.tensor(g.tcy, dtype=dd, requires_grad=True)]
    args += [getattr(c, n).clone().requires_grad_(True) for n in NAMES]
    assert torch.autograd.gradcheck(lambda *a: PW.apply(*a), tuple(args), fast_mode=True)
    # winds only: the coefficient kernel is skipped, results as PWAdvect
    y = wl.cotangents(5, 4, 3, seed=805, dtype=np.float64)
    xs = [x.clone().requires_grad_(True) for x in (u, v, w)]
    outs = PW.apply(*xs, torch.tensor(g.tcx, dtype=dd), torch.tensor(g.tcy, dtype=dd), c.tzc1, c.tzc2, c.tzd1, c.tzd2)
    sum((o * t).sum() for o, t in zip(outs, _dev(y))).backward()
    ref = oracle.adjoint(g.u, g.v, g.w, g.coeffs, *y)
    for x, rr in zip(xs, ref):
        assert np.allclose(x.grad.cpu().numpy(), rr, rtol=1e-12, atol=1e-12)


def test_coeff_grad_argument_errors():
    g = wl.make_grid(20, 8, 4, seed=706)
    (u, v, w), _ = dev_grid(g)
    r = [torch.zeros((4, 8, 20), device="cuda") for _ in range(3)]
    with pytest.raises(B.PWError):
        B.advect_coeff_grad(*(x.to(torch.bfloat16) for x in (u, v, w)), *(x.to(torch.bfloat16) for x in r))


# ------------------------------------------------- fused backward (one pass)

def _same_bits(a, b):
    it = {torch.float32: torch.int32, torch.float64: torch.int64}[a.dtype]
    return a.dtype == b.dtype and a.shape == b.shape and torch.equal(a.view(it), b.view(it))


@pytest.mark.parametrize("case", [(130, 70, 20, np.float32, 1), (1, 1, 1, np.float32, 1), (129, 5, 2, np.float32, 1),
                                  (61, 9, 17, np.float64, 1), (70, 9, 6, np.float32, 2), (257, 3, 4, np.float64, 1)],
                         ids=lambda c: "%dx%dx%d_%s_h%d" % (c[0], c[1], c[2], np.dtype(c[3]).name, c[4]))
def test_fused_backward_equals_separate_calls(case):
    """pw_advect_adjoint_coeff_grad: wind gradients bit for bit those of
    advect_adjoint, coefficient gradients bit for bit those of
    advect_coeff_grad, both within the oracle bounds."""
    nx, ny, nz, dt, halo = case
    g = wl.make_grid(nx, ny, nz, seed=980 + nx, dtype=dt, halo=halo)
    r = wl.cotangents(nx, ny, nz, seed=981 + nx, dtype=dt)
    (u, v, w), c = dev_grid(g)
    rd = _dev(r, u.dtype)
    (gu, gv, gw), cg = B.advect_adjoint_coeff_grad(u, v, w, c, *rd, halo=halo)
    ref_w = B.advect_adjoint(u, v, w, c, *rd, halo=halo)
    ref_c = B.advect_coeff_grad(u, v, w, *rd, halo=halo)
    torch.cuda.synchronize()
    for a, b in zip((gu, gv, gw), ref_w):
        assert _same_bits(a, b)
    for n in ("tcx", "tcy", "tcx_level", "tcy_level") + NAMES:
        assert _same_bits(cg[n], ref_c[n]), n
    # oracle: coefficients (as in check) and winds
    rq = [np.asarray(x, dt).astype(np.float64) for x in r]
    refc = oracle.coeff_grad(g.u, g.v, g.w, *rq, halo=halo)
    mag = magnitudes(g, rq)
    tol = 1e-6 if dt == np.float32 else 1e-13
    for n in ("tcx", "tcy") + NAMES:
        assert np.all(np.abs(cg[n].cpu().numpy() - refc[n]) <= tol * mag[n]), n
    from gpu_util import adjoint_scale
    refw = oracle.adjoint(g.u, g.v, g.w, g.coeffs, *rq, halo=halo)
    scale = adjoint_scale(g.u, g.v, g.w, g.coeffs, rq, halo=halo)
    for a, b, s in zip((gu, gv, gw), refw, scale):
        assert np.all(np.abs(a.cpu().numpy() - b) <= tol * s)


def test_fused_backward_tile_independent_winds_and_reproducible():
    """Every adjoint launch shape gives the same wind gradients in the fused
    pass as alone; two fused calls agree bit for bit."""
    g = wl.make_grid(150, 21, 13, seed=990)
    r = wl.cotangents(150, 21, 13, seed=991)
    (u, v, w), c = dev_grid(g)
    rd = _dev(r, u.dtype)
    (a1, b1, c1), cg1 = B.advect_adjoint_coeff_grad(u, v, w, c, *rd)
    (a2, b2, c2), cg2 = B.advect_adjoint_coeff_grad(u, v, w, c, *rd)
    torch.cuda.synchronize()
    for x, y in zip((a1, b1, c1), (a2, b2, c2)):
        assert _same_bits(x, y)
    for n in cg1:
        assert _same_bits(cg1[n], cg2[n])
    for tile in [(1, 1, 5, 1, 1), (1, 2, 9, 4, 2), (1, 4, 64, 8, 1)]:
        alone = B.advect_adjoint(u, v, w, c, *rd, tile=tile)
        torch.cuda.synchronize()
        for x, y in zip((a1, b1, c1), alone):
            assert _same_bits(x, y), tile


def test_fused_backward_nan_in_unread_cells():
    """Non-finite values in cells no output reads reach neither the wind nor
    the coefficient gradients of the fused pass."""
    from gpu_util import poison_unread
    g = wl.make_grid(70, 11, 6, seed=992)
    r = wl.cotangents(70, 11, 6, seed=993)
    (u, v, w), c = dev_grid(g)
    clean = B.advect_adjoint_coeff_grad(u, v, w, c, *_dev(r, u.dtype))
    poison_unread(g)
    (u, v, w), c = dev_grid(g)
    dirty = B.advect_adjoint_coeff_grad(u, v, w, c, *_dev(r, u.dtype))
    torch.cuda.synchronize()
    for x, y in zip(clean[0], dirty[0]):
        assert torch.equal(x, y)
    for n in clean[1]:
        assert torch.equal(clean[1][n], dirty[1][n])


def test_c4_fused_backward_time(report):
    """256 x 256 x 128 FP32: the fused backward against the adjoint alone and
    the two separate calls (timed, reported)."""
    cfg = wl.C4
    g = wl.config_grid(cfg)
    r = wl.cotangents(cfg["nx"], cfg["ny"], cfg["nz"], cfg["cot_seed"])
    (u, v, w), c = dev_grid(g)
    rd = _dev(r, u.dtype)
    outs = tuple(torch.empty_like(u) for _ in range(3))
    gout = torch.empty(6 * g.nz + 2, dtype=torch.float64, device="cuda")

    def timed(fn, n=50):
        for _ in range(5):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    t_fused = timed(lambda: B.advect_adjoint_coeff_grad(u, v, w, c, *rd, out=outs, grad_out=gout))
    t_adj = timed(lambda: B.advect_adjoint(u, v, w, c, *rd, out=outs))
    t_cg = timed(lambda: B.advect_coeff_grad(u, v, w, *rd, out=gout))
    report["fused_backward_f32_256x256x128_ms"] = dict(fused=round(t_fused, 4), adjoint=round(t_adj, 4),
                                                       coeff_grad=round(t_cg, 4),
                                                       fused_over_adjoint=round(t_fused / t_adj, 3))
