"""GPU tests of the halo fill against the oracle's per-axis definition.

The fill only moves and negates values, so the bar is exact: every cell of
the GPU result equals the oracle's, sign of zero included, for every
storage type, mode combination and halo width, with strided layouts, and the
interior and any cells outside the padded views stay untouched bit for bit.
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
from oracle import halo as H
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


TDT = {"float32": torch.float32, "float64": torch.float64, "bfloat16": torch.bfloat16, "float16": torch.float16}


def _fields(shape, n, seed, tdt):
    rng = np.random.default_rng(seed)
    return [torch.from_numpy(rng.uniform(-2, 2, shape)).to(tdt).to("cuda") for _ in range(n)]


def _host64(t):
    return t.cpu().to(torch.float64).numpy()


def _check(fields, modes, halo):
    before = [_host64(f) for f in fields]
    if len(modes) == 3 and isinstance(modes[0], str):
        modes = [modes] * len(fields)
    B.halo_fill(fields, modes, halo=halo)
    torch.cuda.synchronize()
    for f, b, m in zip(fields, before, modes):
        ref = H.fill(b, halo, m)
        got = _host64(f)
        assert np.array_equal(got, ref), (m, np.argwhere(got != ref)[:5])
        # signed zeros too: a zeroed cell that a later axis negates is -0
        assert np.array_equal(np.signbit(got), np.signbit(ref)), (m, np.argwhere(np.signbit(got) != np.signbit(ref))[:5])


MODES = [m for m in H.MODES]


@pytest.mark.parametrize("dt", list(TDT))
def test_every_mode_combination(dt):
    """All 6^3 (x, y, z) combinations on a ragged grid, three fields per call
    with different rules each."""
    fields = _fields((5 + 2, 4 + 2, 7 + 2), 3, 700, TDT[dt])
    combos = list(itertools.product(MODES, MODES, MODES))
    for i in range(0, len(combos), 3):
        _check(fields, combos[i:i + 3], 1)


@pytest.mark.parametrize("halo", [2, 3])
def test_wide_halo(halo):
    combos = list(itertools.product(MODES, MODES, MODES))
    fields = _fields((4 + 2 * halo, 3 + 2 * halo, 5 + 2 * halo), 8, 701, torch.float32)
    for i in range(0, len(combos), 8):
        _check(fields[:len(combos[i:i + 8])], combos[i:i + 8], halo)


def test_periodic_wraps_more_than_once():
    """Halo wider than the interior (n = 1, 2 with h = 3)."""
    fields = _fields((1 + 6, 2 + 6, 1 + 6), 2, 702, torch.float64)
    _check(fields, [("periodic", "periodic", "periodic"), ("copy", "periodic", "zero")], 3)


def test_strided_layout_leaves_outside_cells_alone():
    """Padded views inside larger allocations (row and plane padding): cells
    outside the views are never written."""
    halo = 1
    nz, ny, nx = 6, 5, 67
    big = _fields((nz + 2 + 1, ny + 2 + 3, nx + 2 + 13), 3, 703, torch.float32)
    keep = [b.clone() for b in big]
    views = [b[:nz + 2, :ny + 2, :nx + 2] for b in big]
    _check(views, [("periodic", "copy", "zero"), ("periodic", "periodic", "copy"), ("reflect", "zero", "reflect_neg")],
           halo)
    for b, k in zip(big, keep):
        assert torch.equal(b[nz + 2:], k[nz + 2:]) and torch.equal(b[:, ny + 2:], k[:, ny + 2:])
        assert torch.equal(b[:, :, nx + 2:], k[:, :, nx + 2:])


def test_interior_untouched_bitwise():
    fields = _fields((9 + 2, 7 + 2, 130 + 2), 3, 704, torch.float32)
    inner = [f[1:-1, 1:-1, 1:-1].clone() for f in fields]
    B.halo_fill(fields, ("periodic", "periodic", "reflect_neg"))
    torch.cuda.synchronize()
    for f, i in zip(fields, inner):
        assert torch.equal(f[1:-1, 1:-1, 1:-1].view(torch.int32), i.view(torch.int32))


def test_512x512x64_lid_conditions(report):
    """The 512 x 512 x 64 FP32 winds with periodic x, y and a free-slip lid
    (u, v zero-gradient, w zero), every cell against the oracle; then the
    fill's time."""
    cfg = wl.C1
    g = wl.config_grid(cfg)
    fields = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in (g.u, g.v, g.w)]
    modes = [("periodic", "periodic", "copy"), ("periodic", "periodic", "copy"), ("periodic", "periodic", "zero")]
    _check(fields, modes, 1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(20):
        B.halo_fill(fields, modes)
    ev[0].record()
    for _ in range(200):
        B.halo_fill(fields, modes)
    ev[1].record()
    torch.cuda.synchronize()
    report["halo_fill_f32_512x512x64_us"] = ev[0].elapsed_time(ev[1]) / 200 * 1e3


def test_periodic_fill_then_forward_conserves_energy():
    """End to end: GPU periodic fill, then the GPU forward in FP64 on integer
    winds with the cyclic dyadic coefficients: sum(u su + v sv + w sw) over
    the interior is exactly zero."""
    rng = np.random.default_rng(705)
    nz, ny, nx = 8, 12, 70
    pads = []
    for _ in range(3):
        a = rng.uniform(-9, 9, (nz + 2, ny + 2, nx + 2))
        a[1:-1, 1:-1, 1:-1] = rng.integers(-4, 5, (nz, ny, nx))
        pads.append(torch.from_numpy(a).to("cuda"))
    B.halo_fill(pads, ("periodic", "periodic", "periodic"))
    tzc2 = rng.choice([0.5, 0.25, 0.125], nz)
    tzd2 = rng.choice([0.5, 0.25, 0.125], nz)
    c = dict(tcx=0.25, tcy=0.125, tzc1=np.roll(tzc2, 1), tzc2=tzc2, tzd1=np.roll(tzd2, 1), tzd2=tzd2)
    out = B.advect(*pads, B.Coeffs.from_host(c, dtype=torch.float64))
    torch.cuda.synchronize()
    e = sum(float(torch.sum(p[1:-1, 1:-1, 1:-1] * s)) for p, s in zip(pads, out))
    assert e == 0.0
    ref = oracle.forward(*[_host64(p) for p in pads], c)
    for a, b in zip(out, ref):
        assert np.array_equal(a.cpu().numpy(), b)


def test_halo_fill_argument_errors():
    f = _fields((6, 6, 6), 2, 706, torch.float32)
    with pytest.raises(ValueError):
        B.halo_fill(f, ("periodic", "sideways", "copy"))
    with pytest.raises(B.PWError):
        B.halo_fill([f[0], f[0]], ("periodic",) * 3)          # the same array twice
    g = _fields((2 + 6, 7 + 6, 7 + 6), 1, 707, torch.float32)
    with pytest.raises(B.PWError):
        B.halo_fill(g, ("keep", "keep", "reflect"), halo=3)   # nz = 2 < h = 3


def test_zfast_arrays_with_axes_exchanged():
    """A z-fastest array ([i, j, k], k contiguous) is filled by the same call
    with the x and z rules exchanged: the result is the x-fastest fill,
    transposed, bit for bit."""
    rng = np.random.default_rng(708)
    a = torch.from_numpy(rng.uniform(-2, 2, (9 + 2, 5 + 2, 70 + 2))).to(torch.float32).cuda()   # (k, j, i)
    z = a.permute(2, 1, 0).contiguous()                                                         # (i, j, k)
    B.halo_fill([a], ("periodic", "copy", "reflect_neg"))
    B.halo_fill([z], ("reflect_neg", "copy", "periodic"))
    torch.cuda.synchronize()
    assert torch.equal(z.permute(2, 1, 0), a)


# ------------------------------------------------------------------ fold

@pytest.mark.parametrize("dt", ["float32", "float64"])
@pytest.mark.parametrize("halo", [1, 2])
def test_fold_every_rule_combination_integer_bitwise(dt, halo):
    """Integer gradients (every sum exact): the GPU fold equals the oracle's
    bit for bit for all 6^3 rule combinations, three fields per call."""
    rng = np.random.default_rng(720 + halo)
    shape = (5 + 2 * halo, 4 + 2 * halo, 9 + 2 * halo)
    combos = list(itertools.product(MODES, MODES, MODES))
    for i in range(0, len(combos), 3):
        cs = combos[i:i + 3]
        host = [rng.integers(-9, 10, shape).astype(np.float64) for _ in cs]
        dev = [torch.from_numpy(x).to(TDT[dt]).cuda() for x in host]
        B.halo_fold(dev, cs, halo=halo)
        torch.cuda.synchronize()
        for d, x, m in zip(dev, host, cs):
            assert np.array_equal(d.cpu().to(torch.float64).numpy(), H.fold(x, halo, m)), m


def test_fold_random_and_dot_product_fp64():
    rng = np.random.default_rng(722)
    shape = (9 + 2, 7 + 2, 130 + 2)
    for modes in [("periodic", "periodic", "copy"), ("reflect_neg", "copy", "reflect"), ("copy", "zero", "periodic")]:
        x = rng.uniform(-1, 1, shape)
        y = rng.uniform(-1, 1, shape)
        fx = torch.from_numpy(x).cuda()
        fy = torch.from_numpy(y).cuda()
        B.halo_fill([fx], modes)
        B.halo_fold([fy], modes)
        torch.cuda.synchronize()
        assert np.allclose(fy.cpu().numpy(), H.fold(y, 1, modes), rtol=0, atol=1e-15)
        lhs = float(torch.sum(fx * torch.from_numpy(y).cuda()))
        rhs = float(torch.sum(torch.from_numpy(x).cuda() * fy))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs), modes


def test_fold_strided_layout_leaves_outside_cells_alone():
    nz, ny, nx = 6, 5, 67
    rng = np.random.default_rng(723)
    big = [torch.from_numpy(rng.integers(-5, 6, (nz + 3, ny + 5, nx + 15)).astype(np.float32)).cuda()
           for _ in range(2)]
    keep = [b.clone() for b in big]
    views = [b[:nz + 2, :ny + 2, :nx + 2] for b in big]
    modes = [("periodic", "copy", "zero"), ("reflect", "periodic", "reflect_neg")]
    ref = [H.fold(v.cpu().numpy().astype(np.float64), 1, m) for v, m in zip(views, modes)]
    B.halo_fold(views, modes)
    torch.cuda.synchronize()
    for v, r, b, k in zip(views, ref, big, keep):
        assert np.array_equal(v.cpu().numpy().astype(np.float64), r)
        assert torch.equal(b[nz + 2:], k[nz + 2:]) and torch.equal(b[:, ny + 2:], k[:, ny + 2:])
        assert torch.equal(b[:, :, nx + 2:], k[:, :, nx + 2:])


def test_adjoint_of_the_forward_with_boundaries():
    """<J_bc d, r> = <d, J_bc^T r> in FP64 with J_bc = tangent at fill(x) on
    fill(d), and J_bc^T r (adjoint kernel + fold) against the oracle's
    fold(adjoint(fill(x), r))."""
    g = wl.make_grid(70, 12, 9, seed=724, dtype=np.float64)
    r = wl.cotangents(70, 12, 9, seed=725, dtype=np.float64)
    d = wl.direction(70, 12, 9, seed=726)
    from gpu_util import dev_grid
    (u, v, w), c = dev_grid(g)
    rd = [torch.from_numpy(x).cuda() for x in r]
    dd = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in d]
    for bc in [("periodic", "periodic", "copy"), ("copy", "periodic", "periodic")]:
        grads = B.advect_bc_adjoint(u, v, w, c, bc, *rd)
        xf = [x.clone() for x in (u, v, w)]
        df = [x.clone() for x in dd]
        B.halo_fill(xf, bc)
        B.halo_fill(df, bc)
        tl = B.advect_tangent(*xf, c, *df)
        torch.cuda.synchronize()
        lhs = sum(float(torch.sum(a * b)) for a, b in zip(tl, rd))
        rhs = sum(float(torch.sum(a * b)) for a, b in zip(dd, grads))
        assert abs(lhs - rhs) <= 1e-11 * abs(rhs), bc
        filled = [H.fill(x, 1, bc) for x in (g.u, g.v, g.w)]
        ref = [H.fold(x, 1, bc) for x in oracle.adjoint(*filled, g.coeffs, *r)]
        for a, b in zip(grads, ref):
            assert np.allclose(a.cpu().numpy(), b, rtol=0, atol=1e-12 * np.max(np.abs(b)))
