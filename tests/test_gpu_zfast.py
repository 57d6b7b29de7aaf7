"""GPU tests of the z-fastest (column-major) forward kernel.

Two independent bars: the FP64 oracle, A-scaled as for the x-fastest
kernel (FP32 1e-6, FP64 1e-13, 16-bit storage the same as FP32 on the
stored values), and bit-for-bit equality with the x-fastest kernel on the
transposed arrays (both kernels use the same per-point arithmetic).
"""
import sys

import numpy as np
import pytest

from gpu_util import dev_grid, oracle_errors
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


def _zf(x):
    """(k, j, i) tensor -> (i, j, k) contiguous, i.e. stored z-fastest."""
    return x.permute(2, 1, 0).contiguous()


def run_both(g, storage=None, tile=None, xtile=None, halo=1):
    (u, v, w), c = dev_grid(g, storage=storage)
    zo = B.advect_zfast(_zf(u), _zf(v), _zf(w), c, halo=halo, tile=tile)
    xo = B.advect(u, v, w, c, halo=halo, tile=xtile)
    torch.cuda.synchronize()
    z = [o.permute(2, 1, 0).cpu().numpy() for o in zo]
    x = [o.cpu().numpy() for o in xo]
    return z, x


SHAPES = [(130, 70, 20), (64, 64, 64), (1, 1, 1), (65, 3, 1), (1, 200, 5), (9, 7, 129), (5, 4, 200),
          (33, 9, 64), (7, 5, 63), (3, 2, 256), (300, 3, 65)]
TILES = [None, (1, 1, 5, 4, 1), (1, 2, 9, 1, 1), (2, 1, 7, 8, 1), (2, 2, 64, 2, 1), (4, 1, 3, 4, 1),
         (4, 2, 16, 1, 1), (1, 4, 11, 4, 1), (2, 4, 1, 1, 1), (1, 8, 13, 4, 2), (2, 2, 64, 2, 2),
         (1, 8, 5, 1, 1), (4, 1, 6, 8, 2)]


@pytest.mark.parametrize("tile", TILES, ids=str)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_f32_zfast_matches_oracle_and_xfast(shape, tile):
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=800 + nx + 3 * ny + 7 * nz)
    z, x = run_both(g, tile=tile)
    errs = oracle_errors(z, g.u, g.v, g.w, g.coeffs)
    assert max(e[0] for e in errs) <= 1e-6, errs
    for a, b in zip(z, x):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("tile", [None, (1, 1, 3, 1, 1), (2, 2, 64, 8, 1), (1, 4, 7, 4, 1), (1, 8, 9, 4, 2),
                                  (2, 1, 5, 1, 2)], ids=str)
def test_f64_zfast(tile):
    g = wl.make_grid(70, 33, 130, seed=801, dtype=np.float64)
    z, x = run_both(g, tile=tile)
    errs = oracle_errors(z, g.u, g.v, g.w, g.coeffs)
    assert max(e[0] for e in errs) <= 1e-13, errs
    for a, b in zip(z, x):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("storage", ["bfloat16", "float16"])
@pytest.mark.parametrize("tile", [None, (1, 2, 8, 4, 1), (2, 1, 5, 1, 1), (4, 2, 16, 4, 1), (1, 8, 7, 4, 2)],
                         ids=str)
def test_16bit_zfast_bitwise_with_xfast(storage, tile):
    g = wl.make_grid(77, 21, 150, seed=802)
    sdt = getattr(torch, storage)
    z, x = run_both(g, storage=sdt, tile=tile)
    for a, b in zip(z, x):
        assert np.array_equal(a, b)
    # and against the oracle on the stored (rounded) values
    (u, v, w), _ = dev_grid(g, storage=sdt)
    st = [t.float().cpu().numpy() for t in (u, v, w)]
    errs = oracle_errors(z, *st, g.coeffs)
    assert max(e[0] for e in errs) <= 1e-6, errs


@pytest.mark.parametrize("halo", [2, 3])
def test_zfast_wider_halo(halo):
    g = wl.make_grid(40, 9, 70, seed=803, halo=halo)
    z, x = run_both(g, halo=halo, tile=(2, 2, 9, 4, 1))
    errs = oracle_errors(z, g.u, g.v, g.w, g.coeffs, halo=halo)
    assert max(e[0] for e in errs) <= 1e-6, errs
    for a, b in zip(z, x):
        assert np.array_equal(a, b)


def test_zfast_strided_layout():
    """Padded column and x-plane strides on input and output: cells outside
    the output views stay untouched."""
    g = wl.make_grid(50, 11, 70, seed=804)
    (u, v, w), c = dev_grid(g)
    ins = []
    for t in (u, v, w):
        big = torch.full((52, 13 + 2, 72 + 9), 7.0, device="cuda")
        big[:, :13, :72] = _zf(t)
        ins.append(big[:, :13, :72])
    outs_big = [torch.full((50, 11 + 3, 70 + 6), -3.0, device="cuda") for _ in range(3)]
    outs = [o[:, :11, :70] for o in outs_big]
    B.advect_zfast(*ins, c, out=outs)
    ref = B.advect(u, v, w, c)
    torch.cuda.synchronize()
    for o, r, ob in zip(outs, ref, outs_big):
        assert torch.equal(o.permute(2, 1, 0), r)
        assert bool((ob[:, 11:] == -3.0).all()) and bool((ob[:, :, 70:] == -3.0).all())


def test_zfast_integer_bitwise():
    g = wl.integer_grid(130, 11, 70, seed=805)
    z, _ = run_both(g)
    import oracle
    ref = oracle.forward(g.u, g.v, g.w, g.coeffs)
    for a, b in zip(z, ref):
        assert np.array_equal(a.astype(np.float64), b)


def test_zfast_512x512x64_parity(report):
    """The 512 x 512 x 64 FP32 grid stored z-fastest in the library's launch
    shape: every output against the oracle and bit-equal to the x-fastest
    kernel."""
    cfg = wl.C1
    g = wl.config_grid(cfg)
    z, x = run_both(g)
    errs = oracle_errors(z, g.u, g.v, g.w, g.coeffs)
    report["zfast_f32_512x512x64"] = dict(zip(("su", "sv", "sw"), (e[0] for e in errs)))
    assert max(e[0] for e in errs) <= 1e-6, errs
    for a, b in zip(z, x):
        assert np.array_equal(a, b)


def test_zfast_argument_errors():
    g = wl.make_grid(20, 8, 4, seed=806)
    (u, v, w), c = dev_grid(g)
    zu, zv, zw = _zf(u), _zf(v), _zf(w)
    with pytest.raises(B.PWError):
        B.advect_zfast(zu, zv, zw, c, tile=(8, 1, 8, 4, 1))
    with pytest.raises(ValueError):
        B.advect_zfast(u.permute(2, 1, 0), v.permute(2, 1, 0), w.permute(2, 1, 0), c)   # z not contiguous
    out = [torch.empty((20, 8, 4), device="cuda") for _ in range(3)]
    bad = zv.view(-1)[:20 * 8 * 4].view(20, 8, 4)
    with pytest.raises(B.PWError):
        B.advect_zfast(zu, zv, zw, c, out=(out[0], bad, out[2]))


@pytest.mark.parametrize("storage", [None, "bfloat16"])
@pytest.mark.parametrize("tile", [None, (1, 4, 9, 4, 2), (2, 2, 64, 1, 1), (4, 1, 5, 8, 2), (1, 8, 3, 4, 1)], ids=str)
@pytest.mark.parametrize("shape", [(37, 9, 70), (64, 8, 64), (5, 3, 150)], ids=lambda s: "x".join(map(str, s)))
def test_zfast_epilogue_bitwise_with_xfast(shape, tile, storage):
    """out = c + alpha F on z-fastest arrays equals the x-fastest epilogue on
    the transposed arrays bit for bit: accumulation in place (alpha = 1) and
    a separate addend with alpha = -0.25."""
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=820 + nz)
    (u, v, w), c = dev_grid(g, storage=None if storage is None else getattr(torch, storage))
    rng = np.random.default_rng(821 + nz)
    c0 = [torch.from_numpy(rng.uniform(-5, 5, (nz, ny, nx)).astype(np.float32)).cuda() for _ in range(3)]
    zin = [_zf(x) for x in (u, v, w)]
    # accumulation in place
    xo = [x.clone() for x in c0]
    B.advect_epilogue(u, v, w, c, xo, alpha=1.0, out=xo)
    zo = [_zf(x) for x in c0]
    B.advect_zfast_epilogue(*zin, c, zo, alpha=1.0, out=zo, tile=tile)
    # separate addends, alpha = -0.25
    xs = B.advect_epilogue(u, v, w, c, c0, alpha=-0.25)
    zs = B.advect_zfast_epilogue(*zin, c, [_zf(x) for x in c0], alpha=-0.25, tile=tile)
    torch.cuda.synchronize()
    for a, b in zip(zo, xo):
        assert torch.equal(a.permute(2, 1, 0), b)
    for a, b in zip(zs, xs):
        assert torch.equal(a.permute(2, 1, 0), b)


def test_zfast_epilogue_argument_errors():
    g = wl.make_grid(20, 8, 4, seed=822)
    (u, v, w), c = dev_grid(g)
    zin = [_zf(x) for x in (u, v, w)]
    out = [torch.zeros((20, 8, 4), device="cuda") for _ in range(3)]
    with pytest.raises(B.PWError):   # addend cu is the output sv: neither its own output nor disjoint
        B.advect_zfast_epilogue(*zin, c, [out[1], out[1], out[2]], out=out)
    with pytest.raises(B.PWError):
        B.advect_zfast_epilogue(*zin, c, out, alpha=float("nan"), out=out)
    with pytest.raises(ValueError):
        B.advect_zfast_epilogue(*zin, c, [x.double() for x in out], out=out)
