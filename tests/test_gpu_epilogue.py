"""GPU tests of the fused epilogue out = c + alpha * F(u, v, w): accumulation
in place and a fused explicit time step on padded views, against the FP64
oracle.

Tolerance: |out - (c + alpha F_ref)| <= 1e-6 * |alpha| * A + 2^-23 * |out|
(FP32: the forward's own A-scaled bound plus the one rounding of the fma);
bit for bit where the epilogue is exact (alpha = 1, c = 0) and across launch
shapes.
"""
import sys

import numpy as np
import pytest

import oracle
from gpu_util import dev_grid
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


def _check(got, c, alpha, ref, mag, eps=2.0 ** -23, tol=1e-6):
    for o, cc, r, m in zip(got, c, ref, mag):
        o = o.cpu().numpy().astype(np.float64)
        exp = np.asarray(cc, np.float64) + alpha * r
        err = np.abs(o - exp)
        assert np.all(err <= tol * abs(alpha) * m + eps * np.abs(exp) + 1e-30), float(np.max(err))


@pytest.mark.parametrize("tile", [None, (4, 2, 64, 1, 2), (1, 1, 5, 4), (2, 4, 3, 8, 1)])
@pytest.mark.parametrize("shape", [(130, 70, 20), (1, 1, 1), (257, 3, 4), (61, 9, 17)],
                         ids=lambda s: "x".join(map(str, s)))
def test_accumulate_in_place(shape, tile):
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=900 + nx)
    (u, v, w), c = dev_grid(g)
    rng = np.random.default_rng(901 + nx)
    c0 = [rng.uniform(-5, 5, (nz, ny, nx)).astype(np.float32) for _ in range(3)]
    out = [torch.from_numpy(x).cuda() for x in c0]
    B.advect_epilogue(u, v, w, c, out, alpha=1.0, out=out, tile=tile)
    ref, mag = oracle.forward(g.u, g.v, g.w, g.coeffs, magnitude=True)
    _check(out, c0, 1.0, ref, mag)


def test_time_step_on_padded_views():
    """u_next[interior] = u[interior] + dt * F(u, v, w), written into the
    interior of padded next-state arrays whose halos stay untouched."""
    g = wl.make_grid(100, 30, 12, seed=902)
    (u, v, w), c = dev_grid(g)
    dt = 0.37
    nxt = [torch.full_like(x, 123.0) for x in (u, v, w)]
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    B.advect_epilogue(u, v, w, c, [x[inner] for x in (u, v, w)], alpha=dt, out=[x[inner] for x in nxt])
    ref, mag = oracle.forward(g.u, g.v, g.w, g.coeffs, magnitude=True)
    _check([x[inner] for x in nxt], [x[inner] for x in (g.u, g.v, g.w)], dt, ref, mag)
    for x in nxt:   # halo untouched
        h = x.clone()
        h[inner] = 123.0
        assert torch.all(h == 123.0)


@pytest.mark.parametrize("storage", [None, "bfloat16", "float16", "float64"])
def test_alpha_one_zero_addend_is_plain_forward_bitwise(storage):
    dt = np.float64 if storage == "float64" else np.float32
    g = wl.make_grid(150, 37, 23, seed=903, dtype=dt)
    st = None if storage in (None, "float64") else getattr(torch, storage)
    (u, v, w), c = dev_grid(g, storage=st)
    plain = B.advect(u, v, w, c)
    zeros = [torch.zeros_like(x) for x in plain]
    fused = B.advect_epilogue(u, v, w, c, zeros, alpha=1.0)
    for a, b in zip(plain, fused):
        assert torch.equal(a, b)


def test_epilogue_tile_invariance_bitwise():
    g = wl.make_grid(300, 9, 7, seed=904)
    (u, v, w), c = dev_grid(g)
    add = [torch.randn((7, 9, 300), device="cuda") for _ in range(3)]
    base = B.advect_epilogue(u, v, w, c, add, alpha=0.5, tile=(1, 2, 4, 4, 1))
    for t in [(4, 2, 7, 1, 2), (2, 4, 64, 2, 1), (4, 1, 1, 8, 2)]:
        got = B.advect_epilogue(u, v, w, c, add, alpha=0.5, tile=t)
        for a, b in zip(base, got):
            assert torch.equal(a, b), t


def test_epilogue_argument_errors():
    g = wl.make_grid(20, 8, 4, seed=905)
    (u, v, w), c = dev_grid(g)
    out = [torch.zeros((4, 8, 20), device="cuda") for _ in range(3)]
    with pytest.raises(B.PWError):   # an addend that is another output
        B.advect_epilogue(u, v, w, c, [out[1], out[1], out[2]], out=out)
    with pytest.raises(B.PWError):
        B.advect_epilogue(u, v, w, c, out, alpha=float("nan"), out=out)


def test_epilogue_is_one_fma_of_the_plain_output():
    """out = fma(alpha, F_plain, c) with F_plain the plain kernel's output
    bit for bit: alpha a power of two makes alpha * F_plain exact, so the
    float64 sum with c is exact wherever the exponents are close (checked per
    point) and its rounding to float32 is the fma's single rounding."""
    g = wl.make_grid(190, 23, 17, seed=905)
    (u, v, w), c = dev_grid(g)
    plain = [x.cpu().numpy() for x in B.advect(u, v, w, c)]
    rng = np.random.default_rng(906)
    c0 = [rng.uniform(-5, 5, plain[0].shape).astype(np.float32) for _ in range(3)]
    alpha = -0.25
    out = [torch.from_numpy(x).cuda() for x in c0]
    B.advect_epilogue(u, v, w, c, out, alpha=alpha, out=out)
    torch.cuda.synchronize()
    checked = 0
    for o, f, cc in zip(out, plain, c0):
        prod = alpha * f.astype(np.float64)
        s = prod + cc.astype(np.float64)
        exact = (s - cc.astype(np.float64)) == prod
        want = s.astype(np.float32)
        got = o.cpu().numpy()
        assert np.array_equal(got[exact], want[exact])
        checked += int(exact.sum())
    assert checked >= 0.99 * 3 * plain[0].size


def _pitched(src, extra_rows, extra_cols, fill):
    """A view of src's contents inside a larger buffer (extra columns and rows
    per plane), and the buffer."""
    big = torch.full((src.shape[0], src.shape[1] + extra_rows, src.shape[2] + extra_cols), fill,
                     dtype=src.dtype, device=src.device)
    big[:, :src.shape[1], :src.shape[2]] = src
    return big, big[:, :src.shape[1], :src.shape[2]]


def _outside_unchanged(big, shape, fill):
    t = big.clone()
    t[:, :shape[1], :shape[2]] = fill
    return bool((t == fill).all())


def test_epilogue_strided_layout_bitwise():
    """Inputs and accumulated outputs as views into larger buffers: the dense
    result bit for bit, nothing outside the output views written."""
    g = wl.make_grid(150, 37, 23, seed=905)
    (u, v, w), c = dev_grid(g)
    rng = np.random.default_rng(906)
    acc = [torch.from_numpy(rng.uniform(-1, 1, (23, 37, 150)).astype(np.float32)).to("cuda") for _ in range(3)]
    dense = [x.clone() for x in acc]
    B.advect_epilogue(u, v, w, c, dense, alpha=0.25, out=dense)
    xs = [_pitched(x, 2, 5, 1.5)[1] for x in (u, v, w)]
    outs = [_pitched(x, 1, 3, -4.0) for x in acc]
    views = [vw for _, vw in outs]
    B.advect_epilogue(*xs, c, views, alpha=0.25, out=views)
    torch.cuda.synchronize()
    for d, (b, vw) in zip(dense, outs):
        assert torch.equal(d, vw)
        assert _outside_unchanged(b, d.shape, -4.0)
