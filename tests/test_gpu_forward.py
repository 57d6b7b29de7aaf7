"""GPU parity tests of the forward kernel (through the C ABI) against the FP64
oracle on the same seeded inputs.

Tolerances (error scaled by A(p), the sum of |term| magnitudes of the point,
which bounds the rounding error of any evaluation order):
  FP32 storage and arithmetic: 1e-6     (bound ~8 * 2^-24 = 4.8e-7)
  FP64:                        1e-13    (bound ~8 * 2^-53)
  BF16 / FP16 storage, against the oracle on the unrounded FP32 values: 1e-2
      (storage rounding bound 2u: 7.8e-3 BF16, 9.8e-4 FP16), and against the
      oracle on the rounded values: 1e-6 (arithmetic only)
Integer winds with dyadic coefficients are exact in every dtype, so there the
comparison is bit for bit.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from gpu_util import dev_grid, full_grid_errors, oracle_errors, poison_unread
from paper_2301_13016_amd import binding as B
from paper_2301_13016_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture(autouse=True)
def _announce(request):
    sys.__stderr__.write("\n[gpu-test] %s\n" % request.node.nodeid)
    sys.__stderr__.flush()
    yield


def run(g, storage=None, tile=None, halo=1):
    (u, v, w), c = dev_grid(g, storage=storage)
    out = B.advect(u, v, w, c, halo=halo, tile=tile)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


SHAPES = [(130, 70, 20), (64, 64, 64), (1, 1, 1), (65, 3, 1), (1, 200, 5), (200, 1, 3), (62, 8, 2), (63, 9, 17)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_f32_matches_oracle(shape):
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=100 + nx + ny + nz)
    errs = oracle_errors(run(g), g.u, g.v, g.w, g.coeffs)
    for (ea, en), name in zip(errs, "su sv sw".split()):
        assert ea <= 1e-6, (name, ea, en)


def test_f64_config0_matches_oracle(report):
    cfg = wl.C0
    g = wl.config_grid(cfg)
    errs = oracle_errors(run(g), g.u, g.v, g.w, g.coeffs)
    report["fwd_f64_64x64x64"] = dict(a_scaled=dict(zip(("su", "sv", "sw"), (e[0] for e in errs))),
                                      normwise=dict(zip(("su", "sv", "sw"), (e[1] for e in errs))))
    for ea, en in errs:
        assert ea <= 1e-13, (ea, en)


@pytest.mark.parametrize("storage", [None, "float64", "bfloat16", "float16"])
@pytest.mark.parametrize("shape", [(4, 4, 4), (130, 70, 20), (63, 5, 9)], ids=lambda s: "x".join(map(str, s)))
def test_integer_inputs_bitwise_all_dtypes(storage, shape):
    nx, ny, nz = shape
    dt = np.float64 if storage == "float64" else np.float32
    g = wl.integer_grid(nx, ny, nz, seed=7 + nx, dtype=dt)
    st = None if storage in (None, "float64") else getattr(torch, storage)
    got = run(g, storage=st)
    ref = oracle.forward(g.u, g.v, g.w, g.coeffs)
    for o, r in zip(got, ref):
        assert np.array_equal(o.astype(np.float64), r)


TILES = [(1, 1, 1, 1), (1, 1, 7, 4), (1, 2, 3, 8), (1, 4, 16, 4), (2, 4, 5, 2), (2, 1, 64, 4), (2, 2, 2, 1),
         (4, 1, 64, 8), (4, 2, 5, 1), (4, 1, 1, 4), (4, 2, 16, 2),
         # two planes prefetched: short chunks (1, 2, 3 levels) exercise the five-plane ring's clamping
         (1, 1, 1, 1, 2), (1, 2, 2, 8, 2), (2, 4, 3, 1, 2), (4, 2, 7, 1, 2), (4, 1, 64, 4, 2), (2, 2, 5, 8, 2),
         # four columns x four rows
         (4, 4, 9, 1), (4, 4, 23, 4, 2), (4, 4, 2, 8, 1)]


@pytest.mark.parametrize("shape", [(150, 37, 23), (300, 9, 7), (259, 5, 6), (513, 3, 4)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tile_shape_invariance_bitwise(shape):
    g = wl.make_grid(*shape, seed=5)
    base = run(g, tile=(1, 4, 16, 4))
    for t in TILES:
        got = run(g, tile=t)
        for a, b in zip(base, got):
            assert np.array_equal(a, b), t


@pytest.mark.parametrize("tile", [(1, 2, 16, 4), (2, 4, 16, 4), (4, 2, 16, 1), (4, 2, 64, 1, 2), (2, 4, 3, 4, 2)])
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 2, 2), (255, 4, 3), (257, 3, 2), (130, 70, 20)],
                         ids=lambda s: "x".join(map(str, s)))
def test_f32_every_tile_kind_matches_oracle(shape, tile):
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=400 + nx)
    errs = oracle_errors(run(g, tile=tile), g.u, g.v, g.w, g.coeffs)
    assert max(e for e, _ in errs) <= 1e-6, (tile, errs)


@pytest.mark.parametrize("storage", ["bfloat16", "float16", "float64"])
def test_prefetch_depth_invariance_other_dtypes(storage):
    """The five-plane ring (two planes prefetched) gives bit-identical results
    to the four-plane ring for 16-bit and FP64 storage too."""
    dt = np.float64 if storage == "float64" else np.float32
    g = wl.make_grid(300, 11, 9, seed=12, dtype=dt)
    st = None if storage == "float64" else getattr(torch, storage)
    px = 2 if storage == "float64" else 4
    base = run(g, storage=st, tile=(1, 2, 4, 4))
    four_rows = [(2, 4, 9, 1, 1), (1, 4, 3, 4, 2)] if storage == "float64" else [(4, 4, 5, 1, 1)]
    for t in [(px, 2, 9, 1, 2), (px, 1, 2, 4, 2), (1, 1, 1, 8, 2)] + four_rows:
        got = run(g, storage=st, tile=t)
        for a, b in zip(base, got):
            assert np.array_equal(a, b), t


def test_deterministic_across_runs():
    g = wl.make_grid(200, 50, 30, seed=6)
    a = run(g)
    b = run(g)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("halo", [2, 3])
def test_wider_halo(halo):
    g = wl.make_grid(70, 20, 9, seed=8, halo=halo)
    errs = oracle_errors(run(g, halo=halo), g.u, g.v, g.w, g.coeffs, halo=halo)
    assert max(e for e, _ in errs) <= 1e-6


def test_pitched_strides_and_untouched_inputs():
    """Inputs and outputs as views into larger buffers: padded rows pitched to
    a multiple of 64 elements, outputs with their own pitch; inputs and the
    gaps of the output buffers must come back untouched."""
    g = wl.make_grid(100, 30, 12, seed=9)
    pz, py, px = g.u.shape
    (u, v, w), c = dev_grid(g)
    big = [torch.full((pz, py, 128), 7.0, device="cuda") for _ in range(3)]
    for bb, x in zip(big, (u, v, w)):
        bb[:, :, :px] = x
    vin = [bb[:, :, :px] for bb in big]
    obig = [torch.full((12, 31, 112), -3.0, device="cuda") for _ in range(3)]
    outs = tuple(ob[:, :30, :100] for ob in obig)
    before = [bb.clone() for bb in big]
    B.advect(*vin, c, out=outs)
    torch.cuda.synchronize()
    for bb, b0 in zip(big, before):
        assert torch.equal(bb, b0)
    for ob in obig:
        assert torch.all(ob[:, 30:, :] == -3.0) and torch.all(ob[:, :, 100:] == -3.0)
    errs = oracle_errors([o.cpu().numpy() for o in outs], g.u, g.v, g.w, g.coeffs)
    assert max(e for e, _ in errs) <= 1e-6


@pytest.mark.parametrize("storage", ["bfloat16", "float16"])
def test_low_precision_storage_errors(storage):
    g = wl.make_grid(190, 40, 16, seed=10)
    st = getattr(torch, storage)
    got = run(g, storage=st)
    # total error against the unrounded FP32 values
    errs = oracle_errors(got, g.u, g.v, g.w, g.coeffs)
    bound = 1e-2 if storage == "bfloat16" else 2e-3
    for ea, _ in errs:
        assert ea <= bound, (storage, ea)
    # arithmetic error against the rounded values actually stored
    (u, v, w), _ = dev_grid(g, storage=st)
    q = [x.float().cpu().numpy() for x in (u, v, w)]
    errs_q = oracle_errors(got, *q, g.coeffs)
    for ea, _ in errs_q:
        assert ea <= 1e-6, (storage, ea)


@pytest.fixture(scope="module")
def grid_1024():
    return wl.config_grid(wl.C2)


def test_precision_grid_full_parity(grid_1024, report):
    """The 1024 x 1024 x 256 grid in every storage type (FP32, BF16, FP16 and
    FP64; the launches the benchmark times), compared at EVERY interior point
    with one FP64 oracle pass on the unrounded FP32 values (BF16/FP16: total
    error of storage rounding plus arithmetic).  The worst A-scaled and
    normwise errors per field go into the report."""
    g = grid_1024
    outs = {}
    for storage in ("float32", "bfloat16", "float16"):
        st = getattr(torch, storage)
        (u, v, w), c = dev_grid(g, storage=None if storage == "float32" else st)
        outs[storage] = B.advect(u, v, w, c)
        del u, v, w
    (u, v, w), _ = dev_grid(g)
    c64 = B.Coeffs.from_host(g.coeffs, dtype=torch.float64)
    outs["float64"] = B.advect(u.double(), v.double(), w.double(), c64)
    del u, v, w
    torch.cuda.synchronize()
    assert all(o.dtype == torch.float64 for o in outs["float64"])
    errs = full_grid_errors(outs, g)
    rep = report.setdefault("precision_1024x1024x256", {})
    for storage, (worst, nw) in errs.items():
        rep[storage] = dict(a_scaled=dict(zip(("su", "sv", "sw"), worst)),
                            normwise=dict(zip(("su", "sv", "sw"), nw)), points="all")
    bound = {"float32": 1e-6, "bfloat16": 1e-2, "float16": 2e-3, "float64": 1e-13}
    for storage, (worst, _) in errs.items():
        assert max(worst) <= bound[storage], (storage, worst)


def test_headline_grid_full_parity(report):
    """The 512 x 512 x 64 FP32 grid in the launch shape the benchmark times,
    compared with the oracle at every one of its 16.8 M points."""
    cfg = wl.C1
    g = wl.config_grid(cfg)
    (u, v, w), c = dev_grid(g)
    out = B.advect(u, v, w, c)
    torch.cuda.synchronize()
    # every output finite and written (the kernel covers the whole interior)
    for o in out:
        assert torch.isfinite(o).all()
    worst, nw = full_grid_errors({"f32": out}, g)["f32"]
    report["fwd_f32_512x512x64"] = dict(a_scaled=dict(zip(("su", "sv", "sw"), worst)),
                                        normwise=dict(zip(("su", "sv", "sw"), nw)), points="all")
    assert max(worst) <= 1e-6, worst


@pytest.mark.parametrize("storage", [None, "float64", "bfloat16"])
@pytest.mark.parametrize("shape,halo", [((70, 13, 9), 1), ((130, 5, 3), 1), ((61, 9, 17), 2), ((1, 1, 1), 1)],
                         ids=lambda x: "x".join(map(str, x)) if isinstance(x, tuple) else "h%d" % x)
def test_unread_cells_do_not_reach_any_output(shape, halo, storage):
    """NaN and +-Inf in every padded cell no output reads leave the forward,
    tangent and coefficient-gradient results bit-identical to those of the
    clean grid."""
    nx, ny, nz = shape
    clean = wl.make_grid(nx, ny, nz, seed=31 + nx, halo=halo,
                         dtype=np.float64 if storage == "float64" else np.float32)
    dirty = wl.make_grid(nx, ny, nz, seed=31 + nx, halo=halo,
                         dtype=np.float64 if storage == "float64" else np.float32)
    poison_unread(dirty)
    st = getattr(torch, storage) if storage in ("bfloat16",) else None
    a = run(clean, storage=st, halo=halo)
    b = run(dirty, storage=st, halo=halo)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    if storage == "bfloat16":
        return
    d = [torch.from_numpy(x).to("cuda").to(torch.float64 if storage else torch.float32)
         for x in wl.direction(nx, ny, nz, seed=32, halo=halo)]
    r = [torch.from_numpy(x).to("cuda").to(d[0].dtype) for x in wl.cotangents(nx, ny, nz, seed=33)]
    outs = []
    for g in (clean, dirty):
        (u, v, w), c = dev_grid(g)
        t = B.advect_tangent(u, v, w, c, *d, halo=halo)
        cg = B.advect_coeff_grad(u, v, w, *r, halo=halo)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in t] + [cg[n].cpu().numpy() for n in sorted(cg)])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


SHARED_TILES = {
    None: [(4, 1), (4, 2), (4, 4)],                          # FP32
    "bfloat16": [(4, 2), (4, 4), (8, 2)],
    "float16": [(4, 2), (8, 2)],
    "float64": [(2, 2), (2, 4)],
}


@pytest.mark.parametrize("storage", [None, "bfloat16", "float16", "float64"])
@pytest.mark.parametrize("shape,halo", [((130, 70, 20), 1), ((512, 9, 7), 1), ((300, 3, 5), 1), ((64, 1, 3), 1),
                                        ((257, 37, 9), 2), ((1, 1, 1), 1), ((1030, 6, 4), 1)],
                         ids=lambda x: "x".join(map(str, x)) if isinstance(x, tuple) else "h%d" % x)
def test_shared_row_tiles_bitwise(shape, halo, storage):
    """Workgroups whose wavefronts pass their edge rows through LDS give the
    same outputs, bit for bit, as independent strips of the same shape: every
    instantiated shape, 2 and 4 wavefronts per group, with and without
    non-temporal own rows, one and several z-chunks (chunks of one, two and
    three levels, a last chunk shorter than the rest), ragged y (wavefronts
    past the grid) and x (edge strips), halo 1 and 2."""
    nx, ny, nz = shape
    g = wl.make_grid(nx, ny, nz, seed=41 + nx + ny, halo=halo,
                     dtype=np.float64 if storage == "float64" else np.float32)
    st = getattr(torch, storage) if storage in ("bfloat16", "float16") else None
    for px, ry in SHARED_TILES[storage]:
        ref = run(g, storage=st, tile=(px, ry, 3, 1, 1), halo=halo)
        for wpb in (2, 4):
            for share in (1, 2):
                for zl in sorted({nz, 3, 2, 1}):
                    got = run(g, storage=st, tile=(px, ry, zl, wpb, 1, share), halo=halo)
                    for a, b in zip(ref, got):
                        assert np.array_equal(a, b), (px, ry, zl, wpb, share)


def test_shared_row_tiles_match_oracle(report):
    """The shared-row FP32 shapes against the FP64 oracle at every point."""
    g = wl.make_grid(300, 45, 13, seed=43)
    worst = 0.0
    for tile in [(4, 1, 13, 4, 1, 2), (4, 2, 7, 4, 1, 1), (4, 4, 13, 2, 1, 2)]:
        errs = oracle_errors(run(g, tile=tile), g.u, g.v, g.w, g.coeffs)
        worst = max(worst, max(e for e, _ in errs))
    report["shared_rows_f32_300x45x13"] = dict(a_scaled_worst=worst)
    assert worst <= 1e-6


def test_shared_row_tiles_epilogue_and_bc():
    """The fused epilogue runs in shared-row workgroups, bit-identical to
    independent strips; boundary rules by addressing with a shared-row tile
    run the same shape with independent strips (same result)."""
    g = wl.make_grid(260, 19, 11, seed=44)
    (u, v, w), c = dev_grid(g)
    rng = np.random.default_rng(45)
    add = [torch.from_numpy(rng.uniform(-1, 1, (11, 19, 260)).astype(np.float32)).to("cuda") for _ in range(3)]
    ref = B.advect_epilogue(u, v, w, c, add, alpha=0.5, tile=(4, 2, 4, 1, 1))
    for tile in [(4, 2, 11, 4, 1, 1), (4, 1, 5, 2, 1, 2), (4, 4, 11, 4, 1, 2)]:
        got = B.advect_epilogue(u, v, w, c, add, alpha=0.5, tile=tile)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(ref, got)), tile
    bc = ("periodic", "periodic", "copy")
    rb = B.advect_bc(u, v, w, c, bc, tile=(4, 2, 11, 4, 1, 0))
    gb = B.advect_bc(u, v, w, c, bc, tile=(4, 2, 11, 4, 1, 1))
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(rb, gb))


def test_host_pointer_rejected():
    """Host outputs: the binding refuses them (device mismatch), and the C
    entry point itself, called with host pointers, returns
    PW_ERR_INVALID_ARG without launching anything."""
    g = wl.make_grid(8, 8, 8, seed=11)
    (u, v, w), c = dev_grid(g)
    host_out = [torch.empty((8, 8, 8)) for _ in range(3)]
    with pytest.raises(ValueError):
        B.advect(u, v, w, c, out=host_out)
    st = B.pw_advect(B.pw_grid(8, 8, 8, 1), None, B.PW_F32, u.data_ptr(), v.data_ptr(), w.data_ptr(),
                     c.c_struct(), *(o.data_ptr() for o in host_out))
    assert st == B.PW_ERR_INVALID_ARG


def test_stream_probe_modes():
    """The bandwidth probe copies bit for bit in every variant (sizes that
    end mid-stride), its write mode stores its documented pattern, and its
    read mode leaves the sink alone for ordinary data."""
    n = 1_000_000 * 4                       # floats: 16 MB, not a multiple of any stride
    src = torch.randn(n, device="cuda")
    for loads in (1, 2, 4, 8):
        for flags in range(4):
            dst = torch.zeros_like(src)
            B.stream_probe(0, loads, flags, src, dst, blocks=37)
            torch.cuda.synchronize()
            assert torch.equal(src, dst), (loads, flags)
    w = torch.zeros(4096, dtype=torch.int32, device="cuda")
    B.stream_probe(2, 4, 2, None, w, blocks=3)
    idx = torch.arange(1024, device="cuda", dtype=torch.int32)
    want = torch.stack([idx, torch.ones_like(idx), 2 * torch.ones_like(idx), 3 * torch.ones_like(idx)], 1).reshape(-1)
    torch.cuda.synchronize()
    assert torch.equal(w, want)
    sink = torch.zeros(1024, dtype=torch.int32, device="cuda")
    B.stream_probe(1, 8, 1, src, sink, blocks=64)
    torch.cuda.synchronize()
    assert int(sink.abs().sum()) == 0


def test_stream_copies_are_exact():
    """The calibration kernels copy bit for bit (one and three streams, sizes
    that end mid-grid-stride)."""
    n = 1_000_004   # floats: a multiple of 4, not of the launch's stride
    src = [torch.randn(n, device="cuda") for _ in range(3)]
    dst = [torch.empty_like(x) for x in src]
    B.stream_copy3(src, dst)
    one = torch.empty_like(src[0])
    B.stream_copy(src[1], one)
    torch.cuda.synchronize()
    for a, b in zip(src, dst):
        assert torch.equal(a, b)
    assert torch.equal(one, src[1])


def test_pwadv_log_prints_one_line_per_launch():
    """PWADV_LOG=1: each launching call prints its entry point, grid, storage
    type, launch shape and the shape's source on stderr (in a child process,
    since the switch is read once per process)."""
    import subprocess
    import textwrap
    code = textwrap.dedent("""
        import sys
        sys.path.insert(0, %r)
        import numpy as np, torch
        from paper_2301_13016_amd import binding as B
        from paper_2301_13016_amd import workloads as wl
        g = wl.make_grid(70, 9, 5, seed=1)
        x = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (g.u, g.v, g.w)]
        c = B.Coeffs.from_host(g.coeffs, device="cuda")
        B.advect(*x, c)
        B.advect(*x, c, tile=(2, 2, 5, 4))
        r = [torch.ones((5, 9, 70), device="cuda") for _ in range(3)]
        B.advect_adjoint(*x, c, *r)
        B.advect_coeff_grad(*x, *r)
        B.halo_fill(x, ("periodic", "periodic", "copy"))
        torch.cuda.synchronize()
    """) % ROOT
    env = dict(os.environ, PWADV_LOG="1")
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stderr.splitlines() if ln.startswith("pwadv: ")]
    assert any(ln.startswith("pwadv: pw_advect 70x9x5 halo 1 f32 tile (") and ln.endswith(("default", "tuned"))
               for ln in lines), lines
    assert any("pw_advect 70x9x5 halo 1 f32 tile (2, 2, 5, 4, 1, 0) given" in ln for ln in lines), lines
    assert any(ln.startswith("pwadv: pw_advect_adjoint 70x9x5") for ln in lines), lines
    assert any(ln.startswith("pwadv: pw_advect_coeff_grad 70x9x5") and ln.endswith("shape rule") for ln in lines)
    assert any(ln.startswith("pwadv: pw_halo_fill 70x9x5 halo 1 f32") for ln in lines), lines
    env.pop("PWADV_LOG")
    q = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert q.returncode == 0 and "pwadv: " not in q.stderr
    # a shape from PWADV_TILE is named as such; an explicit tile still wins
    env.update(PWADV_LOG="1", PWADV_TILE="2x1x3x2x2")
    t = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    assert t.returncode == 0, t.stderr[-2000:]
    lines = [ln for ln in t.stderr.splitlines() if ln.startswith("pwadv: ")]
    assert any("pw_advect 70x9x5 halo 1 f32 tile (2, 1, 3, 2, 2, 0) PWADV_TILE" in ln for ln in lines), lines
    assert any("pw_advect 70x9x5 halo 1 f32 tile (2, 2, 5, 4, 1, 0) given" in ln for ln in lines), lines


def test_pwadv_tile_override_bitwise(monkeypatch):
    """Forward calls without a tile take PWADV_TILE's shape: the outputs equal
    those of the same shape given explicitly, bit for bit, for the plain, the
    epilogue and the boundary-rule forward; shape changes no result."""
    g = wl.make_grid(130, 21, 9, seed=57)
    (u, v, w), c = dev_grid(g)
    add = [torch.full((9, 21, 130), 0.5, device="cuda") for _ in range(3)]
    bc = ("periodic", "periodic", "copy")
    for tile in [(4, 2, 5, 4, 1, 2), (2, 1, 3, 2, 2, 0), (1, 4, 9, 1, 1, 0)]:
        want = [B.advect(u, v, w, c, tile=tile), B.advect_epilogue(u, v, w, c, add, alpha=0.25, tile=tile),
                B.advect_bc(u, v, w, c, bc, tile=tile)]
        monkeypatch.setenv("PWADV_TILE", "x".join(map(str, tile)))
        got = [B.advect(u, v, w, c), B.advect_epilogue(u, v, w, c, add, alpha=0.25), B.advect_bc(u, v, w, c, bc)]
        monkeypatch.delenv("PWADV_TILE")
        torch.cuda.synchronize()
        for wt, gt in zip(want, got):
            assert all(torch.equal(a, b) for a, b in zip(wt, gt)), tile
    monkeypatch.setenv("PWADV_TILE", "5x1x1")
    with pytest.raises(B.PWError):
        B.advect(u, v, w, c)
