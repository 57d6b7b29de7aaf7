"""GPU tests of the batched persistent form, its HIP-graph capture/replay and
the autotuners.  The per-point arithmetic is the single-grid kernel's, so
batched results must equal single-grid launches bit for bit, and both must
match the FP64 oracle to the FP32 bound (A-scaled 1e-6)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from gpu_util import dev_grid, full_grid_errors, oracle_errors
from paper_2301_13016_amd import binding as B
from paper_2301_13016_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(autouse=True)
def _announce(request):
    sys.__stderr__.write("\n[gpu-test] %s\n" % request.node.nodeid)
    sys.__stderr__.flush()
    yield


SMALL = [(70, 13, 9), (1, 1, 1), (129, 4, 17), (64, 64, 3), (200, 7, 33), (5, 90, 2), (256, 2, 5), (300, 3, 4)]


def make_subs(grids):
    subs, host = [], []
    for g in grids:
        (u, v, w), c = dev_grid(g)
        outs = tuple(torch.full((g.nz, g.ny, g.nx), float("nan"), device="cuda") for _ in range(3))
        subs.append((u, v, w, c, outs))
        host.append(g)
    return subs, host


def single(sub):
    u, v, w, c, _ = sub
    out = B.advect(u, v, w, c)
    return [o.clone() for o in out]


@pytest.fixture(scope="module")
def small_batch():
    grids = [wl.make_grid(*s, seed=500 + i) for i, s in enumerate(SMALL)]
    return make_subs(grids)


@pytest.mark.parametrize("tile", [None, (1, 2, 8, 4), (2, 1, 16, 1), (4, 2, 5, 2), (1, 4, 64, 8), (2, 4, 32, 1, 2),
                                  (4, 1, 7, 4, 2), (0, 4, 32, 1), (0, 2, 9, 4, 2), (0, 1, 64, 8)])
def test_batch_equals_single_grid_and_oracle(small_batch, tile):
    subs, grids = small_batch
    ref = [single(s) for s in subs]
    for s in subs:
        for o in s[4]:
            o.fill_(float("nan"))
    b = B.Batch(subs, tile=tile)
    b.run()
    torch.cuda.synchronize()
    for s, r, g in zip(subs, ref, grids):
        for o, rr in zip(s[4], r):
            assert torch.equal(o, rr)
        errs = oracle_errors([o.cpu().numpy() for o in s[4]], g.u, g.v, g.w, g.coeffs)
        assert max(e for e, _ in errs) <= 1e-6
    b.close()


def test_graph_capture_replay(small_batch):
    """Capture once, replay several times with unrelated eager work and
    synchronisations in between; every replay reproduces the eager result."""
    subs, _ = small_batch
    b = B.Batch(subs)
    b.run()
    torch.cuda.synchronize()
    eager = [[o.clone() for o in s[4]] for s in subs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.capture(stream)
    torch.cuda.synchronize()
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        for s in subs:
            for o in s[4]:
                o.zero_()
        scratch.mul_(1.0001).add_(0.5)      # unrelated eager work
        single(subs[rep % len(subs)])        # and an eager library call
        torch.cuda.synchronize()
        b.replay(stream)
        stream.synchronize()
        for s, e in zip(subs, eager):
            for o, x in zip(s[4], e):
                assert torch.equal(o, x), rep
    b.close()


def test_replay_requires_capture_and_tune_invalidates(small_batch):
    subs, _ = small_batch
    b = B.Batch(subs)
    with pytest.raises(B.PWError):
        b.replay()
    stream = torch.cuda.Stream()
    b.capture(stream)
    ref = [[o.clone() for o in s[4]] for s in subs]
    tile = b.tune()
    assert b.info()[0] == tile
    with pytest.raises(B.PWError):   # re-tiling dropped the graph
        b.replay()
    b.run()
    torch.cuda.synchronize()
    for s, e in zip(subs, ref):
        for o, x in zip(s[4], e):
            assert torch.equal(o, x)
    b.close()


@pytest.fixture(scope="module")
def batch_c3():
    grids = wl.batch_grids()
    return make_subs(grids)


def test_c3_batch_matches_plain_launches(batch_c3, report):
    """The 64 uneven subdomains: one persistent launch equals 64 plain
    launches bit for bit, and every point of every subdomain matches the
    oracle."""
    subs, grids = batch_c3
    ref = [single(s) for s in subs]
    b = B.Batch(subs)
    b.tune()
    b.run()
    torch.cuda.synchronize()
    for s, r in zip(subs, ref):
        for o, rr in zip(s[4], r):
            assert torch.equal(o, rr)
    worst = 0.0
    for i, g in enumerate(grids):
        worst = max(worst, max(full_grid_errors({"b": subs[i][4]}, g, slab=64)["b"][0]))
    tile, items, groups = b.info()
    report["batch_c3"] = dict(points=sum(g.points for g in grids), tile=tile, work_items=items,
                              workgroups=groups, worst_err_a_scaled=worst)
    assert worst <= 1e-6
    b.close()


def test_single_grid_tuner_and_cache_file(tmp_path):
    """pw_tune in a fresh process: writes the cache file (one line per
    kernel), results are unchanged (shape never changes results), and a
    second process reads the same shapes back from the file."""
    cache = tmp_path / "tune.txt"
    code = r'''
import sys, numpy as np, torch
sys.path.insert(0, %r); sys.path.insert(0, %r)
from paper_2301_13016_amd import binding as B, workloads as wl
from gpu_util import dev_grid
if sys.argv[1] == "tune":
    g = wl.make_grid(300, 40, 24, seed=9)
    (u, v, w), c = dev_grid(g)
    a = [o.clone() for o in B.advect(u, v, w, c)]
    B.tune(300, 40, 24, torch.float32)
    b = B.advect(u, v, w, c)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b))
print("SHAPES", [B.launch_shape(k, 300, 40, 24, torch.float32) for k in ("forward", "adjoint", "tangent")])
print("OK")
''' % (ROOT, os.path.join(ROOT, "tests"))
    env = dict(os.environ, PWADV_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", code, "tune"], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "OK" in r.stdout
    lines = cache.read_text().splitlines()
    assert len(lines) == 3 and all(l.startswith("pwadv-tune-v3 ") for l in lines)
    assert sorted(int(l.split()[1]) for l in lines) == [0, 1, 2]
    shapes = [l for l in r.stdout.splitlines() if l.startswith("SHAPES")]
    r2 = subprocess.run([sys.executable, "-c", code, "read"], env=env, capture_output=True, text=True, timeout=300)
    assert r2.returncode == 0, r2.stderr[-2000:]
    assert [l for l in r2.stdout.splitlines() if l.startswith("SHAPES")] == shapes


def test_batch_strided_layouts_bitwise():
    """Subdomains whose inputs and outputs are views into larger buffers
    (each with its own pitch): every subdomain equals its dense single-grid
    result bit for bit, and nothing outside the output views is written."""
    shapes = [(70, 13, 9), (129, 4, 17), (200, 7, 5), (33, 40, 3)]
    grids = [wl.make_grid(*s, seed=560 + i) for i, s in enumerate(shapes)]
    dense_subs, _ = make_subs(grids)
    refs = [single(s) for s in dense_subs]
    subs, bigs = [], []
    for i, (u, v, w, c, outs) in enumerate(dense_subs):
        er, ec = 1 + i, 3 + 2 * i

        def pitched(src, fill):
            big = torch.full((src.shape[0], src.shape[1] + er, src.shape[2] + ec), fill, dtype=src.dtype,
                             device=src.device)
            big[:, :src.shape[1], :src.shape[2]] = src
            return big, big[:, :src.shape[1], :src.shape[2]]

        xs = [pitched(x, 2.0)[1] for x in (u, v, w)]
        os_ = [pitched(o, -6.0) for o in outs]
        bigs.append(os_)
        subs.append((*xs, c, tuple(vw for _, vw in os_)))
    for tile in (None, (0, 4, 16, 1), (2, 2, 8, 4, 2)):
        for os_ in bigs:
            for _, vw in os_:
                vw.fill_(float("nan"))
        b = B.Batch(subs, tile=tile)
        b.run()
        torch.cuda.synchronize()
        for ref, os_ in zip(refs, bigs):
            for r, (big, vw) in zip(ref, os_):
                assert torch.equal(r, vw), tile
                outside = big.clone()
                outside[:, :vw.shape[1], :vw.shape[2]] = -6.0
                assert bool((outside == -6.0).all()), tile
        b.close()


def test_per_subdomain_width_rule(small_batch):
    """With 0 columns per lane a subdomain gets 2 columns per lane where that
    leaves no more lanes idle than 1 (nx rounded up to 128 equals nx rounded
    up to 64), else 1: the work list has exactly the strips that rule gives."""
    subs, grids = small_batch
    ry, zlen = 2, 8

    def items(nx, ny, nz, px):
        chunks = -(-nz // zlen)
        zl = -(-nz // chunks)
        return -(-nx // (64 * px)) * -(-ny // ry) * -(-nz // zl)

    def width(nx):
        return 2 if -(-nx // 128) * 128 == -(-nx // 64) * 64 else 1

    b = B.Batch(subs, tile=(0, ry, zlen, 1))
    tile, n_items, _ = b.info()
    assert tile[0] == 0
    assert n_items == sum(items(g.nx, g.ny, g.nz, width(g.nx)) for g in grids)
    assert {width(g.nx) for g in grids} == {1, 2}
    b.close()
    b = B.Batch(subs, tile=(2, ry, zlen, 1))
    assert b.info()[1] == sum(items(g.nx, g.ny, g.nz, 2) for g in grids)
    b.close()


def test_table_generator_retiming():
    """The built-in table's generator re-times a forward pick against its
    neighbours on separately allocated fields: it returns the pick or a
    neighbour, with a median for every shape it could run, and the shape it
    returns runs and equals the pick's result bit for bit."""
    from paper_2301_13016_amd import tune_defaults as TD
    pick = (2, 2, 5, 4, 1, 0)
    best, med = TD.confirm_forward(B, torch, 70, 9, 5, torch.float32, pick, rounds=3)
    assert best in TD.neighbours(pick, 5) and tuple(pick) in med and best in med
    assert all(m > 0 for m in med.values())
    g = wl.make_grid(70, 9, 5, seed=71)
    (u, v, w), c = dev_grid(g)
    a = [o.clone() for o in B.advect(u, v, w, c, tile=pick)]
    b = B.advect(u, v, w, c, tile=best)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b))
