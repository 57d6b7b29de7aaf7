"""Host logic of bench.py: the algorithmic byte counts its rates divide by,
its refusal of more than one GPU, and when it trusts the committed HBM
counter readings.  No GPU work."""
import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _cells(nx, ny, nz, h):
    """(padded, interior) cell counts by marking the interior of a padded array."""
    pad = np.zeros((nz + 2 * h, ny + 2 * h, nx + 2 * h), dtype=bool)
    pad[h:h + nz, h:h + ny, h:h + nx] = True
    return pad.size, int(pad.sum())


def test_forward_bytes():
    """Every padded input element read once, every interior output written once."""
    assert bench.algo_bytes(512, 512, 64, 1, 4) == 410_569_824
    for nx, ny, nz, h, ib, ob in [(7, 5, 3, 1, 4, 4), (9, 2, 4, 2, 2, 4), (3, 3, 3, 1, 8, 8)]:
        padded, interior = _cells(nx, ny, nz, h)
        assert bench.algo_bytes(nx, ny, nz, h, ib, ob) == 3 * padded * ib + 3 * interior * ob


def test_adjoint_and_tangent_bytes():
    """Adjoint: u, v, w and the cotangents read, padded gradients written;
    tangent: values and directions read (padded), interior outputs written."""
    for nx, ny, nz, h, es in [(256, 256, 128, 1, 4), (6, 4, 5, 2, 8)]:
        padded, interior = _cells(nx, ny, nz, h)
        assert bench.adjoint_bytes(nx, ny, nz, h, es) == (6 * padded + 3 * interior) * es
        assert bench.tangent_bytes(nx, ny, nz, h, es) == (6 * padded + 3 * interior) * es
    # the ratio the c4 comparisons quote (1.51x the forward's bytes)
    r = bench.adjoint_bytes(256, 256, 128, 1) / bench.algo_bytes(256, 256, 128, 1, 4)
    assert abs(r - 1.508) < 1e-3


def test_halo_bytes():
    """Every halo cell written once and its source read once; a zeroed lid
    (z rule ZERO) reads nothing for its planes."""
    for nx, ny, nz, h in [(512, 512, 64, 1), (5, 7, 3, 2)]:
        padded, interior = _cells(nx, ny, nz, h)
        cells = padded - interior
        periodic_copy = [(1, 1, 2)] * 3
        assert bench.halo_bytes(nx, ny, nz, h, 4, periodic_copy) == 3 * 2 * cells * 4
        lid = [(1, 1, 2), (1, 1, 2), (1, 1, bench.B_HALO_ZERO)]
        zplanes = 2 * h * (ny + 2 * h) * (nx + 2 * h)
        assert bench.halo_bytes(nx, ny, nz, h, 4, lid) == (3 * 2 * cells - zplanes) * 4


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_reading_needs_the_same_kernel(monkeypatch, tmp_path):
    """The committed counter readings count only while the headline kernel's
    sources and its table row are the ones they were taken on."""
    ent = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["pw_forward_f32_512x512x64"]
    monkeypatch.setattr(bench, "kernel_fingerprint", lambda: ent["source_sha256_16"])
    assert bench.measured_traffic("pw_forward_f32_512x512x64") == int(ent["traffic_bytes"])
    assert bench.measured_traffic("no_such_kernel") is None
    monkeypatch.setattr(bench, "kernel_fingerprint", lambda: "0" * 16)
    assert bench.measured_traffic("pw_forward_f32_512x512x64") is None


def test_fingerprint_follows_the_sources(monkeypatch, tmp_path):
    """A change to any hashed source, or to the headline row of the shape
    table, changes the fingerprint; other table rows do not."""
    import shutil
    csrc = os.path.join(ROOT, "paper_2301_13016_amd", "csrc")
    fake = tmp_path / "paper_2301_13016_amd" / "csrc"
    fake.mkdir(parents=True)
    for name in ("pw_stencil.h", "pw_forward_impl.h", "pw_forward_f32.hip", "pw_forward_lds_f32.hip",
                 "pw_tune_defaults.inc"):
        shutil.copy(os.path.join(csrc, name), fake / name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_fingerprint()
    inc = fake / "pw_tune_defaults.inc"
    text = inc.read_text()
    other = [ln for ln in text.splitlines() if ln.startswith("{0, 0, 10, 10, 8,")][0]
    inc.write_text(text.replace(other, other.replace("{0, 0, 10, 10, 8, 4,", "{0, 0, 10, 10, 8, 2,")))
    assert bench.kernel_fingerprint() == base                                # another row: same
    head = [ln for ln in text.splitlines() if ln.startswith("{0, 0, 9, 9, 6,")][0]
    changed = head.replace("{0, 0, 9, 9, 6, 4,", "{0, 0, 9, 9, 6, 2,")
    inc.write_text(text.replace(head, changed))                              # the headline row
    assert bench.kernel_fingerprint() != base
    inc.write_text(text)
    (fake / "pw_stencil.h").write_text((fake / "pw_stencil.h").read_text() + "\n// x\n")
    assert bench.kernel_fingerprint() != base


def test_unknown_form_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--forms", "precision,bogus"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "bogus" in r.stderr and r.stdout == ""
