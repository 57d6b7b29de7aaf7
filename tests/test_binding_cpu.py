"""CPU tests of the Python binding's argument checks (no GPU, no library call).

The C ABI sizes every buffer from the grid, the storage dtype and the first
output's strides, so a tensor of the wrong shape, dtype or layout that reached
it would be read or written out of bounds.  The binding therefore checks every
tensor it passes -- outputs, gradients, directions, cotangents, addends and the
coefficient arrays -- before any call into the library.  Here the library
entry point is replaced by a sentinel: a rejected call must raise ValueError
without reaching it, and a valid call must reach it.
"""
import types

import pytest

torch = pytest.importorskip("torch")

from paper_2301_13016_amd import binding as B  # noqa: E402


class Reached(Exception):
    pass


@pytest.fixture(autouse=True)
def no_library(monkeypatch):
    def fake():
        raise Reached()
    monkeypatch.setattr(B, "lib", fake)


STREAM = types.SimpleNamespace(cuda_stream=0)
NX, NY, NZ = 6, 5, 4


def winds(dtype=torch.float32, device="cpu", halo=1):
    shp = (NZ + 2 * halo, NY + 2 * halo, NX + 2 * halo)
    return [torch.zeros(shp, dtype=dtype, device=device) for _ in range(3)]


def coeffs(dtype=torch.float32, nz=NZ, device="cpu"):
    mk = lambda: torch.ones(nz, dtype=dtype, device=device)  # noqa: E731
    return B.Coeffs(0.0025, 0.0025, mk(), mk(), mk(), mk())


def interior(dtype=torch.float32, n=3, device="cpu"):
    return [torch.zeros((NZ, NY, NX), dtype=dtype, device=device) for _ in range(n)]


def test_valid_calls_reach_the_library():
    u, v, w = winds()
    c = coeffs()
    calls = [
        lambda: B.advect(u, v, w, c, stream=STREAM),
        lambda: B.advect(u, v, w, c, out=interior(), stream=STREAM),
        lambda: B.advect_epilogue(u, v, w, c, interior(), stream=STREAM),
        lambda: B.advect_bc(u, v, w, c, ("periodic", "periodic", "copy"), stream=STREAM),
        lambda: B.advect_adjoint(u, v, w, c, *interior(), stream=STREAM),
        lambda: B.advect_tangent(u, v, w, c, *winds(), stream=STREAM),
        lambda: B.advect_coeff_grad(u, v, w, *interior(), stream=STREAM),
        lambda: B.advect_adjoint_coeff_grad(u, v, w, c, *interior(), stream=STREAM),
        lambda: B.advect_bc(u, v, w, c, [("periodic", "periodic", "copy")] * 2 + [("periodic", "periodic", "zero")],
                            stream=STREAM),
        lambda: B.halo_fill([u, v, w], ("periodic",) * 3, stream=STREAM),
        lambda: B.Batch([(u, v, w, c, interior())]),
    ]
    for call in calls:
        with pytest.raises(Reached):
            call()
    zu, zv, zw = (x.permute(2, 1, 0).contiguous() for x in (u, v, w))
    zo = [torch.zeros((NX, NY, NZ)) for _ in range(3)]
    with pytest.raises(Reached):
        B.advect_zfast(zu, zv, zw, c, stream=STREAM)
    with pytest.raises(Reached):
        B.advect_zfast_epilogue(zu, zv, zw, c, zo, stream=STREAM)
    # FP64 grids with FP64 coefficients, 16-bit storage with FP32 coefficients
    with pytest.raises(Reached):
        B.advect(*winds(torch.float64), coeffs(torch.float64), stream=STREAM)
    with pytest.raises(Reached):
        B.advect(*winds(torch.bfloat16), coeffs(), stream=STREAM)


@pytest.mark.parametrize("bad", ["bf16", "shape", "strides", "device", "f64"])
def test_forward_outputs_checked(bad):
    u, v, w = winds()
    out = interior()
    if bad == "bf16":
        out[1] = out[1].to(torch.bfloat16)
    elif bad == "shape":
        out[2] = torch.zeros((NZ, NY, NX - 1))
    elif bad == "strides":
        out[0] = torch.zeros((NZ, NY, NX + 2))[:, :, :NX]
    elif bad == "device":
        out[0] = torch.zeros((NZ, NY, NX), device="meta")
    else:
        out = interior(torch.float64)
    with pytest.raises(ValueError):
        B.advect(u, v, w, coeffs(), out=out, stream=STREAM)


@pytest.mark.parametrize("bad", ["dtype", "short", "strided", "device"])
def test_coefficients_checked(bad):
    u, v, w = winds()
    c = coeffs()
    if bad == "dtype":
        c.tzd1 = c.tzd1.double()
    elif bad == "short":
        c.tzc2 = c.tzc2[:NZ - 1]
    elif bad == "strided":
        c.tzc1 = torch.ones(2 * NZ)[::2]
    else:
        c.tzd2 = torch.ones(NZ, device="meta")
    with pytest.raises(ValueError):
        B.advect(u, v, w, c, stream=STREAM)
    with pytest.raises(ValueError):
        B.advect_adjoint(u, v, w, c, *interior(), stream=STREAM)
    with pytest.raises(ValueError):
        B.advect_tangent(u, v, w, c, *winds(), stream=STREAM)


def test_fp64_grid_needs_fp64_coefficients():
    with pytest.raises(ValueError):
        B.advect(*winds(torch.float64), coeffs(torch.float32), stream=STREAM)
    with pytest.raises(ValueError):
        B.advect(*winds(torch.float32), coeffs(torch.float64), stream=STREAM)


def test_inputs_must_agree():
    u, v, w = winds()
    with pytest.raises(ValueError):
        B.advect(u, v.double(), w, coeffs(), stream=STREAM)
    with pytest.raises(ValueError):
        B.advect(u, v, torch.zeros_like(w, device="meta"), coeffs(), stream=STREAM)
    with pytest.raises(ValueError):
        B.advect(u[0], v[0], w[0], coeffs(), stream=STREAM)


@pytest.mark.parametrize("bad", ["cot_shape", "cot_dtype", "grad_dtype", "grad_shape", "grad_strides"])
def test_adjoint_arguments_checked(bad):
    u, v, w = winds()
    r = interior()
    g = [torch.zeros_like(u) for _ in range(3)]
    if bad == "cot_shape":
        r[1] = torch.zeros((NZ, NY + 1, NX))
    elif bad == "cot_dtype":
        r[2] = r[2].double()
    elif bad == "grad_dtype":
        g[1] = g[1].to(torch.float16)
    elif bad == "grad_shape":
        g[0] = torch.zeros((NZ + 2, NY + 2, NX + 1))
    else:
        g[2] = torch.zeros((NZ + 2, NY + 2, NX + 3))[:, :, :NX + 2]
    with pytest.raises(ValueError):
        B.advect_adjoint(u, v, w, coeffs(), *r, out=g, stream=STREAM)


@pytest.mark.parametrize("bad", ["dir_dtype", "out_dtype", "out_shape"])
def test_tangent_arguments_checked(bad):
    u, v, w = winds()
    d = winds()
    out = interior()
    if bad == "dir_dtype":
        d[0] = d[0].double()
    elif bad == "out_dtype":
        out[1] = out[1].to(torch.bfloat16)
    else:
        out[2] = torch.zeros((NZ - 1, NY, NX))
    with pytest.raises(ValueError):
        B.advect_tangent(u, v, w, coeffs(), *d, out=out, stream=STREAM)


@pytest.mark.parametrize("bad", ["cot_shape", "grad_dtype", "grad_out_len", "grad_out_dtype", "coeff_len"])
def test_fused_backward_arguments_checked(bad):
    u, v, w = winds()
    r = interior()
    g = [torch.zeros_like(u) for _ in range(3)]
    c = coeffs()
    go = torch.zeros(6 * NZ + 2, dtype=torch.float64)
    if bad == "cot_shape":
        r[0] = torch.zeros((NZ, NY, NX + 1))
    elif bad == "grad_dtype":
        g[2] = g[2].double()
    elif bad == "grad_out_len":
        go = torch.zeros(6 * NZ + 1, dtype=torch.float64)
    elif bad == "grad_out_dtype":
        go = torch.zeros(6 * NZ + 2, dtype=torch.float32)
    else:
        c = coeffs(nz=NZ - 1)
    with pytest.raises(ValueError):
        B.advect_adjoint_coeff_grad(u, v, w, c, *r, out=g, grad_out=go, stream=STREAM)


def test_bc_rules_checked():
    u, v, w = winds()
    with pytest.raises(ValueError):
        B.advect_bc(u, v, w, coeffs(), ("periodic", "sideways", "copy"), stream=STREAM)
    with pytest.raises(ValueError):
        B.advect_bc(u, v, w, coeffs(), [("periodic",) * 3] * 2, stream=STREAM)   # two triples for three fields


def test_coeff_grad_cotangents_checked():
    u, v, w = winds()
    r = interior()
    r[0] = torch.zeros((NZ, NY, NX + 1))
    with pytest.raises(ValueError):
        B.advect_coeff_grad(u, v, w, *r, stream=STREAM)
    with pytest.raises(ValueError):
        B.advect_coeff_grad(u, v, w, *interior(torch.float64), stream=STREAM)


def test_epilogue_and_bc_addends_checked():
    u, v, w = winds()
    a = interior()
    a[1] = a[1].double()
    with pytest.raises(ValueError):
        B.advect_epilogue(u, v, w, coeffs(), a, stream=STREAM)
    with pytest.raises(ValueError):
        B.advect_bc(u, v, w, coeffs(), ("periodic",) * 3, addends=a, stream=STREAM)
    short = interior()
    short[0] = torch.zeros((NZ, NY, NX - 2))
    with pytest.raises(ValueError):
        B.advect_epilogue(u, v, w, coeffs(), short, stream=STREAM)


def test_zfast_outputs_checked():
    u, v, w = (x.permute(2, 1, 0).contiguous() for x in winds())
    bad = [torch.zeros((NX, NY, NZ)) for _ in range(3)]
    bad[1] = torch.zeros((NZ, NY, NX))            # x-fastest shape for a z-fastest call
    with pytest.raises(ValueError):
        B.advect_zfast(u, v, w, coeffs(), out=bad, stream=STREAM)
    with pytest.raises(ValueError):
        B.advect_zfast_epilogue(u, v, w, coeffs(), bad, stream=STREAM)


def test_batch_subdomains_checked():
    u, v, w = winds()
    out = interior()
    out[2] = out[2].to(torch.float16)
    with pytest.raises(ValueError):
        B.Batch([(u, v, w, coeffs(), out)])
    with pytest.raises(ValueError):
        B.Batch([(*winds(torch.float64), coeffs(torch.float64), interior(torch.float64))])
    with pytest.raises(ValueError):
        B.Batch([(u, v, w, coeffs(nz=NZ - 1), interior())])


def test_halo_fields_checked():
    u, v, w = winds()
    with pytest.raises(ValueError):
        B.halo_fill([u, v.double()], ("periodic",) * 3, stream=STREAM)
    with pytest.raises(ValueError):
        B.halo_fill([u, torch.zeros_like(v, device="meta")], ("periodic",) * 3, stream=STREAM)


def test_one_cell_grid_passes():
    u = [torch.zeros((3, 3, 3)) for _ in range(3)]
    with pytest.raises(Reached):
        B.advect(*u, coeffs(nz=1), stream=STREAM)
