"""GPU test of the allocation-free coefficient-gradient entry point
(pw_advect_coeff_grad_static), called through the C ABI.

It runs the same kernels as pw_advect_coeff_grad with the library's static
device scratch in place of the caller's workspace, so its result must equal
that entry point's bit for bit: checked on two calls in a row, the second on
a smaller grid (the scratch keeps the first call's partials, which the second
must not see), and against the FP64 oracle at the FP32 bar.  Device memory
free before and after the calls must not change.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2301_13016_amd import binding as B
from paper_2301_13016_amd import workloads as wl
from scales import coeff_grad_scale

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture(autouse=True)
def _announce(request):
    sys.__stderr__.write("\n[gpu-test] %s\n" % request.node.nodeid)
    sys.__stderr__.flush()
    yield


def _case(nx, ny, nz, seed, dtype):
    g = wl.make_grid(nx, ny, nz, seed=seed, dtype=dtype)
    r = wl.cotangents(nx, ny, nz, seed=seed + 1, dtype=dtype)
    dev = lambda xs: [torch.from_numpy(np.ascontiguousarray(x)).to("cuda") for x in xs]  # noqa: E731
    return g, r, dev((g.u, g.v, g.w)), dev(r)


def _raw_args(u, r):
    grid = B.pw_grid(u.shape[2] - 2, u.shape[1] - 2, u.shape[0] - 2, 1)
    layout = B.pw_layout(u.stride(1), u.stride(0), r[0].stride(1), r[0].stride(0))
    return grid, layout


def _with_workspace(x, r, out, stream):
    grid, layout = _raw_args(x[0], r)
    dt = B.PW_F64 if x[0].dtype == torch.float64 else B.PW_F32
    need = ctypes.c_int64()
    assert B.lib().pw_advect_coeff_grad_workspace(ctypes.byref(grid), dt, ctypes.byref(need)) == B.PW_OK
    ws = torch.empty(max(1, need.value // 8), dtype=torch.float64, device="cuda")
    st = B.lib().pw_advect_coeff_grad(ctypes.byref(grid), ctypes.byref(layout), dt,
                                      *(t.data_ptr() for t in x), *(t.data_ptr() for t in r),
                                      out.data_ptr(), ws.data_ptr(), need.value, stream)
    assert st == B.PW_OK, B.pw_last_error()
    torch.cuda.synchronize()
    return ws


def _static(x, r, out, stream):
    grid, layout = _raw_args(x[0], r)
    dt = B.PW_F64 if x[0].dtype == torch.float64 else B.PW_F32
    st = B.pw_advect_coeff_grad_static(grid, layout, dt, *(t.data_ptr() for t in x), *(t.data_ptr() for t in r),
                                       out.data_ptr(), stream)
    assert st == B.PW_OK, B.pw_last_error()


def _check_oracle(got, g, r):
    names = ("tzc1", "tzc2", "tzd1", "tzd2", "tcx_level", "tcy_level")
    nz = g.nz
    ref = oracle.coeff_grad(g.u, g.v, g.w, *[np.asarray(x, np.float64) for x in r])
    mag = coeff_grad_scale(g.u, g.v, g.w, r, nz)
    gh = got.cpu().numpy()
    for i, n in enumerate(names[:4]):
        assert np.all(np.abs(gh[i * nz:(i + 1) * nz] - ref[n]) <= 1e-6 * mag[n]), n
    for i, n in ((6 * nz, "tcx"), (6 * nz + 1, "tcy")):
        assert abs(gh[i] - ref[n]) <= 1e-6 * mag[n], n


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_static_scratch_equals_workspace_entry_point(dtype):
    big = _case(200, 70, 24, seed=950, dtype=dtype)
    small = _case(70, 9, 5, seed=960, dtype=dtype)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    refs = []
    for g, r, x, rd in (big, small):
        out = torch.empty(6 * g.nz + 2, dtype=torch.float64, device="cuda")
        _with_workspace(x, rd, out, stream)
        refs.append(out)
    torch.cuda.synchronize()
    outs = [torch.full((6 * g.nz + 2,), float("nan"), dtype=torch.float64, device="cuda") for g, *_ in (big, small)]
    free0 = torch.cuda.mem_get_info()[0]
    for (g, r, x, rd), out in zip((big, small), outs):     # two calls in a row, the second smaller
        _static(x, rd, out, stream)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0
    for (g, r, _, _), out, ref in zip((big, small), outs, refs):
        assert torch.equal(out, ref)
        _check_oracle(out, g, r)
    # the binding's path with a given output allocates nothing either
    again = torch.empty_like(outs[1])
    g, r, x, rd = small
    B.advect_coeff_grad(*x, *rd, out=again, static_scratch=True)
    torch.cuda.synchronize()
    assert torch.equal(again, refs[1])


def test_static_scratch_rejects_oversized_grids():
    g, r, x, rd = _case(40, 8, 4, seed=970, dtype=np.float32)
    grid = B.pw_grid(4096, 2048, 64, 1)   # 67 x 2050 strips x 64 levels x 48 B = 403 MiB of partials
    layout = B.pw_layout(4098, 4098 * 2050, 4096, 4096 * 2048)
    out = torch.empty(6 * 64 + 2, dtype=torch.float64, device="cuda")
    st = B.pw_advect_coeff_grad_static(grid, layout, B.PW_F32, *(t.data_ptr() for t in x),
                                       *(t.data_ptr() for t in rd), out.data_ptr(), None)
    assert st == B.PW_ERR_UNSUPPORTED and "static scratch" in B.pw_last_error()
