"""The allocation-free entry point (lens_deflect_noalloc), called through the
C ABI, against lens_deflect with the same plan: bit-for-bit equal outputs on
two calls in a row, the second with a smaller grid.  The first grid is the
1e6-star benchmark field at p = 16, whose per-call buffers (~90 MB) exceed
the entry point's 64 MiB, so it runs in row bands."""
import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _call(lib, fn, *args):
    from paper_2211_00354_amd import _lib
    _lib.check(getattr(lib, fn)(*args))


def test_noalloc_matches_lens_deflect(lf):
    import torch
    from paper_2211_00354_amd import _lib
    lib = _lib.load()
    f, g = wl.powerlaw_disk()
    xy = torch.from_numpy(f.xy).cuda()
    m = torch.from_numpy(f.m).cuda()
    grid = lf.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny)
    print("[case] noalloc plan: 1e6 stars, 8192^2 grid, mixed p=16", flush=True)
    plan = lf.Plan(xy, m, kappa_s=f.kappa_s, gamma=f.gamma, grid=grid, precision="mixed", p=16)
    o = lf._opts("fmm", "mixed", 16)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    small = lf.Grid(g.x0 + 1000 * g.dx, g.y0 + 3000 * g.dy, g.dx, g.dy, 1000, 700)
    for k, gr in enumerate((grid, small)):
        n = gr.nx * gr.ny
        ref = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda")
        out = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda")
        gc = gr.c()
        print(f"[case] noalloc call {k}: {gr.nx}x{gr.ny}", flush=True)
        _call(lib, "lens_deflect", plan.handle, None, ctypes.byref(gc), None, n, ref.data_ptr(),
              None, ctypes.byref(o), stream)
        _call(lib, "lens_deflect_noalloc", plan.handle, None, ctypes.byref(gc), out.data_ptr(),
              ctypes.byref(o), stream)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        np.testing.assert_array_equal(a, b)
        del ref, out
    # rays outside the plan's region are refused before anything is enqueued
    far = lf.Grid(g.x0 - 5000.0, g.y0, g.dx, g.dy, 16, 16)
    fc = far.c()
    buf = torch.zeros((256, 2), dtype=torch.float64, device="cuda")
    st = lib.lens_deflect_noalloc(plan.handle, None, ctypes.byref(fc), buf.data_ptr(),
                                  ctypes.byref(o), stream)
    assert st == _lib.LENS_EINVAL
    assert bool((buf == 0).all())
    plan.close()
