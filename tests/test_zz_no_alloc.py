"""cbct_forward_noalloc (the allocation-free forward projection) against
cbct_forward, through the C ABI.

Both run the same kernels on the same inputs, so the results must be equal bit
for bit.  Two no-alloc calls in a row, the second on a smaller geometry, check
that what the first left in the shared scratch array does not leak into the
second; host-side rejections (size, tables not yet on the device) enqueue
nothing.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BIG = dict(nx=64, ny=64, nz=64, vx=1.0, vy=1.0, vz=1.0, nu=96, nv=96, du=1.5, dv=1.5,
           dso=1000.0, dsd=1536.0, n_views=48)
SMALL = dict(nx=21, ny=19, nz=17, vx=1.0, vy=1.1, vz=0.9, nu=40, nv=30, du=1.3, dv=1.2,
             dso=400.0, dsd=620.0, n_views=11)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_08574_amd import cbct
    return cbct


def _raw_noalloc(lib, g, x, y, scale=1.0):
    import torch
    dt = {torch.float32: lib.F32, torch.bfloat16: lib.BF16, torch.float16: lib.F16}[x.dtype]
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib._lib.cbct_forward_noalloc(g.handle, ctypes.c_void_p(x.data_ptr()), dt,
                                         ctypes.c_float(scale), ctypes.c_void_p(y.data_ptr()), s)


def test_noalloc_matches_cbct_forward_twice_in_a_row(lib):
    import torch
    print("no-alloc: 64^3/48 views then 21x19x17/11 views, f32 and bf16", flush=True)
    gb, gs = lib.Geometry(**BIG), lib.Geometry(**SMALL)
    rng = np.random.default_rng(11)
    xb = torch.from_numpy(rng.uniform(size=gb.vol_shape).astype(np.float32)).cuda()
    xs = torch.from_numpy(rng.uniform(size=gs.vol_shape).astype(np.float32)).cuda()
    # reference results (these calls also place both geometries' tables)
    rb = lib.forward(gb, xb)
    rs = lib.forward(gs, xs)
    yb = torch.full(gb.proj_shape, float("nan"), device="cuda")
    ys = torch.full(gs.proj_shape, float("nan"), device="cuda")
    assert _raw_noalloc(lib, gb, xb, yb) == lib.OK, lib.last_error()
    assert _raw_noalloc(lib, gs, xs, ys) == lib.OK, lib.last_error()
    torch.cuda.synchronize()
    assert torch.equal(yb, rb)
    assert torch.equal(ys, rs)
    # 16-bit input with a scale, again large then small
    xb16, xs16 = xb.to(torch.bfloat16), xs.to(torch.float16)
    rb16 = lib.forward(gb, xb16, x_scale=0.5)
    rs16 = lib.forward(gs, xs16, x_scale=2.0)
    yb.fill_(float("nan"))
    ys.fill_(float("nan"))
    assert _raw_noalloc(lib, gb, xb16, yb, 0.5) == lib.OK, lib.last_error()
    assert _raw_noalloc(lib, gs, xs16, ys, 2.0) == lib.OK, lib.last_error()
    torch.cuda.synchronize()
    assert torch.equal(yb, rb16)
    assert torch.equal(ys, rs16)
    # the binding marshals to the same symbol
    assert torch.equal(lib.forward_noalloc(gs, xs, torch.empty_like(ys)), rs)


def test_noalloc_rejections_enqueue_nothing(lib):
    import torch
    # tables not yet on this device: a fresh geometry handle
    g = lib.Geometry(**dict(SMALL, n_views=7))
    x = torch.zeros(g.vol_shape, device="cuda")
    y = torch.full(g.proj_shape, 3.0, device="cuda")
    assert _raw_noalloc(lib, g, x, y) == lib.ERR_INVALID
    assert "tables" in lib.last_error()
    torch.cuda.synchronize()
    assert bool((y == 3.0).all())
    # temporaries beyond the fixed array: 256^3 with 720 views of 512^2 (never
    # launched; the size is checked on the host first)
    big = lib.Geometry(nx=256, ny=256, nz=256, vx=1.0, vy=1.0, vz=1.0, nu=512, nv=512,
                       du=0.8, dv=0.8, dso=1000.0, dsd=1536.0, n_views=720)
    rc = lib._lib.cbct_forward_noalloc(big.handle, ctypes.c_void_p(256), lib.F32,
                                       ctypes.c_float(1.0), ctypes.c_void_p(256), None)
    assert rc == lib.ERR_INVALID
    assert "scratch" in lib.last_error()
    # null arguments
    assert lib._lib.cbct_forward_noalloc(g.handle, None, lib.F32, ctypes.c_float(1.0), None,
                                         None) == lib.ERR_INVALID
