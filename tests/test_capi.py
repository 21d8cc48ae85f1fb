"""Host-side checks of the C-ABI library (no GPU needed): symbols, validation, sizes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2509_08574_amd import cbct
    return cbct


def _declared():
    src = open(os.path.join(ROOT, "include", "cbct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("cbct_", "piccs_"))))


def test_every_declared_symbol_is_exported(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    declared = _declared()
    assert "cbct_forward" in declared and "piccs_krylov_solve" in declared
    for name in declared:
        assert hasattr(so, name), name
    assert sorted(lib.EXPORTS) == sorted(declared)


C1 = dict(nx=64, ny=64, nz=64, vx=1.0, vy=1.0, vz=1.0, nu=96, nv=96, du=1.5, dv=1.5,
          dso=1000.0, dsd=1536.0, n_views=48)


def test_geometry_sizes(lib):
    g = lib.Geometry(**C1)
    assert g.sizes() == (64 ** 3, 48 * 96 * 96)


@pytest.mark.parametrize("patch, msg", [
    (dict(nx=0), "sizes"),
    (dict(vz=-1.0), "voxel"),
    (dict(dsd=900.0), "DSO < DSD"),
    (dict(dso=50.0, dsd=100.0), "bounding sphere"),
    (dict(dsd=1040.0), "detector intersects"),
    (dict(nv=4000, dv=1.0), "cone angle"),
    (dict(du=0.0), "pitch"),
])
def test_invalid_geometry_is_rejected(lib, patch, msg):
    d = dict(C1)
    d.update(patch)
    with pytest.raises(lib.CbctError) as ei:
        lib.Geometry(**d)
    assert ei.value.code == lib.ERR_INVALID
    assert msg in str(ei.value)


def test_workspace_bytes_and_param_checks(lib):
    g = lib.Geometry(**C1)
    p = lib.SolveParams(1.0, 2.0, 0.1, 3, 5)
    n = lib.workspace_bytes(g, p)
    pad = (64 * 64 * 66 + 128) * 4
    assert n >= 13 * pad + 2 * 48 * 96 * 96 * 4
    assert n < 13 * pad + 2 * 48 * 96 * 96 * 4 + 8 * 1024 * 1024
    assert lib.workspace_bytes(g, lib.SolveParams(1.0, 2.0, 0.1, 3, 5,
                                                  method=lib.METHOD_PIPLE)) == n
    # reorthogonalisation keeps the outer step's n_inner v's as padded volumes
    nr = lib.workspace_bytes(g, lib.SolveParams(1.0, 2.0, 0.1, 3, 5, reorth=1))
    assert nr >= n + 5 * pad
    for bad in (lib.SolveParams(-1.0, 2.0, 0.1, 3, 5), lib.SolveParams(1.0, 2.0, 0.1, 0, 5),
                lib.SolveParams(1.0, 2.0, float("nan"), 3, 5),
                lib.SolveParams(1.0, 2.0, 0.1, 3, 5, method=2),
                lib.SolveParams(1.0, 2.0, 0.1, 3, 5, reorth=2)):
        with pytest.raises(lib.CbctError):
            lib.workspace_bytes(g, bad)


def test_precision_forms_and_their_workspace(lib):
    """The five precision forms are accepted; the *_ADJ16 forms add the 16-bit copy
    of u-hat (2 bytes per projection sample, 8 bytes of padding) to the mixed
    forms' workspace; an unknown form is rejected."""
    g = lib.Geometry(**C1)
    ws = {pr: lib.workspace_bytes(g, lib.SolveParams(1.0, 2.0, 0.1, 3, 5, precision=pr))
          for pr in (lib.PREC_FP32, lib.PREC_MIXED_BF16, lib.PREC_MIXED_F16,
                     lib.PREC_MIXED_BF16_ADJ16, lib.PREC_MIXED_F16_ADJ16)}
    assert ws[lib.PREC_MIXED_BF16] == ws[lib.PREC_MIXED_F16] > ws[lib.PREC_FP32]
    assert ws[lib.PREC_MIXED_BF16_ADJ16] == ws[lib.PREC_MIXED_F16_ADJ16]
    extra = ws[lib.PREC_MIXED_BF16_ADJ16] - ws[lib.PREC_MIXED_BF16]
    assert 2 * 48 * 96 * 96 + 8 <= extra <= 2 * 48 * 96 * 96 + 8 + 256
    for bad in (-1, 5):
        with pytest.raises(lib.CbctError):
            lib.workspace_bytes(g, lib.SolveParams(1.0, 2.0, 0.1, 3, 5, precision=bad))


def test_back_views_knob_is_validated(lib):
    g = lib.Geometry(**C1)
    for v in (0, 1, 7, 48, 1000):
        g.set_back_views(v)
    with pytest.raises(lib.CbctError) as ei:
        g.set_back_views(-1)
    assert ei.value.code == lib.ERR_INVALID
    so = ctypes.CDLL(lib.LIB_PATH)
    so.cbct_geom_set_back_views.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert so.cbct_geom_set_back_views(None, 4) == lib.ERR_INVALID


def test_null_arguments_are_rejected(lib):
    g = lib.Geometry(**C1)
    so = lib._lib
    assert so.cbct_forward(g.handle, None, 0, 1.0, None, None) == lib.ERR_INVALID
    assert "null" in lib.last_error()
    assert so.cbct_geom_sizes(None, None, None) == lib.ERR_INVALID


def _al(n):
    return (n + 255) // 256 * 256


def test_server_footprint_is_the_sum_of_its_buffers(lib):
    p = lib.SolveParams(1.0, 1.0, 0.1, 3, 10, precision=lib.PREC_MIXED_BF16)
    g = lib.Geometry(**C1)
    f = lib.server_footprint(C1, p)
    M, N = 64 ** 3, 48 * 96 * 96
    assert f["request"] == _al(4 * N) + _al(4 * M) + _al(lib.workspace_bytes(g, p))
    assert f["resident"] == 2 * _al(4 * M)
    # per (view, u): two float4/float2 coefficient entries, a segment header
    # and up to nx + ny - 1 + 4 segments of 8 bytes; per row / column / view a
    # few floats; each part padded to 256 bytes
    rays = 48 * 96
    core = rays * (16 + 8 + 8 + 8 * (64 + 64 - 1 + 4)) + 96 * (16 + 4) + 96 * 4 + 48 * 8
    assert core <= f["tables"] <= core + 8 * 256
    with pytest.raises(lib.CbctError) as ei:
        lib.server_footprint(dict(C1, nx=0), p)
    assert ei.value.code == lib.ERR_INVALID


def test_server_argument_checks(lib):
    so = lib._lib
    assert so.cbct_server_submit(None, None, None) == lib.ERR_INVALID
    assert so.cbct_server_poll(None, 1, None, None) == lib.ERR_INVALID
    assert so.cbct_server_stats_get(None, None) == lib.ERR_INVALID
    assert so.cbct_server_add_prior(None, 0, None, None) == lib.ERR_INVALID
    assert so.cbct_server_destroy(None) == lib.OK
    cfg = lib.ServerConfig(1 << 20, 0, 0, 0)
    h = ctypes.c_void_p()
    assert so.cbct_server_create(ctypes.byref(cfg), ctypes.byref(h)) == lib.ERR_INVALID
    assert "max_slots" in lib.last_error()


def test_server_create_without_a_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    cfg = lib.ServerConfig(1 << 20, 2, 0, 0)
    h = ctypes.c_void_p()
    rc = lib._lib.cbct_server_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc in (lib.ERR_INVALID, lib.ERR_DEVICE) and not h.value


def test_fdk_argument_checks(lib):
    g = lib.Geometry(**C1)
    so = lib._lib
    assert so.cbct_fdk(g.handle, None, None, None) == lib.ERR_INVALID
    wide = lib.Geometry(**dict(C1, nu=4800, du=0.03))
    assert so.cbct_fdk(wide.handle, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == \
        lib.ERR_INVALID
    assert "too long" in lib.last_error()
