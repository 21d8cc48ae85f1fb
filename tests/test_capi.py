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
    for bad in (lib.SolveParams(-1.0, 2.0, 0.1, 3, 5), lib.SolveParams(1.0, 2.0, 0.1, 0, 5),
                lib.SolveParams(1.0, 2.0, float("nan"), 3, 5)):
        with pytest.raises(lib.CbctError):
            lib.workspace_bytes(g, bad)


def test_null_arguments_are_rejected(lib):
    g = lib.Geometry(**C1)
    so = lib._lib
    assert so.cbct_forward(g.handle, None, 0, 1.0, None, None) == lib.ERR_INVALID
    assert "null" in lib.last_error()
    assert so.cbct_geom_sizes(None, None, None) == lib.ERR_INVALID
