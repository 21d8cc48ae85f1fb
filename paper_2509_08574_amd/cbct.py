"""Thin ctypes binding of ``libcbct.so`` (the C ABI declared in include/cbct.h).

Argument marshalling only: every step runs in the HIP library.  Device arrays
are torch tensors on a ROCm device (float32, contiguous); the current torch
stream is passed as the HIP stream.  There is no fallback: if the library is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbct.so")

OK, PENDING = 0, 1
ERR_INVALID, ERR_OOM, ERR_DEVICE, ERR_BUSY, ERR_NOT_FOUND, ERR_NUMERIC = -1, -2, -3, -4, -5, -6
F32, BF16, F16 = 0, 1, 2
PREC_FP32, PREC_MIXED_BF16, PREC_MIXED_F16 = 0, 1, 2
PREC_MIXED_BF16_ADJ16, PREC_MIXED_F16_ADJ16 = 3, 4
METHOD_PICCS, METHOD_PIPLE = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(python paper_2509_08574_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)

EXPORTS = ["cbct_last_error", "cbct_geom_create", "cbct_geom_destroy", "cbct_geom_sizes",
           "cbct_geom_nnz", "cbct_forward", "cbct_back", "piccs_weights",
           "piccs_workspace_bytes", "piccs_krylov_solve", "cbct_col_sizes", "cbct_vol_to_cols",
           "cbct_cols_to_vol", "cbct_proj_to_cols", "cbct_cols_to_proj", "cbct_forward_cols",
           "cbct_back_cols", "cbct_server_create", "cbct_server_add_prior", "cbct_server_submit",
           "cbct_server_poll", "cbct_server_stats_get", "cbct_server_destroy",
           "cbct_server_footprint", "cbct_fdk", "cbct_forward_noalloc",
           "cbct_geom_set_back_views"]


class GeomDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
        ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("dso", ctypes.c_double), ("dsd", ctypes.c_double),
        ("n_views", ctypes.c_int32),
        ("angles", ctypes.POINTER(ctypes.c_double)),
    ]


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("tau", ctypes.c_double), ("n_outer", ctypes.c_int32),
                ("n_inner", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reorth", ctypes.c_int32), ("method", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("inner_done", ctypes.c_int32), ("outer_done", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("resid_hist", ctypes.POINTER(ctypes.c_double))]


_vp = ctypes.c_void_p
_lib.cbct_last_error.restype = ctypes.c_char_p
_lib.cbct_geom_create.argtypes = [ctypes.POINTER(GeomDesc), ctypes.POINTER(_vp)]
_lib.cbct_geom_destroy.argtypes = [_vp]
_lib.cbct_geom_destroy.restype = None
_lib.cbct_geom_sizes.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]
_lib.cbct_geom_nnz.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), _vp]
_lib.cbct_geom_set_back_views.argtypes = [_vp, ctypes.c_int]
_lib.cbct_forward.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_float, _vp, _vp]
_lib.cbct_back.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_float, _vp, _vp]
_lib.cbct_forward_noalloc.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_float, _vp, _vp]
FORWARD_NOALLOC_MAX_BYTES = 256 << 20  # CBCT_FORWARD_NOALLOC_MAX_BYTES
_lib.piccs_weights.argtypes = [_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp]
_lib.piccs_workspace_bytes.argtypes = [_vp, ctypes.POINTER(Params),
                                       ctypes.POINTER(ctypes.c_size_t)]
_lib.piccs_krylov_solve.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(Params), _vp,
                                    ctypes.c_size_t, ctypes.POINTER(Report), _vp]


_lib.cbct_fdk.argtypes = [_vp, _vp, _vp, _vp]


def fdk(g: "Geometry", y: torch.Tensor, x: torch.Tensor | None = None, stream=None):
    """cbct_fdk: FDK reconstruction of line integrals y[view][v][u] into x[z][y][x]."""
    _need(y, g.proj_shape)
    if x is None:
        x = torch.empty(g.vol_shape, dtype=torch.float32, device=y.device)
    _need(x, g.vol_shape)
    _check(_lib.cbct_fdk(g.handle, _ptr(y), _ptr(x), _stream(stream)))
    return x


_i64p = ctypes.POINTER(ctypes.c_int64)
_lib.cbct_col_sizes.argtypes = [_vp, _i64p, _i64p, _i64p]
for _n in ("cbct_vol_to_cols", "cbct_cols_to_vol", "cbct_cols_to_proj", "cbct_forward_cols",
           "cbct_back_cols"):
    getattr(_lib, _n).argtypes = [_vp, _vp, _vp, _vp]
_lib.cbct_proj_to_cols.argtypes = [_vp, _vp, _vp, ctypes.c_int, _vp]


class CbctError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise CbctError(rc, _lib.cbct_last_error().decode())
    return rc


def last_error() -> str:
    return _lib.cbct_last_error().decode()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


_DT = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}


class Geometry:
    """Owning wrapper of a ``cbct_geom`` handle (see include/cbct.h for conventions)."""

    def __init__(self, nx, ny, nz, vx, vy, vz, nu, nv, du, dv, dso, dsd, n_views, angles=None):
        self.desc = GeomDesc(nx, ny, nz, vx, vy, vz, nu, nv, du, dv, dso, dsd, n_views, None)
        self._angles = None
        if angles is not None:
            arr = (ctypes.c_double * n_views)(*[float(a) for a in angles])
            self._angles = arr
            self.desc.angles = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
        h = _vp()
        _check(_lib.cbct_geom_create(ctypes.byref(self.desc), ctypes.byref(h)))
        self.handle = h
        self.vol_shape = (nz, ny, nx)
        self.proj_shape = (n_views, nv, nu)

    @classmethod
    def from_dict(cls, d):
        keys = ("nx", "ny", "nz", "vx", "vy", "vz", "nu", "nv", "du", "dv", "dso", "dsd",
                "n_views")
        return cls(**{k: d[k] for k in keys}, angles=d.get("angles"))

    def sizes(self):
        m, n = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.cbct_geom_sizes(self.handle, ctypes.byref(m), ctypes.byref(n)))
        return m.value, n.value

    def nnz(self, stream=None):
        v = ctypes.c_int64()
        _check(_lib.cbct_geom_nnz(self.handle, ctypes.byref(v), _stream(stream)))
        return v.value

    def set_back_views(self, views):
        """Views per launch of A^T (0 = automatic); results are the same bits."""
        _check(_lib.cbct_geom_set_back_views(self.handle, int(views)))

    def close(self):
        if getattr(self, "handle", None):
            _lib.cbct_geom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 -- interpreter shutdown
            pass


def _need(t, shape, dtypes=(torch.float32,)):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous device tensor")
    if tuple(t.shape) != tuple(shape) or t.dtype not in dtypes:
        raise ValueError(f"expected shape {shape} dtype in {dtypes}, got {tuple(t.shape)} "
                         f"{t.dtype}")


def forward(g: Geometry, x: torch.Tensor, y: torch.Tensor | None = None, x_scale=1.0,
            stream=None) -> torch.Tensor:
    """y = A x (cbct_forward)."""
    _need(x, g.vol_shape, tuple(_DT))
    if y is None:
        y = torch.empty(g.proj_shape, dtype=torch.float32, device=x.device)
    _need(y, g.proj_shape)
    _check(_lib.cbct_forward(g.handle, _ptr(x), _DT[x.dtype], float(x_scale), _ptr(y),
                             _stream(stream)))
    return y


def forward_noalloc(g: Geometry, x: torch.Tensor, y: torch.Tensor, x_scale=1.0,
                    stream=None) -> torch.Tensor:
    """y = A x (cbct_forward_noalloc: the library's fixed scratch array, no
    allocation; the geometry must already have been used on this device)."""
    _need(x, g.vol_shape, tuple(_DT))
    _need(y, g.proj_shape)
    _check(_lib.cbct_forward_noalloc(g.handle, _ptr(x), _DT[x.dtype], float(x_scale), _ptr(y),
                                     _stream(stream)))
    return y


def back(g: Geometry, y: torch.Tensor, x: torch.Tensor | None = None, y_scale=1.0,
         stream=None) -> torch.Tensor:
    """x = A^T y (cbct_back)."""
    _need(y, g.proj_shape, tuple(_DT))
    if x is None:
        x = torch.empty(g.vol_shape, dtype=torch.float32, device=y.device)
    _need(x, g.vol_shape)
    _check(_lib.cbct_back(g.handle, _ptr(y), _DT[y.dtype], float(y_scale), _ptr(x),
                          _stream(stream)))
    return x


def weights(g: Geometry, x, xp, tau, stream=None):
    """(w1, w2) TV weights (piccs_weights)."""
    _need(x, g.vol_shape)
    _need(xp, g.vol_shape)
    w1 = torch.empty_like(x)
    w2 = torch.empty_like(x)
    _check(_lib.piccs_weights(g.handle, _ptr(x), _ptr(xp), float(tau), _ptr(w1), _ptr(w2),
                              _stream(stream)))
    return w1, w2


@dataclass
class SolveParams:
    alpha: float
    lam: float
    tau: float
    n_outer: int
    n_inner: int
    precision: int = PREC_FP32
    reorth: int = 0
    method: int = 0  # METHOD_PICCS or METHOD_PIPLE

    def c(self):
        return Params(self.alpha, self.lam, self.tau, self.n_outer, self.n_inner,
                      self.precision, self.reorth, self.method)


def workspace_bytes(g: Geometry, p: SolveParams) -> int:
    v = ctypes.c_size_t()
    cp = p.c()
    _check(_lib.piccs_workspace_bytes(g.handle, ctypes.byref(cp), ctypes.byref(v)))
    return v.value


def alloc_workspace(g: Geometry, p: SolveParams, device="cuda"):
    n = workspace_bytes(g, p)
    return torch.empty(n + 256, dtype=torch.uint8, device=device)


def _aligned(ws: torch.Tensor):
    base = ws.data_ptr()
    off = (-base) % 256
    return base + off, ws.numel() - off


def solve(g: Geometry, b, xp, x, p: SolveParams, workspace=None, report=True, stream=None):
    """piccs_krylov_solve; x is updated in place.  Returns (x, report dict or None)."""
    _need(b, g.proj_shape)
    _need(xp, g.vol_shape)
    _need(x, g.vol_shape)
    if workspace is None:
        workspace = alloc_workspace(g, p, device=x.device)
    wp, wn = _aligned(workspace)
    cp = p.c()
    rep = None
    hist = None
    if report:
        nh = p.n_outer * p.n_inner
        hist = (ctypes.c_double * nh)()
        rep = Report(0, 0, 0, ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)))
    _check(_lib.piccs_krylov_solve(g.handle, _ptr(b), _ptr(xp), _ptr(x), ctypes.byref(cp),
                                   ctypes.c_void_p(wp), ctypes.c_size_t(wn),
                                   ctypes.byref(rep) if rep is not None else None,
                                   _stream(stream)))
    if rep is None:
        return x, None
    return x, {"inner_done": rep.inner_done, "outer_done": rep.outer_done,
               "breakdown": rep.breakdown, "phibar": list(hist)}


# ---------------------------------------------------------------- column layout

def col_sizes(g: Geometry):
    """(vol_floats, vol_offset, proj_floats) of the kernels' native layouts."""
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.cbct_col_sizes(g.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def vol_to_cols(g: Geometry, x, cols=None, stream=None):
    _need(x, g.vol_shape)
    vf, _, _ = col_sizes(g)
    if cols is None:
        cols = torch.empty(vf, dtype=torch.float32, device=x.device)
    _check(_lib.cbct_vol_to_cols(g.handle, _ptr(x), _ptr(cols), _stream(stream)))
    return cols


def cols_to_vol(g: Geometry, cols, x=None, stream=None):
    if x is None:
        x = torch.empty(g.vol_shape, dtype=torch.float32, device=cols.device)
    _check(_lib.cbct_cols_to_vol(g.handle, _ptr(cols), _ptr(x), _stream(stream)))
    return x


def proj_to_cols(g: Geometry, y, ycols=None, weighted=False, stream=None):
    _need(y, g.proj_shape)
    if ycols is None:
        ycols = torch.empty(y.numel(), dtype=torch.float32, device=y.device)
    _check(_lib.cbct_proj_to_cols(g.handle, _ptr(y), _ptr(ycols), int(bool(weighted)),
                                  _stream(stream)))
    return ycols


def cols_to_proj(g: Geometry, ycols, y=None, stream=None):
    if y is None:
        y = torch.empty(g.proj_shape, dtype=torch.float32, device=ycols.device)
    _check(_lib.cbct_cols_to_proj(g.handle, _ptr(ycols), _ptr(y), _stream(stream)))
    return y


def forward_cols(g: Geometry, cols, ycols, stream=None):
    _check(_lib.cbct_forward_cols(g.handle, _ptr(cols), _ptr(ycols), _stream(stream)))
    return ycols


def back_cols(g: Geometry, ywcols, cols, stream=None):
    _check(_lib.cbct_back_cols(g.handle, _ptr(ywcols), _ptr(cols), _stream(stream)))
    return cols


# ---------------------------------------------------------------- serving

X0_PREVIOUS, X0_PRIOR = 0, 1


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("device", ctypes.c_int32), ("max_queue", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("patient", ctypes.c_int32), ("geom", GeomDesc),
                ("b_host", ctypes.POINTER(ctypes.c_float)), ("params", Params),
                ("x0", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("report", Report)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "capacity", "used", "peak_used", "resident", "queued", "in_flight", "peak_in_flight",
        "done_unpolled", "completed", "failed", "geom_placements", "geom_evictions")]


_lib.cbct_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]
_lib.cbct_server_add_prior.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(GeomDesc), _vp]
_lib.cbct_server_submit.argtypes = [_vp, ctypes.POINTER(Request),
                                    ctypes.POINTER(ctypes.c_uint64)]
_lib.cbct_server_poll.argtypes = [_vp, ctypes.c_uint64, _vp, ctypes.POINTER(Result)]
_lib.cbct_server_stats_get.argtypes = [_vp, ctypes.POINTER(ServerStats)]
_lib.cbct_server_destroy.argtypes = [_vp]
_szp = ctypes.POINTER(ctypes.c_size_t)
_lib.cbct_server_footprint.argtypes = [ctypes.POINTER(GeomDesc), ctypes.POINTER(Params), _szp,
                                       _szp, _szp]


def server_footprint(geom: dict, params: SolveParams) -> dict:
    """Device bytes per running request, per cached geometry and per patient."""
    desc, _keep = _desc(geom)
    cp = params.c()
    r, t, p = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.cbct_server_footprint(ctypes.byref(desc), ctypes.byref(cp), ctypes.byref(r),
                                      ctypes.byref(t), ctypes.byref(p)))
    return {"request": r.value, "tables": t.value, "resident": p.value}


def _desc(d):
    """GeomDesc from a geometry dict; returns (desc, keep-alive angles array)."""
    keys = ("nx", "ny", "nz", "vx", "vy", "vz", "nu", "nv", "du", "dv", "dso", "dsd", "n_views")
    desc = GeomDesc(*[d[k] for k in keys], None)
    arr = None
    if d.get("angles") is not None:
        arr = (ctypes.c_double * d["n_views"])(*[float(a) for a in d["angles"]])
        desc.angles = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
    return desc, arr


def _host_f32(a, n):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != n:
        raise ValueError(f"expected {n} elements, got {a.size}")
    return a


class Server:
    """cbct_server_*: continuous batching of IRN-PICCS requests on one device.

    Host arrays are numpy float32 (copied by the library at submit / add_prior).
    """

    def __init__(self, hbm_budget_bytes=0, max_slots=4, device=0, max_queue=0):
        cfg = ServerConfig(hbm_budget_bytes, max_slots, device, max_queue)
        h = _vp()
        _check(_lib.cbct_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._nvox = {}

    def add_prior(self, patient: int, geom: dict, xp):
        desc, _keep = _desc(geom)
        n = geom["nx"] * geom["ny"] * geom["nz"]
        a = _host_f32(xp, n)
        _check(_lib.cbct_server_add_prior(self.handle, patient, ctypes.byref(desc),
                                          ctypes.c_void_p(a.ctypes.data)))
        self._nvox[patient] = n

    def submit(self, patient: int, geom: dict, b, params: SolveParams, x0=X0_PREVIOUS) -> int:
        """Returns the ticket; raises CbctError (code ERR_BUSY / ERR_OOM / ...) on refusal."""
        desc, _keep = _desc(geom)
        n = geom["n_views"] * geom["nu"] * geom["nv"]
        a = _host_f32(b, n)
        req = Request(patient, desc, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                      params.c(), x0)
        t = ctypes.c_uint64()
        _check(_lib.cbct_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, out=None, hist_len: int = 0):
        """Returns None while pending; else (status, x or None, result dict)."""
        res = Result()
        hist = None
        if hist_len:
            hist = (ctypes.c_double * hist_len)()
            res.report.resid_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        rc = _lib.cbct_server_poll(self.handle, ticket,
                                   ctypes.c_void_p(out.ctypes.data) if out is not None else None,
                                   ctypes.byref(res))
        if rc == PENDING:
            return None
        if rc == ERR_NOT_FOUND:  # unknown or already collected ticket
            raise CbctError(rc, last_error())
        info = {"status": res.status, "t_submit": res.t_submit, "t_admit": res.t_admit,
                "t_done": res.t_done, "inner_done": res.report.inner_done,
                "outer_done": res.report.outer_done, "breakdown": res.report.breakdown,
                "error": last_error() if rc != OK else ""}
        if hist is not None:
            info["phibar"] = list(hist)
        return rc, out, info

    def wait(self, ticket: int, out=None, hist_len: int = 0, timeout: float = 120.0,
             interval: float = 2e-4):
        import time
        t_end = time.monotonic() + timeout
        while True:
            r = self.poll(ticket, out, hist_len)
            if r is not None:
                return r
            if time.monotonic() > t_end:
                raise TimeoutError(f"ticket {ticket} not done after {timeout} s")
            time.sleep(interval)

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.cbct_server_stats_get(self.handle, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            h, self.handle = self.handle, None
            _check(_lib.cbct_server_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
