"""TEST INFRASTRUCTURE -- reference oracle, not part of the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg
may import this module.  It shares no code with the HIP path: the projector
lives in ``oracle/siddon.c`` (plain FP64 Siddon, built by ``oracle/build.py``),
everything else here is plain NumPy in float64.

What it computes, and where the paper defines it:

* ``forward`` / ``back``: the sensing matrix A of the linear CT model and its
  literal transpose (Sec. 2.1, eq. "tomo"; Sec. 2.2.2: Krylov solvers only
  use products with A and A^T).  Exact ray-driven chord lengths.
* ``D`` / ``DT``: the 3-D forward-difference operator D = [D_x; D_y; D_z] built
  from the 1-D matrix D_1 with rows (1, -1) (Sec. 2.2.1).  Reading: D_1 is
  padded with a zero last row so that the three directional differences live
  on the same voxel grid (the isotropic TV of eq. "TV1" adds them entry-wise).
* ``weights``: [W*]_ii = (sqrt(g_x^2 + g_y^2 + g_z^2) + tau^2)^(-1/2) of the
  smoothed TV (Sec. 2.2.1, definition of W~*), one weight per voxel shared by
  the three directions.
* ``aug_forward`` / ``aug_back`` / ``aug_rhs``: the augmented least-squares
  system A~ = [A; alpha W1 D; lambda W2 D], b~ = [b; 0; lambda W2 D x_p]
  (Sec. 2.2.2, the augmented problem equivalent to eq. "PICCS_rec").
* ``lsqr``: Paige & Saunders' LSQR (ACM TOMS 8(1), 1982), the inner Krylov
  solver named in Sec. 2.2.2; ``cgls``: the mathematically equivalent CGLS.
* ``irn_piccs``: the IRN outer loop of eq. "PICCS_rec" with
  W1_k = W~(D x_{k-1}), W2_k = W~(D x_{k-1} - D x_p).
* ``irn_objective``: the smoothed PICCS functional that IRN majorises
  (Sec. 2.2.1: each reweighted problem is a quadratic tangent majorant).

Volumes are float64 arrays of shape (nz, ny, nx); projections (V, nv, nu).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        # CBCT_ORACLE_LIB selects another build of siddon.c (the sanitizer test)
        path = os.environ.get("CBCT_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _build  # noqa: WPS433 (local build helper)

            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        gp = P(_CGeom)
        dp = P(ctypes.c_double)
        ip = P(ctypes.c_int64)
        lib.or_forward.argtypes = [gp, dp, dp, ctypes.c_int]
        lib.or_back.argtypes = [gp, dp, dp, ctypes.c_int]
        lib.or_forward_rays.argtypes = [gp, dp, ip, ctypes.c_int64, dp]
        lib.or_back_voxels.argtypes = [gp, dp, ip, ctypes.c_int64, dp]
        lib.or_ray_chords.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp,
                                      ctypes.c_int]
        lib.or_segment_chords.argtypes = [gp, dp, dp, ip, dp, ctypes.c_int]
        lib.or_count_nnz.argtypes = [gp]
        lib.or_count_nnz.restype = ctypes.c_int64
        lib.or_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


class _CGeom(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
        ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("dso", ctypes.c_double), ("dsd", ctypes.c_double),
        ("n_views", ctypes.c_int32),
        ("angles", ctypes.POINTER(ctypes.c_double)),
    ]


@dataclass
class Geometry:
    """Circular-orbit cone-beam geometry (mm, radians).

    ``angles`` defaults to theta_k = 2 pi k / n_views (endpoint excluded).
    """

    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    nu: int
    nv: int
    du: float
    dv: float
    dso: float
    dsd: float
    n_views: int
    angles: np.ndarray | None = None
    _c: _CGeom | None = field(default=None, repr=False)

    def __post_init__(self):
        if self.angles is None:
            self.angles = 2.0 * math.pi * np.arange(self.n_views, dtype=np.float64) / self.n_views
        self.angles = np.ascontiguousarray(self.angles, dtype=np.float64)
        assert self.angles.shape == (self.n_views,)

    @classmethod
    def from_dict(cls, d: dict) -> "Geometry":
        keys = ("nx", "ny", "nz", "vx", "vy", "vz", "nu", "nv", "du", "dv", "dso", "dsd",
                "n_views")
        kw = {k: d[k] for k in keys}
        return cls(**kw, angles=d.get("angles"))

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (self.n_views, self.nv, self.nu)

    def c(self) -> _CGeom:
        if self._c is None:
            self._c = _CGeom(self.nx, self.ny, self.nz, self.vx, self.vy, self.vz,
                             self.nu, self.nv, self.du, self.dv, self.dso, self.dsd,
                             self.n_views,
                             self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return self._c


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


# --------------------------------------------------------------------------
# A and A^T (Sec. 2.1 / 2.2.2)

def forward(g: Geometry, x: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """y = A x, with A[i][j] the chord length (mm) of ray i in voxel j."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(g.vol_shape)
    y = np.zeros(g.proj_shape, dtype=np.float64)
    if _lib().or_forward(ctypes.byref(g.c()), _dptr(x), _dptr(y), int(nthreads)) != 0:
        raise RuntimeError("oracle forward failed")
    return y


def back(g: Geometry, y: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """x = A^T y, the same chord enumeration scattered into voxels."""
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.proj_shape)
    x = np.zeros(g.vol_shape, dtype=np.float64)
    if _lib().or_back(ctypes.byref(g.c()), _dptr(y), _dptr(x), int(nthreads)) != 0:
        raise RuntimeError("oracle back failed")
    return x


def forward_rays(g: Geometry, x: np.ndarray, rays: np.ndarray) -> np.ndarray:
    """(A x)_r for ray ids r = (view*nv + iv)*nu + iu."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(g.vol_shape)
    rays = np.ascontiguousarray(rays, dtype=np.int64)
    out = np.zeros(rays.shape[0], dtype=np.float64)
    if _lib().or_forward_rays(ctypes.byref(g.c()), _dptr(x), _iptr(rays), rays.shape[0],
                              _dptr(out)) != 0:
        raise RuntimeError("oracle forward_rays failed")
    return out


def back_voxels(g: Geometry, y: np.ndarray, vox: np.ndarray) -> np.ndarray:
    """(A^T y)_j for voxel ids j = (k*ny + jy)*nx + i."""
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.proj_shape)
    vox = np.ascontiguousarray(vox, dtype=np.int64)
    out = np.zeros(vox.shape[0], dtype=np.float64)
    if _lib().or_back_voxels(ctypes.byref(g.c()), _dptr(y), _iptr(vox), vox.shape[0],
                             _dptr(out)) != 0:
        raise RuntimeError("oracle back_voxels failed")
    return out


def ray_chords(g: Geometry, view: int, iu: int, iv: int):
    """(voxel ids, chord lengths) of one detector ray."""
    cap = g.nx + g.ny + g.nz + 4
    idx = np.zeros(cap, dtype=np.int64)
    ln = np.zeros(cap, dtype=np.float64)
    n = _lib().or_ray_chords(ctypes.byref(g.c()), view, iu, iv, _iptr(idx), _dptr(ln), cap)
    if n < 0:
        raise RuntimeError("oracle ray_chords failed")
    return idx[:n].copy(), ln[:n].copy()


def segment_chords(g: Geometry, S, P):
    """(voxel ids, chord lengths) of an arbitrary segment S -> P."""
    cap = g.nx + g.ny + g.nz + 4
    S = np.ascontiguousarray(S, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    idx = np.zeros(cap, dtype=np.int64)
    ln = np.zeros(cap, dtype=np.float64)
    n = _lib().or_segment_chords(ctypes.byref(g.c()), _dptr(S), _dptr(P), _iptr(idx),
                                 _dptr(ln), cap)
    if n < 0:
        raise RuntimeError("oracle segment_chords failed")
    return idx[:n].copy(), ln[:n].copy()


def dense_A(g: Geometry) -> np.ndarray:
    """Dense N x M matrix of A (tiny geometries only)."""
    M = g.nx * g.ny * g.nz
    N = g.n_views * g.nv * g.nu
    A = np.zeros((N, M))
    r = 0
    for view in range(g.n_views):
        for iv in range(g.nv):
            for iu in range(g.nu):
                idx, ln = ray_chords(g, view, iu, iv)
                np.add.at(A[r], idx, ln)
                r += 1
    return A


def count_nnz(g: Geometry) -> int:
    return int(_lib().or_count_nnz(ctypes.byref(g.c())))


def num_threads() -> int:
    return int(_lib().or_num_threads())


# --------------------------------------------------------------------------
# D, D^T and the weights (Sec. 2.2.1)

def D(x: np.ndarray) -> np.ndarray:
    """Forward differences (x_i - x_{i+1}) along x, y, z; zero at each axis' last index.

    Returns shape (3, nz, ny, nx) with components (D_x, D_y, D_z); D_x runs
    along the fastest axis.
    """
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros((3,) + x.shape)
    g[0, :, :, :-1] = x[:, :, :-1] - x[:, :, 1:]
    g[1, :, :-1, :] = x[:, :-1, :] - x[:, 1:, :]
    g[2, :-1, :, :] = x[:-1, :, :] - x[1:, :, :]
    return g


def DT(y: np.ndarray) -> np.ndarray:
    """Transpose of ``D``: per axis (D_1^T y)_i = y_i [i < n-1] - y_{i-1} [i >= 1]."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros(y.shape[1:])
    out[:, :, :-1] += y[0, :, :, :-1]
    out[:, :, 1:] -= y[0, :, :, :-1]
    out[:, :-1, :] += y[1, :, :-1, :]
    out[:, 1:, :] -= y[1, :, :-1, :]
    out[:-1, :, :] += y[2, :-1, :, :]
    out[1:, :, :] -= y[2, :-1, :, :]
    return out


def weight_of_gradient(g: np.ndarray, tau: float) -> np.ndarray:
    """[W~*]_ii = 1 / sqrt( sqrt(g_x^2 + g_y^2 + g_z^2) + tau^2 )."""
    mag = np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
    return 1.0 / np.sqrt(mag + tau * tau)


def weights(x: np.ndarray, xp: np.ndarray, tau: float):
    """(W1, W2) = (W~(D x), W~(D x - D x_p)) per voxel (Sec. 2.2.2)."""
    x = np.asarray(x, dtype=np.float64)
    xp = np.asarray(xp, dtype=np.float64)
    return weight_of_gradient(D(x), tau), weight_of_gradient(D(x) - D(xp), tau)


# --------------------------------------------------------------------------
# The augmented system (Sec. 2.2.2)

@dataclass
class Augmented:
    """A~ = [A; alpha W1 D; lambda W2 D] and b~ = [b; 0; lambda W2 D x_p].

    Vectors in the data space are tuples (u_b, u_1, u_2) with u_b of the
    projection shape and u_1, u_2 of shape (3,) + volume shape.
    """

    g: Geometry
    alpha: float
    lam: float
    w1: np.ndarray
    w2: np.ndarray
    A: object = None   # optional callable overriding forward(g, .)
    AT: object = None  # optional callable overriding back(g, .)

    def _A(self, x):
        return self.A(x) if self.A is not None else forward(self.g, x)

    def _AT(self, y):
        return self.AT(y) if self.AT is not None else back(self.g, y)

    def forward(self, x):
        Dx = D(x)
        return (self._A(x), self.alpha * self.w1[None] * Dx, self.lam * self.w2[None] * Dx)

    def back(self, u):
        ub, u1, u2 = u
        return (self._AT(ub) + self.alpha * DT(self.w1[None] * u1)
                + self.lam * DT(self.w2[None] * u2))

    def rhs(self, b, xp):
        return (np.asarray(b, dtype=np.float64), np.zeros((3,) + self.g.vol_shape),
                self.lam * self.w2[None] * D(xp))


def dnorm(u) -> float:
    """Euclidean norm of a data-space tuple (or of a plain array)."""
    if isinstance(u, tuple):
        return math.sqrt(sum(float(np.vdot(p, p)) for p in u))
    return math.sqrt(float(np.vdot(u, u)))


def _sub(a, b):
    return tuple(p - q for p, q in zip(a, b)) if isinstance(a, tuple) else a - b


def _scale(c, a):
    return tuple(c * p for p in a) if isinstance(a, tuple) else c * a


def _axpy(c, x, y):  # c*x + y
    return tuple(c * p + q for p, q in zip(x, y)) if isinstance(x, tuple) else c * x + y


BREAKDOWN = 1e-300


@dataclass
class LsqrResult:
    x: np.ndarray
    phibar: list          # phi-bar after each iteration (= ||b~ - A~ x_i|| in exact arithmetic)
    iters: int
    breakdown: bool
    beta1: float
    alpha1: float


def lsqr(Aop, ATop, b, x0, n_iter: int, reorth: bool = False) -> LsqrResult:
    """LSQR (Paige & Saunders 1982), fixed iteration count, started at x0.

    Aop / ATop map model space <-> data space (arrays or tuples of arrays).
    Breakdown (beta or alpha <= 1e-300) stops early.  With ``reorth`` the new
    v is made orthogonal to all previous v by classical Gram-Schmidt applied
    twice (one-sided reorthogonalisation; not in the paper, optional).
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    u = _sub(b, Aop(x))
    beta = dnorm(u)
    if beta <= BREAKDOWN:
        return LsqrResult(x, [], 0, True, beta, 0.0)
    u = _scale(1.0 / beta, u)
    v = ATop(u)
    alpha = dnorm(v)
    if alpha <= BREAKDOWN:
        return LsqrResult(x, [], 0, True, beta, alpha)
    v = v / alpha
    beta1, alpha1 = beta, alpha
    V = [v.copy()] if reorth else None
    w = v.copy()
    phibar, rhobar = beta, alpha
    hist = []
    it = 0
    broke = False
    for _ in range(n_iter):
        u = _axpy(-alpha, u, Aop(v))
        beta = dnorm(u)
        if beta > BREAKDOWN:
            u = _scale(1.0 / beta, u)
        vraw = ATop(u) - beta * v
        if reorth:
            for _pass in range(2):  # classical Gram-Schmidt, applied twice
                coef = [float(np.vdot(q, vraw)) for q in V]
                for cq, q in zip(coef, V):
                    vraw = vraw - cq * q
        alpha = dnorm(vraw)
        if alpha > BREAKDOWN:
            v = vraw / alpha
        rho = math.sqrt(rhobar * rhobar + beta * beta)
        c = rhobar / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        hist.append(phibar)
        it += 1
        if reorth and alpha > BREAKDOWN:
            V.append(v.copy())
        if beta <= BREAKDOWN or alpha <= BREAKDOWN:
            broke = True
            break
    return LsqrResult(x, hist, it, broke, beta1, alpha1)


def cgls(Aop, ATop, b, x0, n_iter: int):
    """CGLS on min ||A x - b||, fixed iteration count, started at x0."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = _sub(b, Aop(x))
    s = ATop(r)
    p = s.copy()
    gamma = float(np.vdot(s, s))
    hist = []
    for _ in range(n_iter):
        if gamma <= BREAKDOWN ** 2:
            break
        q = Aop(p)
        qq = dnorm(q) ** 2
        if qq <= BREAKDOWN ** 2:
            break
        a = gamma / qq
        x = x + a * p
        r = _axpy(-a, q, r)
        s = ATop(r)
        gnew = float(np.vdot(s, s))
        p = s + (gnew / gamma) * p
        gamma = gnew
        hist.append(dnorm(r))
    return x, hist


@dataclass
class IrnResult:
    x: np.ndarray
    phibar: list          # concatenated LSQR phi-bar histories
    outer: list           # per outer iteration: x_k
    breakdown: bool


def irn_piccs(g: Geometry, b, xp, x0, alpha, lam, tau, n_outer, n_inner,
              reorth=False, A=None, AT=None, keep_iterates=False) -> IrnResult:
    """IRN-PICCS (eq. "PICCS_rec"): n_outer reweightings, n_inner LSQR steps each.

    Outer step k: W1 = W~(D x_{k-1}), W2 = W~(D x_{k-1} - D x_p); then LSQR on the
    augmented system restarted from x_{k-1} gives x_k.
    """
    x = np.array(x0, dtype=np.float64, copy=True).reshape(g.vol_shape)
    xp = np.asarray(xp, dtype=np.float64).reshape(g.vol_shape)
    hist, outs = [], []
    broke = False
    for _k in range(n_outer):
        w1, w2 = weights(x, xp, tau)
        aug = Augmented(g, alpha, lam, w1, w2, A=A, AT=AT)
        res = lsqr(aug.forward, aug.back, aug.rhs(b, xp), x, n_inner, reorth=reorth)
        x = res.x
        hist.extend(res.phibar)
        broke = broke or res.breakdown
        if keep_iterates:
            outs.append(x.copy())
    return IrnResult(x, hist, outs, broke)


@dataclass
class AugmentedPiple:
    """IRN-PIPLE's augmented system (eq. "seq_W_2" written as one least-squares
    problem): A~ = [A; alpha W1 D; lambda I] and b~ = [b; 0; lambda x_p].

    Data-space tuples are (u_b, u_1, u_2) with u_1 of shape (3,) + volume shape
    and u_2 of the volume shape.
    """

    g: Geometry
    alpha: float
    lam: float
    w1: np.ndarray
    A: object = None
    AT: object = None

    def forward(self, x):
        Ax = self.A(x) if self.A is not None else forward(self.g, x)
        return (Ax, self.alpha * self.w1[None] * D(x), self.lam * x)

    def back(self, u):
        ub, u1, u2 = u
        ATu = self.AT(ub) if self.AT is not None else back(self.g, ub)
        return ATu + self.alpha * DT(self.w1[None] * u1) + self.lam * u2

    def rhs(self, b, xp):
        return (np.asarray(b, dtype=np.float64), np.zeros((3,) + self.g.vol_shape),
                self.lam * np.asarray(xp, dtype=np.float64).reshape(self.g.vol_shape))


def irn_piple(g: Geometry, b, xp, x0, alpha, lam, tau, n_outer, n_inner,
              reorth=False, A=None, AT=None, keep_iterates=False) -> IrnResult:
    """IRN-PIPLE (eq. "seq_W_2"): TV(x) by IRN weights, ||x - x_p||^2 exactly.

    Outer step k: W1 = W~(D x_{k-1}); then LSQR on [A; alpha W1 D; lambda I] x ~
    [b; 0; lambda x_p] restarted from x_{k-1} gives x_k.
    """
    x = np.array(x0, dtype=np.float64, copy=True).reshape(g.vol_shape)
    xp = np.asarray(xp, dtype=np.float64).reshape(g.vol_shape)
    hist, outs = [], []
    broke = False
    for _k in range(n_outer):
        w1 = weight_of_gradient(D(x), tau)
        aug = AugmentedPiple(g, alpha, lam, w1, A=A, AT=AT)
        res = lsqr(aug.forward, aug.back, aug.rhs(b, xp), x, n_inner, reorth=reorth)
        x = res.x
        hist.extend(res.phibar)
        broke = broke or res.breakdown
        if keep_iterates:
            outs.append(x.copy())
    return IrnResult(x, hist, outs, broke)


def psi(s: np.ndarray, tau: float) -> np.ndarray:
    """psi(s) = 2 sqrt(s) - 2 tau^2 ln(1 + sqrt(s)/tau^2), so psi'(s) = 1/(sqrt(s) + tau^2)."""
    r = np.sqrt(s)
    t2 = tau * tau
    return 2.0 * r - 2.0 * t2 * np.log1p(r / t2)


def piple_objective(g: Geometry, x, b, xp, alpha, lam, tau, A=None) -> float:
    """F(x) = ||Ax-b||^2 + alpha^2 sum psi(|Dx|^2) + lambda^2 ||x - x_p||^2 (eq.
    "PIRPLE_problem" with the smoothed TV whose tangent majorant is eq. "seq_W_2")."""
    x = np.asarray(x, dtype=np.float64).reshape(g.vol_shape)
    Ax = A(x) if A is not None else forward(g, x)
    r = Ax - np.asarray(b, dtype=np.float64).reshape(Ax.shape)
    s1 = (D(x) ** 2).sum(axis=0)
    d = x - np.asarray(xp, dtype=np.float64).reshape(g.vol_shape)
    return (float(np.vdot(r, r)) + alpha ** 2 * float(psi(s1, tau).sum())
            + lam ** 2 * float(np.vdot(d, d)))


def irn_objective(g: Geometry, x, b, xp, alpha, lam, tau, A=None) -> float:
    """F(x) = ||Ax-b||^2 + alpha^2 sum psi(|Dx|^2) + lambda^2 sum psi(|D(x-x_p)|^2).

    psi' equals the squared IRN weight, and psi is concave, so each reweighted
    quadratic of eq. "PICCS_rec" is a tangent majorant of F (Sec. 2.2.1).
    """
    x = np.asarray(x, dtype=np.float64).reshape(g.vol_shape)
    Ax = A(x) if A is not None else forward(g, x)
    r = Ax - np.asarray(b, dtype=np.float64).reshape(Ax.shape)
    g1 = D(x)
    g2 = g1 - D(np.asarray(xp, dtype=np.float64).reshape(g.vol_shape))
    s1 = (g1 ** 2).sum(axis=0)
    s2 = (g2 ** 2).sum(axis=0)
    return (float(np.vdot(r, r)) + alpha ** 2 * float(psi(s1, tau).sum())
            + lam ** 2 * float(psi(s2, tau).sum()))


# --------------------------------------------------------------------------
# FDK (Feldkamp, Davis & Kress 1984): a direct cone-beam reconstruction used as
# a first image when no prior exists.  Circular orbit, flat detector, full scan.

def ramp_kernel(n_half: int, dp: float) -> np.ndarray:
    """Samples h(n dp), n = -n_half..n_half, of the band-limited ramp filter
    (inverse transform of |f| on |f| <= 1/(2 dp)): 1/(4 dp^2) at 0, 0 at even n,
    -1/(n pi dp)^2 at odd n."""
    n = np.arange(-n_half, n_half + 1)
    h = np.zeros(n.shape, dtype=np.float64)
    h[n == 0] = 1.0 / (4.0 * dp * dp)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (np.pi * n[odd] * dp) ** 2
    return h


def fdk_view_weights(g: Geometry) -> np.ndarray:
    """Angular quadrature weight of each view: half the angle between its two
    neighbours on the circle (2 pi / V for equally spaced views)."""
    a = np.mod(np.asarray(g.angles, dtype=np.float64), 2.0 * np.pi)
    order = np.argsort(a)
    s = a[order]
    nxt = np.roll(s, -1)
    nxt[-1] += 2.0 * np.pi
    prv = np.roll(s, 1)
    prv[0] -= 2.0 * np.pi
    w = np.empty_like(a)
    w[order] = 0.5 * (nxt - prv)
    return w


def fdk_filter(g: Geometry, y: np.ndarray) -> np.ndarray:
    """Cosine-weighted, ramp-filtered projections Q[view][v][u] (Feldkamp's
    first two steps), with the detector rescaled to the isocentre plane."""
    V, nv, nu = g.proj_shape
    y = np.asarray(y, dtype=np.float64).reshape(V, nv, nu)
    u = ((np.arange(nu) + 0.5) * g.du - 0.5 * nu * g.du)[None, None, :]
    v = ((np.arange(nv) + 0.5) * g.dv - 0.5 * nv * g.dv)[None, :, None]
    w = g.dsd / np.sqrt(g.dsd ** 2 + u * u + v * v)
    dp = g.du * g.dso / g.dsd
    h = ramp_kernel(nu - 1, dp)
    out = np.empty_like(y)
    yw = y * w
    for k in range(V):
        for r in range(nv):
            # full linear convolution, keep the nu central outputs
            out[k, r] = dp * np.convolve(yw[k, r], h, mode="full")[nu - 1:2 * nu - 1]
    return out


def fdk_backproject(g: Geometry, q: np.ndarray) -> np.ndarray:
    """Voxel-driven weighted backprojection: x(r) = sum over views of
    (dbeta / 2) (DSO / U)^2 Q(u(r), v(r)), U = DSO - r . s_hat the depth of r
    along the central ray, (u, v) the detector point of r, bilinear
    interpolation with zero outside the detector."""
    V, nv, nu = g.proj_shape
    q = np.asarray(q, dtype=np.float64).reshape(V, nv, nu)
    xc = (np.arange(g.nx) + 0.5) * g.vx - 0.5 * g.nx * g.vx
    yc = (np.arange(g.ny) + 0.5) * g.vy - 0.5 * g.ny * g.vy
    zc = (np.arange(g.nz) + 0.5) * g.vz - 0.5 * g.nz * g.vz
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    out = np.zeros(g.vol_shape, dtype=np.float64)
    wv = fdk_view_weights(g)
    for k, th in enumerate(g.angles):
        c, s = math.cos(th), math.sin(th)
        U = g.dso - (X * c + Y * s)
        lat = -X * s + Y * c
        fu = g.dsd * lat / U / g.du + 0.5 * nu - 0.5
        fv = g.dsd * Z / U / g.dv + 0.5 * nv - 0.5
        i0 = np.floor(fu).astype(np.int64)
        j0 = np.floor(fv).astype(np.int64)
        au = fu - i0
        av = fv - j0
        val = np.zeros(g.vol_shape)
        for di, wu in ((0, 1.0 - au), (1, au)):
            for dj, wvv in ((0, 1.0 - av), (1, av)):
                ii, jj = i0 + di, j0 + dj
                ok = (ii >= 0) & (ii < nu) & (jj >= 0) & (jj < nv)
                val += np.where(ok, wu * wvv * q[k, np.clip(jj, 0, nv - 1),
                                                np.clip(ii, 0, nu - 1)], 0.0)
        out += 0.5 * wv[k] * (g.dso / U) ** 2 * val
    return out


def fdk_backproject_at(g: Geometry, q: np.ndarray, flat_idx) -> np.ndarray:
    """fdk_backproject evaluated only at the voxels with flat [z][y][x] indices
    flat_idx (same formula, one voxel at a time)."""
    V, nv, nu = g.proj_shape
    q = np.asarray(q, dtype=np.float64).reshape(V, nv, nu)
    wv = fdk_view_weights(g)
    out = np.zeros(len(flat_idx))
    for n, f in enumerate(flat_idx):
        k, rem = divmod(int(f), g.nx * g.ny)
        j, i = divmod(rem, g.nx)
        X = (i + 0.5) * g.vx - 0.5 * g.nx * g.vx
        Y = (j + 0.5) * g.vy - 0.5 * g.ny * g.vy
        Zc = (k + 0.5) * g.vz - 0.5 * g.nz * g.vz
        acc = 0.0
        for v, th in enumerate(g.angles):
            c, s = math.cos(th), math.sin(th)
            U = g.dso - (X * c + Y * s)
            fu = g.dsd * (-X * s + Y * c) / U / g.du + 0.5 * nu - 0.5
            fv = g.dsd * Zc / U / g.dv + 0.5 * nv - 0.5
            i0, j0 = math.floor(fu), math.floor(fv)
            au, av = fu - i0, fv - j0
            val = 0.0
            for di, wu in ((0, 1.0 - au), (1, au)):
                for dj, wvv in ((0, 1.0 - av), (1, av)):
                    ii, jj = i0 + di, j0 + dj
                    if 0 <= ii < nu and 0 <= jj < nv:
                        val += wu * wvv * q[v, jj, ii]
            acc += 0.5 * wv[v] * (g.dso / U) ** 2 * val
        out[n] = acc
    return out


def fdk(g: Geometry, y: np.ndarray) -> np.ndarray:
    """FDK reconstruction of line-integral projections y[view][v][u]."""
    return fdk_backproject(g, fdk_filter(g, y))
