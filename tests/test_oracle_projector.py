"""Pins of the FP64 oracle projector against facts fixed independently of it.

The sensing matrix A of the linear CT model (paper Sec. 2.1, eq. "tomo") is read
as exact chord lengths; these tests check the oracle's Siddon enumeration
against hand-derived values, an independent per-voxel slab computation, closed
forms for boxes and ellipsoids, a symmetry of the circular orbit, and the
adjoint identity that A^T must satisfy (Sec. 2.2.2).
"""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- helpers (independent)

def endpoints(g, view, iu, iv):
    th = g.angles[view]
    c, s = math.cos(th), math.sin(th)
    uc = (iu + 0.5) * g.du - g.nu * g.du / 2
    vc = (iv + 0.5) * g.dv - g.nv * g.dv / 2
    S = np.array([g.dso * c, g.dso * s, 0.0])
    P = np.array([(g.dso - g.dsd) * c - uc * s, (g.dso - g.dsd) * s + uc * c, vc])
    return S, P


def slab_chord(S, P, lo, hi):
    """Length of segment S->P inside the box [lo, hi] (Kay-Kajiya slabs)."""
    d = P - S
    t0, t1 = 0.0, 1.0
    for a in range(3):
        if d[a] == 0.0:
            if not (lo[a] < S[a] < hi[a]):
                return 0.0
            continue
        ta, tb = (lo[a] - S[a]) / d[a], (hi[a] - S[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return max(0.0, t1 - t0) * float(np.linalg.norm(d))


def vox_box(g, i, j, k):
    lo = np.array([-g.nx * g.vx / 2 + i * g.vx, -g.ny * g.vy / 2 + j * g.vy,
                   -g.nz * g.vz / 2 + k * g.vz])
    return lo, lo + np.array([g.vx, g.vy, g.vz])


def tiny(orc, nx=5, ny=6, nz=7, nu=8, nv=6, V=7, h=(1.0, 1.1, 0.9)):
    return orc.Geometry(nx=nx, ny=ny, nz=nz, vx=h[0], vy=h[1], vz=h[2], nu=nu, nv=nv, du=1.7,
                        dv=1.6, dso=30.0, dsd=50.0, n_views=V)


# ---------------------------------------------------------------- golden hand cases

def _golden_cases():
    cases, cur = [], None
    with open(os.path.join(HERE, "golden", "chords_hand.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "case":
                cur = {"name": tok[1], "chords": {}}
                cases.append(cur)
            elif tok[0] == "grid":
                cur["grid"] = [float(t) for t in tok[1:]]
            elif tok[0] in ("S", "P"):
                cur[tok[0]] = [float(t) for t in tok[1:]]
            elif tok[0] == "chord":
                cur["chords"][int(tok[1])] = eval(tok[2], {"sqrt": math.sqrt})  # noqa: S307
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_golden_hand_chords(orc, case):
    nx, ny, nz, vx, vy, vz = case["grid"]
    g = orc.Geometry(nx=int(nx), ny=int(ny), nz=int(nz), vx=vx, vy=vy, vz=vz, nu=1, nv=1,
                     du=1, dv=1, dso=10, dsd=20, n_views=1)
    idx, ln = orc.segment_chords(g, case["S"], case["P"])
    got = {}
    for i, l in zip(idx, ln):
        got[int(i)] = got.get(int(i), 0.0) + l
    assert set(got) == set(case["chords"])
    for j, want in case["chords"].items():
        assert got[j] == pytest.approx(want, rel=1e-14, abs=1e-14)


# ---------------------------------------------------------------- closed forms / brute force

def test_all_ones_equals_box_length(orc):
    g = tiny(orc, nx=6, ny=5, nz=4, nu=11, nv=9, V=5)
    y = orc.forward(g, np.ones(g.vol_shape))
    lo = np.array([-g.nx * g.vx / 2, -g.ny * g.vy / 2, -g.nz * g.vz / 2])
    for view in range(g.n_views):
        for iv in range(g.nv):
            for iu in range(g.nu):
                S, P = endpoints(g, view, iu, iv)
                want = slab_chord(S, P, lo, -lo)
                assert y[view, iv, iu] == pytest.approx(want, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("dims", [(5, 6, 7), (4, 4, 3), (3, 5, 2)])
def test_dense_A_equals_slab_brute_force(orc, dims):
    g = tiny(orc, *dims)
    A = orc.dense_A(g)
    B = np.zeros_like(A)
    r = 0
    for view in range(g.n_views):
        for iv in range(g.nv):
            for iu in range(g.nu):
                S, P = endpoints(g, view, iu, iv)
                for k in range(g.nz):
                    for j in range(g.ny):
                        for i in range(g.nx):
                            lo, hi = vox_box(g, i, j, k)
                            B[r, (k * g.ny + j) * g.nx + i] = slab_chord(S, P, lo, hi)
                r += 1
    assert np.count_nonzero(A) > 0
    np.testing.assert_allclose(A, B, rtol=0, atol=1e-12)


def test_box_phantom_closed_form(orc):
    g = orc.Geometry(nx=12, ny=10, nz=8, vx=1.0, vy=1.0, vz=1.0, nu=20, nv=14, du=1.3, dv=1.3,
                     dso=40.0, dsd=70.0, n_views=6)
    x = np.zeros(g.vol_shape)
    (i0, i1), (j0, j1), (k0, k1) = (3, 9), (2, 7), (1, 6)
    rho = 0.7
    x[k0:k1, j0:j1, i0:i1] = rho
    y = orc.forward(g, x)
    lo = np.array([-6 + i0, -5 + j0, -4 + k0], dtype=float)
    hi = np.array([-6 + i1, -5 + j1, -4 + k1], dtype=float)
    for view in range(g.n_views):
        for iv in range(g.nv):
            for iu in range(g.nu):
                S, P = endpoints(g, view, iu, iv)
                assert y[view, iv, iu] == pytest.approx(rho * slab_chord(S, P, lo, hi),
                                                        rel=1e-12, abs=1e-12)


def _ellipsoid_chord(S, P, c, Q):
    d = P - S
    a = d @ Q @ d
    b = d @ Q @ (S - c)
    cc = (S - c) @ Q @ (S - c) - 1.0
    disc = b * b - a * cc
    if disc <= 0:
        return 0.0
    return 2.0 * math.sqrt(disc) / a * float(np.linalg.norm(d))


def test_ellipsoid_projection_converges_first_order(orc):
    """Centre-point voxelised ellipsoids: A x -> density * chord at O(h)."""
    L = 32.0  # physical cube edge [mm]
    c = np.array([1.3, -2.1, 0.7])
    semi = np.array([9.0, 6.0, 7.5])
    ang = 0.4
    R = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0],
                  [0, 0, 1.0]])
    Q = R @ np.diag(1 / semi ** 2) @ R.T
    rng = np.random.default_rng(7)
    errs = []
    for n in (16, 32, 64):
        h = L / n
        g = orc.Geometry(nx=n, ny=n, nz=n, vx=h, vy=h, vz=h, nu=40, nv=40, du=1.2, dv=1.2,
                         dso=100.0, dsd=160.0, n_views=4)
        ctr = (np.arange(n) + 0.5) * h - L / 2
        Z, Y, X = np.meshgrid(ctr, ctr, ctr, indexing="ij")
        Pm = np.stack([X, Y, Z], -1) - c
        x = (np.einsum("...i,ij,...j->...", Pm, Q, Pm) <= 1.0).astype(float)
        rays = rng.integers(0, g.n_views * g.nv * g.nu, size=400) if n == 16 else rays
        y = orc.forward_rays(g, x, rays)
        e = []
        for r, yr in zip(rays, y):
            view, rem = divmod(int(r), g.nv * g.nu)
            iv, iu = divmod(rem, g.nu)
            S, P = endpoints(g, view, iu, iv)
            e.append(abs(yr - _ellipsoid_chord(S, P, c, Q)))
        errs.append(float(np.mean(e)))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    # first-order convergence: halving h roughly halves the mean error
    assert all(1.4 < q < 3.0 for q in ratios), (errs, ratios)
    assert errs[-1] < 0.3


def test_rotation_by_quarter_turn_shifts_views(orc):
    n, V = 9, 8
    g = orc.Geometry(nx=n, ny=n, nz=5, vx=1.0, vy=1.0, vz=1.2, nu=13, nv=6, du=1.4, dv=1.5,
                     dso=35.0, dsd=60.0, n_views=V)
    x = np.random.default_rng(3).uniform(size=g.vol_shape)
    # rotate the object by +90 degrees about z: x'[k][a][b] = x[k][n-1-b][a]
    xr = np.empty_like(x)
    for a in range(n):
        for b in range(n):
            xr[:, a, b] = x[:, n - 1 - b, a]
    y = orc.forward(g, x)
    yr = orc.forward(g, xr)
    np.testing.assert_allclose(yr, np.roll(y, V // 4, axis=0), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- adjoint

@pytest.mark.parametrize("geo", ["tiny", "c1"])
def test_dot_product_adjoint(orc, geo):
    if geo == "tiny":
        g = tiny(orc)
    else:
        from paper_2509_08574_amd import synth
        g = orc.Geometry.from_dict(synth.geometry("c1"))
    rng = np.random.default_rng(11)
    x = rng.uniform(size=g.vol_shape)
    y = rng.uniform(size=g.proj_shape)
    lhs = float(np.vdot(orc.forward(g, x), y))
    rhs = float(np.vdot(x, orc.back(g, y, nthreads=1)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_dense_AT_is_transpose(orc):
    g = tiny(orc, 4, 3, 5, nu=5, nv=4, V=3)
    A = orc.dense_A(g)
    N, M = A.shape
    AT = np.zeros((M, N))
    for r in range(N):
        e = np.zeros(N)
        e[r] = 1.0
        AT[:, r] = orc.back(g, e.reshape(g.proj_shape), nthreads=1).ravel()
    assert np.array_equal(AT, A.T)


def test_sampled_rows_and_columns_match_full(orc):
    g = tiny(orc, 6, 7, 5, nu=9, nv=7, V=6)
    rng = np.random.default_rng(5)
    x = rng.uniform(size=g.vol_shape)
    y = rng.uniform(size=g.proj_shape)
    Ax = orc.forward(g, x).ravel()
    ATy = orc.back(g, y, nthreads=1).ravel()
    rays = rng.choice(Ax.size, 40, replace=False)
    vox = rng.choice(ATy.size, 40, replace=False)
    np.testing.assert_allclose(orc.forward_rays(g, x, rays), Ax[rays], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(orc.back_voxels(g, y, vox), ATy[vox], rtol=1e-12, atol=1e-12)


def test_nnz_count_matches_dense(orc):
    g = tiny(orc)
    assert orc.count_nnz(g) == np.count_nonzero(orc.dense_A(g))
