"""Pins of the oracle's FDK reconstruction (Feldkamp, Davis & Kress 1984).

The ramp kernel against its closed-form frequency response; the angular
quadrature weights; and a whole reconstruction of an off-centre sphere from
projections computed here in closed form (not by the oracle's projector), which
fixes the overall scale, the signs of the detector coordinates and the
backprojection geometry.
"""
import math

import numpy as np


def test_ramp_kernel_frequency_response(orc):
    """dp * sum_n h_n cos(2 pi f n dp) = |f| for |f| < 1/(2 dp) (band-limited ramp)."""
    dp = 0.7
    n_half = 4000
    h = orc.ramp_kernel(n_half, dp)
    n = np.arange(-n_half, n_half + 1)
    for f in (0.02, 0.1, 0.3, 0.45, 0.49):
        f = f / dp
        H = dp * float(np.sum(h * np.cos(2 * np.pi * f * n * dp)))
        # the tail beyond n_half is O(1 / (pi^2 n_half dp)) in absolute terms
        assert abs(H - abs(f)) < 2.0 / (np.pi ** 2 * n_half * dp), (f, H)


def test_view_weights(orc):
    g = orc.Geometry(nx=4, ny=4, nz=4, vx=1, vy=1, vz=1, nu=8, nv=8, du=1, dv=1, dso=50,
                     dsd=80, n_views=12)
    np.testing.assert_allclose(orc.fdk_view_weights(g), 2 * np.pi / 12, rtol=1e-14)
    ang = np.sort(np.random.default_rng(1).uniform(0, 2 * np.pi, 9))
    g = orc.Geometry(nx=4, ny=4, nz=4, vx=1, vy=1, vz=1, nu=8, nv=8, du=1, dv=1, dso=50,
                     dsd=80, n_views=9, angles=ang)
    w = orc.fdk_view_weights(g)
    assert abs(w.sum() - 2 * np.pi) < 1e-12
    k = 4
    assert abs(w[k] - 0.5 * (ang[k + 1] - ang[k - 1])) < 1e-14


def sphere_projections(g, centre, radius):
    """Closed-form chord length (mm) of every pixel-centre ray through a sphere."""
    V, nv, nu = g.proj_shape
    out = np.zeros((V, nv, nu))
    u = (np.arange(nu) + 0.5) * g.du - 0.5 * nu * g.du
    v = (np.arange(nv) + 0.5) * g.dv - 0.5 * nv * g.dv
    c = np.asarray(centre, dtype=np.float64)
    for k, th in enumerate(g.angles):
        S = np.array([g.dso * math.cos(th), g.dso * math.sin(th), 0.0])
        C = np.array([(g.dso - g.dsd) * math.cos(th), (g.dso - g.dsd) * math.sin(th), 0.0])
        eu = np.array([-math.sin(th), math.cos(th), 0.0])
        P = C[None, None, :] + u[None, :, None] * eu + v[:, None, None] * np.array([0, 0, 1.0])
        d = P - S
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        w = S - c
        t = d @ w
        dist2 = w @ w - t * t
        out[k] = 2.0 * np.sqrt(np.maximum(radius * radius - dist2, 0.0))
    return out


def test_fdk_recovers_an_off_centre_sphere(orc):
    g = orc.Geometry(nx=40, ny=40, nz=32, vx=1.5, vy=1.5, vz=1.5, nu=96, nv=80, du=1.6,
                     dv=1.6, dso=400.0, dsd=600.0, n_views=120)
    centre, radius, rho = (9.0, -6.0, 4.0), 11.0, 1.0
    x = orc.fdk(g, rho * sphere_projections(g, centre, radius))
    zc = (np.arange(g.nz) + 0.5) * g.vz - 0.5 * g.nz * g.vz
    yc = (np.arange(g.ny) + 0.5) * g.vy - 0.5 * g.ny * g.vy
    xc = (np.arange(g.nx) + 0.5) * g.vx - 0.5 * g.nx * g.vx
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    inside = r < radius - 3.0
    outside = (r > radius + 4.0) & (np.sqrt(X ** 2 + Y ** 2) < 22.0) & (np.abs(Z) < 16.0)
    assert abs(x[inside].mean() - rho) < 0.03 * rho
    assert abs(x[outside].mean()) < 0.03 * rho
    # the reconstructed mass sits where the sphere is (catches flipped axes)
    m = x > 0.5 * rho
    for A, c0 in ((X, centre[0]), (Y, centre[1]), (Z, centre[2])):
        assert abs(A[m].mean() - c0) < 0.4


def test_fdk_is_linear(orc):
    g = orc.Geometry(nx=8, ny=7, nz=6, vx=1, vy=1, vz=1, nu=12, nv=10, du=1.2, dv=1.2, dso=60,
                     dsd=100, n_views=10)
    rng = np.random.default_rng(3)
    y1, y2 = rng.normal(size=(2,) + g.proj_shape)
    np.testing.assert_allclose(orc.fdk(g, 2.5 * y1 + y2), 2.5 * orc.fdk(g, y1) + orc.fdk(g, y2),
                               rtol=1e-10, atol=1e-12)


def test_fdk_distance_weighting_far_from_the_axis(orc):
    """Short source distance, sphere far off-centre in the mid-plane: the
    (DSO/U)^2 weighting matters at second order in rho/DSO (about 13 % here)
    and must recover the density."""
    g = orc.Geometry(nx=48, ny=48, nz=12, vx=2.0, vy=2.0, vz=2.0, nu=180, nv=40, du=1.6,
                     dv=1.6, dso=100.0, dsd=160.0, n_views=180)
    centre, radius, rho = (36.0, 0.0, 0.0), 8.0, 1.0
    x = orc.fdk(g, rho * sphere_projections(g, centre, radius))
    zc = (np.arange(g.nz) + 0.5) * g.vz - 0.5 * g.nz * g.vz
    yc = (np.arange(g.ny) + 0.5) * g.vy - 0.5 * g.ny * g.vy
    xc = (np.arange(g.nx) + 0.5) * g.vx - 0.5 * g.nx * g.vx
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    r = np.sqrt((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2)
    inside = r < radius - 3.0
    assert inside.sum() > 20
    assert abs(x[inside].mean() - rho) < 0.04 * rho


def test_sampled_backprojection_matches_the_full_one(orc):
    g = orc.Geometry(nx=9, ny=8, nz=7, vx=1, vy=1, vz=1, nu=14, nv=12, du=1.1, dv=1.1, dso=60,
                     dsd=100, n_views=11)
    q = np.random.default_rng(5).normal(size=g.proj_shape)
    full = orc.fdk_backproject(g, q).ravel()
    idx = np.random.default_rng(6).choice(full.size, 40, replace=False)
    np.testing.assert_allclose(orc.fdk_backproject_at(g, q, idx), full[idx], rtol=1e-12,
                               atol=1e-12)
