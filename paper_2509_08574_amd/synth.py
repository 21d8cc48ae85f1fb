"""Seeded synthetic inputs: workload configurations, phantoms, noise, random vectors.

This module is shared by the tests, the benchmark and the oracle checks.  It
holds none of the reconstruction method's arithmetic: it draws phantoms
(voxelised ellipsoids and needle cylinders), random test vectors and
measurement noise applied to line integrals computed elsewhere.  Everything is
seeded through ``numpy.random.default_rng``.

Phantom recipe (the paper's own data -- the TIGRE head phantom and the thorax
scan with its 3D Slicer ground truth -- is not available, so these stand in):
* ellipsoids with uniformly random orientation (random unit quaternion),
  centres uniform in the inner 70 % of the volume, semi-axes uniform in the
  configured range (voxels), densities U[0.1, 1.0], added together;
* voxelisation by the voxel-centre test;
* a needle is a finite cylinder whose voxels are *set* to its value (2.0);
* noise: counts ~ Poisson(I0 exp(-mu p)) with mu = 0.02 / mm per density unit,
  counts clamped to >= 1, b = -ln(counts / I0) / mu.
"""
from __future__ import annotations

import math

import numpy as np

MU_WATER_PER_MM = 0.02


def _rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _grid(shape):
    nz, ny, nx = shape
    return (np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5)


def add_ellipsoid(vol: np.ndarray, centre, semi, R, value, mode="add", zrange=None):
    """Voxel-centre voxelisation of {p : |R^T (p - c) / a| <= 1} (voxel units, (x,y,z)),
    optionally restricted to the z planes zrange = (z0, z1)."""
    nz, ny, nx = vol.shape
    rmax = float(max(semi))
    lo = [max(0, int(math.floor(centre[a] - rmax)) - 1) for a in range(3)]
    hi = [min(n, int(math.ceil(centre[a] + rmax)) + 1) for a, n in enumerate((nx, ny, nz))]
    if zrange is not None:
        lo[2], hi[2] = max(lo[2], zrange[0]), min(hi[2], zrange[1])
    if any(h <= l for l, h in zip(lo, hi)):
        return
    yc = (np.arange(lo[1], hi[1]) + 0.5 - centre[1])[None, :, None]
    xc = (np.arange(lo[0], hi[0]) + 0.5 - centre[0])[None, None, :]
    # z slabs of a few planes keep the temporaries in cache (same arithmetic)
    for z0 in range(lo[2], hi[2], 8):
        z1 = min(z0 + 8, hi[2])
        zc = (np.arange(z0, z1) + 0.5 - centre[2])[:, None, None]
        acc = 0.0
        for m in range(3):  # (R^T p)_m / a_m, summed in squares
            q = (xc * R[0, m] + yc * R[1, m] + zc * R[2, m]) / semi[m]
            acc = acc + q * q
        inside = acc <= 1.0
        sub = vol[z0:z1, lo[1]:hi[1], lo[0]:hi[0]]
        if mode == "add":
            sub[inside] += value
        else:
            sub[inside] = value


def cylinder_indices(shape, centre, axis, radius, length):
    """Flat indices (into a [z][y][x] array of `shape`) of the voxels whose
    centres lie in a finite cylinder (voxel units, (x, y, z))."""
    nz, ny, nx = shape
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    ext = length / 2.0 + radius + 1
    lo = [max(0, int(math.floor(centre[a] - ext))) for a in range(3)]
    hi = [min(n, int(math.ceil(centre[a] + ext)) + 1) for a, n in enumerate((nx, ny, nz))]
    if any(h <= l for l, h in zip(lo, hi)):
        return np.zeros(0, dtype=np.int64)
    zc = (np.arange(lo[2], hi[2]) + 0.5 - centre[2])[:, None, None]
    yc = (np.arange(lo[1], hi[1]) + 0.5 - centre[1])[None, :, None]
    xc = (np.arange(lo[0], hi[0]) + 0.5 - centre[0])[None, None, :]
    t = xc * axis[0] + yc * axis[1] + zc * axis[2]
    r2 = xc * xc + yc * yc + zc * zc - t * t
    kz, jy, ix = np.nonzero((np.abs(t) <= length / 2.0) & (r2 <= radius * radius))
    return ((kz + lo[2]) * ny + (jy + lo[1])) * nx + (ix + lo[0])


def add_cylinder(vol: np.ndarray, centre, axis, radius, length, value):
    """Set the voxels whose centres lie in a finite cylinder to ``value`` (voxel units)."""
    vol.reshape(-1)[cylinder_indices(vol.shape, centre, axis, radius, length)] = value


def ellipsoid_phantom(shape, n_ell, semi_range, seed, dens_range=(0.1, 1.0), threads=1):
    """Sum of ``n_ell`` random ellipsoids; returns (volume, list of ellipsoid params).

    With threads > 1 the volume is filled by z slabs in parallel; every voxel
    receives the same additions in the same order, so the result is identical.
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    vol = np.zeros(shape, dtype=np.float64)
    ells = []
    for _ in range(n_ell):
        c = np.array([rng.uniform(0.15 * n, 0.85 * n) for n in (nx, ny, nz)])
        a = rng.uniform(semi_range[0], semi_range[1], size=3)
        R = _rotation(rng)
        rho = rng.uniform(*dens_range)
        ells.append((c, a, R, rho))

    def fill(z0, z1):
        for c, a, R, rho in ells:
            add_ellipsoid(vol, c, a, R, rho, zrange=(z0, z1))

    if threads <= 1:
        fill(0, nz)
    else:
        from concurrent.futures import ThreadPoolExecutor
        step = -(-nz // (4 * threads))
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda z: fill(z, min(z + step, nz)), range(0, nz, step)))
    return vol, ells


def random_unit(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def noisy_line_integrals(p: np.ndarray, I0: float, seed: int, mu=MU_WATER_PER_MM):
    """Poisson transmission noise on line integrals p (mm x density)."""
    rng = np.random.default_rng(seed)
    lam = I0 * np.exp(-mu * np.asarray(p, dtype=np.float64))
    counts = np.maximum(rng.poisson(lam), 1).astype(np.float64)
    return -np.log(counts / I0) / mu


def random_volume(shape, seed, lo=0.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def random_proj(shape, seed, lo=0.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


# --------------------------------------------------------------------------
# Workload configurations.  Geometry keys match the C descriptor fields.

def geometry(name: str) -> dict:
    g = {
        # 64^3 at 1 mm, 96x96 detector at 1.5 mm, 48 views.
        "c1": dict(nx=64, ny=64, nz=64, vx=1.0, vy=1.0, vz=1.0, nu=96, nv=96, du=1.5, dv=1.5,
                   dso=1000.0, dsd=1536.0, n_views=48),
        # 256^3 at 1 mm, 512x512 at 0.8 mm, 90 views.
        "c2": dict(nx=256, ny=256, nz=256, vx=1.0, vy=1.0, vz=1.0, nu=512, nv=512, du=0.8,
                   dv=0.8, dso=1000.0, dsd=1536.0, n_views=90),
        # 720-view scan of the same object (prior acquisition).
        "c2_prior": dict(nx=256, ny=256, nz=256, vx=1.0, vy=1.0, vz=1.0, nu=512, nv=512,
                         du=0.8, dv=0.8, dso=1000.0, dsd=1536.0, n_views=720),
        # 512^3 at 0.5 mm, 1024x768 at 0.4 mm, 120 views.
        "c3_512": dict(nx=512, ny=512, nz=512, vx=0.5, vy=0.5, vz=0.5, nu=1024, nv=768,
                       du=0.4, dv=0.4, dso=1000.0, dsd=1536.0, n_views=120),
        # 512x512x400 at 0.4 mm, 1024x1024 at 0.3 mm, 180 views.
        "c5": dict(nx=512, ny=512, nz=400, vx=0.4, vy=0.4, vz=0.4, nu=1024, nv=1024, du=0.3,
                   dv=0.3, dso=1000.0, dsd=1536.0, n_views=180),
    }
    return dict(g[name])


def serving_geometry(n: int, n_views: int) -> dict:
    """Serving-stream geometry: FOV 256 mm, voxel 256/n mm, detector 2n x 2n at 0.8*256/n mm."""
    h = 256.0 / n
    return dict(nx=n, ny=n, nz=n, vx=h, vy=h, vz=h, nu=2 * n, nv=2 * n, du=0.8 * h,
                dv=0.8 * h, dso=1000.0, dsd=1536.0, n_views=n_views)


# Regularisation parameters (alpha, lambda, tau), chosen once by the oracle-side
# sweep oracle/sweep_params.py on the 64^3 case (best relative error to the
# ground truth), and the outer x inner split of the iteration count per workload.
SOLVE_PARAMS = {
    "c1": dict(alpha=1.0, lam=1.0, tau=0.1, n_outer=3, n_inner=5, I0=1e5, seed=1),
    "c2": dict(alpha=1.0, lam=1.0, tau=0.1, n_outer=5, n_inner=10, I0=5e4, seed=2),
    "c5": dict(alpha=1.0, lam=1.0, tau=0.1, n_outer=4, n_inner=10, I0=5e4, seed=5),
}


def c1_case(seed: int = 1):
    """The 64^3 / 48-view case: prior, current object (prior + sphere + needle)."""
    shape = (64, 64, 64)
    prior, _ = ellipsoid_phantom(shape, 10, (4.0, 24.0), seed)
    rng = np.random.default_rng(seed + 1000)
    cur = prior.copy()
    c = np.array([rng.uniform(0.3 * 64, 0.7 * 64) for _ in range(3)])
    add_ellipsoid(cur, c, (4.0, 4.0, 4.0), np.eye(3), 0.5)
    nc = np.array([rng.uniform(0.35 * 64, 0.65 * 64) for _ in range(3)])
    add_cylinder(cur, nc, random_unit(rng), 1.0, 40.0, 2.0)
    return prior, cur


def c2_case(seed: int = 2):
    """The 256^3 / 90-view case: 30-ellipsoid object and its lesion-growth change."""
    shape = (256, 256, 256)
    base, ells = ellipsoid_phantom(shape, 30, (16.0, 96.0), seed)
    k = int(np.argmin([np.prod(a) for (_, a, _, _) in ells]))
    c, a, R, rho = ells[k]
    cur = base.copy()
    add_ellipsoid(cur, c, a, R, -rho)          # remove the original lesion
    add_ellipsoid(cur, c, 1.3 * a, R, rho)     # and add it grown by 1.3
    # Thirty overlapping ellipsoids sum to several times water; scale the object
    # to a peak of 1 (water) so that line integrals stay at mu * p = O(1-5).
    scale = 1.0 / base.max()
    return base * scale, cur * scale


# --------------------------------------------------------------------------
# Serving stream: repeated scans of several patients, each the patient's prior
# plus a needle moved along its own axis.

SERVING_SIZES = (128, 256, 384)
SERVING_PARAMS = dict(alpha=1.0, lam=1.0, tau=0.1, n_outer=3, n_inner=10, I0=5e4)


def serving_patient(i: int, sizes=SERVING_SIZES):
    """Patient i (seed 400 + i): (n, prior volume, needle (centre, axis)).

    The prior is a 30-ellipsoid object (semi-axes U[4, 24] * n/64 voxels),
    scaled to a peak of 1, with a needle (radius 1 voxel, length 40 voxels,
    value 2.0) set into it at a seeded position and direction.
    """
    rng = np.random.default_rng(400 + i)
    n = int(sizes[rng.integers(len(sizes))])
    base, _ = ellipsoid_phantom((n, n, n), 30, (4.0 * n / 64, 24.0 * n / 64), 400 + i)
    base *= 1.0 / base.max()
    centre = np.array([rng.uniform(0.35 * n, 0.65 * n) for _ in range(3)])
    axis = random_unit(rng)
    prior = base.copy()
    add_cylinder(prior, centre, axis, 1.0, 40.0, 2.0)
    return n, prior, (base, centre, axis)


def serving_needle(patient_state, shift_voxels: float):
    """Flat voxel indices of the needle moved by shift_voxels along its axis
    (the voxels set to 2.0 in the current object)."""
    base, centre, axis = patient_state
    return cylinder_indices(base.shape, centre + shift_voxels * axis, axis, 1.0, 40.0)


def serving_current(patient_state, shift_voxels: float):
    """The patient's object with the needle moved by shift_voxels along its axis."""
    cur = patient_state[0].copy()
    cur.reshape(-1)[serving_needle(patient_state, shift_voxels)] = 2.0
    return cur


def serving_request_draw(i: int, n_patients: int):
    """Request i (seed 4000 + i): (patient, number of views, needle shift in voxels)."""
    rng = np.random.default_rng(4000 + i)
    return (int(rng.integers(n_patients)), int(rng.integers(30, 121)),
            float(rng.uniform(2.0, 5.0)))


# --------------------------------------------------------------------------
# Stand-ins shaped like the paper's two experiments (Sec. 3), whose data are
# not available: a digital head with a cubic tumour (128^3, 128^2 detector, 20
# views) and a thorax with a needle (256^3, 512 x 364 detector at 0.776 mm,
# DSO 810, DSD 1195, 20 / 50 / 180 views).  Densities are relative to water.

def head_geometry(n_views: int = 20) -> dict:
    """128^3 at 1.6 mm, 128^2 detector at 2.4 mm (the head's geometry is not
    stated; these distances are the common 1000 / 1536 mm)."""
    return dict(nx=128, ny=128, nz=128, vx=1.6, vy=1.6, vz=1.6, nu=128, nv=128, du=2.4,
                dv=2.4, dso=1000.0, dsd=1536.0, n_views=n_views)


def head_case(seed: int = 31):
    """(prior, current): skull shell around brain tissue with seeded internal
    structures; the current scan adds an 8 x 8 x 8-voxel cubic tumour."""
    rng = np.random.default_rng(seed)
    n = 128
    vol = np.zeros((n, n, n))
    c = np.array([64.0, 64.0, 64.0])
    add_ellipsoid(vol, c, (46.0, 56.0, 50.0), np.eye(3), 1.6)    # skull
    add_ellipsoid(vol, c, (42.0, 52.0, 46.0), np.eye(3), -0.6)   # brain = 1.0
    for _ in range(14):                                           # internal structure
        cc = c + rng.uniform(-28, 28, size=3)
        add_ellipsoid(vol, cc, rng.uniform(3.0, 12.0, size=3), _rotation(rng),
                      rng.uniform(-0.12, 0.12))
    cur = vol.copy()
    t0 = (c + rng.uniform(-18, 18, size=3)).astype(int) - 4
    cur[t0[2]:t0[2] + 8, t0[1]:t0[1] + 8, t0[0]:t0[0] + 8] += 0.15
    return vol, cur


def thorax_geometry(n_views: int) -> dict:
    """256^3 at 1.05 mm; the scanner of Sec. 3.2: DSO 810 mm, DSD 1195 mm, 512 x
    364 detector at 0.776 mm."""
    return dict(nx=256, ny=256, nz=256, vx=1.05, vy=1.05, vz=1.05, nu=512, nv=364,
                du=0.776, dv=0.776, dso=810.0, dsd=1195.0, n_views=n_views)


def thorax_case(seed: int = 32):
    """(prior, current): body, two lungs, spine and seeded nodules; the current
    scan adds a needle (radius 1 voxel, length 60 voxels, value 2.0) in a lung."""
    rng = np.random.default_rng(seed)
    n = 256
    vol = np.zeros((n, n, n))
    c = np.array([128.0, 128.0, 128.0])
    add_ellipsoid(vol, c, (118.0, 88.0, 400.0), np.eye(3), 1.0)           # body (all z)
    for sx in (-1, 1):                                                     # lungs
        add_ellipsoid(vol, c + [sx * 48.0, -8.0, 0.0], (36.0, 52.0, 100.0), np.eye(3), -0.75)
    add_ellipsoid(vol, c + [0.0, 66.0, 0.0], (14.0, 14.0, 400.0), np.eye(3), 0.8)  # spine
    for _ in range(10):                                                    # nodules, vessels
        sx = rng.choice([-1, 1])
        cc = c + [sx * 48.0, -8.0, 0.0] + rng.uniform(-25, 25, size=3)
        add_ellipsoid(vol, cc, rng.uniform(2.0, 7.0, size=3), _rotation(rng), 0.7)
    cur = vol.copy()
    axis = random_unit(rng)
    add_cylinder(cur, c + [-48.0, -8.0, 0.0], axis, 1.0, 60.0, 2.0)
    return vol, cur


# --------------------------------------------------------------------------
# Large cases: the 512^3 precision comparison and the repeated-scan sequence.

def c3_case(seed: int = 3):
    """512^3 at 0.5 mm: the 256^3 object family at twice the resolution
    (30 ellipsoids, semi-axes U[32, 192] voxels, scaled to a peak of 1), the
    smallest one grown by 1.3.  Returns (prior = object without the change,
    current)."""
    shape = (512, 512, 512)
    base, ells = ellipsoid_phantom(shape, 30, (32.0, 192.0), seed, threads=8)
    k = int(np.argmin([np.prod(a) for (_, a, _, _) in ells]))
    c, a, R, rho = ells[k]
    cur = base.copy()
    add_ellipsoid(cur, c, a, R, -rho)
    add_ellipsoid(cur, c, 1.3 * a, R, rho)
    scale = 1.0 / base.max()
    return base * scale, cur * scale


def c5_case(seed: int = 5):
    """512 x 512 x 400 at 0.4 mm: 30 ellipsoids (semi-axes U[32, 192] voxels)
    scaled to a peak of 1, and a needle (radius 2.5 voxels, length 100 voxels,
    value 2.0) at a seeded position and direction.  Returns (anatomy, needle
    centre, needle axis); scan s (1..10) has the needle advanced by 7.5 (s - 1)
    voxels along its axis (3 mm per scan)."""
    rng = np.random.default_rng(seed + 100)
    shape = (400, 512, 512)
    base, _ = ellipsoid_phantom(shape, 30, (32.0, 192.0), seed, threads=8)
    base *= 1.0 / base.max()
    centre = np.array([rng.uniform(0.35 * n, 0.55 * n) for n in (512, 512, 400)])
    axis = random_unit(rng)
    return base, centre, axis


def c5_scan(base, centre, axis, scan: int) -> np.ndarray:
    """Flat voxel indices of the needle in scan `scan` (1-based)."""
    return cylinder_indices(base.shape, centre + 7.5 * (scan - 1) * axis, axis, 2.5, 100.0)
