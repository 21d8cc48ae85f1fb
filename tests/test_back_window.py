"""CPU check of the adjoint projector's candidate-row window (no GPU).

The gather form of A^T (k_back) visits, for each voxel cell and each detector
column (view, u) whose rays cross the cell's x-y column, only a window of C
consecutive detector rows.  Every chord the forward projector produces for that
cell must come from a row inside that window, or A^T would silently drop it.
This test emulates, in numpy float32, the device's arithmetic for both sides:

* the float32 plane tables built on the host (per (view, u): x and y plane
  coefficients; per detector row: z coefficients), from the same float64
  formulas rounded the same way;
* the forward's chord of row v in cell k over the column interval [aa, ab]:
  med3(ab, zA, zB) - med3(aa, zA, zB) with zA, zB the cell's two z-plane
  parameters of that row (the forward's c0 / c1 and the adjoint's candidate
  chord are this same expression);
* the detector columns the adjoint visits per view: the images of the voxel
  column's four corners through the approximate reciprocal of their depth,
  widened by a column margin; every (view, u) whose rays cross the voxel column
  must be among them;
* the window's first row, from the approximate reciprocal of the ray parameter
  (v_rcp_f32, at most 1 ulp from the exact reciprocal), folded into
  floor(clamp(-flo, -(nv - C), 0)); and the window size C computed on the host.

Fused multiply-adds are emulated by a float64 product-and-sum rounded to
float32.  That rounding can differ from a true fma by one ulp, so every
quantity that decides the window start is evaluated with each reciprocal and
each result moved by -1, 0, +1 ulp, and a row counts as carrying a chord if
its overlap exceeds minus two ulps of the interval ends.  The check passes only
if every such row lies inside the window for every one of those variants.

Cells checked: the bottom, top and middle z slices (where the sign of the cell
height switches between the window formulas) of the volume's corner and edge
columns and of seeded interior columns, over every view and every detector
column that crosses them, for the benchmark geometries and the tallest accepted
detector.
"""
import math

import numpy as np
import pytest

from paper_2509_08574_amd import synth

F = np.float32


def fma32(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64)
            + np.asarray(c, np.float64)).astype(F)


def med3(t, a, b):
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    return np.maximum(np.minimum(t, hi), lo)


def axis_coeffs(S, d, lo, h, n, a_ref):
    """Float32 plane coefficients (r, c) of one axis for arrays of ray origins S
    and directions d: plane p is crossed at a' = fma(p - n//2, r, c)."""
    d = np.asarray(d, np.float64)
    dpos = d / h
    pos_ref = (S - lo) / h + a_ref * dpos
    rel = pos_ref - (n >> 1)
    par = np.abs(dpos) <= 1e-30
    r = np.where(par, 1e30, 1.0 / np.where(par, 1.0, dpos)).astype(F)
    kc = np.where(pos_ref <= 0.0, -1.0, np.where(pos_ref >= n, float(n), np.floor(pos_ref)))
    c_par = (-(kc - (n >> 1) + 0.5) * 1e30).astype(F)
    c = np.where(par, c_par, (-rel * r.astype(np.float64)).astype(F))
    return r, c


def back_candidates(d):
    """The window size C the host chooses (upper bound on the rows that can meet
    one cell within one column interval, plus the start margin, with 2 % + 0.01
    rows for rounding)."""
    hx, hy = d["nx"] * F(d["vx"]) / 2.0, d["ny"] * F(d["vy"]) / 2.0
    rxy = math.sqrt(float(hx) ** 2 + float(hy) ** 2)
    umax = d["nu"] * float(F(d["du"])) / 2.0
    dsd, dso, dv = float(F(d["dsd"])), float(F(d["dso"])), float(F(d["dv"]))
    amin = (dso - rxy) / math.sqrt(dsd * dsd + umax * umax)
    diag = math.sqrt(float(F(d["vx"])) ** 2 + float(F(d["vy"])) ** 2)
    dA = diag / dsd
    hz = float(F(d["vz"]))
    rz = d["nz"] * hz / 2.0
    span = (hz / amin + rz * dA / (amin * amin)) / dv + margin_rows(d["nv"])
    return min(int(math.floor(span * 1.02 + 0.01)) + 1, d["nv"])


def margin_cols(nu):
    """Detector columns by which the visited range is widened on each side."""
    return 1e-3 + 8.0 * nu * 2.0 ** -23


def margin_rows(nv):
    """Rows by which a window starts early (1e-3 plus eight ulps' worth of nv * 2^-23)."""
    return 1e-3 + 8.0 * nv * 2.0 ** -23


def ulp_steps(x):
    x = np.asarray(x, F)
    return [np.nextafter(x, F(-np.inf)), x, np.nextafter(x, F(np.inf))]


class Tables:
    def __init__(self, d):
        self.d = d
        nx, ny, nz, nu, nv = d["nx"], d["ny"], d["nz"], d["nu"], d["nv"]
        a_ref = d["dso"] / d["dsd"]
        V = d["n_views"]
        ang = np.asarray(d.get("angles") or 2.0 * np.pi * np.arange(V) / V, np.float64)
        c, s = np.cos(ang)[:, None], np.sin(ang)[:, None]
        u = (np.arange(nu) + 0.5) * d["du"] - nu * d["du"] / 2.0
        Sx, Sy = d["dso"] * c, d["dso"] * s
        Px = (d["dso"] - d["dsd"]) * c - u[None] * s
        Py = (d["dso"] - d["dsd"]) * s + u[None] * c
        self.rx, self.cx = axis_coeffs(Sx, Px - Sx, -nx * d["vx"] / 2.0, d["vx"], nx, a_ref)
        self.ry, self.cy = axis_coeffs(Sy, Py - Sy, -ny * d["vy"] / 2.0, d["vy"], ny, a_ref)
        vmm = (np.arange(nv) + 0.5) * d["dv"] - nv * d["dv"] / 2.0
        self.rg, self.cz = axis_coeffs(np.zeros(nv), vmm, -nz * d["vz"] / 2.0, d["vz"], nz,
                                       a_ref)
        self.C = back_candidates(d)
        # kernel constants, formed in float32 as in the launch and the kernel
        self.a_ref = F(F(d["dso"]) / F(d["dsd"]))
        self.a_ref_dv = F(self.a_ref * F(d["dv"]))
        self.fv_off = F(0.5 * nv - 0.5 - margin_rows(nv))
        self.nrwin = F(-(nv - self.C))
        self.z_lo = F(F(F(-0.5) * F(nz)) * F(d["vz"]))

    def interval(self, i, j):
        """(aa, ab) over every (view, u) for voxel column (i, j)."""
        d = self.d
        px, py = F(i - (d["nx"] >> 1)), F(j - (d["ny"] >> 1))
        ex0, ex1 = fma32(px, self.rx, self.cx), fma32(px + F(1), self.rx, self.cx)
        ey0, ey1 = fma32(py, self.ry, self.cy), fma32(py + F(1), self.ry, self.cy)
        aa = np.maximum(np.minimum(ex0, ex1), np.minimum(ey0, ey1))
        ab = np.minimum(np.maximum(ex0, ex1), np.maximum(ey0, ey1))
        return aa, ab

    def u_range_bounds(self, i, j):
        """Per view: the start and end of the visited detector columns that hold
        for every rounding variant (the latest start, the earliest end)."""
        d = self.d
        nx, ny, nu = d["nx"], d["ny"], d["nu"]
        hx, hy = F(d["vx"]), F(d["vy"])
        xlo = F(F(F(i) - F(F(0.5) * F(nx))) * hx)
        ylo = F(F(F(j) - F(F(0.5) * F(ny))) * hy)
        xhi, yhi = F(xlo + hx), F(ylo + hy)
        fu_scale = F(F(d["dsd"]) / F(d["du"]))
        fu_off = F(F(F(0.5) * F(nu)) - F(0.5))
        mu = F(margin_cols(nu))
        V = d["n_views"]
        ang = np.asarray(d.get("angles") or 2.0 * np.pi * np.arange(V) / V, np.float64)
        cs, sn = np.cos(ang).astype(F), np.sin(ang).astype(F)
        # per corner, the lowest and highest image over the variants
        img_lo, img_hi = [], []
        for X, Y in ((xlo, ylo), (xhi, ylo), (xlo, yhi), (xhi, yhi)):
            depth = (F(d["dso"]) - (X * cs + Y * sn).astype(F)).astype(F)
            lat = (Y * cs - X * sn).astype(F)
            rc = (1.0 / depth.astype(np.float64)).astype(F)
            vals = [fu for r in ulp_steps(rc)
                    for fu in ulp_steps(fma32((lat * r).astype(F), fu_scale, fu_off))]
            img_lo.append(np.min(vals, axis=0))
            img_hi.append(np.max(vals, axis=0))
        # the kernel starts at ceil(min over corners - margin); the latest such
        # start takes each corner's highest variant
        start = np.maximum(0, np.ceil(np.min(img_hi, axis=0) - mu).astype(np.int64))
        end = np.minimum(nu - 1, np.floor(np.max(img_lo, axis=0) + mu).astype(np.int64))
        return start, end

    def window_starts(self, k, aa, ab):
        """(lowest, highest) window start over the rounding variants, per entry."""
        d = self.d
        zk0 = fma32(F(k), F(d["vz"]), self.z_lo)
        t = np.where(zk0 >= 0, ab, aa)
        den = fma32(t, F(d["dv"]), self.a_ref_dv)
        exact = (1.0 / den.astype(np.float64)).astype(F)
        lo_r, hi_r = None, None
        for ia in ulp_steps(exact):
            for nflo in ulp_steps(fma32(-zk0, ia, -self.fv_off)):
                m = np.floor(med3(nflo, self.nrwin, F(0.0))).astype(np.int64)
                r0 = -m
                lo_r = r0 if lo_r is None else np.minimum(lo_r, r0)
                hi_r = r0 if hi_r is None else np.maximum(hi_r, r0)
        return lo_r, hi_r

    def chord_rows(self, k, aa, ab, rows):
        """Mask [entry, row] of rows whose chord with cell k over [aa, ab] is
        positive (the overlap of [aa, ab] with the cell's interval of that row,
        med3(ab, zA, zB) - med3(aa, zA, zB)), counting also rows that miss by up
        to two ulps of the cell's plane parameters."""
        fk = F(k - (self.d["nz"] >> 1))
        rg, cz = self.rg[rows], self.cz[rows]
        zA, zB = fma32(fk, rg, cz), fma32(fk + F(1), rg, cz)
        zmin, zmax = np.minimum(zA, zB), np.maximum(zA, zB)
        for _ in range(2):
            zmin, zmax = np.nextafter(zmin, F(-np.inf)), np.nextafter(zmax, F(np.inf))
        return np.minimum(ab[:, None], zmax) > np.maximum(aa[:, None], zmin)


def columns(d, n_random=24, seed=0):
    """The four corner columns first, then edge and seeded interior columns."""
    nx, ny = d["nx"], d["ny"]
    corners = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]
    cols = {(nx // 2, 0), (nx // 2, ny - 1), (0, ny // 2), (nx - 1, ny // 2)}
    for t in range(0, max(nx, ny), max(1, max(nx, ny) // 8)):
        cols |= {(min(t, nx - 1), 0), (min(t, nx - 1), ny - 1), (0, min(t, ny - 1)),
                 (nx - 1, min(t, ny - 1))}
    rng = np.random.default_rng(seed)
    for _ in range(n_random):
        cols.add((int(rng.integers(nx)), int(rng.integers(ny))))
    return list(dict.fromkeys(corners)) + sorted(cols - set(corners))


def check_geometry(d, full_rows_cols=4, band=6):
    """Returns the number of (cell, view, u) windows checked; asserts coverage."""
    T = Tables(d)
    nz, nv, C = d["nz"], d["nv"], T.C
    ks = sorted({0, 1, nz // 2 - 1, nz // 2, nz - 2, nz - 1} & set(range(nz)))
    checked = 0
    for ci, (i, j) in enumerate(columns(d)):
        aa, ab = T.interval(i, j)
        # every detector column whose rays cross (i, j) must be visited
        start, end = T.u_range_bounds(i, j)
        views, us = np.nonzero(ab > aa)
        assert ((us >= start[views]) & (us <= end[views])).all(), (
            f"column ({i}, {j}): a detector column crossing it lies outside the visited range")
        sel = ab > aa
        aa, ab = aa[sel], ab[sel]
        if aa.size == 0:
            continue
        for k in ks:
            r_lo, r_hi = T.window_starts(k, aa, ab)
            if ci < full_rows_cols:
                rows = np.arange(nv)[None, :].repeat(aa.size, 0)
            else:
                # rows around the window; the corner columns above check every row
                base = np.clip(r_lo - band, 0, None)
                rows = np.minimum(base[:, None] + np.arange(C + 2 * band)[None, :], nv - 1)
            mask = T.chord_rows(k, aa, ab, rows)
            bad = mask & ((rows < r_hi[:, None]) | (rows > (r_lo + C - 1)[:, None]))
            assert not bad.any(), (
                f"column ({i}, {j}) cell {k}: a chord row lies outside its window "
                f"(C = {C}); first offending entry {np.argwhere(bad)[0]}")
            checked += aa.size
    return checked


GEOMS = {
    "c2": synth.geometry("c2"),
    "c3_512": synth.geometry("c3_512"),
    "c5": synth.geometry("c5"),
    # the tallest accepted detector (16384 rows): row positions near 8192 carry
    # float32 rounding of about 5e-4 rows
    "max_nv": dict(nx=5, ny=4, nz=8, vx=0.01, vy=0.01, vz=1.0, nu=2, nv=16384, du=0.05,
                   dv=0.5, dso=40.0, dsd=70.0, n_views=3),
    # a tall volume seen on 16384 rows: its top and bottom cells meet rows about
    # 6700 rows from the centre (row positions 1500 and 14900), where a float32
    # row position is rounded by up to 5e-4 rows
    "far_rows": dict(nx=4, ny=4, nz=3200, vx=0.5, vy=0.5, vz=1.0, nu=8, nv=16384, du=0.5,
                     dv=0.4, dso=3000.0, dsd=5000.0, n_views=16),
    # a wide detector (16384 columns) whose outer voxel columns project about
    # 6000 columns from the centre, where float32 column positions are rounded
    # by up to 5e-4 columns
    "far_cols": dict(nx=3000, ny=3000, nz=4, vx=1.0, vy=1.0, vz=1.0, nu=16384, nv=8,
                     du=0.4, dv=1.0, dso=4000.0, dsd=6500.0, n_views=16),
}


@pytest.mark.parametrize("name", list(GEOMS))
def test_every_forward_chord_is_inside_its_adjoint_window(name):
    d = GEOMS[name]
    n = check_geometry(d)
    assert n > 0


def test_window_size_is_small_and_bounded():
    # the benchmark geometries keep the window at three or four rows; every
    # geometry here is one the adjoint accepts (at most 8 rows per window)
    for name in ("c2", "c3_512", "c5"):
        assert 2 <= back_candidates(GEOMS[name]) <= 4, name
    for name, d in GEOMS.items():
        assert back_candidates(d) <= 8, name


def test_planted_narrow_window_is_caught():
    """With one row fewer than the host's bound the check must fail somewhere
    (it is not vacuous)."""
    d = GEOMS["c2"]
    T = Tables(d)
    C = T.C - 1
    found = False
    for (i, j) in columns(d, n_random=4)[:12]:
        aa, ab = T.interval(i, j)
        sel = ab > aa
        aa, ab = aa[sel], ab[sel]
        for k in (0, d["nz"] - 1, d["nz"] // 2):
            r_lo, r_hi = T.window_starts(k, aa, ab)
            rows = np.minimum(np.clip(r_lo - 6, 0, None)[:, None] + np.arange(C + 12)[None, :],
                              d["nv"] - 1)
            mask = T.chord_rows(k, aa, ab, rows)
            found |= bool((mask & (rows > (r_lo + C - 1)[:, None])).any())
    assert found
