// Chord arithmetic shared by the forward projector and its transpose.
//
// Both kernels evaluate every chord with exactly these float32 operations
// (the library is built with -ffp-contract=off), so the matrix applied by the
// back projector is entry-for-entry the transpose of the forward one.
//
// Ray parameter.  A ray runs from the source S (alpha = 0) to a pixel centre P
// (alpha = 1); its length is L = |P - S|, so a parameter interval d(alpha)
// covers d(alpha) * L mm.  Kernels use a' = alpha - DSO/DSD, which is zero at
// the depth of the isocentre and small across the volume (better float32
// resolution than alpha itself).
//
// Plane crossings.  Plane indices are counted from the middle of each axis,
// o = n / 2 (integer division).  In voxel-index units the ray's x position is
// o + xi(a'), xi(a') = xi0 + a' * dxi, so x-plane p (p = 0..nx) is crossed at
// a' = (p - o - xi0) / dxi = fma(p - o, rx, cx) with rx = 1/dxi in float and
// cx = -xi0 * rx rounded once from float64 on the host; likewise for y (ry,
// cy) and z (rg, cz).  Coefficients come from per-(view, u) and per-row
// tables.  Relative plane indices keep the cancellation in the fma to the
// ray's distance from the axis midpoint.
//
// Rays are traversed column by column (a column = all z cells of one (i, j)):
// every ray of one detector column u crosses the same sequence of (i, j)
// columns over the same a'-intervals, and within one column's interval
// [aa, ab] a ray meets at most two z cells (the geometry check guarantees it
// crosses at most one z plane there).  With k the cell at aa and an the
// a'-value of its exit plane, the two chords are
//     c0 = min(ab, an) - aa      in cell k,
//     c1 = ab - min(ab, an)      in cell k + s   (s = z direction, +-1),
// in parameter units; multiplying by L gives millimetres.
#pragma once

#include <hip/hip_runtime.h>

namespace cbct {

__device__ __forceinline__ float plane_alpha(float p, float r, float c) { return fmaf(p, r, c); }

// Cell of the x (or y) grid that contains the ray at parameter a, i.e. the
// cell whose entry plane is crossed at or before a and whose exit plane after
// a; clamped to [0, n-1].  Works in indices relative to o = n / 2 and returns
// the absolute cell.  c0 is the relative index position at a' = 0 (guess only).
__device__ __forceinline__ int xy_cell(float a, float c0, float r, float c, int n) {
    const int o = n >> 1;
    const float lo = (float)(-o), hi = (float)(n - 1 - o);
    const float d = 1.0f / r;
    float t = floorf(fmaf(a, d, c0));
    t = fminf(fmaxf(t, lo), hi);
    const float up = r > 0.0f ? 1.0f : 0.0f;
    const float s = r > 0.0f ? 1.0f : -1.0f;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const float tn = t + s;
        if (!(plane_alpha(t + up, r, c) > a) && tn >= lo && tn <= hi) t = tn;
        const float tp = t - s;
        if (plane_alpha(t + 1.0f - up, r, c) > a && tp >= lo && tp <= hi) t = tp;
    }
    return (int)t + o;
}

// z state of one ray at parameter a: cell k (absolute, clamped to the pad
// cells -1 / nz), exit plane pe of that cell (relative to o = nz / 2) and its
// parameter an.  The cell is the one whose entry plane lies strictly before a
// and whose exit plane lies at or after a.  A ray outside the z range sits in
// the pad cell on its side: below the volume moving up it is in cell -1 whose
// exit plane is 0 (and symmetrically above), so it enters the volume exactly
// at the boundary plane.
// zr = (z0, rg, cz, dz) for the ray's detector row.
__device__ __forceinline__ void zlane_init(float a, float4 zr, int nz, int &k, float &pe,
                                           float &an) {
    const float z0 = zr.x, rg = zr.y, cz = zr.z, dz = zr.w;
    const int o = nz >> 1;
    const float up = rg > 0.0f ? 1.0f : 0.0f;
    const float s = rg > 0.0f ? 1.0f : -1.0f;
    float kt = floorf(fmaf(a, dz, z0));
    if (!(plane_alpha(kt + up, rg, cz) >= a)) kt += s;
    if (!(plane_alpha(kt + 1.0f - up, rg, cz) < a)) kt -= s;
    kt = fminf(fmaxf(kt, (float)(-1 - o)), (float)(nz - o));
    k = (int)kt + o;
    pe = kt + up;
    an = plane_alpha(pe, rg, cz);
}

// Block id remap for the 8 XCDs of MI355X: the dispatcher hands consecutive
// block ids to XCDs round-robin; this gives every XCD a contiguous range of
// logical tiles so that neighbouring tiles share that XCD's L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned n) {
    const unsigned q = n >> 3, r = n & 7u;
    const unsigned x = b & 7u, idx = b >> 3;
    return x * q + (x < r ? x : r) + idx;
}

}  // namespace cbct
