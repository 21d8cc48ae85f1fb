"""Host-side checks of the kernels' block-to-work maps (no GPU needed).

The maps are restated here from csrc/chord.h (xcd_remap), csrc/proj.hip (the
forward's view-grouped block order) and csrc/piccs.hip (the stencils' plane
slabs, one or two planes per thread), and checked for what the kernels rely on:
every unit of work is taken exactly once, idle blocks are exactly the padding,
and the XCD shares are contiguous.
"""
import itertools

import pytest


def xcd_remap(b, n):
    q, r = n >> 3, n & 7
    x, idx = b & 7, b >> 3
    return x * q + (x if x < r else r) + idx


@pytest.mark.parametrize("n", [1, 7, 8, 9, 64, 1000, 4099])
def test_xcd_remap_is_a_permutation_with_contiguous_shares(n):
    seen = [xcd_remap(b, n) for b in range(n)]
    assert sorted(seen) == list(range(n))
    # blocks dispatched to one XCD (b mod 8 fixed) map to one contiguous range, in order
    for x in range(8):
        mine = [xcd_remap(b, n) for b in range(x, n, 8)]
        assert mine == list(range(mine[0], mine[0] + len(mine))) if mine else True


def fwd_rpl(nv):
    def padded(rpl):
        rb, h = 64 * rpl, nv // 2
        return ((h + rb - 1) // rb + (nv - h + rb - 1) // rb) * rb
    if nv // 2 < 128:
        return 1
    best = min(padded(2), padded(3))
    if nv // 2 >= 256 and 20 * padded(4) < 21 * best:
        return 4
    if nv // 2 >= 192 and 20 * padded(3) < 21 * padded(2):
        return 3
    return 2


@pytest.mark.parametrize("nviews, nu, nv, group", [
    (7, 11, 13, 3), (9, 30, 150, 3), (180, 64, 1024, 3), (90, 40, 512, 3), (1, 12, 10, 3),
    (13, 37, 150, 4), (11, 23, 70, 5)])
def test_forward_block_order_covers_every_column_block_once(nviews, nu, nv, group):
    rb_rows = 64 * fwd_rpl(nv)
    h = nv // 2
    nlo, nhi = (h + rb_rows - 1) // rb_rows, (nv - h + rb_rows - 1) // rb_rows
    nrb, nub = nlo + nhi, (nu + 3) >> 2
    ngroups = (nviews + group - 1) // group
    nb = ngroups * group * nrb * nub
    work, idle = [], 0
    for blk in range(nb):
        b = xcd_remap(blk, nb)
        vl, t0 = b % group, b // group
        ub, t = t0 % nub, t0 // nub
        rb, view = t % nrb, (t // nrb) * group + vl
        if view < nviews:
            work.append((view, ub, rb))
        else:
            idle += 1
    assert sorted(work) == sorted(itertools.product(range(nviews), range(nub), range(nrb)))
    assert idle == (ngroups * group - nviews) * nrb * nub


def vox_cells(nx, ny, nz, planes):
    nkb, nxb = (nz + 63) >> 6, (nx + 3) >> 2
    P = nkb * nxb
    S = (P + 7) >> 3
    nblocks = 8 * S * ((ny + planes - 1) // planes)
    cells = []
    for blk in range(nblocks):
        s = blk >> 3
        jg = s // S
        p = (blk & 7) * S + (s - jg * S)
        for w in range(4):
            for lane in range(64):
                i, k, j = (p // nkb) * 4 + w, (p % nkb) * 64 + lane, jg * planes
                if not (p < P and i < nx and k < nz):
                    continue
                cells.append((i, j, k))
                if planes == 2 and j + 1 < ny:
                    cells.append((i, j + 1, k))
    return cells


@pytest.mark.parametrize("nx, ny, nz", [(13, 1, 70), (13, 2, 70), (13, 7, 70), (4, 8, 64),
                                        (21, 19, 17), (9, 5, 130)])
@pytest.mark.parametrize("planes", [1, 2])
def test_stencil_slabs_cover_every_cell_once(nx, ny, nz, planes):
    cells = vox_cells(nx, ny, nz, planes)
    assert len(cells) == nx * ny * nz
    assert set(cells) == set(itertools.product(range(nx), range(ny), range(nz)))
