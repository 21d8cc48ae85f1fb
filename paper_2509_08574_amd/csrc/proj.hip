// Cone-beam projector pair for gfx950: forward A and its exact transpose A^T.
//
// A is the sensing matrix of the linear CT model (paper Sec. 2.1, eq. "tomo"),
// read as exact ray/voxel chord lengths; Krylov solvers touch it only through
// products with A and A^T (Sec. 2.2.2).  Chord arithmetic: chord.h.
//
// Forward (k_fwd): one wave per (view, detector column u, 64 to 256 detector
// rows); each lane walks one to four rows.  All rays of one detector column
// share their x-y path, so the wave walks the voxel columns (i, j) it crosses
// in lock-step (uniform control flow) while every lane tracks its own z cell.
// Volumes are stored column-major (z fastest), so at each step the lanes read a
// short contiguous run of one column: coalesced gathers for every view angle.
//
// Back (k_back): one wave per voxel column (i, j), columns taken in 8 x 16
// tiles.  For every view, the wave visits the detector columns u whose rays
// cross (i, j) and recomputes the forward walk's x-y interval [aa, ab]; each
// lane then gathers, for each of its cells, a short window of detector rows
// whose chords with that cell are the forward kernel's c0 / c1 bit for bit.
// The views run in chunks of one launch each (back_views_per_launch); every
// cell is summed over the views in a fixed order, with no atomics.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>

#include "chord.h"
#include "internal.h"

namespace cbct {

// ---------------------------------------------------------------- segment tables

// One thread per detector column (view, iu): the x-y traversal shared by all
// rows of that column.  The sequence of (exit parameter, voxel column) uses the
// same plane values k_back recomputes per column from its four bounding planes.
__global__ void __launch_bounds__(256)
k_segtab(GeoK G, int2 *__restrict__ seghdr, int2 *__restrict__ seg) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= G.nviews * G.nu) return;
    const float4 cxy = G.xy[r];    // (rx, cx, ry, cy)
    const float2 c0 = G.xy0[r];    // (xi0, eta0)
    // plane indices relative to the axis midpoints
    const int ox = G.nx >> 1, oy = G.ny >> 1;
    const float ax0 = plane_alpha((float)(-ox), cxy.x, cxy.y);
    const float axN = plane_alpha((float)(G.nx - ox), cxy.x, cxy.y);
    const float ay0 = plane_alpha((float)(-oy), cxy.z, cxy.w);
    const float ayN = plane_alpha((float)(G.ny - oy), cxy.z, cxy.w);
    const float a_in = fmaxf(fminf(ax0, axN), fminf(ay0, ayN));
    const float a_out = fminf(fmaxf(ax0, axN), fmaxf(ay0, ayN));
    int2 *out = seg + (size_t)r * G.seg_stride;
    int n = 0;
    if (a_out > a_in) {
        const int sx = cxy.x > 0.0f ? 1 : -1, sy = cxy.z > 0.0f ? 1 : -1;
        int i = xy_cell(a_in, c0.x, cxy.x, cxy.y, G.nx);
        int j = xy_cell(a_in, c0.y, cxy.z, cxy.w, G.ny);
        float axn = plane_alpha((float)(i - ox + (sx > 0)), cxy.x, cxy.y);
        float ayn = plane_alpha((float)(j - oy + (sy > 0)), cxy.z, cxy.w);
        const int nmax = G.seg_stride - kSegPad;
        while (n < nmax) {
            const float ab = fminf(axn, ayn);
            out[n++] = make_int2(__float_as_int(ab), j * G.nx + i);
            const bool adx = axn == ab, ady = ayn == ab;
            if (adx) {
                i += sx;
                axn = plane_alpha((float)(i - ox + (sx > 0)), cxy.x, cxy.y);
            }
            if (ady) {
                j += sy;
                ayn = plane_alpha((float)(j - oy + (sy > 0)), cxy.z, cxy.w);
            }
            if ((unsigned)i >= (unsigned)G.nx || (unsigned)j >= (unsigned)G.ny) break;
        }
    }
    // no-op entries: zero-length segments at the exit parameter, column 0
    const int last = n > 0 ? out[n - 1].x : __float_as_int(a_in);
    for (int q = 0; q < kSegPad; ++q) out[n + q] = make_int2(last, 0);
    seghdr[r] = make_int2(__float_as_int(a_in), n);
}

void launch_segment_tables(const GeoK &G, int2 *seghdr, int2 *seg, hipStream_t s) {
    const int nr = G.nviews * G.nu;
    hipLaunchKernelGGL(k_segtab, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, G, seghdr,
                       seg);
    CBCT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- forward

// Detector rows are grouped in blocks that never straddle the detector's
// centre: rows [0, h) (rays going down, v < 0) in blocks counted down from h,
// rows [h, nv) (rays going up) in blocks counted up from h, h = nv / 2.  The z
// direction is therefore uniform within a wave.

constexpr int kBufWord3 = 0x00020000;  // raw buffer resource, 32-bit dwords (gfx9 family)

__device__ __forceinline__ float ldb(__amdgpu_buffer_rsrc_t r, int off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Storage element of the forward projector's input volume: float32, or a
// 16-bit shadow (bf16, or fp16 holding value * scale) widened on load.
template <int DT>
struct Elem;
template <>
struct Elem<CBCT_F32> {
    static constexpr int size = 4;
    __device__ static float load(__amdgpu_buffer_rsrc_t r, int off) { return ldb(r, off); }
};
template <>
struct Elem<CBCT_BF16> {
    static constexpr int size = 2;
    __device__ static float load(__amdgpu_buffer_rsrc_t r, int off) {
        const unsigned h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return __uint_as_float(h << 16);
    }
};
template <>
struct Elem<CBCT_F16> {
    static constexpr int size = 2;
    __device__ static float load(__amdgpu_buffer_rsrc_t r, int off) {
        const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
        return __half2float(__ushort_as_half(h));
    }
};
// Pair words (CBCT_BF16_PAIR / CBCT_F16_PAIR): 4 bytes per cell, word k holding
// cells k and k + 1.
template <>
struct Elem<CBCT_BF16_PAIR> {
    static constexpr int size = 4;
    __device__ static void load2(__amdgpu_buffer_rsrc_t r, int off, float &lo, float &hi) {
        const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        lo = __uint_as_float(w << 16);
        hi = __uint_as_float(w & 0xffff0000u);
    }
};
template <>
struct Elem<CBCT_F16_PAIR> {
    static constexpr int size = 4;
    __device__ static void load2(__amdgpu_buffer_rsrc_t r, int off, float &lo, float &hi) {
        const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        lo = __half2float(__ushort_as_half((unsigned short)(w & 0xffffu)));
        hi = __half2float(__ushort_as_half((unsigned short)(w >> 16)));
    }
};
template <int DT>
constexpr bool kPairs = DT == CBCT_BF16_PAIR || DT == CBCT_F16_PAIR;

// Bytes of one column's buffer record, counted from one cell below the column:
// reads past it return 0.  Single cells: up to cell nz + 1 (the next column's
// bottom pad).  Pair words: up to word nz (top pad and the next column's bottom
// pad); word nz + 1 would carry the next column's first cell in its high half.
template <int DT>
__host__ __device__ constexpr int fwd_record_bytes(int nz) {
    return kPairs<DT> ? (nz + 2) * 4 : (nz + 3) * Elem<DT>::size;
}

// One x-y segment [aa, ab] of a row's walk: chords c0 (cell k) and c1 (cell
// k + DIR), z-crossing update, then the next column's reads are issued before
// this segment's products so their latency overlaps the arithmetic.
//
// The z state is the integer index pk of the current cell's exit plane
// (relative to nz / 2); the exit plane's parameter is fma(pk, rg, cz) and the
// lower of the two cells read sits at byte offset (pk + nz/2 + 1) * size from
// one cell below the column, in both directions.  Moving up, a ray that has
// left the volume reads the next column's bottom pad and then offsets past
// the buffer record (both read as zero), so only the downward walk needs a
// clamp, at offset 0.
template <int DIR, int MODE, int DT>
struct FwdLane {
    using E = Elem<DT>;
    float aa, an, rg, cz, acc;
    int pk;           // exit plane of the current cell, relative to nz / 2
    int ob;           // byte offset of the lower cell read, from one cell below the column
    int obase;        // nz / 2 + 1
    int nrec, Z, nz;
    const char *vol_c;
    unsigned cnt;

    __device__ __forceinline__ void step(int2 e, float lo, float hi, int2 enext, float &nlo,
                                         float &nhi) {
        const float ab = __int_as_float(e.x);
        const float m = fminf(ab, an);
        const float c0 = m - aa;
        const float c1 = ab - m;
        const float vcur = DIR > 0 ? lo : hi, vnext = DIR > 0 ? hi : lo;
        if constexpr (MODE == FWD_COUNT) {
            const int kc = ob / E::size - (DIR > 0 ? 1 : 0);
            cnt += (c0 > 0.0f && kc >= 0 && kc < nz) ? 1u : 0u;
            cnt += (c1 > 0.0f && kc + DIR >= 0 && kc + DIR < nz) ? 1u : 0u;
        }
        // at most one z plane per segment: step the plane index by 0 or DIR and
        // re-evaluate the exit plane either way (the same fma on the same index
        // gives the same value), rather than selecting between two candidates
        const int cross = an < ab ? 1 : 0;
        pk += DIR > 0 ? cross : -cross;
        an = plane_alpha((float)pk, rg, cz);
        ob = (pk + obase) * E::size;
        if constexpr (DIR < 0) ob = max(ob, -E::size);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(vol_c + (uint64_t)(uint32_t)enext.y * (uint32_t)(Z * E::size)), 0, nrec,
            kBufWord3);
        if constexpr (DT == CBCT_F32) {
            // The next segment reads its second cell (k + DIR) only if it crosses
            // a z plane; otherwise that cell's chord is exactly 0 and the read is
            // skipped (0 stands in, so the product adds exactly nothing).  With
            // float32 storage the reads are the projector's limit (lane data
            // delivered by the L1), not arithmetic.
            const bool next_crosses = an < __int_as_float(enext.x);
            if constexpr (DIR > 0) {
                nlo = E::load(rs, ob);
                if (next_crosses) nhi = E::load(rs, ob + E::size);
            } else {
                nhi = E::load(rs, ob + E::size);
                if (next_crosses) nlo = E::load(rs, ob);
            }
        } else if constexpr (kPairs<DT>) {
            // one aligned word holds both cells: (k, k + 1) moving up, (k - 1, k)
            // moving down
            E::load2(rs, ob, nlo, nhi);
        } else {
            // 16-bit storage halves the data; a masked 16-bit read would be merged
            // into half a register and waited for at once, so both cells are read
            nlo = E::load(rs, ob);
            nhi = E::load(rs, ob + E::size);
        }
        if constexpr (MODE != FWD_COUNT) {
            acc = fmaf(c0, vcur, acc);
            acc = fmaf(c1, vnext, acc);
        }
        aa = ab;
    }
};

// Walk the x-y segments of one detector column for RPL rows per lane moving in
// z direction DIR.  Two segments per loop trip with alternating registers, so
// the one-ahead reads never need to be copied (and waited for) early; with two
// or four rows per lane the walks share the segment stream and multiply the reads in
// flight.
template <int DIR, int MODE, int RPL, int DT>
__device__ __forceinline__ void fwd_walk(const GeoK &G, const void *vol, const int2 *sp,
                                         int nseg, float a_in, const float4 *czr, float *acc,
                                         unsigned *cnt) {
    using E = Elem<DT>;
    FwdLane<DIR, MODE, DT> L[RPL];
    // b0, b1 start at zero: a skipped second-cell read leaves the previous value
    float a0[RPL], a1[RPL], b0[RPL] = {}, b1[RPL] = {};
    int2 e0 = sp[0], e1 = sp[1], e2 = sp[2];
    const char *vol_c = (const char *)vol;
    const __amdgpu_buffer_rsrc_t rs0 = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(vol_c + (size_t)e0.y * G.Z * E::size), 0, fwd_record_bytes<DT>(G.nz),
        kBufWord3);
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
        int k;
        float pe;
        zlane_init(a_in, czr[p], G.nz, k, pe, L[p].an);
        L[p].aa = a_in;
        L[p].rg = czr[p].y;
        L[p].cz = czr[p].z;
        L[p].acc = 0.0f;
        L[p].cnt = 0;
        L[p].pk = (int)pe;
        L[p].obase = G.nz >> 1;
        L[p].ob = (k + (DIR > 0 ? 1 : 0)) * E::size;  // = (pk + obase) * size
        L[p].nrec = fwd_record_bytes<DT>(G.nz);
        L[p].Z = G.Z;
        L[p].nz = G.nz;
        L[p].vol_c = vol_c;
        if constexpr (kPairs<DT>) {
            E::load2(rs0, L[p].ob, a0[p], a1[p]);
        } else {
            a0[p] = E::load(rs0, L[p].ob);
            a1[p] = E::load(rs0, L[p].ob + E::size);
        }
    }
    // Entries past the last segment are no-op segments (zero length, exit
    // parameter, column 0), so the walk runs in whole pairs and reads table
    // entries one pair ahead.
    for (int n = 0; n < nseg; n += 2) {
        const int2 e3 = sp[n + 3], e4 = sp[n + 4];
#pragma unroll
        for (int p = 0; p < RPL; ++p) L[p].step(e0, a0[p], a1[p], e1, b0[p], b1[p]);
#pragma unroll
        for (int p = 0; p < RPL; ++p) L[p].step(e1, b0[p], b1[p], e2, a0[p], a1[p]);
        e0 = e2;
        e1 = e3;
        e2 = e4;
    }
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
        acc[p] = L[p].acc;
        cnt[p] = L[p].cnt;
    }
}

// Detector rows the forward grid covers with `rpl` rows per lane: each half is
// rounded up to whole blocks of 64 * rpl rows (blocks never straddle the centre).
__host__ __device__ inline int fwd_padded_rows(int nv, int rpl) {
    const int rb = 64 * rpl, h = nv / 2;
    return ((h + rb - 1) / rb + (nv - h + rb - 1) / rb) * rb;
}

// Rows per lane of the forward kernel.  Rows of one lane share the segment
// stream's scalar work, which co-limits the walk, so more rows per lane cost
// less per row (four against two: about 6 %); but larger blocks can leave lanes
// idle.  The most rows per lane (4, 3, 2) whose blocks pad the detector by under
// 5 % more rows than the tightest choice; one below 128 rows per half.
__host__ __device__ inline int fwd_rpl(int nv) {
    if (nv / 2 < 128) return 1;
    const int best = min(fwd_padded_rows(nv, 2), fwd_padded_rows(nv, 3));
    if (nv / 2 >= 256 && 20 * fwd_padded_rows(nv, 4) < 21 * best) return 4;
    if (nv / 2 >= 192 && 20 * fwd_padded_rows(nv, 3) < 21 * fwd_padded_rows(nv, 2)) return 3;
    return 2;
}

// Views per group in the forward's block order.  Blocks of a few consecutive
// views at the same detector columns and rows run side by side on one XCD; their
// rays cross nearly the same voxels (the views are a few degrees apart), which
// the XCD's L2 then serves to all of them.  Measured per A (views per group:
// ms), 512 x 512 x 400 / 180 views: 1: 34.5, 2: 33.7, 3: 31.7, 6: 32.1;
// 256^3 / 90 views: 1: 2.17, 2: 2.10, 3: 2.05, 6: 2.06.  Results are the same
// bits for every grouping.
#ifndef CBCT_FWD_VIEW_GROUP
#define CBCT_FWD_VIEW_GROUP 3
#endif
constexpr int kFwdViewGroup = CBCT_FWD_VIEW_GROUP;

template <int MODE, int RPL, int DT>
__global__ void __launch_bounds__(256)
k_fwd(GeoK G, FwdArgs a) {
    if constexpr (MODE == FWD_SOLVER) {
        if (*a.brk == 2) return;
    }
    constexpr int RB = 64 * RPL;  // rows per wave
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = G.nv / 2;
    const int nlo = (h + RB - 1) / RB, nhi = (G.nv - h + RB - 1) / RB, nrb = nlo + nhi;
    const int nub = (G.nu + 3) >> 2;
    // block order within an XCD's share: kFwdViewGroup consecutive views, then
    // 4-column u blocks, then row blocks, then view groups
    const unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const int vl = (int)(b % (unsigned)kFwdViewGroup);
    const unsigned t0 = b / (unsigned)kFwdViewGroup;
    const int ub = (int)(t0 % (unsigned)nub);
    const unsigned t = t0 / (unsigned)nub;
    const int rb = (int)(t % (unsigned)nrb);
    const int view_g = (int)(t / (unsigned)nrb) * kFwdViewGroup + vl;
    const bool vok = view_g < G.nviews;  // the last group may be short
    const int view = vok ? view_g : G.nviews - 1;
    const bool up = rb >= nlo;
    const int iu = ub * 4 + w;
    const int iuc = iu < G.nu ? iu : G.nu - 1;

    int iv[RPL], ivc[RPL];
    bool rowok[RPL];
    float4 czr[RPL];
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
        iv[p] = up ? h + (rb - nlo) * RB + 64 * p + lane : h - (rb + 1) * RB + 64 * p + lane;
        rowok[p] = up ? iv[p] < G.nv : iv[p] >= 0;
        ivc[p] = rowok[p] ? iv[p] : (up ? G.nv - 1 : 0);
        czr[p] = G.zr[ivc[p]];
    }

    const int r = view * G.nu + iuc;  // wave-uniform
    const int2 hdr = G.seghdr[r];
    const int nseg = vok ? hdr.y : 0;
    const int2 *sp = G.seg + (size_t)r * G.seg_stride;

    float acc[RPL];
    unsigned cnt[RPL];
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
        acc[p] = 0.0f;
        cnt[p] = 0;
    }
    if (nseg > 0) {
        const float a_in = __int_as_float(hdr.x);
        if (up)
            fwd_walk<1, MODE, RPL, DT>(G, a.vol, sp, nseg, a_in, czr, acc, cnt);
        else
            fwd_walk<-1, MODE, RPL, DT>(G, a.vol, sp, nseg, a_in, czr, acc, cnt);
    }

    if constexpr (MODE == FWD_COUNT) {
        unsigned c = 0;
#pragma unroll
        for (int p = 0; p < RPL; ++p) c += (vok && iu < G.nu && rowok[p]) ? cnt[p] : 0u;
        if (c) atomicAdd(a.count, (unsigned long long)c);
        return;
    }
    double sq = 0.0;
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
        const bool ok = vok && iu < G.nu && rowok[p];
        const size_t o = ((size_t)view * G.nu + iuc) * G.nv + ivc[p];
        const float L2 = G.Lu2[iuc] + G.Lv2[ivc[p]];
        if constexpr (MODE == FWD_PLAIN) {
            if (ok) a.out[o] = sqrtf(L2) * acc[p] * a.scale;
        } else {
            // u-hat = L * u, u = s1 * (A v) + s2 * u_old  =>  u-hat = s1 L^2 acc + s2 u-hat_old
            const float s1 = (float)*a.s1, s2 = (float)*a.s2;
            float un = s1 * (L2 * acc[p]);
            if (s2 != 0.0f) un = fmaf(s2, a.uin[o], un);
            if (ok) {
                a.out[o] = un;
                sq += (double)un * (double)un / (double)L2;  // |u|^2 = u-hat^2 / L^2
                // the adjoint's 16-bit input (*_ADJ16 forms): the same value rounded
                if (a.u16) {
                    unsigned short h;
                    if (a.u16_dt == CBCT_BF16)
                        h = __bfloat16_as_ushort(__float2bfloat16(un));
                    else
                        h = __half_as_ushort(__float2half(un * (float)*a.u16_scale));
                    ((unsigned short *)a.u16)[o] = h;
                }
            }
        }
    }
    if constexpr (MODE == FWD_SOLVER) {
        // block reduction (fixed order -> deterministic)
        for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
        __shared__ double red[4];
        if (lane == 0) red[w] = sq;
        __syncthreads();
        if (threadIdx.x == 0) a.partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

int64_t forward_blocks(const GeoK &G) {
    const int RB = 64 * fwd_rpl(G.nv), h = G.nv / 2;
    const int nrb = (h + RB - 1) / RB + (G.nv - h + RB - 1) / RB;
    const int64_t vg = (G.nviews + kFwdViewGroup - 1) / kFwdViewGroup * kFwdViewGroup;
    return vg * nrb * ((G.nu + 3) / 4);
}

template <int RPL, int DT>
static void launch_forward_rpl(const GeoK &G, int mode, const FwdArgs &a, hipStream_t s,
                               dim3 grid) {
    const dim3 block(256);
    if (mode == FWD_PLAIN)
        hipLaunchKernelGGL((k_fwd<FWD_PLAIN, RPL, DT>), grid, block, 0, s, G, a);
    else if (mode == FWD_SOLVER)
        hipLaunchKernelGGL((k_fwd<FWD_SOLVER, RPL, DT>), grid, block, 0, s, G, a);
    else
        hipLaunchKernelGGL((k_fwd<FWD_COUNT, RPL, DT>), grid, block, 0, s, G, a);
}

template <int DT>
static void launch_forward_dt(const GeoK &G, int mode, const FwdArgs &a, hipStream_t s,
                              dim3 grid) {
    if (fwd_rpl(G.nv) == 4)
        launch_forward_rpl<4, DT>(G, mode, a, s, grid);
    else if (fwd_rpl(G.nv) == 3)
        launch_forward_rpl<3, DT>(G, mode, a, s, grid);
    else if (fwd_rpl(G.nv) == 2)
        launch_forward_rpl<2, DT>(G, mode, a, s, grid);
    else
        launch_forward_rpl<1, DT>(G, mode, a, s, grid);
}

void launch_forward(const GeoK &G, int mode, const FwdArgs &a, hipStream_t s, int dtype) {
    const int64_t nb = forward_blocks(G);
    if (nb > 0x7fffffff) throw Error(CBCT_ERR_INVALID, "forward grid too large");
    const dim3 grid((unsigned)nb);
    if (dtype == CBCT_BF16)
        launch_forward_dt<CBCT_BF16>(G, mode, a, s, grid);
    else if (dtype == CBCT_F16)
        launch_forward_dt<CBCT_F16>(G, mode, a, s, grid);
    else if (dtype == CBCT_BF16_PAIR)
        launch_forward_dt<CBCT_BF16_PAIR>(G, mode, a, s, grid);
    else if (dtype == CBCT_F16_PAIR)
        launch_forward_dt<CBCT_F16_PAIR>(G, mode, a, s, grid);
    else
        launch_forward_dt<CBCT_F32>(G, mode, a, s, grid);
    CBCT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- back

// Gather form of A^T.  One wave owns one voxel column (i, j) and a block of up to
// 64*nq cells (nq <= 8); lane l accumulates cells k = k0 + l + 64 q.  For every
// view, the detector columns u whose rays cross (i, j) give the column interval
// [aa, ab] (same float32 plane values as the forward traversal); the rows that
// can meet cell k are those whose height z = (a_ref + a') v lies in the cell for
// some a' in [aa, ab], a range of at most C rows (C computed on the host from the
// geometry).  Each candidate row's chord is the overlap of [aa, ab] with the
// cell's own z-plane interval,
//     c = med3(ab, zA, zB) - med3(aa, zA, zB)   (med3 = clamp into [min, max]),
// zA, zB = fma(k - o, rg, cz), fma(k + 1 - o, rg, cz), o = nz / 2.  Because the forward kernel's cell
// state satisfies entry(k) < aa <= exit(k) at every segment start and meets at
// most one z plane per segment, this equals its c0 / c1 bit for bit and is 0 for
// every cell the forward does not touch: the two kernels apply the same matrix.
// No atomics; every cell is summed in a fixed order.
// Tile of voxel columns (x by y) whose waves run side by side.  Timed per A^T
// with the view chunks (ms at 512 x 512 x 400 / 256^3): 16 x 16 39.4 / 2.71,
// 8 x 16 38.6 / 2.66, 4 x 16 38.5 / 2.65, 4 x 32 38.9 / 2.66, 8 x 32 39.0 / 2.67,
// 16 x 8 40.1 / 2.80, 8 x 8 40.0 / 2.76, 32 x 32 40.0 / 2.77.  Same bits for all.
#ifndef CBCT_BACK_TILE_W
#define CBCT_BACK_TILE_W 8
#endif
#ifndef CBCT_BACK_TILE_H
#define CBCT_BACK_TILE_H 16
#endif
constexpr int kBackTileW = CBCT_BACK_TILE_W, kBackTileH = CBCT_BACK_TILE_H;

// Window samples of A^T's input: float32, or 16-bit values widened on load.
// A 16-bit window of up to four rows is one 8-byte read at the window's first
// row (2-byte aligned; the device runs in unaligned-access mode), whose last
// sample may lie past the detector column (the buffer is padded by 8 bytes).
template <int DT>
struct BackIn;
template <>
struct BackIn<CBCT_F32> {
    using T = float;
    template <int C>
    __device__ static void window(const float *y, float (&v)[C]) {
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = y[c];
    }
};
template <int DT>
struct BackIn16 {
    using T = unsigned short;
    __device__ static float widen(unsigned short h) {
        if constexpr (DT == CBCT_BF16)
            return __uint_as_float((unsigned)h << 16);
        else
            return __half2float(__ushort_as_half(h));
    }
    template <int C>
    __device__ static void window(const unsigned short *y, float (&v)[C]) {
        if constexpr (C <= 4) {
            const uint2 w = *(const uint2 *)y;
            const unsigned h[4] = {w.x & 0xffffu, w.x >> 16, w.y & 0xffffu, w.y >> 16};
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = widen((unsigned short)h[c]);
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) v[c] = widen(y[c]);
        }
    }
};
template <>
struct BackIn<CBCT_BF16> : BackIn16<CBCT_BF16> {};
template <>
struct BackIn<CBCT_F16> : BackIn16<CBCT_F16> {};

template <int C, int DT>
__global__ void __launch_bounds__(256)
k_back(GeoK G, const void *__restrict__ yin, float *__restrict__ out, const int *brk,
       const double *in_scale, float a_ref, float z_lo_mm, float fv_off, float fu_margin,
       int kspan, int nq, int v0, int v1) {
    if (brk && *brk == 2) return;
    using YT = typename BackIn<DT>::T;
    const YT *yhat = (const YT *)yin;
    extern __shared__ float lds[];
    float2 *zrs = (float2 *)lds;  // per-row (rg, cz)
    for (int t = threadIdx.x; t < G.nv; t += 256) {
        const float4 z = G.zr[t];
        zrs[t] = make_float2(z.y, z.z);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nzs = (G.nz + kspan - 1) / kspan;        // z splits per column
    const int64_t lw = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * 4 + w;
    // columns in kBackTileW x kBackTileH tiles, tiles row-major: the waves
    // resident on one XCD cover a compact patch of the x-y plane, whose
    // detector footprint in each view is narrow and stays in that XCD's L2
    const int64_t cw = lw / nzs;
    const int zs = (int)(lw % nzs);
    const int ntx = (G.nx + kBackTileW - 1) / kBackTileW;
    const int64_t tile = cw / (kBackTileW * kBackTileH);
    const int rt = (int)(cw % (kBackTileW * kBackTileH));
    const int i = (int)(tile % ntx) * kBackTileW + rt % kBackTileW;
    const int j = (int)(tile / ntx) * kBackTileH + rt / kBackTileW;
    if (i >= G.nx || j >= G.ny) return;
    const int64_t col = (int64_t)j * G.nx + i;
    const int kbase = zs * kspan;

    constexpr int QM = 8;
    float acc[QM], fk[QM], fk1[QM], zk0[QM];
    bool kok[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int k = kbase + lane + 64 * q;
        kok[q] = q < nq && k < G.nz;
        // views v0 .. v1 - 1 continue the sums of the views before v0 (unscaled
        // float32 partial sums stored by the previous launch)
        acc[q] = v0 > 0 && kok[q] ? out[(size_t)col * G.Z + k + 1] : 0.0f;
        fk[q] = (float)(k - (G.nz >> 1));      // plane index relative to nz / 2
        fk1[q] = fk[q] + 1.0f;
        zk0[q] = fmaf((float)k, G.hz, z_lo_mm);   // cell's lower z [mm]
    }
    const float fi = (float)i, fj = (float)j;
    // the column's lower plane indices relative to the axis midpoints
    const float px = (float)(i - (G.nx >> 1)), py = (float)(j - (G.ny >> 1));
    const float xlo = (fi - 0.5f * G.nx) * G.hx, xhi = xlo + G.hx;
    const float ylo = (fj - 0.5f * G.ny) * G.hy, yhi = ylo + G.hy;
    const float fu_scale = G.dsd / G.du, fu_off = 0.5f * G.nu - 0.5f;
    // row index of height z at ray parameter A: z / (A dv) + nv/2 - 1/2; fv_off
    // is nv/2 - 1/2 less the window's safety margin (rows), formed on the host
    const float a_ref_dv = a_ref * G.dv;
    const float nrwin = -(float)(G.nv - C);  // minus the last allowed window start

    // The detector footprint of the column is the same for every lane: once per
    // 64 views lane t computes it for view view + t, and each view then reads
    // its own back with readlane instead of all 64 lanes recomputing it.
    int fu0v = 0, fu1v = -1;
    for (int view = v0; view < v1; ++view) {
        const int tv = (view - v0) & 63;
        if (tv == 0) {
            // detector u range of the column's x-y square: a ray with a positive
            // chord crosses the square's interior, so its pixel lies strictly between
            // the extreme corner images (fu_margin columns cover the approximate
            // reciprocal and the rounding of the column positions)
            const int vw = view + lane;
            fu0v = 0;
            fu1v = -1;
            if (vw < v1) {
                const float2 cs = G.trig[vw];
                float umin = 3.0e38f, umax = -3.0e38f;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float X = (c & 1) ? xhi : xlo, Y = (c & 2) ? yhi : ylo;
                    const float depth = G.dso - (X * cs.x + Y * cs.y);
                    const float lat = Y * cs.x - X * cs.y;
                    const float fu =
                        fmaf(lat * __builtin_amdgcn_rcpf(depth), fu_scale, fu_off);
                    umin = fminf(umin, fu);
                    umax = fmaxf(umax, fu);
                }
                fu0v = max(0, (int)ceilf(umin - fu_margin));
                fu1v = min(G.nu - 1, (int)floorf(umax + fu_margin));
            }
        }
        const int iu0 = __builtin_amdgcn_readlane(fu0v, tv);
        const int iu1 = __builtin_amdgcn_readlane(fu1v, tv);
        for (int iu = iu0; iu <= iu1; ++iu) {
            const float4 cxy = G.xy[(size_t)view * G.nu + iu];
            const float ex0 = plane_alpha(px, cxy.x, cxy.y);
            const float ex1 = plane_alpha(px + 1.0f, cxy.x, cxy.y);
            const float ey0 = plane_alpha(py, cxy.z, cxy.w);
            const float ey1 = plane_alpha(py + 1.0f, cxy.z, cxy.w);
            const float aa = fmaxf(fminf(ex0, ex1), fminf(ey0, ey1));
            const float ab = fminf(fmaxf(ex0, ex1), fmaxf(ey0, ey1));
            if (!(ab > aa)) continue;
            // heights reached by row v over the interval: z = A v, A in [A1, A2]
            const float iA1 = __builtin_amdgcn_rcpf(fmaf(aa, G.dv, a_ref_dv));
            const float iA2 = __builtin_amdgcn_rcpf(fmaf(ab, G.dv, a_ref_dv));
            const YT *yrow = yhat + ((size_t)view * G.nu + iu) * G.nv;
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                if (q >= nq) break;
                // the first row whose centre can satisfy z_k <= A v, then a window of C
                // rows kept inside [0, nv): every row meeting the cell is in it, and
                // rows that miss the cell contribute exactly zero below.  The start
                // r0 = clamp(ceil(flo), 0, nv - C) is formed negated, as
                // -r0 = floor(clamp(-flo, -(nv - C), 0)): one floor-convert instead of
                // a ceil, a clamp and a convert, and the same integer.  |r0| < 2^14,
                // so both byte offsets are 24-bit products.
                const float nflo = fmaf(-zk0[q], zk0[q] >= 0.0f ? iA2 : iA1, -fv_off);
                const int m = (int)floorf(__builtin_amdgcn_fmed3f(nflo, nrwin, 0.0f));
                const float2 *zq = (const float2 *)((const char *)zrs + __mul24(m, -8));
                const YT *yq = (const YT *)((const char *)yrow +
                                            (uint32_t)__mul24(m, -(int)sizeof(YT)));
                float yv[C];
                BackIn<DT>::template window<C>(yq, yv);
                float a = acc[q];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float2 z = zq[c];
                    const float zA = plane_alpha(fk[q], z.x, z.y);
                    const float zB = plane_alpha(fk1[q], z.x, z.y);
                    // med3(t, zA, zB) clamps t into the cell's interval: where the two
                    // intervals overlap these are max(aa, zmin) and min(ab, zmax), and
                    // where they do not both clamp to the same end, giving 0.  The
                    // clamp is non-decreasing in t and aa < ab, so hi - lo >= 0.
                    const float lo = __builtin_amdgcn_fmed3f(aa, zA, zB);
                    const float hi = __builtin_amdgcn_fmed3f(ab, zA, zB);
                    a = fmaf(hi - lo, yv[c], a);
                }
                acc[q] = a;  // lanes past the column's end are never stored
            }
        }
    }
    float *oc = out + (size_t)col * G.Z;
    // a scaled 16-bit input carries the power-of-two scale: the last launch
    // divides it out (exact)
    const float inv = DT == CBCT_F16 && v1 == G.nviews ? (float)(1.0 / *in_scale) : 1.0f;
#pragma unroll
    for (int q = 0; q < QM; ++q)
        if (kok[q]) oc[kbase + lane + 64 * q + 1] = DT == CBCT_F16 ? acc[q] * inv : acc[q];
    if (zs == 0 && lane == 0) oc[0] = 0.0f;
    if (zs == nzs - 1 && lane == 0) oc[G.nz + 1] = 0.0f;
}

// Safety margin (rows) by which a window starts before the first row whose
// centre can meet the cell.  It covers the float32 rounding of the window
// start, which grows with the row position: the row offset nv/2 - 1/2 and the
// start itself are rounded to half an ulp each (an ulp of a position below nv
// is at most nv * 2^-23 rows), and the approximate reciprocal adds up to one
// ulp of the distance from the centre row (below nv/2 rows); plus the table
// rounding of the rows' plane parameters, a small fraction of 1e-3 rows.  The
// margin is 1e-3 rows plus eight ulps' worth of nv * 2^-23.
static double back_margin_rows(int nv) { return 1e-3 + 8.0 * nv * std::ldexp(1.0, -23); }
// The same margin for the detector columns visited per view, whose corner
// images carry the same kinds of rounding at positions below nu.
static double back_margin_cols(int nu) { return 1e-3 + 8.0 * nu * std::ldexp(1.0, -23); }

// Upper bound on the number of detector rows that can meet one cell within one
// column interval: rows span (z_k / A1 .. z_k+1 / A2) with A the absolute ray
// parameter, so the span is at most (hz / A_min + R_z (A_max - A_min) / A_min^2) / dv;
// a window starting the margin early must reach that far, and 2 % plus 0.01 rows
// cover the rounding of the bound.
static int back_candidates(const GeoK &G) {
    const double hx = G.nx * (double)G.hx / 2, hy = G.ny * (double)G.hy / 2;
    const double rxy = std::sqrt(hx * hx + hy * hy);
    const double umax = G.nu * (double)G.du / 2;
    const double amin = (G.dso - rxy) / std::sqrt((double)G.dsd * G.dsd + umax * umax);
    const double diag = std::sqrt((double)G.hx * G.hx + (double)G.hy * G.hy);
    const double dA = diag / G.dsd;  // parameter extent of one column interval
    const double rz = G.nz * (double)G.hz / 2;
    const double span = (G.hz / amin + rz * dA / (amin * amin)) / G.dv + back_margin_rows(G.nv);
    return (int)std::floor(span * 1.02 + 0.01) + 1;
}

// Views per launch of A^T.  A block sums its cells over the views in order, and
// the blocks resident on one XCD (about 224, i.e. 7 tiles of 8 x 16 columns)
// are spread over the views they have reached: blocks finish and are replaced
// at different times.  Over all views, the detector data those blocks touch
// overflows the XCD's 4 MB L2 at the larger geometries (hit rate 0.50 at
// 512 x 512 x 400 with 180 views).  One launch per chunk of views bounds that
// spread.  The chunk is sized so that a 16-column square's detector footprint
// per view (the detector columns it can cast its shadow on, times the rows a
// voxel column spans) over the chunk's views stays near 3.5 MB.  A
// cell's float32 partial sum passes from launch to launch through the output,
// unchanged, so every chunk size gives the same bits.  Measured per A^T (views
// per launch: ms): 512 x 512 x 400, 180 views: all 49.0, 45: 41.5, 20: 40.2,
// 12: 41.3, 8: 43.9; 256^3, 90 views: all 2.81, 45: 2.74, 20: 2.78, 12: 2.91.
static int back_views_per_launch(const GeoK &G, size_t sample_bytes) {
    if (G.back_views > 0) return std::min(G.back_views, G.nviews);
    const double h = std::max(G.hx, G.hy), mag = (double)G.dsd / G.dso;
    const double cols = 16.0 * h * std::sqrt(2.0) * mag / G.du + 2.0;  // 16-column square
    const double rows = std::min((double)G.nv, G.nz * (double)G.hz * mag / G.dv);
    const double per_view = cols * rows * (double)sample_bytes;
    // in double until it is known to fit: a footprint far below a byte per view
    // (a degenerate voxel height) would overflow an int
    const double vd = per_view > 0.0 ? std::floor(3.5e6 / per_view) : (double)G.nviews;
    if (vd >= (double)G.nviews) return G.nviews;
    const int v = std::max(8, (int)vd);
    if (v >= G.nviews) return G.nviews;
    const int chunks = (G.nviews + v - 1) / v;
    return (G.nviews + chunks - 1) / chunks;  // equal chunks
}

template <int DT>
static void launch_back_dt(const GeoK &G, const void *yhat, float *out, const int *brk,
                           const double *scale, hipStream_t s) {
    // cells per wave: 64 * nq, nq <= 8; columns taller than 512 cells are split
    const int nq = std::min(8, (G.nz + 63) / 64);
    const int kspan = 64 * nq;
    const int nzs = (G.nz + kspan - 1) / kspan;
    const int64_t ntiles = (int64_t)((G.nx + kBackTileW - 1) / kBackTileW) *
                           ((G.ny + kBackTileH - 1) / kBackTileH);
    const int64_t nwaves = ntiles * kBackTileW * kBackTileH * nzs;
    const int64_t nb = (nwaves + 3) / 4;
    if (nb > 0x7fffffff) throw Error(CBCT_ERR_INVALID, "back grid too large");
    const size_t shm = sizeof(float2) * (size_t)G.nv;
    const float a_ref = G.dso / G.dsd;
    const float z_lo_mm = -0.5f * G.nz * G.hz;
    const float fv_off = (float)(0.5 * G.nv - 0.5 - back_margin_rows(G.nv));
    const float fu_margin = (float)back_margin_cols(G.nu);
    // window of C rows; never more rows than the detector has
    const int C = std::min(back_candidates(G), G.nv);
    const int vc = back_views_per_launch(G, sizeof(typename BackIn<DT>::T));
    auto go = [&](auto kern) {
        for (int v0 = 0; v0 < G.nviews; v0 += vc)
            hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(256), shm, s, G, yhat, out, brk,
                               scale, a_ref, z_lo_mm, fv_off, fu_margin, kspan, nq, v0,
                               std::min(G.nviews, v0 + vc));
    };
    switch (C) {
        case 1: go(k_back<1, DT>); break;
        case 2: go(k_back<2, DT>); break;
        case 3: go(k_back<3, DT>); break;
        case 4: go(k_back<4, DT>); break;
        case 5: go(k_back<5, DT>); break;
        case 6: go(k_back<6, DT>); break;
        case 7: go(k_back<7, DT>); break;
        case 8: go(k_back<8, DT>); break;
        default:
            throw Error(CBCT_ERR_INVALID, "detector rows too fine for the back projector (more "
                                          "than 8 rows can meet one voxel)");
    }
    CBCT_HIP(hipGetLastError());
}

void launch_back(const GeoK &G, const void *yhat, float *out, const int *brk, hipStream_t s,
                 int dt, const double *scale) {
    if (dt == CBCT_BF16)
        launch_back_dt<CBCT_BF16>(G, yhat, out, brk, scale, s);
    else if (dt == CBCT_F16)
        launch_back_dt<CBCT_F16>(G, yhat, out, brk, scale, s);
    else
        launch_back_dt<CBCT_F32>(G, yhat, out, brk, scale, s);
}

// ---------------------------------------------------------------- layout kernels

template <typename T>
__global__ void __launch_bounds__(256)
k_transpose(const T *__restrict__ in, T *__restrict__ out, int R, int C, int64_t ib,
            int64_t ir, int64_t ioff, int64_t ob, int64_t oc, int64_t ooff,
            const float *__restrict__ Lu2, const float *__restrict__ Lv2) {
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int bc = blockIdx.x, br = blockIdx.y, bb = blockIdx.z;
    const int64_t ibase = (int64_t)bb * ib + ioff, obase = (int64_t)bb * ob + ooff;
    for (int q = ty; q < 32; q += 8) {
        const int r = br * 32 + q, c = bc * 32 + tx;
        if (r < R && c < C) {
            T v = in[ibase + (int64_t)r * ir + c];
            if constexpr (sizeof(T) == 4) {
                if (Lu2) v *= sqrtf(Lu2[c] + Lv2[r]);
            }
            tile[q][tx] = v;
        }
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int c = bc * 32 + q, r = br * 32 + tx;
        if (r < R && c < C) out[obase + (int64_t)c * oc + r] = tile[tx][q];
    }
}

void launch_transpose(const float *in, float *out, int B, int R, int C, int64_t ib, int64_t ir,
                      int64_t ioff, int64_t ob, int64_t oc, int64_t ooff, const float *Lu2,
                      const float *Lv2, hipStream_t s) {
    dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32), (unsigned)B);
    hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, s, in, out, R, C, ib, ir, ioff, ob,
                       oc, ooff, Lu2, Lv2);
    CBCT_HIP(hipGetLastError());
}

// 16-bit x[k][j][i] -> 16-bit column volume (pads untouched).
static void vol_to_cols16(const GeoK &G, const unsigned short *x, unsigned short *cols,
                          hipStream_t s) {
    dim3 grid((unsigned)((G.nx + 31) / 32), (unsigned)((G.nz + 31) / 32), (unsigned)G.ny);
    hipLaunchKernelGGL(k_transpose<unsigned short>, grid, dim3(256), 0, s, x, cols, G.nz, G.nx,
                       (int64_t)G.nx, (int64_t)G.nx * G.ny, (int64_t)0, (int64_t)G.nx * G.Z,
                       (int64_t)G.Z, (int64_t)1, (const float *)nullptr, (const float *)nullptr);
    CBCT_HIP(hipGetLastError());
}

__global__ void k_fill(float *p, int64_t n, float v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) p[t] = v;
}

void launch_fill(float *p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return;
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
    CBCT_HIP(hipGetLastError());
}

// x[k][j][i] -> cols (cell (i,j,k) at (j*nx+i)*Z + k + 1): batch j, rows k, cols i.
void vol_to_cols(const GeoK &G, const float *x, float *cols, hipStream_t s) {
    launch_transpose(x, cols, G.ny, G.nz, G.nx, G.nx, (int64_t)G.nx * G.ny, 0,
                     (int64_t)G.nx * G.Z, G.Z, 1, nullptr, nullptr, s);
}

// cols -> x: batch j, rows i, cols k.
void cols_to_vol(const GeoK &G, const float *cols, float *x, hipStream_t s) {
    launch_transpose(cols, x, G.ny, G.nx, G.nz, (int64_t)G.nx * G.Z, G.Z, 1, G.nx,
                     (int64_t)G.nx * G.ny, 0, nullptr, nullptr, s);
}

// y[view][v][u] -> ycol[view][u][v] (optionally times L(u, v)): batch view, rows v, cols u.
void proj_to_cols(const GeoK &G, const float *y, float *ycol, bool scale_by_L, hipStream_t s) {
    const int64_t per = (int64_t)G.nu * G.nv;
    launch_transpose(y, ycol, G.nviews, G.nv, G.nu, per, G.nu, 0, per, G.nv, 0,
                     scale_by_L ? G.Lu2 : nullptr, scale_by_L ? G.Lv2 : nullptr, s);
}

// ycol[view][u][v] -> y[view][v][u]: batch view, rows u, cols v.
void cols_to_proj(const GeoK &G, const float *ycol, float *y, hipStream_t s) {
    const int64_t per = (int64_t)G.nu * G.nv;
    launch_transpose(ycol, y, G.nviews, G.nu, G.nv, per, G.nv, 0, per, G.nu, 0, nullptr, nullptr,
                     s);
}

// ---------------------------------------------------------------- 16-bit operand conversion

__global__ void k_to_f32(const void *in, int dtype, float scale, float *out, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        float v;
        if (dtype == CBCT_BF16) {
            const unsigned short h = ((const unsigned short *)in)[t];
            v = __uint_as_float((unsigned)h << 16);
        } else if (dtype == CBCT_F16) {
            v = (float)((const __half *)in)[t];
        } else {
            v = ((const float *)in)[t];
        }
        out[t] = v * scale;
    }
}

static void to_f32(const void *in, cbct_dtype dt, float scale, float *out, int64_t n,
                   hipStream_t s) {
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)nb), dim3(256), 0, s, in, (int)dt, scale, out, n);
    CBCT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- API-layout forward

void forward_api_bytes(const cbct_geom *g, cbct_dtype xt, size_t *cols_bytes,
                       size_t *ycol_bytes) {
    const size_t es = xt == CBCT_F32 ? 4 : 2;
    *cols_bytes = es * (size_t)g->pad_floats();
    *ycol_bytes = sizeof(float) * (size_t)g->n_proj();
}

void forward_api(const GeoK &G, const cbct_geom *g, const void *x, cbct_dtype xt,
                 float x_scale, float *y, void *cols, float *ycol, hipStream_t s) {
    size_t cols_bytes = 0, ycol_bytes = 0;
    forward_api_bytes(g, xt, &cols_bytes, &ycol_bytes);
    // padded column copy in the input's own storage type (pads and guards zero);
    // the kernel widens 16-bit values on load and applies x_scale in its epilogue
    launch_fill((float *)cols, (int64_t)(cols_bytes / 4), 0.0f, s);
    FwdArgs a{};
    if (xt == CBCT_F32) {
        float *P = (float *)cols + kGuard;
        vol_to_cols(G, (const float *)x, P, s);
        a.vol = P;
    } else {
        unsigned short *P = (unsigned short *)cols + kGuard;
        vol_to_cols16(G, (const unsigned short *)x, P, s);
        a.vol = P;
    }
    a.out = ycol;
    a.scale = x_scale;
    launch_forward(G, FWD_PLAIN, a, s, xt);
    cols_to_proj(G, ycol, y, s);
}

}  // namespace cbct

using namespace cbct;

namespace {

// Stream-ordered temporary device buffer (freed on the same stream).
struct StreamBuf {
    void *p = nullptr;
    hipStream_t s;
    explicit StreamBuf(size_t bytes, hipStream_t st) : s(st) {
        if (bytes) CBCT_HIP(hipMallocAsync(&p, bytes, st));
    }
    StreamBuf(const StreamBuf &) = delete;
    StreamBuf &operator=(const StreamBuf &) = delete;
    ~StreamBuf() {
        if (p) (void)hipFreeAsync(p, s);
    }
    float *f() const { return (float *)p; }
};

int translate(const std::exception &ex) {
    if (auto e = dynamic_cast<const Error *>(&ex)) {
        set_last_error(e->what());
        return e->code;
    }
    set_last_error(ex.what());
    return CBCT_ERR_INVALID;
}

void check_dtype(cbct_dtype t, float scale) {
    CBCT_REQUIRE(t == CBCT_F32 || t == CBCT_BF16 || t == CBCT_F16, "unknown dtype");
    CBCT_REQUIRE(std::isfinite(scale) && scale > 0.0f, "scale must be finite and > 0");
}

}  // namespace

extern "C" {

int cbct_forward(const cbct_geom *gc, const void *x, cbct_dtype xt, float x_scale, float *y,
                 void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && x && y, "null argument");
        check_dtype(xt, x_scale);
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        hipStream_t s = (hipStream_t)hip_stream;
        GeoK G = geo_for_device(g);
        size_t cols_bytes = 0, ycol_bytes = 0;
        forward_api_bytes(g, xt, &cols_bytes, &ycol_bytes);
        StreamBuf cols(cols_bytes, s);
        StreamBuf ycol(ycol_bytes, s);
        forward_api(G, g, x, xt, x_scale, y, cols.p, ycol.f(), s);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_back(const cbct_geom *gc, const void *y, cbct_dtype yt, float y_scale, float *x,
              void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && x && y, "null argument");
        check_dtype(yt, y_scale);
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        hipStream_t s = (hipStream_t)hip_stream;
        GeoK G = geo_for_device(g);
        const int64_t N = g->n_proj();
        StreamBuf cols(sizeof(float) * g->pad_floats(), s);
        StreamBuf ycol(sizeof(float) * N, s);
        const float *yf = (const float *)y;
        StreamBuf conv(yt == CBCT_F32 && y_scale == 1.0f ? 0 : sizeof(float) * N, s);
        if (!(yt == CBCT_F32 && y_scale == 1.0f)) {
            to_f32(y, yt, y_scale, conv.f(), N, s);
            yf = conv.f();
        }
        proj_to_cols(G, yf, ycol.f(), true, s);
        float *P = cols.f() + kGuard;
        launch_back(G, ycol.f(), P, nullptr, s);
        cols_to_vol(G, P, x, s);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_col_sizes(const cbct_geom *gc, int64_t *vol_floats, int64_t *vol_offset,
                   int64_t *proj_floats) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc, "null geometry");
        if (vol_floats) *vol_floats = gc->pad_floats();
        if (vol_offset) *vol_offset = kGuard;
        if (proj_floats) *proj_floats = gc->n_proj();
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_vol_to_cols(const cbct_geom *gc, const float *x, float *cols, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && x && cols, "null argument");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        hipStream_t s = (hipStream_t)hip_stream;
        GeoK G = geo_for_device(g);
        launch_fill(cols, g->pad_floats(), 0.0f, s);
        vol_to_cols(G, x, cols + kGuard, s);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_cols_to_vol(const cbct_geom *gc, const float *cols, float *x, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && x && cols, "null argument");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        GeoK G = geo_for_device(g);
        cols_to_vol(G, cols + kGuard, x, (hipStream_t)hip_stream);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_proj_to_cols(const cbct_geom *gc, const float *y, float *ycols, int weighted,
                      void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && y && ycols, "null argument");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        GeoK G = geo_for_device(g);
        proj_to_cols(G, y, ycols, weighted != 0, (hipStream_t)hip_stream);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_cols_to_proj(const cbct_geom *gc, const float *ycols, float *y, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && y && ycols, "null argument");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        GeoK G = geo_for_device(g);
        cols_to_proj(G, ycols, y, (hipStream_t)hip_stream);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_forward_cols(const cbct_geom *gc, const float *cols, float *ycols, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && cols && ycols, "null argument");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        GeoK G = geo_for_device(g);
        FwdArgs a{};
        a.vol = cols + kGuard;
        a.out = ycols;
        a.scale = 1.0f;
        launch_forward(G, FWD_PLAIN, a, (hipStream_t)hip_stream);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_back_cols(const cbct_geom *gc, const float *ywcols, float *cols, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && cols && ywcols, "null argument");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        hipStream_t s = (hipStream_t)hip_stream;
        GeoK G = geo_for_device(g);
        // guards are outside every column the kernel writes
        launch_fill(cols, kGuard, 0.0f, s);
        launch_fill(cols + kGuard + g->n_col() * G.Z, kGuard, 0.0f, s);
        launch_back(G, ywcols, cols + kGuard, nullptr, s);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_geom_nnz(const cbct_geom *gc, int64_t *nnz, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && nnz, "null argument");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        hipStream_t s = (hipStream_t)hip_stream;
        GeoK G = geo_for_device(g);
        StreamBuf cols(sizeof(float) * g->pad_floats(), s);
        StreamBuf cnt(sizeof(unsigned long long), s);
        CBCT_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s));
        launch_fill(cols.f(), g->pad_floats(), 0.0f, s);
        FwdArgs a{};
        a.vol = cols.f() + kGuard;
        a.count = (unsigned long long *)cnt.p;
        launch_forward(G, FWD_COUNT, a, s);
        unsigned long long h = 0;
        CBCT_HIP(hipMemcpyAsync(&h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, s));
        CBCT_HIP(hipStreamSynchronize(s));
        *nnz = (int64_t)h;
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

}  // extern "C"
