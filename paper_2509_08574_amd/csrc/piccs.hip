// IRN-PICCS solver on the device: TV weights, the regulariser blocks of the
// augmented operator, LSQR's reductions and scalar recurrence, vector updates.
//
// Method (paper Sec. 2.2.2): for k = 1..n_outer, with W1 = W~(D x_{k-1}) and
// W2 = W~(D x_{k-1} - D x_p), run n_inner LSQR iterations from x_{k-1} on
//   A~ = [A; alpha W1 D; lambda W2 D],   b~ = [b; 0; lambda W2 D x_p].
// LSQR (Paige & Saunders 1982) keeps u (data space) and v (model space)
// unnormalised in storage: U = beta * u, V = alpha * v.  Every kernel reads its
// scale factors from a float64 scalar block that the reduction kernels update
// (k_psum's first stage over many blocks, then k_red's single block, which also
// runs LSQR's scalar step), so the host enqueues the whole solve without waiting.
//
// Data-space vector: u_b (projections, stored as u-hat = L * u_b in column
// layout, L = ray length), u1 and u2 (three difference components each, in
// padded column volumes).  Model-space vectors: padded column volumes.
#include <rocprofiler-sdk-roctx/roctx.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>

#include "chord.h"
#include "internal.h"

namespace cbct {

enum Sc {
    SC_ALPHA = 0, SC_BETA, SC_RHOBAR, SC_PHIBAR,
    SC_FWD_S1, SC_FWD_S2, SC_REG_S1, SC_REG_S2, SC_BACK_S1, SC_BACK_S2,
    SC_XW_A, SC_XW_B, SC_XW_C,
    SC_M1, SC_P1, SC_ZERO,
    SC_INNER_DONE, SC_OUTER_DONE, SC_NBRK,
    SC_V16_SCALE,  // power-of-two scale of the 16-bit shadow of V (mixed forms)
    SC_U16_SCALE,  // power-of-two scale of the 16-bit copy of u-hat (fp16 ADJ16 form)
    SC_NUMERIC,    // 1 once a norm came out non-finite (the solve stopped there)
    SC_COUNT = 32
};
// flag 0: breakdown state of the current inner solve: 0 running, 1 last
// update pending, 2 stopped.
constexpr double kTiny = 1e-30;

// ---------------------------------------------------------------- helpers

struct VoxIdx {
    int i, j, k;
    bool ok;
    int64_t c;  // index relative to the padded base P
};

// Tiles of 64 cells along z by 4 columns along x, one wave per column.  The
// dispatcher hands block b to XCD b mod 8 and each XCD runs its blocks roughly
// in order, so the mapping below gives XCD x the x-th contiguous eighth (a slab
// of S tiles) of every y-plane, plane after plane.  A tile's z and x neighbours
// then lie in the same slab, and its y neighbour one slab later, on the same XCD:
// the cache lines two tiles share (columns start 4 bytes past a line, and Z is
// not a multiple of 32) are fetched into one L2, not into two.
// With NP = 2 each thread takes the cell in plane j and the one in plane j + 1
// (j even), and "plane" above means such a pair of planes.
template <int NP = 1>
__device__ __forceinline__ VoxIdx vox_index(const GeoK &G) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned nkb = (unsigned)(G.nz + 63) >> 6, nxb = (unsigned)(G.nx + 3) >> 2;
    const unsigned P = nkb * nxb, S = (P + 7) >> 3;
    const unsigned b = blockIdx.x, s = b >> 3;
    const unsigned j = s / S;
    const unsigned p = (b & 7) * S + (s - j * S);  // tile within plane j
    VoxIdx v;
    v.j = (int)j * NP;
    v.i = (int)(p / nkb) * 4 + w;
    v.k = (int)(p % nkb) * 64 + lane;
    v.ok = p < P && v.i < G.nx && v.k < G.nz;
    v.c = ((int64_t)v.j * G.nx + v.i) * G.Z + v.k + 1;
    return v;
}

// Blocks of a launch over the volume: 8 slabs of S tiles per y-plane (the last
// slab may hold up to 7 idle tiles, which still write a zero partial).
template <int NP = 1>
static int64_t vox_blocks(const GeoK &G) {
    const int64_t P = (int64_t)((G.nz + 63) / 64) * ((G.nx + 3) / 4);
    return 8 * ((P + 7) / 8) * ((G.ny + NP - 1) / NP);
}

// Sum of `v` over the block (256 threads), written to part[blockIdx.x].
__device__ __forceinline__ void block_partial(double v, double *part) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------- weights

// w1 = (sqrt(|D x|^2) + tau^2)^(-1/2), w2 = (sqrt(|D x - D xp|^2) + tau^2)^(-1/2)
// (paper Sec. 2.2.1, definition of W~*; Sec. 2.2.2 for the PICCS pair), from a
// cell's values and its forward neighbours along x, y, z; a neighbour past the
// volume's far face contributes a zero difference.
__device__ __forceinline__ void tv_weights(float x0, float p0, float xx, float xy, float xz,
                                           float px, float py, float pz, bool hx_, bool hy_,
                                           bool hz_, float tau2, float &w1, float &w2) {
    const float gx = hx_ ? x0 - xx : 0.f, gy = hy_ ? x0 - xy : 0.f, gz = hz_ ? x0 - xz : 0.f;
    const float hx = hx_ ? gx - (p0 - px) : 0.f, hy = hy_ ? gy - (p0 - py) : 0.f,
                hz = hz_ ? gz - (p0 - pz) : 0.f;
    w1 = 1.0f / sqrtf(sqrtf(gx * gx + gy * gy + gz * gz) + tau2);
    w2 = 1.0f / sqrtf(sqrtf(hx * hx + hy * hy + hz * hz) + tau2);
}

// Two cells per thread, in planes j and j + 1: plane j's y neighbour is plane
// j + 1's own cell, and each thread keeps twice the reads in flight (with one
// cell per thread this kernel streams two arrays and has too few bytes in flight
// to approach the HBM rate).
__global__ void __launch_bounds__(256)
k_weights(GeoK G, const float *__restrict__ x, const float *__restrict__ xp, float tau2,
          float *__restrict__ w1, float *__restrict__ w2) {
    const VoxIdx v = vox_index<2>(G);
    if (!v.ok) return;
    const int64_t sy = (int64_t)G.nx * G.Z;
    const bool hx_ = v.i < G.nx - 1, hz_ = v.k < G.nz - 1;
    const bool two = v.j + 1 < G.ny;        // plane j + 1 exists (= plane j has a y neighbour)
    const bool hy1 = v.j + 2 < G.ny;        // plane j + 1 has a y neighbour
    // every read is issued unconditionally (offset 0 where a neighbour or the
    // second plane does not exist) and the face conditions select afterwards
    const int64_t ox = hx_ ? G.Z : 0, oz = hz_ ? 1 : 0;
    const int64_t c0 = v.c, c1 = two ? c0 + sy : c0, oy1 = hy1 ? sy : 0;
    const float x0 = x[c0], p0 = xp[c0], x1 = x[c1], p1 = xp[c1];
    const float xx0 = x[c0 + ox], xz0 = x[c0 + oz], px0 = xp[c0 + ox], pz0 = xp[c0 + oz];
    const float xx1 = x[c1 + ox], xz1 = x[c1 + oz], px1 = xp[c1 + ox], pz1 = xp[c1 + oz];
    const float xy1 = x[c1 + oy1], py1 = xp[c1 + oy1];
    float a, b;
    tv_weights(x0, p0, xx0, x1, xz0, px0, p1, pz0, hx_, two, hz_, tau2, a, b);
    w1[c0] = a;
    w2[c0] = b;
    if (two) {
        tv_weights(x1, p1, xx1, xy1, xz1, px1, py1, pz1, hx_, hy1, hz_, tau2, a, b);
        w1[c1] = a;
        w2[c1] = b;
    }
}

// ---------------------------------------------------------------- regulariser, forward

// (u1, u2) <- s1 * (alpha W1 D v, lambda W2 D(v - vp)) + s2 * (u1, u2)
// (the second and third blocks of A~ v, or of b~ - A~ x when vp is given);
// partial sums of |u1|^2 + |u2|^2 per block.  PIPLE: the third block is
// lambda (v - vp), one component per voxel (W2 unused).
template <bool HAS_VP, bool PIPLE>
__global__ void __launch_bounds__(256)
k_regF(GeoK G, const float *__restrict__ V, const float *__restrict__ Vp,
       const float *__restrict__ W1, const float *__restrict__ W2, float *__restrict__ u1,
       float *__restrict__ u2, int64_t cstride, float alpha, float lam, const double *s1p,
       const double *s2p, double *part, const int *brk) {
    if (*brk == 2) return;
    const VoxIdx v = vox_index(G);
    const float s1 = (float)*s1p, s2 = (float)*s2p;
    double sum = 0.0;
    if (v.ok) {
        const int64_t c = v.c;
        const bool hi[3] = {v.i < G.nx - 1, v.j < G.ny - 1, v.k < G.nz - 1};
        const int64_t st[3] = {G.Z, (int64_t)G.nx * G.Z, 1};
        // all reads are issued before any is used: neighbour offsets are 0 at the
        // volume's far faces and the face condition selects afterwards; the old
        // u values are read only when they are used (s2 != 0, uniform)
        const bool keep = s2 != 0.0f;
        const float x0 = V[c];
        const float p0 = HAS_VP ? Vp[c] : 0.f;
        float xn[3], pn[3], o1[3], o2[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int64_t o = hi[q] ? st[q] : 0;
            xn[q] = V[c + o];
            pn[q] = HAS_VP ? Vp[c + o] : 0.f;
            o1[q] = keep ? u1[c + q * cstride] : 0.f;
            o2[q] = (keep && !PIPLE) ? u2[c + q * cstride] : 0.f;
        }
        const float o2p = (keep && PIPLE) ? u2[c] : 0.f;
        const float a1 = alpha * W1[c], a2 = PIPLE ? lam : lam * W2[c];
        float acc = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float d = hi[q] ? x0 - xn[q] : 0.f;
            const float e = hi[q] ? (HAS_VP ? d - (p0 - pn[q]) : d) : 0.f;
            float n1 = s1 * (a1 * d);
            if (keep) n1 = fmaf(s2, o1[q], n1);
            u1[c + q * cstride] = n1;
            acc = fmaf(n1, n1, acc);
            if (!PIPLE) {
                float n2 = s1 * (a2 * e);
                if (keep) n2 = fmaf(s2, o2[q], n2);
                u2[c + q * cstride] = n2;
                acc = fmaf(n2, n2, acc);
            }
        }
        if (PIPLE) {
            float n2 = s1 * (a2 * (x0 - p0));
            if (keep) n2 = fmaf(s2, o2p, n2);
            u2[c] = n2;
            acc = fmaf(n2, n2, acc);
        }
        sum = (double)acc;
    }
    block_partial(sum, part);
}

// ---------------------------------------------------------------- regulariser, adjoint

// v <- s1 * (t + alpha D^T(W1 u1) + lambda D^T(W2 u2)) + s2 * v, with t = A^T u-hat
// from the back projector; partial sums of |v|^2 per block.  PIPLE: the third
// term is lambda u2 (one component per voxel).
// D^T per axis: (D_1^T y)_i = y_i [i < n-1] - y_{i-1} [i >= 1].
template <bool PIPLE>
__global__ void __launch_bounds__(256)
k_regA(GeoK G, const float *__restrict__ t, const float *__restrict__ W1,
       const float *__restrict__ W2, const float *__restrict__ u1, const float *__restrict__ u2,
       int64_t cstride, float alpha, float lam, float *__restrict__ V, const double *s1p,
       const double *s2p, double *part, const int *brk) {
    if (*brk == 2) return;
    const VoxIdx v = vox_index(G);
    const float s1 = (float)*s1p, s2 = (float)*s2p;
    double sum = 0.0;
    if (v.ok) {
        const int64_t c = v.c;
        const int64_t st[3] = {G.Z, (int64_t)G.nx * G.Z, 1};
        const bool hi[3] = {v.i < G.nx - 1, v.j < G.ny - 1, v.k < G.nz - 1};
        const bool lo[3] = {v.i > 0, v.j > 0, v.k > 0};
        // all reads are issued before any is used: the backward neighbour's offset is
        // 0 at the volume's near faces and the face condition selects afterwards
        const float w1c = W1[c], w2c = PIPLE ? 0.f : W2[c];
        const float tc = t[c], vo = s2 != 0.0f ? V[c] : 0.f;
        float a0[3], an[3], wn1[3], b0[3], bn[3], wn2[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int64_t o = lo[q] ? st[q] : 0;
            a0[q] = u1[q * cstride + c];
            an[q] = u1[q * cstride + c - o];
            wn1[q] = W1[c - o];
            if (!PIPLE) {
                b0[q] = u2[q * cstride + c];
                bn[q] = u2[q * cstride + c - o];
                wn2[q] = W2[c - o];
            }
        }
        float r1 = 0.f, r2 = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (hi[q]) r1 += w1c * a0[q];
            if (lo[q]) r1 -= wn1[q] * an[q];
            if (!PIPLE) {
                if (hi[q]) r2 += w2c * b0[q];
                if (lo[q]) r2 -= wn2[q] * bn[q];
            }
        }
        if (PIPLE) r2 = u2[c];
        float vn = s1 * (tc + alpha * r1 + lam * r2);
        if (s2 != 0.0f) vn = fmaf(s2, vo, vn);
        V[c] = vn;
        sum = (double)vn * (double)vn;
    }
    block_partial(sum, part);
}

// ---------------------------------------------------------------- vector updates

// x += a w;  w <- b V + c w   (LSQR's solution and direction updates).  Works
// on the whole padded array: pads are zero in every operand and stay zero.
// Mixed forms (DT = bf16 / fp16) also write the forward projector's 16-bit
// shadow V16 = V * scale (scale a power of two, exact).
template <int DT>
__global__ void __launch_bounds__(256)
k_xw(float *__restrict__ x, float *__restrict__ w, const float *__restrict__ V,
     unsigned *__restrict__ V16, float *__restrict__ q, int64_t n, const double *sc,
     const int *brk) {
    if (*brk == 2) return;
    const float a = (float)sc[SC_XW_A], b = (float)sc[SC_XW_B], c = (float)sc[SC_XW_C];
    const float sv = (float)sc[SC_V16_SCALE];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const float wo = (a != 0.0f || c != 0.0f) ? w[t] : 0.0f;
        if (a != 0.0f) x[t] = fmaf(a, wo, x[t]);
        const float v = V[t];
        w[t] = fmaf(c, wo, b * v);
        if (q) q[t] = b * v;  // normalised v, kept for reorthogonalisation
        // shadow word t = (h(V[t]), h(V[t + 1])): V[t + 1] is the next cell of the
        // column, or a zero pad / guard
        if constexpr (DT == CBCT_BF16) {
            const unsigned h0 = __bfloat16_as_ushort(__float2bfloat16(v * sv));
            const unsigned h1 = __bfloat16_as_ushort(__float2bfloat16(V[t + 1] * sv));
            V16[t] = h0 | (h1 << 16);
        } else if constexpr (DT == CBCT_F16) {
            const unsigned h0 = __half_as_ushort(__float2half(v * sv));
            const unsigned h1 = __half_as_ushort(__float2half(V[t + 1] * sv));
            V16[t] = h0 | (h1 << 16);
        }
    }
}

// ---------------------------------------------------------------- reorthogonalisation

// Optional one-sided reorthogonalisation of LSQR's v (not in the paper, whose
// method relies on the short recurrences): classical Gram-Schmidt applied twice
// against the normalised v's of the current outer step, q_0 .. q_{k-1}, with
// float64 arithmetic.  One pass: c_i = <q_i, V> for all i from the same V
// (k_qdot per-block partials, k_qred fixed-order sums), then
// V <- V - sum_i c_i q_i (k_qaxpy), which also leaves per-block partials of
// |V|^2 for the norm that follows.
constexpr int kQBlocks = 1024;

// grid (kQBlocks, k): block (b, i) sums q_i[t] V[t] over its grid-stride share.
__global__ void __launch_bounds__(256)
k_qdot(const float *__restrict__ Q, int64_t qstride, const float *__restrict__ V, int64_t n,
       double *part, const int *brk) {
    if (*brk == 2) return;
    const float *q = Q + (int64_t)blockIdx.y * qstride;
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)kQBlocks * 256)
        s += (double)q[t] * (double)V[t];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(int64_t)blockIdx.y * kQBlocks + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// grid (k), 1024 threads: coef[i] = sum of the kQBlocks partials of q_i, fixed order.
__global__ void __launch_bounds__(1024)
k_qred(const double *__restrict__ part, double *coef, const int *brk) {
    if (*brk == 2) return;
    __shared__ double red[1024];
    red[threadIdx.x] = part[(int64_t)blockIdx.x * kQBlocks + threadIdx.x];
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) coef[blockIdx.x] = red[0];
}

// grid kQBlocks: V <- V - sum_{i<k} coef[i] q_i (float64), partials of |V|^2.
__global__ void __launch_bounds__(256)
k_qaxpy(const float *__restrict__ Q, int64_t qstride, float *__restrict__ V, int64_t n, int k,
        const double *__restrict__ coef, double *part, const int *brk) {
    if (*brk == 2) return;
    double sum = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)kQBlocks * 256) {
        double v = (double)V[t];
        for (int i = 0; i < k; ++i) v -= coef[i] * (double)Q[(int64_t)i * qstride + t];
        const float vf = (float)v;
        V[t] = vf;
        sum += (double)vf * (double)vf;
    }
    block_partial(sum, part);
}

// Power-of-two scale bringing the entries of a vector of norm nrm over m
// entries to root-mean-square about 1 (fp16 range); 1 for bf16 / fp32.
__device__ __forceinline__ double shadow_scale(int dt, double nrm, double m) {
    if (dt != CBCT_F16 || !(nrm > 0.0)) return 1.0;
    return exp2(rint(log2(sqrt(m) / nrm)));
}

// ---------------------------------------------------------------- reductions + recurrence

enum RedMode { RED_INIT_BETA = 0, RED_INIT_ALPHA, RED_BETA, RED_ALPHA };

// One block of 1024 threads: sum two partial arrays in a fixed order (so the
// result is bit-reproducible), then advance LSQR's scalar recurrence.
// Power-of-two scale for the fp16 copy of u-hat written by the next inner
// forward: u-hat = L u with |u| = beta_next, estimated by the current beta, so
// its samples have root-mean-square about beta L_ref / sqrt(N); uref = sqrt(N) /
// L_ref brings that to about 1.  1 for bf16 / fp32.
__device__ __forceinline__ double uhat_scale(int dt, double beta, double uref) {
    if (dt != CBCT_F16 || !(beta > 0.0)) return 1.0;
    return exp2(rint(log2(uref / beta)));
}

// First stage of a norm's reduction when there are many partials: block b sums
// its contiguous share of p0[0, n0) followed by p1[0, n1), in a fixed order, into
// out[b].  One 1024-thread block reading hundreds of thousands of partials is
// bound by its own load latency (about 130 us at 512 x 512 x 400); 256 blocks
// read them in a few microseconds and k_red then sums 256 values.
constexpr int kPsumBlocks = 256;
constexpr int64_t kPsumMin = 16384;  // fewer partials go to k_red directly

__global__ void __launch_bounds__(256)
k_psum(const double *__restrict__ p0, int64_t n0, const double *__restrict__ p1, int64_t n1,
       double *out, const int *brk) {
    if (*brk == 2) return;
    const int64_t n = n0 + n1;
    const int64_t per = (n + kPsumBlocks - 1) / kPsumBlocks;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    double a = 0.0;
    for (int64_t t = lo + threadIdx.x; t < hi; t += 256) a += t < n0 ? p0[t] : p1[t - n0];
    block_partial(a, out);
}

template <int MODE>
__global__ void __launch_bounds__(1024)
k_red(const double *__restrict__ p0, int64_t n0, const double *__restrict__ p1, int64_t n1,
      double *sc, int *fl, double *hist, int it, int dt, double nvox, double uref) {
    const int brk = fl[0];
    if (brk == 2) return;
    if (MODE == RED_BETA && brk == 1) {
        if (threadIdx.x == 0) fl[0] = 2;
        return;
    }
    __shared__ double red[1024];
    // eight independent sums per thread keep eight reads in flight (this one block
    // is all that runs on the GPU meanwhile); combined in a fixed order
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    auto add = [&](const double *__restrict__ p, int64_t n) {
        int64_t t = threadIdx.x;
        for (; t + 7 * 1024 < n; t += 8 * 1024) {
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] += p[t + u * 1024];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (t + u * 1024 < n) a[u] += p[t + u * 1024];
    };
    add(p0, n0);
    add(p1, n1);
    red[threadIdx.x] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double nrm = sqrt(red[0]);
    if (!isfinite(nrm)) {  // NaN / Inf in b, x_0 or x_p, or an overflow: stop here
        sc[SC_NUMERIC] = 1.0;
        fl[0] = 2;
        return;
    }
    if (MODE == RED_INIT_BETA) {            // beta_1 u_1 = b~ - A~ x_0
        sc[SC_BETA] = nrm;
        if (!(nrm > kTiny)) { fl[0] = 2; return; }
        sc[SC_BACK_S1] = 1.0 / nrm;
        sc[SC_BACK_S2] = 0.0;
    } else if (MODE == RED_INIT_ALPHA) {    // alpha_1 v_1 = A~^T u_1; w_1 = v_1
        sc[SC_ALPHA] = nrm;
        if (!(nrm > kTiny)) { fl[0] = 2; return; }
        const double beta = sc[SC_BETA];
        sc[SC_PHIBAR] = beta;
        sc[SC_RHOBAR] = nrm;
        sc[SC_XW_A] = 0.0;
        sc[SC_XW_B] = 1.0 / nrm;
        sc[SC_XW_C] = 0.0;
        const double sv = shadow_scale(dt, nrm, nvox);
        sc[SC_V16_SCALE] = sv;
        sc[SC_FWD_S1] = 1.0 / (nrm * sv);  // the projector reads V * sv
        sc[SC_REG_S1] = 1.0 / nrm;
        sc[SC_FWD_S2] = sc[SC_REG_S2] = -nrm / beta;
        sc[SC_U16_SCALE] = uhat_scale(dt, beta, uref);
    } else if (MODE == RED_BETA) {          // beta u = A~ v - alpha u
        const double alpha = sc[SC_ALPHA];
        sc[SC_BETA] = nrm;
        sc[SC_BACK_S1] = nrm > kTiny ? 1.0 / nrm : 1.0;
        sc[SC_BACK_S2] = -nrm / alpha;
    } else {                                 // alpha v = A~^T u - beta v; Givens; updates
        const double beta = sc[SC_BETA], alpha = nrm;
        const double rhobar = sc[SC_RHOBAR], phibar = sc[SC_PHIBAR];
        const double rho = sqrt(rhobar * rhobar + beta * beta);
        if (!(rho > 0.0)) { fl[0] = 2; return; }
        const double c = rhobar / rho, s = beta / rho;
        const double theta = s * alpha;
        sc[SC_RHOBAR] = -c * alpha;
        sc[SC_PHIBAR] = s * phibar;
        const double phi = c * phibar;
        sc[SC_XW_A] = phi / rho;
        sc[SC_XW_B] = alpha > kTiny ? 1.0 / alpha : 0.0;
        sc[SC_XW_C] = -theta / rho;
        sc[SC_ALPHA] = alpha;
        if (hist) hist[it] = s * phibar;
        sc[SC_INNER_DONE] += 1.0;
        if (!(beta > kTiny) || !(alpha > kTiny)) {
            fl[0] = 1;  // apply this last update, then stop
            sc[SC_FWD_S1] = sc[SC_FWD_S2] = sc[SC_REG_S1] = sc[SC_REG_S2] = 0.0;
        } else {
            const double sv = shadow_scale(dt, alpha, nvox);
            sc[SC_V16_SCALE] = sv;
            sc[SC_FWD_S1] = 1.0 / (alpha * sv);  // the projector reads V * sv
            sc[SC_REG_S1] = 1.0 / alpha;
            sc[SC_FWD_S2] = sc[SC_REG_S2] = -alpha / beta;
            sc[SC_U16_SCALE] = uhat_scale(dt, beta, uref);
        }
    }
}

__global__ void k_solve_begin(double *sc, int *fl, double *hist, int nh) {
    for (int q = 0; q < SC_COUNT; ++q) sc[q] = 0.0;
    for (int q = 0; q < nh; ++q) hist[q] = __longlong_as_double(0x7ff8000000000000LL);  // NaN
    sc[SC_M1] = -1.0;
    sc[SC_P1] = 1.0;
    sc[SC_V16_SCALE] = 1.0;
    sc[SC_U16_SCALE] = 1.0;
    fl[0] = 0;
}

__global__ void k_outer_begin(double *sc, int *fl) {
    if (fl[0] != 0) sc[SC_NBRK] += 1.0;
    fl[0] = 0;
    sc[SC_OUTER_DONE] += 1.0;
}

__global__ void k_solve_end(double *sc, int *fl) {
    if (fl[0] != 0) sc[SC_NBRK] += 1.0;
    fl[0] = 0;
}

// ---------------------------------------------------------------- workspace

struct Workspace {
    float *x, *xp, *w, *V, *t, *W1, *W2, *u1, *u2;  // padded column bases (P pointers)
    unsigned *V16;      // 16-bit shadow of V as pair words (base P), mixed forms
    unsigned *V16buf;   // its allocation start
    size_t v16_bytes;
    int64_t cstride;                                // floats between components
    float *bhat, *uhat;
    unsigned short *uhat16;  // 16-bit copy of u-hat read by the adjoint (*_ADJ16 forms)
    double *pf, *pr, *pa;  // partials: forward, regF, regA
    double *pp;            // first-stage sums of the partials (k_psum)
    int64_t nf, nr;
    float *Q;              // reorthogonalisation basis: n_inner padded volumes (base P)
    double *pq, *qcoef;    // its dot partials [n_inner][kQBlocks] and coefficients
    double *sc, *hist;
    int *fl;
    size_t bytes;
};

static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

// Whether A^T reads a 16-bit copy of u-hat (the *_ADJ16 forms).  The default
// mixed forms read float32: with A^T's view chunks its L2 hit rate is 0.94, and
// the 16-bit window read and its widening then cost more than the bytes they
// save (512 x 512 x 400: A^T 41.3 ms from float32, 42.0 ms from bf16 at its best
// chunk; 256^3: 2.82 against 2.94 ms).
static bool adjoint_reads_u16(const piccs_params *p) {
    return p->precision == CBCT_PREC_MIXED_BF16_ADJ16 ||
           p->precision == CBCT_PREC_MIXED_F16_ADJ16;
}

static Workspace carve(const cbct_geom *g, const GeoK &G, const piccs_params *p, char *base) {
    Workspace W{};
    const size_t vb = al(sizeof(float) * (size_t)g->pad_floats());
    const size_t pb = al(sizeof(float) * (size_t)g->n_proj());
    W.nf = forward_blocks(G);
    W.nr = vox_blocks(G);
    size_t off = 0;
    auto take = [&](size_t b) {
        char *q = base ? base + off : nullptr;
        off += al(b);
        return q;
    };
    float *vols[13];
    for (int q = 0; q < 13; ++q) vols[q] = (float *)take(vb);
    auto P = [&](int q) { return vols[q] ? vols[q] + kGuard : nullptr; };
    W.x = P(0); W.xp = P(1); W.w = P(2); W.V = P(3); W.t = P(4); W.W1 = P(5); W.W2 = P(6);
    W.u1 = P(7); W.u2 = P(10);
    W.cstride = (int64_t)(vb / sizeof(float));
    if (p->precision != CBCT_PREC_FP32) {
        W.v16_bytes = al(sizeof(unsigned) * (size_t)g->pad_floats());
        W.V16buf = (unsigned *)take(W.v16_bytes);
        W.V16 = W.V16buf ? W.V16buf + kGuard : nullptr;
    }
    W.bhat = (float *)take(pb);
    W.uhat = (float *)take(pb);
    if (adjoint_reads_u16(p))
        // 2 bytes per sample, read up to 8 bytes past the last
        W.uhat16 = (unsigned short *)take(sizeof(unsigned short) * (size_t)g->n_proj() + 8);
    W.pf = (double *)take(sizeof(double) * (size_t)W.nf);
    W.pr = (double *)take(sizeof(double) * (size_t)W.nr);
    W.pa = (double *)take(sizeof(double) * (size_t)W.nr);
    W.pp = (double *)take(sizeof(double) * (size_t)kPsumBlocks);
    if (p->reorth) {
        W.pq = (double *)take(sizeof(double) * (size_t)kQBlocks * p->n_inner);
        W.qcoef = (double *)take(sizeof(double) * (size_t)p->n_inner);
        float *q0 = (float *)take(vb * (size_t)p->n_inner);
        W.Q = q0 ? q0 + kGuard : nullptr;
    }
    W.sc = (double *)take(sizeof(double) * SC_COUNT);
    W.fl = (int *)take(sizeof(int) * 16);
    W.hist = (double *)take(sizeof(double) * (size_t)std::max(1, p->n_outer * p->n_inner));
    W.bytes = off;
    return W;
}

void check_solve_params(const piccs_params *p) {
    CBCT_REQUIRE(p != nullptr, "null params");
    CBCT_REQUIRE(std::isfinite(p->alpha) && p->alpha >= 0 && std::isfinite(p->lambda) &&
                     p->lambda >= 0 && std::isfinite(p->tau) && p->tau >= 0,
                 "alpha, lambda, tau must be finite and >= 0");
    CBCT_REQUIRE(p->n_outer >= 1 && p->n_inner >= 1 && p->n_outer <= 100000 &&
                     p->n_inner <= 100000, "n_outer and n_inner must be >= 1");
    CBCT_REQUIRE(p->precision >= CBCT_PREC_FP32 && p->precision <= CBCT_PREC_MIXED_F16_ADJ16,
                 "unknown precision");
    CBCT_REQUIRE(p->reorth == 0 || p->reorth == 1, "reorth must be 0 or 1");
    CBCT_REQUIRE(p->method == CBCT_METHOD_PICCS || p->method == CBCT_METHOD_PIPLE,
                 "unknown method");
}

// Enqueues one whole IRN-PICCS solve on stream s (no host synchronisation).
// When sc_host / hist_host are non-null, the device scalar block and the
// residual history are copied there, stream-ordered, at the end.
void solve_enqueue(cbct_geom *g, const float *b, const float *xp, float *x,
                   const piccs_params *p, void *workspace, size_t ws_bytes, hipStream_t s,
                   double *sc_host, double *hist_host) {
    CBCT_REQUIRE(((uintptr_t)workspace & 255) == 0, "workspace must be 256-byte aligned");
    GeoK G = geo_for_device(g);
    Workspace W = carve(g, G, p, (char *)workspace);
    CBCT_REQUIRE(ws_bytes >= W.bytes, "workspace too small (see piccs_workspace_bytes)");

    const int64_t ncz = g->n_col() * G.Z;
    const unsigned nvb = (unsigned)vox_blocks(G);
    const float alpha = (float)p->alpha, lam = (float)p->lambda;
    const float tau2 = (float)(p->tau * p->tau);
    const bool piple = p->method == CBCT_METHOD_PIPLE;
    auto regF_init = piple ? k_regF<true, true> : k_regF<true, false>;
    auto regF_step = piple ? k_regF<false, true> : k_regF<false, false>;
    auto regA = piple ? k_regA<true> : k_regA<false>;

    // padded column copies of the inputs (pads and guards zero)
    launch_fill(W.x - kGuard, W.cstride * 13, 0.0f, s);
    const int dt = p->precision == CBCT_PREC_MIXED_BF16 ||
                           p->precision == CBCT_PREC_MIXED_BF16_ADJ16
                       ? CBCT_BF16
                   : p->precision == CBCT_PREC_MIXED_F16 || p->precision == CBCT_PREC_MIXED_F16_ADJ16
                       ? CBCT_F16
                       : CBCT_F32;
    if (dt != CBCT_F32) launch_fill((float *)W.V16buf, (int64_t)(W.v16_bytes / 4), 0.0f, s);
    const double nvox = (double)g->n_vox();
    const double uref = std::sqrt((double)g->n_proj()) / g->d.dsd;
    // q: where the normalised v goes for reorthogonalisation, or null
    auto xw = [&](float *q) {
        if (dt == CBCT_BF16)
            hipLaunchKernelGGL(k_xw<CBCT_BF16>, dim3(4096), dim3(256), 0, s, W.x, W.w, W.V,
                               W.V16, q, ncz, W.sc, W.fl);
        else if (dt == CBCT_F16)
            hipLaunchKernelGGL(k_xw<CBCT_F16>, dim3(4096), dim3(256), 0, s, W.x, W.w, W.V,
                               W.V16, q, ncz, W.sc, W.fl);
        else
            hipLaunchKernelGGL(k_xw<CBCT_F32>, dim3(4096), dim3(256), 0, s, W.x, W.w, W.V,
                               (unsigned *)nullptr, q, ncz, W.sc, W.fl);
    };
    const bool reorth = p->reorth != 0;
    auto basis = [&](int i) { return reorth && i < p->n_inner ? W.Q + (int64_t)i * W.cstride
                                                             : (float *)nullptr; };
    // CGS2 of V against q_0 .. q_{k-1}; the second pass leaves |V|^2 partials in W.pq
    auto cgs2 = [&](int k) {
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_qdot, dim3(kQBlocks, k), dim3(256), 0, s, W.Q, W.cstride, W.V,
                               ncz, W.pq, W.fl);
            hipLaunchKernelGGL(k_qred, dim3(k), dim3(1024), 0, s, W.pq, W.qcoef, W.fl);
            hipLaunchKernelGGL(k_qaxpy, dim3(kQBlocks), dim3(256), 0, s, W.Q, W.cstride, W.V,
                               ncz, k, W.qcoef, W.pq, W.fl);
        }
    };
    vol_to_cols(G, x, W.x, s);
    vol_to_cols(G, xp, W.xp, s);
    proj_to_cols(G, b, W.bhat, true, s);  // b-hat = L * b
    hipLaunchKernelGGL(k_solve_begin, dim3(1), dim3(1), 0, s, W.sc, W.fl, W.hist,
                       p->n_outer * p->n_inner);

    FwdArgs fa{};
    fa.out = W.uhat;
    fa.uin = nullptr;
    fa.partial = W.pf;
    fa.brk = W.fl;
    // a norm and its LSQR step (k_red), with k_psum first when the partials are many
    auto red = [&](auto kern, const double *p0, int64_t n0, const double *p1, int64_t n1,
                   int it) {
        if (n0 + n1 > kPsumMin) {
            hipLaunchKernelGGL(k_psum, dim3(kPsumBlocks), dim3(256), 0, s, p0, n0, p1, n1, W.pp,
                               W.fl);
            p0 = W.pp;
            n0 = kPsumBlocks;
            p1 = nullptr;
            n1 = 0;
        }
        hipLaunchKernelGGL(kern, dim3(1), dim3(1024), 0, s, p0, n0, p1, n1, W.sc, W.fl, W.hist,
                           it, dt, nvox, uref);
    };
    // marker ranges (rocprofv3 --marker-trace) around each outer step and each
    // LSQR iteration; they span the host's enqueueing, the kernels run later on s
    int it_global = 0;
    for (int ko = 0; ko < p->n_outer; ++ko) {
        roctxRangePushA("IRN outer step");
        hipLaunchKernelGGL(k_outer_begin, dim3(1), dim3(1), 0, s, W.sc, W.fl);
        hipLaunchKernelGGL(k_weights, dim3((unsigned)vox_blocks<2>(G)), dim3(256), 0, s, G, W.x,
                           W.xp, tau2, W.W1,
                           W.W2);
        // beta_1 u_1 = b~ - A~ x_{k-1} (float32 throughout, as the restart's adjoint)
        fa.vol = W.x; fa.uin = W.bhat; fa.s1 = W.sc + SC_M1; fa.s2 = W.sc + SC_P1;
        fa.u16 = nullptr;
        launch_forward(G, FWD_SOLVER, fa, s);
        hipLaunchKernelGGL(regF_init, dim3(nvb), dim3(256), 0, s, G, W.x, W.xp, W.W1,
                           W.W2, W.u1, W.u2, W.cstride, alpha, lam, W.sc + SC_M1,
                           W.sc + SC_ZERO, W.pr, W.fl);
        red(k_red<RED_INIT_BETA>, W.pf, W.nf, W.pr, W.nr, 0);
        // alpha_1 v_1 = A~^T u_1
        launch_back(G, W.uhat, W.t, W.fl, s);
        hipLaunchKernelGGL(regA, dim3(nvb), dim3(256), 0, s, G, W.t, W.W1, W.W2, W.u1,
                           W.u2, W.cstride, alpha, lam, W.V, W.sc + SC_BACK_S1,
                           W.sc + SC_BACK_S2, W.pa, W.fl);
        red(k_red<RED_INIT_ALPHA>, W.pa, W.nr, nullptr, 0, 0);
        xw(basis(0));
        for (int ki = 0; ki < p->n_inner; ++ki, ++it_global) {
            roctxRangePushA("LSQR iteration");
            fa.vol = dt == CBCT_F32 ? (const void *)W.V : (const void *)W.V16;
            fa.uin = W.uhat; fa.s1 = W.sc + SC_FWD_S1; fa.s2 = W.sc + SC_FWD_S2;
            // *_ADJ16 forms: the inner forward also writes the adjoint's 16-bit input
            fa.u16 = W.uhat16; fa.u16_dt = dt; fa.u16_scale = W.sc + SC_U16_SCALE;  // or null
            launch_forward(G, FWD_SOLVER, fa, s,
                           dt == CBCT_BF16  ? CBCT_BF16_PAIR
                           : dt == CBCT_F16 ? CBCT_F16_PAIR
                                            : CBCT_F32);
            hipLaunchKernelGGL(regF_step, dim3(nvb), dim3(256), 0, s, G, W.V,
                               (const float *)nullptr, W.W1, W.W2, W.u1, W.u2, W.cstride,
                               alpha, lam, W.sc + SC_REG_S1, W.sc + SC_REG_S2, W.pr, W.fl);
            red(k_red<RED_BETA>, W.pf, W.nf, W.pr, W.nr, it_global);
            if (W.uhat16)
                launch_back(G, W.uhat16, W.t, W.fl, s, dt, W.sc + SC_U16_SCALE);
            else
                launch_back(G, W.uhat, W.t, W.fl, s);
            hipLaunchKernelGGL(regA, dim3(nvb), dim3(256), 0, s, G, W.t, W.W1, W.W2, W.u1,
                               W.u2, W.cstride, alpha, lam, W.V, W.sc + SC_BACK_S1,
                               W.sc + SC_BACK_S2, W.pa, W.fl);
            if (reorth) cgs2(ki + 1);
            red(k_red<RED_ALPHA>, reorth ? W.pq : W.pa, reorth ? (int64_t)kQBlocks : W.nr,
                nullptr, 0, it_global);
            xw(basis(ki + 1));
            roctxRangePop();
        }
        roctxRangePop();
    }
    hipLaunchKernelGGL(k_solve_end, dim3(1), dim3(1), 0, s, W.sc, W.fl);
    CBCT_HIP(hipGetLastError());
    cols_to_vol(G, W.x, x, s);

    if (sc_host)
        CBCT_HIP(hipMemcpyAsync(sc_host, W.sc, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost,
                                s));
    if (hist_host)
        CBCT_HIP(hipMemcpyAsync(hist_host, W.hist, sizeof(double) * p->n_outer * p->n_inner,
                                hipMemcpyDeviceToHost, s));
}

int solve_scalar_count() { return SC_COUNT; }

bool solve_numeric_fault(const double *sc) { return sc[SC_NUMERIC] != 0.0; }

void report_from_scalars(const double *sc, piccs_report *rep) {
    rep->inner_done = (int32_t)sc[SC_INNER_DONE];
    rep->outer_done = (int32_t)sc[SC_OUTER_DONE];
    rep->breakdown = (int32_t)sc[SC_NBRK];
}

}  // namespace cbct

using namespace cbct;

namespace {

int translate(const std::exception &ex) {
    if (auto e = dynamic_cast<const Error *>(&ex)) {
        set_last_error(e->what());
        return e->code;
    }
    set_last_error(ex.what());
    return CBCT_ERR_INVALID;
}

}  // namespace

extern "C" {

int piccs_weights(const cbct_geom *gc, const float *x, const float *xp, double tau, float *w1,
                  float *w2, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && x && xp && w1 && w2, "null argument");
        CBCT_REQUIRE(std::isfinite(tau) && tau >= 0, "tau must be finite and >= 0");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        hipStream_t s = (hipStream_t)hip_stream;
        GeoK G = geo_for_device(g);
        const int64_t pf = g->pad_floats();
        float *tmp = nullptr;
        CBCT_HIP(hipMallocAsync((void **)&tmp, sizeof(float) * 4 * pf, s));
        try {
            launch_fill(tmp, 4 * pf, 0.0f, s);
            float *X = tmp + kGuard, *XP = tmp + pf + kGuard, *A = tmp + 2 * pf + kGuard,
                  *B = tmp + 3 * pf + kGuard;
            vol_to_cols(G, x, X, s);
            vol_to_cols(G, xp, XP, s);
            hipLaunchKernelGGL(k_weights, dim3((unsigned)vox_blocks<2>(G)), dim3(256), 0, s, G, X,
                               XP, (float)(tau * tau), A, B);
            CBCT_HIP(hipGetLastError());
            cols_to_vol(G, A, w1, s);
            cols_to_vol(G, B, w2, s);
        } catch (...) {
            (void)hipFreeAsync(tmp, s);
            throw;
        }
        CBCT_HIP(hipFreeAsync(tmp, s));
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int piccs_workspace_bytes(const cbct_geom *gc, const piccs_params *p, size_t *bytes) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && bytes, "null argument");
        check_solve_params(p);
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        GeoK G{};
        G.nx = g->d.nx; G.ny = g->d.ny; G.nz = g->d.nz; G.nu = g->d.nu; G.nv = g->d.nv;
        G.nviews = g->d.n_views; G.Z = g->Z();
        *bytes = carve(g, G, p, nullptr).bytes;
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int piccs_krylov_solve(const cbct_geom *gc, const float *b, const float *xp, float *x,
                       const piccs_params *p, void *workspace, size_t ws_bytes,
                       piccs_report *rep, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && b && xp && x && workspace, "null argument");
        check_solve_params(p);
        hipStream_t s = (hipStream_t)hip_stream;
        const int nh = p->n_outer * p->n_inner;
        std::vector<double> sc(SC_COUNT), hist(rep && rep->resid_hist ? (size_t)nh : 0);
        solve_enqueue(const_cast<cbct_geom *>(gc), b, xp, x, p, workspace, ws_bytes, s,
                      rep ? sc.data() : nullptr, hist.empty() ? nullptr : hist.data());
        if (rep) {
            CBCT_HIP(hipStreamSynchronize(s));
            report_from_scalars(sc.data(), rep);
            if (rep->resid_hist)
                for (int q = 0; q < nh; ++q) rep->resid_hist[q] = hist[(size_t)q];
            if (solve_numeric_fault(sc.data()))
                throw Error(CBCT_ERR_NUMERIC,
                            "non-finite norm in the solve (NaN or Inf in b, x0 or xp, or an "
                            "overflow); x holds the last finite iterate");
        }
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

}  // extern "C"
