// FDK (Feldkamp, Davis & Kress 1984) for the circular orbit and flat detector:
// a direct reconstruction used as a first image when no prior exists.
//
//   k_fdk_filter: each detector row is weighted by DSD / sqrt(DSD^2 + u^2 + v^2)
//     and convolved along u with the band-limited ramp at the isocentre pitch
//     dp = du DSO / DSD (taps 1/(4 dp^2) at 0, -1/(n pi dp)^2 at odd n, times
//     dp).  A block stages a tile of zero-padded rows in LDS; the result is
//     written in the column layout [view][u][v] read by the backprojector.
//   k_fdk_back: voxel-driven backprojection.  One wave per voxel column (i, j),
//     lanes over its cells (as in the adjoint projector): per view, the depth U
//     along the central ray and the detector column u are the same for the
//     whole column, and v varies linearly with z.  Bilinear interpolation, zero
//     outside the detector, weight (dbeta / 2) (DSO / U)^2.
#include <algorithm>

#include "chord.h"
#include "internal.h"

namespace cbct {

// Filter block: `rows` detector rows of one view in LDS, each stored with nu
// zeros on both sides (the taps reach nu - 1 samples away, so the sums need no
// bounds tests) at a stride of 4 mod 32 floats: the 8 rows x 4 consecutive u a
// half-wave reads fall in 32 different banks.
__host__ __device__ inline int fdk_stride(int nu) {
    const int s = 3 * nu;
    return s + ((4 - s % 32) + 32) % 32;
}

__global__ void __launch_bounds__(256)
k_fdk_filter(GeoK G, const float *__restrict__ y, float *__restrict__ q, int rows) {
    extern __shared__ float lds[];
    const int nu = G.nu, nh = nu / 2 + 1, S = fdk_stride(nu);
    float *tap = lds;            // [nh] ramp taps
    float *row = lds + nh;       // [rows][S]
    const int nrt = (G.nv + rows - 1) / rows;
    const int view = blockIdx.x / nrt;
    const int v0 = (blockIdx.x % nrt) * rows;
    const int nr = min(rows, G.nv - v0);
    for (int t = threadIdx.x; t < nh; t += blockDim.x) tap[t] = G.ramp[t];
    for (int t = threadIdx.x; t < rows * S; t += blockDim.x) {
        const int r = t / S, e = t % S - nu;   // e: sample index, outside [0, nu) is padding
        float w = 0.0f;
        if (r < nr && e >= 0 && e < nu) {
            const int v = v0 + r;
            const float L2 = G.Lu2[e] + G.Lv2[v];
            w = y[((size_t)view * G.nv + v) * nu + e] * (G.dsd / sqrtf(L2));
        }
        row[t] = w;
    }
    __syncthreads();
    // outputs t = (u, r) with r fastest (consecutive threads write consecutive
    // v); each thread keeps up to kOut outputs in registers and walks the taps
    // once for all of them
    constexpr int kOut = 16;
    const int nout = rows * nu;
    for (int base = 0; base < nout; base += kOut * 256) {
        const float *rw[kOut];
        float acc[kOut];
#pragma unroll
        for (int j = 0; j < kOut; ++j) {
            const int t = min(base + (int)threadIdx.x + 256 * j, nout - 1);
            rw[j] = row + (t % rows) * S + nu + t / rows;   // sample u of row r
            acc[j] = tap[0] * rw[j][0];
        }
        for (int m = 0; 2 * m + 1 < nu; ++m) {
            const int n = 2 * m + 1;
            const float h = tap[m + 1];
#pragma unroll
            for (int j = 0; j < kOut; ++j) acc[j] = fmaf(h, rw[j][-n] + rw[j][n], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < kOut; ++j) {
            const int t = base + (int)threadIdx.x + 256 * j;
            const int r = t % rows, u = t / rows;
            if (t < nout && r < nr) q[((size_t)view * nu + u) * G.nv + v0 + r] = acc[j];
        }
    }
}

// rows per filter block such that taps and padded rows fit in 64 KB of LDS
static int fdk_rows(int nu) {
    const int S = fdk_stride(nu), nh = nu / 2 + 1;
    return std::max(0, std::min(8, (16384 - nh) / S));
}

__global__ void __launch_bounds__(256)
k_fdk_back(GeoK G, const float *__restrict__ q, float *__restrict__ out, int kspan, int nq) {
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nzs = (G.nz + kspan - 1) / kspan;
    const int64_t lw = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * 4 + w;
    // 16 x 16 tiles of columns: the waves resident on one XCD cover a compact
    // patch of the x-y plane
    const int64_t cw = lw / nzs;
    const int zs = (int)(lw % nzs);
    const int ntx = (G.nx + 15) / 16;
    const int64_t tile = cw / 256;
    const int rt = (int)(cw % 256);
    const int i = (int)(tile % ntx) * 16 + rt % 16;
    const int j = (int)(tile / ntx) * 16 + rt / 16;
    if (i >= G.nx || j >= G.ny) return;
    const int64_t col = (int64_t)j * G.nx + i;
    const int kbase = zs * kspan;

    constexpr int QM = 8;
    float acc[QM], zk[QM];
#pragma unroll
    for (int m = 0; m < QM; ++m) {
        acc[m] = 0.0f;
        zk[m] = ((float)(kbase + lane + 64 * m) + 0.5f - 0.5f * G.nz) * G.hz;  // cell centre z
    }
    const float X = ((float)i + 0.5f - 0.5f * G.nx) * G.hx;
    const float Y = ((float)j + 0.5f - 0.5f * G.ny) * G.hy;
    const float fu_off = 0.5f * G.nu - 0.5f, fv_off = 0.5f * G.nv - 0.5f;
    for (int view = 0; view < G.nviews; ++view) {
        const float2 cs = G.trig[view];
        const float U = G.dso - (X * cs.x + Y * cs.y);
        const float lat = Y * cs.x - X * cs.y;
        const float iU = 1.0f / U;
        const float fu = G.dsd * lat * iU / G.du + fu_off;
        const float fl = floorf(fu);
        const int i0 = (int)fl;
        if (i0 < -1 || i0 > G.nu - 1) continue;   // both taps outside the detector
        const float au = fu - fl;
        const float ratio = G.dso * iU;
        const float wgt = G.fdkw[view] * ratio * ratio;
        const float sv = G.dsd * iU / G.dv;
        const bool ok0 = i0 >= 0, ok1 = i0 + 1 < G.nu;
        const float *q0 = q + ((size_t)view * G.nu + (ok0 ? i0 : 0)) * G.nv;
        const float *q1 = q + ((size_t)view * G.nu + (ok1 ? i0 + 1 : 0)) * G.nv;
#pragma unroll
        for (int m = 0; m < QM; ++m) {
            if (m >= nq) break;
            const float fv = fmaf(zk[m], sv, fv_off);
            const float flv = floorf(fv);
            const int j0 = (int)flv;
            const float av = fv - flv;
            const bool j0ok = j0 >= 0 && j0 < G.nv, j1ok = j0 + 1 >= 0 && j0 + 1 < G.nv;
            const float a00 = ok0 && j0ok ? q0[j0] : 0.0f;
            const float a01 = ok0 && j1ok ? q0[j0 + 1] : 0.0f;
            const float a10 = ok1 && j0ok ? q1[j0] : 0.0f;
            const float a11 = ok1 && j1ok ? q1[j0 + 1] : 0.0f;
            const float lo = fmaf(av, a01 - a00, a00);
            const float hi = fmaf(av, a11 - a10, a10);
            acc[m] = fmaf(wgt, fmaf(au, hi - lo, lo), acc[m]);
        }
    }
    float *oc = out + (size_t)col * G.Z;
#pragma unroll
    for (int m = 0; m < QM; ++m) {
        const int k = kbase + lane + 64 * m;
        if (m < nq && k < G.nz) oc[k + 1] = acc[m];
    }
    if (zs == 0 && lane == 0) oc[0] = 0.0f;
    if (zs == nzs - 1 && lane == 0) oc[G.nz + 1] = 0.0f;
}

}  // namespace cbct

using namespace cbct;

namespace {

int translate_fdk(const std::exception &ex) {
    if (auto e = dynamic_cast<const Error *>(&ex)) {
        set_last_error(e->what());
        return e->code;
    }
    set_last_error(ex.what());
    return CBCT_ERR_INVALID;
}

}  // namespace

extern "C" int cbct_fdk(const cbct_geom *gc, const float *y, float *x, void *hip_stream) {
    void *tmp = nullptr;
    hipStream_t s = (hipStream_t)hip_stream;
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && y && x, "null argument");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        const int nu = g->d.nu;
        const int rows = fdk_rows(nu);
        CBCT_REQUIRE(rows >= 1, "detector rows too long for the FDK filter (nu > 4680)");
        const size_t lds = sizeof(float) * ((size_t)rows * fdk_stride(nu) + nu / 2 + 1);
        const GeoK G = geo_for_device(g);
        const size_t nq_bytes = sizeof(float) * (size_t)g->n_proj();
        const size_t nv_bytes = sizeof(float) * (size_t)g->pad_floats();
        CBCT_HIP(hipMallocAsync(&tmp, nq_bytes + nv_bytes + 256, s));
        float *q = (float *)tmp;
        float *cols = (float *)((char *)tmp + ((nq_bytes + 255) & ~(size_t)255));
        const int nrt = (G.nv + rows - 1) / rows;
        const int64_t nbf = (int64_t)G.nviews * nrt;
        CBCT_REQUIRE(nbf <= 0x7fffffff, "FDK filter grid too large");
        hipLaunchKernelGGL(k_fdk_filter, dim3((unsigned)nbf), dim3(256), lds, s, G, y, q, rows);
        CBCT_HIP(hipGetLastError());
        const int nq = std::min(8, (G.nz + 63) / 64);
        const int kspan = 64 * nq;
        const int nzs = (G.nz + kspan - 1) / kspan;
        const int64_t ntiles = (int64_t)((G.nx + 15) / 16) * ((G.ny + 15) / 16);
        const int64_t nb = (ntiles * 256 * nzs + 3) / 4;
        CBCT_REQUIRE(nb <= 0x7fffffff, "FDK grid too large");
        float *cbase = cols + kGuard;
        hipLaunchKernelGGL(k_fdk_back, dim3((unsigned)nb), dim3(256), 0, s, G, q, cbase, kspan,
                           nq);
        CBCT_HIP(hipGetLastError());
        cols_to_vol(G, cbase, x, s);
        CBCT_HIP(hipFreeAsync(tmp, s));
        return CBCT_OK;
    } catch (const std::exception &e) {
        if (tmp) (void)hipFreeAsync(tmp, s);
        return translate_fdk(e);
    }
}
