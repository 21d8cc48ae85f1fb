// Internal declarations of the CBCT HIP library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cbct.h"

namespace cbct {

// Error carrying a C status code; converted at the ABI boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);
void clear_last_error();

#define CBCT_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::cbct::Error(e_ == hipErrorOutOfMemory ? CBCT_ERR_OOM : CBCT_ERR_DEVICE, \
                                std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

#define CBCT_REQUIRE(cond, msg)                                                         \
    do {                                                                                \
        if (!(cond)) throw ::cbct::Error(CBCT_ERR_INVALID, msg);                        \
    } while (0)

// Number of zero floats before and after every padded volume buffer.
constexpr int kGuard = 64;

// Kernel-side view of a geometry on one device (passed by value).
//
// Internal layouts used by every kernel:
//  * "column" volumes: cell (i, j, k) at P[(j*nx + i)*Z + k + 1] with Z = nz + 2;
//    local entries 0 and Z-1 of each column are zero pads (cells k = -1 and
//    k = nz), and kGuard zero floats precede and follow the array;
//  * "column" projections: sample (view, iu, iv) at Y[(view*nu + iu)*nv + iv].
struct GeoK {
    int nx, ny, nz, nu, nv, nviews;
    int Z;               // nz + 2
    float hx, hy, hz;    // voxel size [mm] (detector footprints and row ranges only)
    float dso, dsd, du, dv;
    // plane indices p enter as p - n/2 (n = nx, ny or nz, integer division)
    const float4 *xy;    // [nviews*nu]: (rx, cx, ry, cy): x plane p at a' = fma(p - nx/2, rx, cx)
    const float2 *xy0;   // [nviews*nu]: (xi0, eta0): x, y index positions at a' = 0, less n/2
    const float4 *zr;    // [nv]: (z0, rg, cz, dz): z plane p at a' = fma(p - nz/2, rg, cz)
    const float *Lu2;    // [nu]: dsd^2 + u^2
    const float *Lv2;    // [nv]: v^2
    const float2 *trig;  // [nviews]: (cos th, sin th)
    // x-y traversal of every detector column (view, iu), precomputed on the
    // device with the same float32 operations the kernels would use:
    // seghdr[r] = (a_in as float bits, number of segments n), and
    // seg[r*seg_stride + q] = (exit parameter ab as float bits, column j*nx + i)
    // for q < n, followed by kSegPad no-op entries (zero-length segment at the
    // exit parameter, column 0) so that a kernel may read past the end.
    const int2 *seghdr;  // [nviews*nu]
    const int2 *seg;     // [nviews*nu*seg_stride]
    int seg_stride;      // nx + ny - 1 + kSegPad (at most nx + ny - 1 segments)
    // FDK: half the angular quadrature weight of each view, and the ramp
    // filter's non-zero taps times the isocentre pitch dp:
    // ramp[0] = 1/(4 dp) (tap 0), ramp[m+1] = -1/((2m+1)^2 pi^2 dp) (taps +-(2m+1)).
    const float *fdkw;   // [nviews]
    const float *ramp;   // [nu/2 + 1]
    int back_views;      // views per launch of A^T; 0 = chosen from the geometry
};

constexpr int kSegPad = 4;

struct DevTables {
    float4 *xy = nullptr;
    float2 *xy0 = nullptr;
    float4 *zr = nullptr;
    float *Lu2 = nullptr;
    float *Lv2 = nullptr;
    float2 *trig = nullptr;
    int2 *seghdr = nullptr;
    int2 *seg = nullptr;
    float *fdkw = nullptr;
    float *ramp = nullptr;
    void *block = nullptr;   // one allocation holding all of the above
    bool external = false;   // block owned by the caller of geo_place
};

}  // namespace cbct

struct cbct_geom {
    cbct_geom_desc d{};
    std::vector<double> angles;
    // Host copies of the float32 tables (built once in cbct_geom_create).
    std::vector<float4> xy;
    std::vector<float2> xy0;
    std::vector<float4> zr;
    std::vector<float> Lu2, Lv2;
    std::vector<float2> trig;
    std::vector<float> fdkw, ramp;
    std::mutex mu;
    std::map<int, cbct::DevTables> dev;
    int back_views = 0;  // cbct_geom_set_back_views (0 = automatic)

    int64_t n_vox() const { return (int64_t)d.nx * d.ny * d.nz; }
    int64_t n_proj() const { return (int64_t)d.n_views * d.nv * d.nu; }
    int64_t n_col() const { return (int64_t)d.nx * d.ny; }
    int Z() const { return d.nz + 2; }
    // floats in one padded column volume buffer, guards included
    int64_t pad_floats() const { return n_col() * Z() + 2 * cbct::kGuard; }
};

namespace cbct {

// Kernel arguments for geometry g on the current device (uploads tables and
// builds the segment tables once per device).
GeoK geo_for_device(cbct_geom *g);
// Enqueues the build of the x-y segment tables of G on s (seghdr/seg allocated).
void launch_segment_tables(const GeoK &G, int2 *seghdr, int2 *seg, hipStream_t s);
// Bytes of device memory held per device by the geometry's tables (one block).
size_t geom_table_bytes(const cbct_geom_desc &d);
// Places the current device's tables of g in caller memory `mem` (256-byte
// aligned, geom_table_bytes bytes), enqueuing the upload and the segment-table
// build on s; work that uses g must be ordered after s.  The geometry never
// frees that memory.  Throws if g already has tables on this device.
void geo_place(cbct_geom *g, void *mem, hipStream_t s);
// Forgets the current device's tables placed by geo_place (no free).
void geo_unplace(cbct_geom *g);

// ---- solver (piccs.hip) ----
void check_solve_params(const piccs_params *p);
// Enqueues a whole solve on s without host synchronisation; copies the scalar
// block (solve_scalar_count doubles) and the residual history to the host
// pointers, when non-null, at the end of the stream's work.
void solve_enqueue(cbct_geom *g, const float *b, const float *xp, float *x,
                   const piccs_params *p, void *workspace, size_t ws_bytes, hipStream_t s,
                   double *sc_host, double *hist_host);
int solve_scalar_count();
void report_from_scalars(const double *sc, piccs_report *rep);
// True if the solve whose scalar block this is stopped on a non-finite norm.
bool solve_numeric_fault(const double *sc);

// ---- projector launchers (proj.hip) ----
// Forward epilogue modes.
enum FwdMode { FWD_PLAIN = 0, FWD_SOLVER = 1, FWD_COUNT = 2 };

struct FwdArgs {
    const void *vol;         // padded column volume base (cell (col, -1)); element type
                             // float32, bf16 or fp16 as passed to launch_forward
    float *out;              // column projections
    const float *uin;        // FWD_SOLVER: previous u-hat (may alias out)
    const double *s1, *s2;   // FWD_SOLVER: device scalars
    double *partial;         // FWD_SOLVER: one double per block
    const int *brk;          // FWD_SOLVER: breakdown flag (2 = stopped)
    unsigned long long *count;  // FWD_COUNT
    float scale;             // FWD_PLAIN: output multiplier (value of one stored unit)
    // FWD_SOLVER, *_ADJ16 forms: 16-bit copy of the new u-hat for the adjoint
    // (bf16, or fp16 holding u-hat * *u16_scale, a power of two), or null
    void *u16;
    int u16_dt;              // CBCT_BF16 or CBCT_F16
    const double *u16_scale;
};
// Internal storage codes beyond cbct_dtype: the solver's 16-bit shadow of a
// volume kept as one 32-bit word per cell holding (cell k, cell k + 1) in its
// low and high halves, so that one aligned read yields both cells a ray step
// may need.  Word k of a column is (h(v[k]), h(v[k+1])), pads included.
constexpr int CBCT_BF16_PAIR = 16, CBCT_F16_PAIR = 17;

void launch_forward(const GeoK &G, int mode, const FwdArgs &a, hipStream_t s,
                    int dtype = CBCT_F32);
int64_t forward_blocks(const GeoK &G);

// Back projection of column projections y-hat (already multiplied by the ray
// length L) into a padded column volume (pads written as zero).  With
// dt = CBCT_BF16 / CBCT_F16, yhat holds 16-bit values (fp16: y-hat * *scale, a
// power of two, divided out at the store) and must be readable 8 bytes past its
// last sample.
void launch_back(const GeoK &G, const void *yhat, float *out, const int *brk, hipStream_t s,
                 int dt = CBCT_F32, const double *scale = nullptr);

// Batched 2-D transpose: out[b*ob + c*oc + r + ooff] = in[b*ib + r*ir + c + ioff] (* L(c,r)
// when Lu2/Lv2 are non-null: used for projections with u = c, v = r).
void launch_transpose(const float *in, float *out, int B, int R, int C, int64_t ib, int64_t ir,
                      int64_t ioff, int64_t ob, int64_t oc, int64_t ooff, const float *Lu2,
                      const float *Lv2, hipStream_t s);
void launch_fill(float *p, int64_t n, float v, hipStream_t s);

// API-layout <-> column-layout helpers.
void vol_to_cols(const GeoK &G, const float *x, float *cols, hipStream_t s);
void cols_to_vol(const GeoK &G, const float *cols, float *x, hipStream_t s);
void proj_to_cols(const GeoK &G, const float *y, float *ycol, bool scale_by_L, hipStream_t s);
void cols_to_proj(const GeoK &G, const float *ycol, float *y, hipStream_t s);


// y = A x from an API-layout volume of storage type xt (value = stored * x_scale)
// into API-layout projections y, through the column layouts held in caller
// temporaries: cols (forward_api_bytes' cols_bytes, 4-byte aligned) and ycol.
void forward_api_bytes(const cbct_geom *g, cbct_dtype xt, size_t *cols_bytes,
                       size_t *ycol_bytes);
void forward_api(const GeoK &G, const cbct_geom *g, const void *x, cbct_dtype xt,
                 float x_scale, float *y, void *cols, float *ycol, hipStream_t s);
// Kernel arguments for g on the current device if its tables are already there
// (never allocates); false otherwise.
bool geo_if_placed(cbct_geom *g, GeoK *out);

}  // namespace cbct
