// Geometry handle: validation, float64 -> float32 ray tables, per-device upload.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace cbct {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }

// Coefficients of one axis of a ray written as
//   index position(a') = o + c0 + a' * dpos,  a' = alpha - a_ref,  o = n / 2,
// from the source coordinate S, direction component d (P - S) and the grid's
// low edge lo, cell size h and cell count n.  Plane p is crossed at
// a' = (p - o - c0) / dpos, evaluated by the kernels as fma(p - o, r, c) with
// r = 1/dpos rounded to float and c = -c0 * r rounded once from float64.
// Counting planes from the middle of the axis and deriving c from the rounded
// r keeps the float32 cancellation in that fma to the ray's distance from the
// axis midpoint: a crossing is off by about eps * |p - o| cells rather than
// eps * p, and a rounding of r only scales the ray about its own a' = 0.
static void axis_coeffs(double S, double d, double lo, double h, int n, double a_ref,
                        float &c0, float &r, float &c, float &dpos_f) {
    const double dpos = d / h;                     // index units per unit alpha
    const double pos_ref = (S - lo) / h + a_ref * dpos;  // index position at a' = 0
    const int o = n >> 1;
    const double rel = pos_ref - o;
    c0 = (float)rel;
    dpos_f = (float)dpos;
    if (std::fabs(dpos) > 1e-30) {
        r = (float)(1.0 / dpos);
        c = (float)(-rel * (double)r);
    } else {
        // A ray parallel to the planes never crosses them.  Its cell is
        // floor(pos) inside the box (a ray lying in an interior plane belongs to
        // the cell above it, as with Siddon's midpoint rule) and none when it
        // lies in or beyond an outer face (cell -1 or n).  Planes at or below
        // that cell get parameter -huge, the others +huge: half a plane spacing
        // times 1e30, so float rounding cannot move a plane to the wrong side.
        const double kc = pos_ref <= 0.0 ? -1.0 : (pos_ref >= n ? (double)n : std::floor(pos_ref));
        r = 1e30f;
        c = (float)(-(kc - o + 0.5) * 1e30);
    }
}

static void build_tables(cbct_geom *g) {
    const cbct_geom_desc &d = g->d;
    const double a_ref = d.dso / d.dsd;
    const double xlo = -d.nx * d.vx / 2.0, ylo = -d.ny * d.vy / 2.0, zlo = -d.nz * d.vz / 2.0;
    g->xy.resize((size_t)d.n_views * d.nu);
    g->xy0.resize((size_t)d.n_views * d.nu);
    g->trig.resize((size_t)d.n_views);
    for (int v = 0; v < d.n_views; ++v) {
        const double th = g->angles[(size_t)v];
        const double c = std::cos(th), s = std::sin(th);
        g->trig[(size_t)v] = make_float2((float)c, (float)s);
        const double Sx = d.dso * c, Sy = d.dso * s;
        for (int iu = 0; iu < d.nu; ++iu) {
            const double u = (iu + 0.5) * d.du - d.nu * d.du / 2.0;
            const double Px = (d.dso - d.dsd) * c - u * s;
            const double Py = (d.dso - d.dsd) * s + u * c;
            float xi0, rx, cx, dx, eta0, ry, cy, dy;
            axis_coeffs(Sx, Px - Sx, xlo, d.vx, d.nx, a_ref, xi0, rx, cx, dx);
            axis_coeffs(Sy, Py - Sy, ylo, d.vy, d.ny, a_ref, eta0, ry, cy, dy);
            g->xy[(size_t)v * d.nu + iu] = make_float4(rx, cx, ry, cy);
            g->xy0[(size_t)v * d.nu + iu] = make_float2(xi0, eta0);
        }
    }
    g->zr.resize((size_t)d.nv);
    g->Lv2.resize((size_t)d.nv);
    for (int iv = 0; iv < d.nv; ++iv) {
        const double vmm = (iv + 0.5) * d.dv - d.nv * d.dv / 2.0;
        float z0, rg, cz, dz;
        axis_coeffs(0.0, vmm, zlo, d.vz, d.nz, a_ref, z0, rg, cz, dz);
        g->zr[(size_t)iv] = make_float4(z0, rg, cz, dz);
        g->Lv2[(size_t)iv] = (float)(vmm * vmm);
    }
    g->Lu2.resize((size_t)d.nu);
    for (int iu = 0; iu < d.nu; ++iu) {
        const double u = (iu + 0.5) * d.du - d.nu * d.du / 2.0;
        g->Lu2[(size_t)iu] = (float)(d.dsd * d.dsd + u * u);
    }
    // FDK quadrature: each view weighs half the angle between its neighbours
    // on the circle (2 pi / V for equal spacing); half of that again is the
    // 1/2 of the full-scan formula.
    {
        const double two_pi = 2.0 * M_PI;
        std::vector<std::pair<double, int>> a((size_t)d.n_views);
        for (int v = 0; v < d.n_views; ++v)
            a[(size_t)v] = {std::fmod(std::fmod(g->angles[(size_t)v], two_pi) + two_pi, two_pi),
                            v};
        std::sort(a.begin(), a.end());
        g->fdkw.resize((size_t)d.n_views);
        for (int q = 0; q < d.n_views; ++q) {
            const double nxt = q + 1 < d.n_views ? a[(size_t)q + 1].first : a[0].first + two_pi;
            const double prv = q > 0 ? a[(size_t)q - 1].first : a.back().first - two_pi;
            g->fdkw[(size_t)a[(size_t)q].second] = (float)(0.25 * (nxt - prv));
        }
    }
    // band-limited ramp at the isocentre pitch, times that pitch
    {
        const double dp = d.du * d.dso / d.dsd;
        g->ramp.resize((size_t)d.nu / 2 + 1);
        g->ramp[0] = (float)(1.0 / (4.0 * dp));
        for (size_t m = 0; m + 1 < g->ramp.size(); ++m) {
            const double n = 2.0 * (double)m + 1.0;
            g->ramp[m + 1] = (float)(-1.0 / (n * n * M_PI * M_PI * dp));
        }
    }
}

static void validate(const cbct_geom_desc *d) {
    CBCT_REQUIRE(d != nullptr, "null geometry descriptor");
    CBCT_REQUIRE(d->nx > 0 && d->ny > 0 && d->nz > 0, "volume sizes must be > 0");
    CBCT_REQUIRE(d->nu > 0 && d->nv > 0 && d->n_views > 0, "detector sizes and n_views must be > 0");
    CBCT_REQUIRE(d->vx > 0 && d->vy > 0 && d->vz > 0, "voxel sizes must be > 0");
    CBCT_REQUIRE(d->du > 0 && d->dv > 0, "detector pitch must be > 0");
    CBCT_REQUIRE(std::isfinite(d->dso) && std::isfinite(d->dsd) && d->dso > 0 && d->dsd > d->dso,
                 "need 0 < DSO < DSD");
    CBCT_REQUIRE(d->nx <= 8192 && d->ny <= 8192 && d->nz <= 8192, "volume side > 8192");
    CBCT_REQUIRE(d->nu <= 16384 && d->nv <= 16384 && d->n_views <= 65536,
                 "detector or view count too large");
    CBCT_REQUIRE((int64_t)d->n_views * d->nu * d->nv < (int64_t)1 << 40, "too many rays");
    const double hx = d->nx * d->vx / 2, hy = d->ny * d->vy / 2, hz = d->nz * d->vz / 2;
    const double rsph = std::sqrt(hx * hx + hy * hy + hz * hz);
    const double rxy = std::sqrt(hx * hx + hy * hy);
    CBCT_REQUIRE(d->dso > rsph, "source inside the volume's bounding sphere");
    CBCT_REQUIRE(d->dsd - d->dso > rxy, "detector intersects the volume");
    // At most one z plane per x-y cell: z moves by |v|/DSD per mm of x-y path
    // at most, and a ray's path through one x-y cell is at most the cell diagonal.
    const double vmax = d->nv * d->dv / 2.0;
    const double diag = std::sqrt(d->vx * d->vx + d->vy * d->vy);
    CBCT_REQUIRE(vmax / d->dsd * diag < 0.95 * d->vz,
                 "cone angle too large for the column traversal (a ray would cross more than "
                 "one z plane inside one x-y cell)");
    if (d->angles)
        for (int v = 0; v < d->n_views; ++v)
            CBCT_REQUIRE(std::isfinite(d->angles[v]), "non-finite view angle");
}

static GeoK make_geok(const cbct_geom *g, const DevTables &t) {
    const cbct_geom_desc &d = g->d;
    GeoK G;
    G.nx = d.nx; G.ny = d.ny; G.nz = d.nz; G.nu = d.nu; G.nv = d.nv; G.nviews = d.n_views;
    G.Z = d.nz + 2;
    G.hx = (float)d.vx; G.hy = (float)d.vy; G.hz = (float)d.vz;
    G.dso = (float)d.dso; G.dsd = (float)d.dsd; G.du = (float)d.du; G.dv = (float)d.dv;
    G.xy = t.xy; G.xy0 = t.xy0; G.zr = t.zr; G.Lu2 = t.Lu2; G.Lv2 = t.Lv2; G.trig = t.trig;
    G.seghdr = t.seghdr; G.seg = t.seg; G.seg_stride = d.nx + d.ny - 1 + kSegPad;
    G.fdkw = t.fdkw; G.ramp = t.ramp;
    G.back_views = g->back_views;
    return G;
}

// Offsets of the device tables inside one block, each part 256-byte aligned.
struct TableLayout {
    size_t xy, xy0, zr, Lu2, Lv2, trig, seghdr, seg, fdkw, ramp, total;
};

static TableLayout table_layout(const cbct_geom_desc &d) {
    const size_t nr = (size_t)d.n_views * d.nu;
    const size_t stride = (size_t)d.nx + d.ny - 1 + kSegPad;
    TableLayout L{};
    size_t o = 0;
    auto put = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) & ~(size_t)255;
        return at;
    };
    L.xy = put(sizeof(float4) * nr);
    L.xy0 = put(sizeof(float2) * nr);
    L.zr = put(sizeof(float4) * d.nv);
    L.Lu2 = put(sizeof(float) * d.nu);
    L.Lv2 = put(sizeof(float) * d.nv);
    L.trig = put(sizeof(float2) * d.n_views);
    L.seghdr = put(sizeof(int2) * nr);
    L.seg = put(sizeof(int2) * nr * stride);
    L.fdkw = put(sizeof(float) * d.n_views);
    L.ramp = put(sizeof(float) * ((size_t)d.nu / 2 + 1));
    L.total = o;
    return L;
}

// Points t into `base` and enqueues the table uploads and the segment-table
// build on s.  The host tables live as long as g.
static void upload_tables(cbct_geom *g, char *base, DevTables &t, hipStream_t s) {
    const cbct_geom_desc &d = g->d;
    const TableLayout L = table_layout(d);
    t.block = base;
    t.xy = (float4 *)(base + L.xy);
    t.xy0 = (float2 *)(base + L.xy0);
    t.zr = (float4 *)(base + L.zr);
    t.Lu2 = (float *)(base + L.Lu2);
    t.Lv2 = (float *)(base + L.Lv2);
    t.trig = (float2 *)(base + L.trig);
    t.seghdr = (int2 *)(base + L.seghdr);
    t.seg = (int2 *)(base + L.seg);
    t.fdkw = (float *)(base + L.fdkw);
    t.ramp = (float *)(base + L.ramp);
    CBCT_HIP(hipMemcpyAsync(t.xy, g->xy.data(), sizeof(float4) * g->xy.size(),
                            hipMemcpyHostToDevice, s));
    CBCT_HIP(hipMemcpyAsync(t.xy0, g->xy0.data(), sizeof(float2) * g->xy0.size(),
                            hipMemcpyHostToDevice, s));
    CBCT_HIP(hipMemcpyAsync(t.zr, g->zr.data(), sizeof(float4) * g->zr.size(),
                            hipMemcpyHostToDevice, s));
    CBCT_HIP(hipMemcpyAsync(t.Lu2, g->Lu2.data(), sizeof(float) * d.nu, hipMemcpyHostToDevice, s));
    CBCT_HIP(hipMemcpyAsync(t.Lv2, g->Lv2.data(), sizeof(float) * d.nv, hipMemcpyHostToDevice, s));
    CBCT_HIP(hipMemcpyAsync(t.trig, g->trig.data(), sizeof(float2) * g->trig.size(),
                            hipMemcpyHostToDevice, s));
    CBCT_HIP(hipMemcpyAsync(t.fdkw, g->fdkw.data(), sizeof(float) * g->fdkw.size(),
                            hipMemcpyHostToDevice, s));
    CBCT_HIP(hipMemcpyAsync(t.ramp, g->ramp.data(), sizeof(float) * g->ramp.size(),
                            hipMemcpyHostToDevice, s));
    GeoK G = make_geok(g, t);
    launch_segment_tables(G, t.seghdr, t.seg, s);
}

GeoK geo_for_device(cbct_geom *g) {
    int dev = 0;
    CBCT_HIP(hipGetDevice(&dev));
    DevTables t;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        auto it = g->dev.find(dev);
        if (it == g->dev.end()) {
            void *block = nullptr;
            hipStream_t s = nullptr;
            try {
                CBCT_HIP(hipMalloc(&block, table_layout(g->d).total));
                CBCT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
                upload_tables(g, (char *)block, t, s);
                CBCT_HIP(hipStreamSynchronize(s));
                CBCT_HIP(hipStreamDestroy(s));
                s = nullptr;
            } catch (...) {
                if (s) (void)hipStreamDestroy(s);
                (void)hipFree(block);
                throw;
            }
            g->dev[dev] = t;
        } else {
            t = it->second;
        }
    }
    return make_geok(g, t);
}

bool geo_if_placed(cbct_geom *g, GeoK *out) {
    int dev = 0;
    CBCT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g->mu);
    auto it = g->dev.find(dev);
    if (it == g->dev.end()) return false;
    *out = make_geok(g, it->second);
    return true;
}

void geo_place(cbct_geom *g, void *mem, hipStream_t s) {
    CBCT_REQUIRE(mem && ((uintptr_t)mem & 255) == 0, "table memory must be 256-byte aligned");
    int dev = 0;
    CBCT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g->mu);
    CBCT_REQUIRE(g->dev.find(dev) == g->dev.end(), "geometry already has device tables");
    DevTables t;
    upload_tables(g, (char *)mem, t, s);
    t.external = true;
    g->dev[dev] = t;
}

void geo_unplace(cbct_geom *g) {
    int dev = 0;
    CBCT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g->mu);
    auto it = g->dev.find(dev);
    if (it != g->dev.end() && it->second.external) g->dev.erase(it);
}

size_t geom_table_bytes(const cbct_geom_desc &d) { return table_layout(d).total; }

}  // namespace cbct

using namespace cbct;

extern "C" {

const char *cbct_last_error(void) { return g_last_error.c_str(); }

int cbct_geom_create(const cbct_geom_desc *d, cbct_geom **out) {
    try {
        clear_last_error();
        CBCT_REQUIRE(out != nullptr, "null output handle");
        *out = nullptr;
        validate(d);
        cbct_geom *g = new cbct_geom();
        g->d = *d;
        g->angles.resize((size_t)d->n_views);
        for (int v = 0; v < d->n_views; ++v)
            g->angles[(size_t)v] = d->angles ? d->angles[v] : 2.0 * M_PI * v / d->n_views;
        g->d.angles = g->angles.data();
        build_tables(g);
        *out = g;
        return CBCT_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return CBCT_ERR_OOM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return CBCT_ERR_INVALID;
    }
}

void cbct_geom_destroy(cbct_geom *g) {
    if (!g) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g->dev) {
        if (kv.second.external) continue;
        (void)hipSetDevice(kv.first);
        (void)hipFree(kv.second.block);
    }
    (void)hipSetDevice(cur);
    delete g;
}

int cbct_geom_set_back_views(cbct_geom *g, int views) {
    if (!g || views < 0) {
        set_last_error(!g ? "null geometry" : "views per adjoint launch must be >= 0");
        return CBCT_ERR_INVALID;
    }
    g->back_views = views;
    return CBCT_OK;
}

int cbct_geom_sizes(const cbct_geom *g, int64_t *n_vox, int64_t *n_proj) {
    if (!g) {
        set_last_error("null geometry");
        return CBCT_ERR_INVALID;
    }
    if (n_vox) *n_vox = g->n_vox();
    if (n_proj) *n_proj = g->n_proj();
    return CBCT_OK;
}

}  // extern "C"
