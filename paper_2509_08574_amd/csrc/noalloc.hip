// Allocation-free forward projection: cbct_forward with its temporaries in a
// fixed device array of this library instead of stream-ordered allocations,
// for callers that cannot allocate (code under graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The array lives in this translation unit's code object, which holds no
// kernels: it is loaded (and the array placed) on a device the first time
// cbct_forward_noalloc runs there, and stays until the process ends.  The
// projector kernels it drives live in proj.hip and take its address as an
// ordinary pointer argument.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>

#include "internal.h"

namespace cbct {

// Largest temporary the call can hold: the padded column copy of the volume
// (4 or 2 bytes per cell, pads and guards included) plus the column-layout
// projections (4 bytes per sample), each rounded up to 256 bytes.  256 MiB
// covers 256^3 volumes with 90 views of 512 x 512.
constexpr size_t kScratchBytes = CBCT_FORWARD_NOALLOC_MAX_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must be a multiple of 256 bytes");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
std::map<int, unsigned char *> g_ptr;  // device ordinal -> address of `scratch` there

// Device address of this device's copy of the array (looked up once per device,
// with that device current; the host-side name is not a device address).
unsigned char *scratch_on_current_device() {
    int dev = 0;
    CBCT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ptr.find(dev);
    if (it != g_ptr.end()) return it->second;
    void *p = nullptr;
    CBCT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CBCT_REQUIRE(p != nullptr && ((uintptr_t)p & 255) == 0,
                 "scratch array has no aligned device address");
    g_ptr[dev] = (unsigned char *)p;
    return (unsigned char *)p;
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

int translate(const std::exception &ex) {
    if (auto e = dynamic_cast<const Error *>(&ex)) {
        set_last_error(e->what());
        return e->code;
    }
    set_last_error(ex.what());
    return CBCT_ERR_INVALID;
}

}  // namespace
}  // namespace cbct

using namespace cbct;

extern "C" {

int cbct_forward_noalloc(const cbct_geom *gc, const void *x, cbct_dtype xt, float x_scale,
                         float *y, void *hip_stream) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gc && x && y, "null argument");
        CBCT_REQUIRE(xt == CBCT_F32 || xt == CBCT_BF16 || xt == CBCT_F16, "unknown dtype");
        CBCT_REQUIRE(std::isfinite(x_scale) && x_scale > 0.0f, "scale must be finite and > 0");
        cbct_geom *g = const_cast<cbct_geom *>(gc);
        size_t cols_bytes = 0, ycol_bytes = 0;
        forward_api_bytes(g, xt, &cols_bytes, &ycol_bytes);
        const size_t need = al256(cols_bytes) + al256(ycol_bytes);
        if (need > kScratchBytes)
            throw Error(CBCT_ERR_INVALID,
                        "cbct_forward_noalloc: geometry needs " + std::to_string(need) +
                            " bytes of scratch, more than the fixed " +
                            std::to_string(kScratchBytes) + " (use cbct_forward)");
        GeoK G{};
        if (!geo_if_placed(g, &G))
            throw Error(CBCT_ERR_INVALID,
                        "cbct_forward_noalloc: the geometry's tables are not on this device "
                        "yet (any allocating call with this geometry places them)");
        unsigned char *base = scratch_on_current_device();
        forward_api(G, g, x, xt, x_scale, y, base, (float *)(base + al256(cols_bytes)),
                    (hipStream_t)hip_stream);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

}  // extern "C"
