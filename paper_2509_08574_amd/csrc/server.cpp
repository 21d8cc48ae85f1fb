// Reconstruction server: continuous batching of IRN-PICCS solves on one device.
//
// One scheduler thread owns the device side.  It admits waiting requests
// (serve_core.h decides which), enqueues each admitted request whole on its
// slot's stream -- H2D of b, x_0 from the patient's resident x_prev or x_p,
// the solve, x written back to x_prev and to a page-locked host buffer -- and
// records an event; it then polls the events of running requests and retires
// them.  Every device byte the server uses lives in one arena allocated at
// create time (the HBM budget), so steady-state serving performs no device
// allocation and no implicit device synchronisation.
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdio>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <memory>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "serve_core.h"

namespace cbct {
namespace {

using serve::align_up;
using serve::Job;
using serve::kNoBlock;

// Page-locked host buffers, kept for reuse until the server ends (freeing
// page-locked memory synchronises the device).
class PinnedPool {
   public:
    void *get(size_t bytes, size_t *cap) {
        const size_t want = bytes ? bytes : 1;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(want);
            if (it != free_.end() && it->first <= 2 * want + (size_t(1) << 20)) {
                *cap = it->first;
                void *p = it->second;
                free_.erase(it);
                return p;
            }
        }
        const size_t n = (want + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
        void *p = nullptr;
        CBCT_HIP(hipHostMalloc(&p, n, hipHostMallocDefault));
        std::lock_guard<std::mutex> lk(mu_);
        all_.push_back(p);
        *cap = n;
        return p;
    }
    void put(void *p, size_t cap) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_.emplace(cap, p);
    }
    ~PinnedPool() {
        for (void *p : all_) (void)hipHostFree(p);
    }

   private:
    std::mutex mu_;
    std::multimap<size_t, void *> free_;
    std::vector<void *> all_;
};

struct Pinned {
    void *p = nullptr;
    size_t cap = 0;
};

struct Payload {
    cbct_geom *g = nullptr;  // owned by the server's geometry cache
    piccs_params params{};
    int32_t x0 = CBCT_X0_PREVIOUS;
    int64_t n_vox = 0, n_proj = 0;
    size_t ws_bytes = 0;
    Pinned b, x, r;          // b copy; result x; scalars + residual history
    hipEvent_t ev = nullptr;
    piccs_report report{};
    roctx_range_id_t range = 0;  // marker range from launch to collection (0: none)
};

struct Resident {
    float *xp = nullptr, *xprev = nullptr;
    int32_t nx = 0, ny = 0, nz = 0;
    double vx = 0, vy = 0, vz = 0;
    bool has_prev = false;
};

// Everything that makes two geometries give the same tables.
using GeomKey = std::tuple<int32_t, int32_t, int32_t, double, double, double, int32_t, int32_t,
                           double, double, double, double, std::vector<double>>;

GeomKey key_of(const cbct_geom_desc &d) {
    std::vector<double> a((size_t)std::max(d.n_views, 0));
    for (int v = 0; v < d.n_views; ++v)
        a[(size_t)v] = d.angles ? d.angles[v] : 2.0 * M_PI * v / d.n_views;
    return GeomKey(d.nx, d.ny, d.nz, d.vx, d.vy, d.vz, d.nu, d.nv, d.du, d.dv, d.dso, d.dsd,
                   std::move(a));
}

struct GeomHost {
    cbct_geom *g = nullptr;
    hipEvent_t ready = nullptr;  // table build finished (recorded at placement)
    GeomKey key;
};

}  // namespace
}  // namespace cbct

using namespace cbct;

struct cbct_server {
    struct Backend;

    cbct_server_config cfg{};
    int device = 0;
    char *base = nullptr;
    std::vector<hipStream_t> streams;
    hipStream_t upload = nullptr;
    PinnedPool pinned;
    std::vector<hipEvent_t> free_events;
    int nsc = 0;

    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::thread worker;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    std::unique_ptr<serve::Scheduler<Payload>> core;
    std::map<int32_t, Resident> residents;
    std::map<GeomKey, int64_t> geom_ids;
    std::unordered_map<int64_t, GeomHost> geoms;
    int64_t next_geom = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    hipEvent_t get_event() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        CBCT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return e;
    }

    void release_payload(Payload &P) {
        pinned.put(P.b.p, P.b.cap);
        pinned.put(P.x.p, P.x.cap);
        pinned.put(P.r.p, P.r.cap);
        P.b = P.x = P.r = Pinned{};
        if (P.ev) free_events.push_back(P.ev);
        P.ev = nullptr;
    }

    void forget_geometry(int64_t id) {
        auto it = geoms.find(id);
        if (it == geoms.end()) return;
        geom_ids.erase(it->second.key);
        if (it->second.ready) (void)hipEventDestroy(it->second.ready);
        cbct_geom_destroy(it->second.g);
        geoms.erase(it);
    }

    struct Backend {
        cbct_server *S;
        double now() { return S->now(); }
        void place_geometry(int64_t key, size_t off, int slot) {
            GeomHost &gh = S->geoms.at(key);
            geo_place(gh.g, S->base + off, S->streams[(size_t)slot]);
            if (!gh.ready) CBCT_HIP(hipEventCreateWithFlags(&gh.ready, hipEventDisableTiming));
            CBCT_HIP(hipEventRecord(gh.ready, S->streams[(size_t)slot]));
        }
        void drop_geometry(int64_t key, bool unused) {
            auto it = S->geoms.find(key);
            if (it == S->geoms.end()) return;
            geo_unplace(it->second.g);
            if (unused) S->forget_geometry(key);
        }
        void launch(Job<Payload> &j) {
            Payload &P = j.payload;
            hipStream_t s = S->streams[(size_t)j.slot];
            char *blk = S->base + j.off;
            float *b_d = (float *)blk;
            float *x_d = (float *)(blk + align_up(sizeof(float) * (size_t)P.n_proj));
            void *ws = blk + align_up(sizeof(float) * (size_t)P.n_proj) +
                       align_up(sizeof(float) * (size_t)P.n_vox);
            P.ev = S->get_event();
            try {
                Resident &R = S->residents.at(j.patient);
                CBCT_HIP(hipStreamWaitEvent(s, S->geoms.at(j.geom).ready, 0));
                CBCT_HIP(hipMemcpyAsync(b_d, P.b.p, sizeof(float) * (size_t)P.n_proj,
                                        hipMemcpyHostToDevice, s));
                const float *x0 =
                    (P.x0 == CBCT_X0_PREVIOUS && R.has_prev) ? R.xprev : R.xp;
                CBCT_HIP(hipMemcpyAsync(x_d, x0, sizeof(float) * (size_t)P.n_vox,
                                        hipMemcpyDeviceToDevice, s));
                double *r = (double *)P.r.p;
                solve_enqueue(P.g, b_d, R.xp, x_d, &P.params, ws, P.ws_bytes, s, r,
                              r + S->nsc);
                CBCT_HIP(hipMemcpyAsync(R.xprev, x_d, sizeof(float) * (size_t)P.n_vox,
                                        hipMemcpyDeviceToDevice, s));
                R.has_prev = true;
                CBCT_HIP(hipMemcpyAsync(P.x.p, x_d, sizeof(float) * (size_t)P.n_vox,
                                        hipMemcpyDeviceToHost, s));
                CBCT_HIP(hipEventRecord(P.ev, s));
                // a marker range per request, from its launch on a slot to its
                // collection (seen by rocprofv3 --marker-trace)
                char name[96];
                std::snprintf(name, sizeof name, "request %llu patient %d slot %d",
                              (unsigned long long)j.ticket, (int)j.patient, j.slot);
                P.range = roctxRangeStartA(name);
            } catch (...) {
                // order completion after whatever was enqueued
                if (hipEventRecord(P.ev, s) != hipSuccess) {
                    (void)hipStreamSynchronize(s);
                    S->free_events.push_back(P.ev);
                    P.ev = nullptr;
                }
                throw;
            }
        }
        bool finished(Job<Payload> &j) {
            Payload &P = j.payload;
            if (!P.ev) return true;
            const hipError_t e = hipEventQuery(P.ev);
            if (e == hipErrorNotReady) return false;
            if (e != hipSuccess && j.status == CBCT_PENDING) {
                j.status = CBCT_ERR_DEVICE;
                j.error = std::string("request failed on the device: ") + hipGetErrorString(e);
            }
            return true;
        }
        void collect(Job<Payload> &j) {
            Payload &P = j.payload;
            if (P.range) roctxRangeStop(P.range);
            P.range = 0;
            if (j.status == CBCT_PENDING) {
                report_from_scalars((const double *)P.r.p, &P.report);
                j.status = CBCT_OK;
                if (solve_numeric_fault((const double *)P.r.p)) {
                    j.status = CBCT_ERR_NUMERIC;
                    j.error = "non-finite norm in the solve (NaN or Inf in b or the start "
                              "image, or an overflow)";
                }
            }
            if (P.ev) S->free_events.push_back(P.ev);
            P.ev = nullptr;
            if (j.status != CBCT_OK) {
                S->pinned.put(P.b.p, P.b.cap);
                P.b = Pinned{};
            }
        }
        void discard(Job<Payload> &j) { S->release_payload(j.payload); }
    };

    Backend be{this};

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            core->step(be);
            if (stop && core->idle()) break;
            if (core->in_flight())
                cv.wait_for(lk, std::chrono::microseconds(100));
            else
                cv.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
};

namespace {

int translate(const std::exception &ex) {
    if (auto e = dynamic_cast<const Error *>(&ex)) {
        set_last_error(e->what());
        return e->code;
    }
    if (dynamic_cast<const std::bad_alloc *>(&ex)) {
        set_last_error("host allocation failed");
        return CBCT_ERR_OOM;
    }
    set_last_error(ex.what());
    return CBCT_ERR_INVALID;
}

// Restores the calling thread's current device on scope exit.
struct DeviceGuard {
    int prev = 0;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        CBCT_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() { (void)hipSetDevice(prev); }
};

}  // namespace

extern "C" {

int cbct_server_create(const cbct_server_config *c, cbct_server **out) {
    cbct_server *S = nullptr;
    try {
        clear_last_error();
        CBCT_REQUIRE(c && out, "null argument");
        *out = nullptr;
        CBCT_REQUIRE(c->max_slots >= 1 && c->max_slots <= 64, "max_slots must be in [1, 64]");
        CBCT_REQUIRE(c->max_queue >= 0, "max_queue must be >= 0");
        int ndev = 0;
        CBCT_HIP(hipGetDeviceCount(&ndev));
        CBCT_REQUIRE(c->device >= 0 && c->device < ndev, "no such device");
        DeviceGuard dg(c->device);
        S = new cbct_server();
        S->cfg = *c;
        S->device = c->device;
        if (S->cfg.max_queue == 0) S->cfg.max_queue = 4096;
        size_t budget = c->hbm_budget_bytes;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            CBCT_HIP(hipMemGetInfo(&fr, &tot));
            budget = fr / 10 * 9;
        }
        budget = budget / serve::kAlign * serve::kAlign;
        CBCT_REQUIRE(budget > 0, "HBM budget too small");
        CBCT_HIP(hipMalloc((void **)&S->base, budget));
        S->cfg.hbm_budget_bytes = budget;
        for (int i = 0; i < c->max_slots; ++i) {
            hipStream_t s = nullptr;
            CBCT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            S->streams.push_back(s);
        }
        CBCT_HIP(hipStreamCreateWithFlags(&S->upload, hipStreamNonBlocking));
        S->nsc = solve_scalar_count();
        S->core = std::make_unique<serve::Scheduler<Payload>>(budget, c->max_slots,
                                                              S->cfg.max_queue);
        S->worker = std::thread([S] { S->loop(); });
        *out = S;
        return CBCT_OK;
    } catch (const std::exception &e) {
        if (S) {
            for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
            if (S->upload) (void)hipStreamDestroy(S->upload);
            if (S->base) (void)hipFree(S->base);
            delete S;
        }
        return translate(e);
    }
}

int cbct_server_add_prior(cbct_server *S, int32_t patient, const cbct_geom_desc *gd,
                          const float *xp_host) {
    try {
        clear_last_error();
        CBCT_REQUIRE(S && gd && xp_host, "null argument");
        cbct_geom *g = nullptr;
        int rc = cbct_geom_create(gd, &g);  // validates the description
        if (rc != CBCT_OK) return rc;
        const int64_t M = g->n_vox();
        cbct_geom_destroy(g);
        size_t off = kNoBlock;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            CBCT_REQUIRE(!S->core->has_patient(patient), "patient already registered");
            off = S->core->add_patient(patient, 2 * align_up(sizeof(float) * (size_t)M));
            if (off == kNoBlock)
                throw Error(CBCT_ERR_OOM, "prior and previous reconstruction do not fit in the "
                                          "HBM budget");
        }
        Resident R;
        R.xp = (float *)(S->base + off);
        R.xprev = (float *)(S->base + off + align_up(sizeof(float) * (size_t)M));
        R.nx = gd->nx; R.ny = gd->ny; R.nz = gd->nz;
        R.vx = gd->vx; R.vy = gd->vy; R.vz = gd->vz;
        {
            DeviceGuard dg(S->device);
            CBCT_HIP(hipMemcpyAsync(R.xp, xp_host, sizeof(float) * (size_t)M,
                                    hipMemcpyHostToDevice, S->upload));
            CBCT_HIP(hipStreamSynchronize(S->upload));
        }
        // visible to submit only once the prior is on the device
        std::lock_guard<std::mutex> lk(S->mu);
        S->residents[patient] = R;
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_server_submit(cbct_server *S, const cbct_request *r, uint64_t *ticket) {
    Payload P;
    try {
        clear_last_error();
        CBCT_REQUIRE(S && r && ticket && r->b_host, "null argument");
        *ticket = 0;
        check_solve_params(&r->params);
        CBCT_REQUIRE(r->x0 == CBCT_X0_PREVIOUS || r->x0 == CBCT_X0_PRIOR, "unknown x0 source");
        CBCT_REQUIRE(r->geom.n_views >= 1 && r->geom.nu >= 1 && r->geom.nv >= 1,
                     "invalid geometry sizes");
        const int64_t N = (int64_t)r->geom.n_views * r->geom.nu * r->geom.nv;
        const int64_t M = (int64_t)r->geom.nx * r->geom.ny * r->geom.nz;
        CBCT_REQUIRE(M >= 1, "invalid geometry sizes");
        // copy b outside the lock (it can be hundreds of MB)
        P.b.p = S->pinned.get(sizeof(float) * (size_t)N, &P.b.cap);
        std::memcpy(P.b.p, r->b_host, sizeof(float) * (size_t)N);
        P.x.p = S->pinned.get(sizeof(float) * (size_t)M, &P.x.cap);
        const size_t nh = (size_t)r->params.n_outer * r->params.n_inner;
        P.r.p = S->pinned.get(sizeof(double) * (solve_scalar_count() + nh), &P.r.cap);
        P.params = r->params;
        P.x0 = r->x0;
        P.n_vox = M;
        P.n_proj = N;

        GeomKey key = key_of(r->geom);
        std::lock_guard<std::mutex> lk(S->mu);
        auto rit = S->residents.find(r->patient);
        if (rit == S->residents.end()) throw Error(CBCT_ERR_NOT_FOUND, "unknown patient");
        const Resident &R = rit->second;
        CBCT_REQUIRE(R.nx == r->geom.nx && R.ny == r->geom.ny && R.nz == r->geom.nz &&
                         R.vx == r->geom.vx && R.vy == r->geom.vy && R.vz == r->geom.vz,
                     "request volume differs from the patient's prior volume");
        int64_t gid;
        auto git = S->geom_ids.find(key);
        if (git != S->geom_ids.end()) {
            gid = git->second;
        } else {
            cbct_geom *g = nullptr;
            const int rc = cbct_geom_create(&r->geom, &g);
            if (rc != CBCT_OK) throw Error(rc, cbct_last_error());
            gid = S->next_geom++;
            GeomHost gh;
            gh.g = g;
            gh.key = key;
            S->geoms.emplace(gid, std::move(gh));
            S->geom_ids.emplace(std::move(key), gid);
        }
        cbct_geom *g = S->geoms.at(gid).g;
        P.g = g;
        const int wrc = piccs_workspace_bytes(g, &r->params, &P.ws_bytes);
        if (wrc != CBCT_OK) throw Error(wrc, cbct_last_error());
        Job<Payload> j;
        j.patient = r->patient;
        j.geom = gid;
        j.geom_bytes = geom_table_bytes(g->d);
        j.bytes = align_up(sizeof(float) * (size_t)N) + align_up(sizeof(float) * (size_t)M) +
                  align_up(P.ws_bytes);
        j.payload = std::move(P);
        P = Payload{};
        const int rc = S->core->submit(std::move(j), S->now(), ticket);
        if (rc != CBCT_OK) {
            S->release_payload(j.payload);
            if (S->core->geometry_refs(gid) == 0 && S->core->geometry_offset(gid) == kNoBlock)
                S->forget_geometry(gid);
            set_last_error(rc == CBCT_ERR_BUSY     ? "server queue full"
                           : rc == CBCT_ERR_OOM    ? "request cannot fit in the HBM budget"
                                                   : "unknown patient");
            return rc;
        }
        S->cv.notify_one();
        return CBCT_OK;
    } catch (const std::exception &e) {
        if (S) S->release_payload(P);
        return translate(e);
    }
}

int cbct_server_poll(cbct_server *S, uint64_t ticket, float *x_host_out, cbct_result *res) {
    try {
        clear_last_error();
        CBCT_REQUIRE(S, "null argument");
        Job<Payload> j;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const int rc = S->core->take(ticket, &j);
            if (rc == CBCT_PENDING) return CBCT_PENDING;
            if (rc == CBCT_ERR_NOT_FOUND) {
                set_last_error("unknown ticket");
                return rc;
            }
        }
        Payload &P = j.payload;
        if (j.status == CBCT_OK && x_host_out)
            std::memcpy(x_host_out, P.x.p, sizeof(float) * (size_t)P.n_vox);
        if (res) {
            double *hist_out = res->report.resid_hist;
            res->status = j.status;
            res->t_submit = j.t_submit;
            res->t_admit = j.t_admit;
            res->t_done = j.t_done;
            res->report = P.report;
            res->report.resid_hist = hist_out;
            if (hist_out && j.status == CBCT_OK) {
                const double *h = (const double *)P.r.p + S->nsc;
                const int nh = P.params.n_outer * P.params.n_inner;
                for (int q = 0; q < nh; ++q) hist_out[q] = h[q];
            }
        }
        if (j.status != CBCT_OK) set_last_error(j.error);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->release_payload(P);
        }
        return j.status;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_server_footprint(const cbct_geom_desc *gd, const piccs_params *p, size_t *request_bytes,
                          size_t *tables_bytes, size_t *resident_bytes) {
    try {
        clear_last_error();
        CBCT_REQUIRE(gd && p, "null argument");
        cbct_geom *g = nullptr;
        int rc = cbct_geom_create(gd, &g);
        if (rc != CBCT_OK) return rc;
        size_t ws = 0;
        rc = piccs_workspace_bytes(g, p, &ws);
        const size_t M = (size_t)g->n_vox(), N = (size_t)g->n_proj();
        const size_t tb = geom_table_bytes(g->d);
        cbct_geom_destroy(g);
        if (rc != CBCT_OK) return rc;
        if (request_bytes)
            *request_bytes = align_up(sizeof(float) * N) + align_up(sizeof(float) * M) +
                             align_up(ws);
        if (tables_bytes) *tables_bytes = align_up(tb);
        if (resident_bytes) *resident_bytes = 2 * align_up(sizeof(float) * M);
        return CBCT_OK;
    } catch (const std::exception &e) {
        return translate(e);
    }
}

int cbct_server_stats_get(cbct_server *S, cbct_server_stats *out) {
    if (!S || !out) {
        set_last_error("null argument");
        return CBCT_ERR_INVALID;
    }
    clear_last_error();
    std::lock_guard<std::mutex> lk(S->mu);
    const serve::Stats st = S->core->stats();
    out->capacity = st.capacity;
    out->used = st.used;
    out->peak_used = st.peak_used;
    out->resident = st.resident;
    out->queued = st.queued;
    out->in_flight = st.in_flight;
    out->peak_in_flight = st.peak_in_flight;
    out->done_unpolled = st.done_unpolled;
    out->completed = st.completed;
    out->failed = st.failed;
    out->geom_placements = st.geom_placements;
    out->geom_evictions = st.geom_evictions;
    return CBCT_OK;
}

int cbct_server_destroy(cbct_server *S) {
    if (!S) return CBCT_OK;
    clear_last_error();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    int status = CBCT_OK;
    {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(S->device);
        std::lock_guard<std::mutex> lk(S->mu);
        S->core->for_each_job([&](Job<Payload> &j) { S->release_payload(j.payload); });
        for (auto &kv : S->geoms) {
            geo_unplace(kv.second.g);
            if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
            cbct_geom_destroy(kv.second.g);
        }
        S->geoms.clear();
        for (hipEvent_t e : S->free_events) (void)hipEventDestroy(e);
        for (hipStream_t s : S->streams)
            if (hipStreamSynchronize(s) != hipSuccess) status = CBCT_ERR_DEVICE;
        for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
        (void)hipStreamDestroy(S->upload);
        (void)hipFree(S->base);
        (void)hipSetDevice(prev);
    }
    S->core.reset();
    delete S;
    if (status != CBCT_OK) set_last_error("device error while draining the server");
    return status;
}

}  // extern "C"
