// Host-only driver of the server's scheduling core with a simulated device,
// for testing admission, residency and ordering without a GPU.  Built with
// the host compiler into libcbct_sim.so; not part of libcbct.so.
//
// The simulated device finishes a request only when the caller says so
// (sim_finish); time is a step counter advanced by every sim_step.
#include <cstdint>
#include <cstring>
#include <set>
#include <stdexcept>
#include <vector>

#include "serve_core.h"

namespace {

using cbct::serve::Job;
using cbct::serve::Scheduler;

struct SimPayload {
    bool done = false;       // set by sim_finish
    bool fail_launch = false;
};

struct Sim;

struct SimBackend {
    Sim *sim;
    double now();
    void place_geometry(int64_t key, size_t off, int slot);
    void drop_geometry(int64_t key, bool unused);
    void launch(Job<SimPayload> &j);
    bool finished(Job<SimPayload> &j) { return j.payload.done || j.status != CBCT_PENDING; }
    void collect(Job<SimPayload> &j) {
        if (j.status == CBCT_PENDING) j.status = CBCT_OK;
    }
    void discard(Job<SimPayload> &) {}
};

struct Sim {
    Scheduler<SimPayload> core;
    SimBackend be;
    double clock = 0;
    std::vector<uint64_t> launch_order;
    std::set<int64_t> placed;      // geometry keys with device tables
    std::set<int64_t> forgotten;   // keys dropped with unused = true
    std::set<uint64_t> fail_next;  // tickets whose launch throws
    int64_t fails_pending = 0;
    Sim(size_t cap, int slots, int q) : core(cap, slots, q), be{this} {}
};

double SimBackend::now() { return sim->clock; }
void SimBackend::place_geometry(int64_t key, size_t, int) {
    if (sim->placed.count(key)) throw std::logic_error("geometry placed twice");
    sim->placed.insert(key);
}
void SimBackend::drop_geometry(int64_t key, bool unused) {
    sim->placed.erase(key);
    if (unused) sim->forgotten.insert(key);
}
void SimBackend::launch(Job<SimPayload> &j) {
    if (!sim->placed.count(j.geom)) throw std::logic_error("launch without geometry tables");
    sim->launch_order.push_back(j.ticket);
    if (j.payload.fail_launch) throw std::runtime_error("simulated launch failure");
}

}  // namespace

extern "C" {

void *sim_create(uint64_t capacity, int32_t max_slots, int32_t max_queue) {
    return new Sim((size_t)capacity, max_slots, max_queue);
}
void sim_destroy(void *h) { delete (Sim *)h; }

// Returns the arena offset of the patient's resident block, or -1.
int64_t sim_add_patient(void *h, int32_t id, uint64_t bytes) {
    Sim *s = (Sim *)h;
    const size_t off = s->core.add_patient(id, (size_t)bytes);
    return off == cbct::serve::kNoBlock ? -1 : (int64_t)off;
}

int32_t sim_submit(void *h, int32_t patient, int64_t geom, uint64_t geom_bytes, uint64_t bytes,
                   int32_t fail_launch, uint64_t *ticket) {
    Sim *s = (Sim *)h;
    Job<SimPayload> j;
    j.patient = patient;
    j.geom = geom;
    j.geom_bytes = (size_t)geom_bytes;
    j.bytes = (size_t)bytes;
    j.payload.fail_launch = fail_launch != 0;
    return s->core.submit(std::move(j), s->clock, ticket);
}

// Advances the clock by one, completes finished jobs and admits; returns the
// number admitted.
int32_t sim_step(void *h) {
    Sim *s = (Sim *)h;
    s->clock += 1.0;
    return s->core.step(s->be);
}

// Marks a running job finished on the simulated device; -1 if not running.
int32_t sim_finish(void *h, uint64_t ticket) {
    Sim *s = (Sim *)h;
    int32_t rc = -1;
    s->core.for_each_job([&](Job<SimPayload> &j) {
        if (j.ticket == ticket && j.t_admit >= 0 && j.t_done < 0) {
            j.payload.done = true;
            rc = 0;
        }
    });
    return rc;
}

// Status of a ticket: CBCT_PENDING, CBCT_ERR_NOT_FOUND, or the finished
// job's status (the job is removed).  Fills times, slot and arena offset.
int32_t sim_poll(void *h, uint64_t ticket, double *t_submit, double *t_admit, double *t_done,
                 int32_t *slot) {
    Sim *s = (Sim *)h;
    Job<SimPayload> j;
    const int rc = s->core.take(ticket, &j);
    if (rc != CBCT_OK) return rc;
    if (t_submit) *t_submit = j.t_submit;
    if (t_admit) *t_admit = j.t_admit;
    if (t_done) *t_done = j.t_done;
    if (slot) *slot = j.slot;
    return j.status;
}

// Running tickets with their arena offsets, slots and sizes; returns count.
int32_t sim_running(void *h, uint64_t *tickets, uint64_t *offs, int32_t *slots, int32_t cap) {
    Sim *s = (Sim *)h;
    int32_t n = 0;
    s->core.for_each_job([&](Job<SimPayload> &j) {
        if (j.t_admit >= 0 && j.t_done < 0) {
            if (n < cap) {
                tickets[n] = j.ticket;
                offs[n] = (uint64_t)j.off;
                slots[n] = j.slot;
            }
            ++n;
        }
    });
    return n;
}

// Launch order so far; returns count.
int32_t sim_launch_order(void *h, uint64_t *out, int32_t cap) {
    Sim *s = (Sim *)h;
    const int32_t n = (int32_t)s->launch_order.size();
    for (int32_t i = 0; i < n && i < cap; ++i) out[i] = s->launch_order[(size_t)i];
    return n;
}

// out[0..11] = capacity, used, peak_used, resident, queued, in_flight,
// peak_in_flight, done_unpolled, completed, failed, geom_placements,
// geom_evictions.
void sim_stats(void *h, int64_t *out) {
    const cbct::serve::Stats st = ((Sim *)h)->core.stats();
    const int64_t v[12] = {st.capacity, st.used, st.peak_used, st.resident,
                           st.queued, st.in_flight, st.peak_in_flight, st.done_unpolled,
                           st.completed, st.failed, st.geom_placements, st.geom_evictions};
    std::memcpy(out, v, sizeof(v));
}

// 1 if the geometry key has device tables in the simulation, 2 if it was
// dropped as unused, 0 otherwise.
int32_t sim_geometry_state(void *h, int64_t key) {
    Sim *s = (Sim *)h;
    if (s->placed.count(key)) return 1;
    return s->forgotten.count(key) ? 2 : 0;
}

// ---- the arena on its own
void *arena_create(uint64_t cap) { return new cbct::serve::Arena((size_t)cap); }
void arena_destroy(void *a) { delete (cbct::serve::Arena *)a; }
int64_t arena_alloc(void *a, uint64_t bytes, int32_t high) {
    auto *A = (cbct::serve::Arena *)a;
    const size_t off = high ? A->alloc_high((size_t)bytes) : A->alloc_low((size_t)bytes);
    return off == cbct::serve::kNoBlock ? -1 : (int64_t)off;
}
int32_t arena_release(void *a, uint64_t off) {
    return ((cbct::serve::Arena *)a)->release((size_t)off) ? 0 : -1;
}
// out = capacity, used, live blocks, free blocks, largest free
void arena_info(void *a, int64_t *out) {
    auto *A = (cbct::serve::Arena *)a;
    out[0] = (int64_t)A->capacity();
    out[1] = (int64_t)A->used();
    out[2] = (int64_t)A->live_blocks();
    out[3] = (int64_t)A->free_blocks();
    out[4] = (int64_t)A->largest_free();
}

}  // extern "C"
