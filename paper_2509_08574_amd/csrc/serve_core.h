// Host-only scheduling core of the reconstruction server (no HIP dependency).
//
// The server keeps everything it places on the device inside one arena of
// `capacity` bytes (the HBM budget):
//   * per patient, resident for the server's lifetime: the prior x_p and the
//     previous reconstruction x_prev (carved from the top of the arena);
//   * per geometry, cached while idle and evicted least-recently-used when
//     memory is short: the projector tables (also from the top);
//   * per admitted request, released when its work has finished: b, x and the
//     solver workspace (first fit from the bottom).
//
// Admission (continuous batching): requests wait in arrival order; the first
// waiting request whose patient has no request on the device is admitted as
// soon as a stream slot is free and its block fits.  A request that does not
// fit blocks the ones behind it (no starvation of large requests); one that
// could not fit even with nothing else on the device fails with
// CBCT_ERR_OOM.  Requests of one patient run one at a time in arrival order
// (each may start from the previous one's result).
//
// Scheduler<P> is driven from one thread under the caller's lock; the
// backend supplies the clock, launches work and reports completion.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <limits>
#include <map>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/cbct.h"

namespace cbct {
namespace serve {

constexpr size_t kAlign = 256;
constexpr size_t kNoBlock = std::numeric_limits<size_t>::max();
inline size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Offsets into [0, capacity) in kAlign granules; free blocks are coalesced.
class Arena {
   public:
    explicit Arena(size_t capacity) : cap_(capacity / kAlign * kAlign) {
        if (cap_) free_[0] = cap_;
    }

    // Lowest-addressed free block that fits (transient request blocks).
    size_t alloc_low(size_t bytes) {
        const size_t n = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[off + n] = sz - n;
            take(off, n);
            return off;
        }
        return kNoBlock;
    }

    // Highest-addressed free block that fits, carved from its top end
    // (long-lived residents gather at the top, away from request blocks).
    size_t alloc_high(size_t bytes) {
        const size_t n = align_up(bytes ? bytes : 1);
        for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(std::next(it).base());
            if (sz > n) free_[off] = sz - n;
            take(off + sz - n, n);
            return off + sz - n;
        }
        return kNoBlock;
    }

    // Returns a block obtained from alloc_low / alloc_high; false if unknown.
    bool release(size_t off) {
        auto it = live_.find(off);
        if (it == live_.end()) return false;
        size_t o = off, n = it->second;
        live_.erase(it);
        used_ -= n;
        auto nx = free_.lower_bound(o);
        if (nx != free_.end() && nx->first == o + n) {
            n += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == o) {
                o = pv->first;
                n += pv->second;
                free_.erase(pv);
            }
        }
        free_[o] = n;
        return true;
    }

    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t live_blocks() const { return live_.size(); }
    size_t free_blocks() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t block_size(size_t off) const {
        auto it = live_.find(off);
        return it == live_.end() ? 0 : it->second;
    }

   private:
    void take(size_t off, size_t n) {
        live_[off] = n;
        used_ += n;
    }
    size_t cap_, used_ = 0;
    std::map<size_t, size_t> free_;             // offset -> size
    std::unordered_map<size_t, size_t> live_;   // offset -> size
};

template <class P>
struct Job {
    uint64_t ticket = 0;
    int32_t patient = 0;
    int64_t geom = -1;        // geometry key (backend-defined)
    size_t bytes = 0;         // transient block: inputs, output, workspace
    size_t geom_bytes = 0;    // device tables of the geometry
    double t_submit = 0, t_admit = -1, t_done = -1;
    int status = CBCT_PENDING;
    std::string error;
    size_t off = kNoBlock;    // transient block while on the device
    int slot = -1;
    P payload{};
};

struct Stats {
    int64_t capacity = 0, used = 0, peak_used = 0, resident = 0;
    int64_t queued = 0, in_flight = 0, peak_in_flight = 0, done_unpolled = 0;
    int64_t completed = 0, failed = 0, geom_placements = 0, geom_evictions = 0;
};

// Backend interface: B must provide
//   double now();
//   void place_geometry(int64_t key, size_t off, int slot);   // may throw
//   void drop_geometry(int64_t key, bool unused);  // forget the device tables;
//                                  // unused: no request refers to the key any more
//   void launch(Job<P> &j);                                    // may throw
//   bool finished(Job<P> &j);                                  // non-blocking
//   void collect(Job<P> &j);     // results; sets j.status to CBCT_OK or an error
//                                // unless it is already an error (failed launch)
//   void discard(Job<P> &j);     // job leaves the scheduler without launch
template <class P>
class Scheduler {
   public:
    Scheduler(size_t capacity, int max_slots, int max_queue)
        : arena_(capacity), max_queue_(max_queue) {
        for (int i = max_slots - 1; i >= 0; --i) free_slots_.push_back(i);
        st_.capacity = (int64_t)arena_.capacity();
    }

    Arena &arena() { return arena_; }
    const Arena &arena() const { return arena_; }

    // Registers a patient with `bytes` of resident device memory; returns the
    // arena offset, or kNoBlock when it does not fit.
    size_t add_patient(int32_t id, size_t bytes) {
        if (patients_.count(id)) return kNoBlock;
        const size_t off = arena_.alloc_high(bytes);
        if (off == kNoBlock) return kNoBlock;
        patients_[id] = Patient{off, arena_.block_size(off), false};
        resident_ += arena_.block_size(off);
        update_peaks();
        return off;
    }
    bool has_patient(int32_t id) const { return patients_.count(id) != 0; }
    size_t patient_offset(int32_t id) const {
        auto it = patients_.find(id);
        return it == patients_.end() ? kNoBlock : it->second.off;
    }

    // Takes ownership of j (ticket assigned here).  Returns CBCT_OK,
    // CBCT_ERR_BUSY (queue full), CBCT_ERR_NOT_FOUND (unknown patient) or
    // CBCT_ERR_OOM (the request can never fit beside the residents).
    int submit(Job<P> &&j, double now, uint64_t *ticket) {
        if (!patients_.count(j.patient)) return CBCT_ERR_NOT_FOUND;
        if ((int64_t)queue_.size() >= max_queue_) return CBCT_ERR_BUSY;
        if (never_fits(j)) return CBCT_ERR_OOM;
        j.ticket = next_ticket_++;
        j.t_submit = now;
        j.status = CBCT_PENDING;
        *ticket = j.ticket;
        const uint64_t t = j.ticket;
        geom_refs_[j.geom] += 1;
        queue_.push_back(t);
        jobs_.emplace(t, std::move(j));
        return CBCT_OK;
    }

    // Completes finished work, then admits what fits.  Returns the number of
    // requests admitted.
    template <class B>
    int step(B &be) {
        reap(be);
        return admit(be);
    }

    template <class B>
    void reap(B &be) {
        for (size_t q = 0; q < running_.size();) {
            Job<P> &j = jobs_.at(running_[q]);
            if (!be.finished(j)) {
                ++q;
                continue;
            }
            be.collect(j);
            j.t_done = be.now();
            finish_device_side(j);
            if (j.status == CBCT_OK) st_.completed++;
            else st_.failed++;
            running_.erase(running_.begin() + (std::ptrdiff_t)q);
        }
    }

    template <class B>
    int admit(B &be) {
        int n = 0;
        for (size_t q = 0; q < queue_.size();) {
            Job<P> &j = jobs_.at(queue_[q]);
            Patient &pt = patients_.at(j.patient);
            if (pt.busy) {  // an earlier request of this patient is on the device
                ++q;
                continue;
            }
            if (free_slots_.empty()) break;
            if (never_fits(j)) {
                fail_queued(be, q, CBCT_ERR_OOM, "request does not fit in the HBM budget");
                continue;
            }
            GeomRes &gr = geoms_[j.geom];
            size_t goff = kNoBlock, off = kNoBlock;
            for (;;) {
                // both blocks are placed afresh after every eviction so that
                // the freed space is used as a whole
                if (gr.off == kNoBlock) goff = arena_.alloc_high(j.geom_bytes);
                if (gr.off != kNoBlock || goff != kNoBlock) off = arena_.alloc_low(j.bytes);
                if (off != kNoBlock) break;
                if (goff != kNoBlock) arena_.release(goff);
                goff = kNoBlock;
                if (!evict_one_idle_geometry(be, j.geom)) break;
            }
            if (off == kNoBlock) {
                if (running_.empty()) {  // nothing left to wait for
                    fail_queued(be, q, CBCT_ERR_OOM,
                                "request does not fit in the free HBM budget");
                    continue;
                }
                break;  // wait for memory; later requests do not pass this one
            }
            j.off = off;
            j.slot = free_slots_.back();
            free_slots_.pop_back();
            j.t_admit = be.now();
            pt.busy = true;
            gr.running++;
            gr.last_use = ++use_clock_;
            queue_.erase(queue_.begin() + (std::ptrdiff_t)q);
            running_.push_back(j.ticket);
            bool ok = true;
            try {
                if (goff != kNoBlock) {
                    gr.off = goff;
                    st_.geom_placements++;
                    be.place_geometry(j.geom, goff, j.slot);
                }
                be.launch(j);
            } catch (const std::exception &e) {
                ok = false;
                j.error = e.what();
            }
            // A failed launch stays "running" until the backend reports the
            // part that did reach the device finished, so its block is not
            // reused under it.
            if (!ok) j.status = CBCT_ERR_DEVICE;
            ++n;
            update_peaks();
        }
        return n;
    }

    // CBCT_PENDING while queued or running, CBCT_ERR_NOT_FOUND if unknown;
    // otherwise moves the finished job into *out and returns CBCT_OK.
    int take(uint64_t ticket, Job<P> *out) {
        auto it = jobs_.find(ticket);
        if (it == jobs_.end()) return CBCT_ERR_NOT_FOUND;
        if (it->second.t_done < 0) return CBCT_PENDING;
        *out = std::move(it->second);
        jobs_.erase(it);
        return CBCT_OK;
    }

    bool idle() const { return queue_.empty() && running_.empty(); }
    size_t in_flight() const { return running_.size(); }
    size_t queued() const { return queue_.size(); }

    // Jobs finished but never taken (for teardown).
    template <class F>
    void for_each_job(F f) {
        for (auto &kv : jobs_) f(kv.second);
    }

    // Drops every idle geometry from the device (for teardown).
    template <class B>
    void evict_all_idle(B &be) {
        while (evict_one_idle_geometry(be, -2)) {
        }
    }

    Stats stats() const {
        Stats s = st_;
        s.used = (int64_t)arena_.used();
        s.resident = (int64_t)resident_;
        s.queued = (int64_t)queue_.size();
        s.in_flight = (int64_t)running_.size();
        int64_t d = 0;
        for (auto &kv : jobs_) d += kv.second.t_done >= 0;
        s.done_unpolled = d;
        return s;
    }

    // Arena offset of a placed geometry (kNoBlock if not on the device).
    size_t geometry_offset(int64_t key) const {
        auto it = geoms_.find(key);
        return it == geoms_.end() ? kNoBlock : it->second.off;
    }
    // Queued + running requests that use the geometry.
    int geometry_refs(int64_t key) const {
        auto it = geom_refs_.find(key);
        return it == geom_refs_.end() ? 0 : it->second;
    }

   private:
    struct Patient {
        size_t off;
        size_t bytes;
        bool busy;
    };
    struct GeomRes {
        size_t off = kNoBlock;
        int running = 0;
        uint64_t last_use = 0;
    };

    bool never_fits(const Job<P> &j) const {
        const size_t need = align_up(j.bytes ? j.bytes : 1) +
                            (geometry_offset(j.geom) == kNoBlock ? align_up(j.geom_bytes) : 0);
        return need > arena_.capacity() - resident_;
    }

    template <class B>
    bool evict_one_idle_geometry(B &be, int64_t keep) {
        int64_t best = -1;
        uint64_t best_use = 0;
        bool found = false;
        for (auto &kv : geoms_) {
            if (kv.first == keep || kv.second.off == kNoBlock || kv.second.running) continue;
            if (!found || kv.second.last_use < best_use) {
                best = kv.first;
                best_use = kv.second.last_use;
                found = true;
            }
        }
        if (!found) return false;
        GeomRes &gr = geoms_[best];
        arena_.release(gr.off);
        gr.off = kNoBlock;
        st_.geom_evictions++;
        const bool unused = geom_refs_[best] == 0;
        if (unused) {
            geoms_.erase(best);
            geom_refs_.erase(best);
        }
        be.drop_geometry(best, unused);
        return true;
    }

    void finish_device_side(Job<P> &j) {
        if (j.off != kNoBlock) arena_.release(j.off);
        j.off = kNoBlock;
        free_slots_.push_back(j.slot);
        patients_.at(j.patient).busy = false;
        GeomRes &gr = geoms_[j.geom];
        gr.running--;
        geom_refs_[j.geom] -= 1;
    }

    template <class B>
    void fail_queued(B &be, size_t q, int status, const char *msg) {
        Job<P> &j = jobs_.at(queue_[q]);
        j.status = status;
        j.error = msg;
        j.t_done = be.now();
        const int64_t key = j.geom;
        be.discard(j);
        st_.failed++;
        queue_.erase(queue_.begin() + (std::ptrdiff_t)q);
        if (--geom_refs_[key] == 0 && geometry_offset(key) == kNoBlock) {
            geoms_.erase(key);
            geom_refs_.erase(key);
            be.drop_geometry(key, true);
        }
    }

    void update_peaks() {
        if ((int64_t)arena_.used() > st_.peak_used) st_.peak_used = (int64_t)arena_.used();
        if ((int64_t)running_.size() > st_.peak_in_flight)
            st_.peak_in_flight = (int64_t)running_.size();
    }

    Arena arena_;
    int64_t max_queue_;
    size_t resident_ = 0;
    uint64_t next_ticket_ = 1, use_clock_ = 0;
    std::deque<uint64_t> queue_;
    std::vector<uint64_t> running_;
    std::vector<int> free_slots_;
    std::unordered_map<uint64_t, Job<P>> jobs_;
    std::map<int32_t, Patient> patients_;
    std::map<int64_t, GeomRes> geoms_;
    std::map<int64_t, int> geom_refs_;
    Stats st_;
};

}  // namespace serve
}  // namespace cbct
