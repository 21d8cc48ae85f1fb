"""Host logic of the reconstruction server: arena allocator and admission.

Drives the same scheduling core as libcbct.so's server (csrc/serve_core.h)
through a host-only library whose simulated device finishes a request only
when the test says so, so every ordering and memory decision is checked
deterministically without a GPU.
"""
import ctypes
import os

import numpy as np
import pytest

# CBCT_SIM_LIB selects another build of serve_sim.cpp (the sanitizer test)
LIB = os.environ.get("CBCT_SIM_LIB") or os.path.join(os.path.dirname(__file__), "..",
                                                     "paper_2509_08574_amd", "libcbct_sim.so")

OK, PENDING, ERR_OOM, ERR_DEVICE, ERR_BUSY, ERR_NOT_FOUND = 0, 1, -2, -3, -4, -5
A = 256  # allocation granule


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libcbct_sim.so not built")
    L = ctypes.CDLL(LIB)
    vp, u64, i64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32
    L.sim_create.restype = vp
    L.sim_create.argtypes = [u64, i32, i32]
    L.sim_destroy.argtypes = [vp]
    L.sim_add_patient.restype = i64
    L.sim_add_patient.argtypes = [vp, i32, u64]
    L.sim_submit.restype = i32
    L.sim_submit.argtypes = [vp, i32, i64, u64, u64, i32, ctypes.POINTER(u64)]
    L.sim_step.restype = i32
    L.sim_step.argtypes = [vp]
    L.sim_finish.restype = i32
    L.sim_finish.argtypes = [vp, u64]
    dp = ctypes.POINTER(ctypes.c_double)
    L.sim_poll.restype = i32
    L.sim_poll.argtypes = [vp, u64, dp, dp, dp, ctypes.POINTER(i32)]
    L.sim_running.restype = i32
    L.sim_running.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(i32),
                              i32]
    L.sim_launch_order.restype = i32
    L.sim_launch_order.argtypes = [vp, ctypes.POINTER(u64), i32]
    L.sim_stats.argtypes = [vp, ctypes.POINTER(i64)]
    L.sim_geometry_state.restype = i32
    L.sim_geometry_state.argtypes = [vp, i64]
    L.arena_create.restype = vp
    L.arena_create.argtypes = [u64]
    L.arena_destroy.argtypes = [vp]
    L.arena_alloc.restype = i64
    L.arena_alloc.argtypes = [vp, u64, i32]
    L.arena_release.restype = i32
    L.arena_release.argtypes = [vp, u64]
    L.arena_info.argtypes = [vp, ctypes.POINTER(i64)]
    return L


STATS = ("capacity", "used", "peak_used", "resident", "queued", "in_flight", "peak_in_flight",
         "done_unpolled", "completed", "failed", "geom_placements", "geom_evictions")


class Sim:
    def __init__(self, L, capacity, slots=4, queue=64):
        self.L, self.h = L, L.sim_create(capacity, slots, queue)

    def close(self):
        self.L.sim_destroy(self.h)

    def patient(self, pid, nbytes):
        return self.L.sim_add_patient(self.h, pid, nbytes)

    def submit(self, pid, nbytes, geom=0, geom_bytes=A, fail=False):
        t = ctypes.c_uint64()
        rc = self.L.sim_submit(self.h, pid, geom, geom_bytes, nbytes, int(fail), ctypes.byref(t))
        return rc, t.value

    def step(self):
        return self.L.sim_step(self.h)

    def finish(self, t):
        assert self.L.sim_finish(self.h, t) == 0

    def poll(self, t):
        ts, ta, td, sl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        rc = self.L.sim_poll(self.h, t, ctypes.byref(ts), ctypes.byref(ta), ctypes.byref(td),
                             ctypes.byref(sl))
        return rc, (ts.value, ta.value, td.value, sl.value)

    def running(self):
        cap = 256
        t = (ctypes.c_uint64 * cap)()
        o = (ctypes.c_uint64 * cap)()
        s = (ctypes.c_int32 * cap)()
        n = self.L.sim_running(self.h, t, o, s, cap)
        return {t[i]: (o[i], s[i]) for i in range(n)}

    def order(self):
        out = (ctypes.c_uint64 * 4096)()
        n = self.L.sim_launch_order(self.h, out, 4096)
        return list(out[:n])

    def stats(self):
        v = (ctypes.c_int64 * 12)()
        self.L.sim_stats(self.h, v)
        return dict(zip(STATS, list(v)))

    def geom_state(self, key):
        return self.L.sim_geometry_state(self.h, key)


@pytest.fixture
def sim(lib):
    made = []

    def make(capacity, slots=4, queue=64):
        s = Sim(lib, capacity, slots, queue)
        made.append(s)
        return s
    yield make
    for s in made:
        s.close()


# ---------------------------------------------------------------- arena

class Arena:
    def __init__(self, L, cap):
        self.L, self.h = L, L.arena_create(cap)

    def alloc(self, n, high=False):
        return self.L.arena_alloc(self.h, n, int(high))

    def release(self, off):
        return self.L.arena_release(self.h, off)

    def info(self):
        v = (ctypes.c_int64 * 5)()
        self.L.arena_info(self.h, v)
        return dict(zip(("capacity", "used", "live", "free_blocks", "largest"), list(v)))

    def close(self):
        self.L.arena_destroy(self.h)


def test_arena_low_high_and_coalescing(lib):
    a = Arena(lib, 100 * A + 17)
    assert a.info()["capacity"] == 100 * A          # rounded down to the granule
    assert a.alloc(1) == 0                          # rounded up to one granule
    assert a.alloc(A + 1) == A                      # two granules, next to it
    top = a.alloc(10 * A, high=True)
    assert top == 90 * A                            # carved from the top end
    assert a.info()["used"] == 13 * A
    assert a.alloc(88 * A) == -1                    # only 87 granules left
    mid = a.alloc(87 * A)
    assert mid == 3 * A
    assert a.info()["largest"] == 0
    for off in (A, 0, mid, top):
        assert a.release(off) == 0
    inf = a.info()
    assert inf["used"] == 0 and inf["live"] == 0 and inf["free_blocks"] == 1
    assert inf["largest"] == 100 * A
    assert a.release(0) == -1                       # not live
    a.close()


def test_arena_random_against_model(lib):
    """Random alloc/release: blocks disjoint, inside the arena, accounting exact,
    everything coalesces back to one block."""
    rng = np.random.default_rng(3)
    cap = 4096 * A
    a = Arena(lib, cap)
    live = {}
    for it in range(3000):
        if live and (rng.uniform() < 0.45 or len(live) > 60):
            off = list(live)[rng.integers(len(live))]
            assert a.release(off) == 0
            del live[off]
        else:
            n = int(rng.integers(1, 200 * A))
            off = a.alloc(n, high=bool(rng.uniform() < 0.3))
            size = -(-n // A) * A
            if off < 0:
                # refused only if no free gap is large enough
                assert a.info()["largest"] < size
                continue
            assert off % A == 0 and off + size <= cap
            for o, s in live.items():
                assert off + size <= o or o + s <= off, "overlapping blocks"
            live[off] = size
        assert a.info()["used"] == sum(live.values())
    for off in list(live):
        assert a.release(off) == 0
    inf = a.info()
    assert inf["free_blocks"] == 1 and inf["largest"] == cap
    a.close()


# ---------------------------------------------------------------- admission

def test_admission_by_footprint(sim):
    s = sim(capacity=100 * A, slots=8)
    for p in (1, 2, 3):
        assert s.patient(p, 10 * A) >= 0          # residents: 30 granules at the top
    ok = [s.submit(p, 30 * A) for p in (1, 2, 3)]
    assert all(rc == OK for rc, _ in ok)
    t = [tk for _, tk in ok]
    assert s.step() == 2                          # 2 x 30 fit beside 30 resident, 3 do not
    assert set(s.running()) == {t[0], t[1]}
    st = s.stats()
    # two blocks, residents and one granule of cached geometry tables
    assert st["used"] == 91 * A and st["queued"] == 1 and st["in_flight"] == 2
    s.finish(t[0])
    assert s.step() == 1                          # retired, then the third admitted
    assert set(s.running()) == {t[1], t[2]}
    assert s.poll(t[0])[0] == OK
    s.finish(t[1])
    s.finish(t[2])
    s.step()
    st = s.stats()
    assert st["peak_used"] <= st["capacity"] and st["peak_in_flight"] == 2
    assert st["resident"] == 30 * A and st["used"] == 31 * A and st["completed"] == 3


def test_slot_limit(sim):
    s = sim(capacity=1000 * A, slots=2)
    for p in range(5):
        s.patient(p, A)
    tk = [s.submit(p, A)[1] for p in range(5)]
    s.step()
    assert set(s.running()) == set(tk[:2])
    slots = {sl for _, sl in s.running().values()}
    assert slots == {0, 1}
    s.finish(tk[0])
    s.step()
    assert set(s.running()) == {tk[1], tk[2]}


def test_patient_requests_run_in_order_one_at_a_time(sim):
    s = sim(capacity=1000 * A, slots=4)
    s.patient(7, A)
    s.patient(8, A)
    a1, a2, a3 = (s.submit(7, A)[1] for _ in range(3))
    b1 = s.submit(8, A)[1]
    s.step()
    # patient 7's later requests wait; patient 8's passes them
    assert set(s.running()) == {a1, b1}
    s.finish(a1)
    s.step()
    assert set(s.running()) == {a2, b1}
    s.finish(a2)
    s.finish(b1)
    s.step()
    assert set(s.running()) == {a3}
    assert s.order() == [a1, b1, a2, a3]


def test_fifo_no_bypass_on_memory(sim):
    """A request waiting for memory is not overtaken by smaller later ones."""
    s = sim(capacity=100 * A, slots=8)
    for p in (1, 2, 3):
        s.patient(p, A)
    t1 = s.submit(1, 60 * A)[1]
    t2 = s.submit(2, 60 * A)[1]       # needs t1's memory
    t3 = s.submit(3, 5 * A)[1]        # would fit now, but is behind t2
    s.step()
    assert set(s.running()) == {t1}
    s.finish(t1)
    s.step()
    assert set(s.running()) == {t2, t3}


def test_refusals_and_pending(sim):
    s = sim(capacity=100 * A, slots=2, queue=2)
    s.patient(1, 40 * A)
    assert s.submit(1, 61 * A)[0] == ERR_OOM        # never fits beside the resident
    assert s.submit(9, A)[0] == ERR_NOT_FOUND       # unknown patient
    t1 = s.submit(1, A)[1]
    t2 = s.submit(1, A)[1]
    assert s.submit(1, A)[0] == ERR_BUSY            # two waiting already
    assert s.poll(t1)[0] == PENDING                 # queued
    s.step()
    assert s.poll(t1)[0] == PENDING                 # running
    assert s.submit(1, A)[0] == OK                  # t1 left the queue
    assert s.poll(12345)[0] == ERR_NOT_FOUND
    s.finish(t1)
    s.step()
    rc, (ts, ta, td, slot) = s.poll(t1)
    assert rc == OK and ts <= ta <= td and slot in (0, 1)
    assert s.poll(t1)[0] == ERR_NOT_FOUND           # collected once
    assert t2 > t1


def test_request_that_stops_fitting_fails_with_oom(sim):
    s = sim(capacity=100 * A, slots=2)
    s.patient(1, 10 * A)
    s.patient(2, 10 * A)
    t1 = s.submit(1, 40 * A)[1]
    t2 = s.submit(2, 70 * A)[1]     # fits when alone, waits for t1's memory
    s.step()
    assert set(s.running()) == {t1}
    assert s.patient(3, 15 * A) >= 0   # residents now 35: 70 no longer fits when idle
    s.finish(t1)
    s.step()
    assert s.poll(t1)[0] == OK
    assert s.poll(t2)[0] == ERR_OOM
    assert s.stats()["failed"] == 1


def test_geometry_tables_cached_and_evicted(sim):
    s = sim(capacity=100 * A, slots=4)
    s.patient(1, 10 * A)
    s.patient(2, 10 * A)
    t1 = s.submit(1, 20 * A, geom=5, geom_bytes=20 * A)[1]
    s.step()
    s.finish(t1)
    s.step()
    assert s.geom_state(5) == 1                 # cached after its request finished
    t2 = s.submit(2, 20 * A, geom=5, geom_bytes=20 * A)[1]
    s.step()
    assert s.stats()["geom_placements"] == 1    # reused, not placed again
    s.finish(t2)
    s.step()
    # a new geometry that only fits if the idle one goes
    t3 = s.submit(1, 45 * A, geom=6, geom_bytes=25 * A)[1]   # 70 > 60 free
    s.step()
    assert t3 in s.running()
    st = s.stats()
    assert st["geom_evictions"] == 1 and st["geom_placements"] == 2
    assert s.geom_state(5) == 2                 # dropped and no request refers to it
    assert s.geom_state(6) == 1


def test_geometry_in_use_is_never_evicted(sim):
    s = sim(capacity=100 * A, slots=4)
    s.patient(1, 5 * A)
    s.patient(2, 5 * A)
    t1 = s.submit(1, 20 * A, geom=1, geom_bytes=30 * A)[1]
    t2 = s.submit(2, 35 * A, geom=2, geom_bytes=30 * A)[1]   # needs geometry 1's memory
    s.step()
    assert set(s.running()) == {t1}
    assert s.geom_state(1) == 1 and s.stats()["geom_evictions"] == 0
    s.finish(t1)
    s.step()
    assert set(s.running()) == {t2}
    assert s.stats()["geom_evictions"] == 1


def test_failed_launch_reports_device_error_and_frees(sim):
    s = sim(capacity=100 * A, slots=2)
    s.patient(1, A)
    t1 = s.submit(1, 50 * A, fail=True)[1]
    s.step()
    s.step()
    rc, _ = s.poll(t1)
    assert rc == ERR_DEVICE
    st = s.stats()
    assert st["used"] == st["resident"] + A and st["failed"] == 1


def test_random_stream_invariants(sim):
    """Random arrivals and completions: memory never over budget, running
    blocks disjoint, each patient's requests launched in submission order,
    every request finishes."""
    rng = np.random.default_rng(11)
    cap = 2000 * A
    s = sim(capacity=cap, slots=5, queue=1000)
    for p in range(8):
        s.patient(p, int(rng.integers(10, 60)) * A)
    submitted = {}
    outcome = {}
    for it in range(1500):
        if rng.uniform() < 0.35 and len(submitted) < 600:
            p = int(rng.integers(8))
            nb = int(rng.integers(1, 700)) * A
            g = int(rng.integers(6))
            rc, t = s.submit(p, nb, geom=g, geom_bytes=(g + 1) * 40 * A)
            if rc == OK:
                submitted[t] = p
            else:
                assert rc in (ERR_OOM, ERR_BUSY)
        run = s.running()
        if run and rng.uniform() < 0.5:
            s.finish(list(run)[rng.integers(len(run))])
        s.step()
        st = s.stats()
        assert st["used"] <= cap
        blocks = sorted((o, t) for t, (o, _) in s.running().items())
        for t in submitted:
            r = s.poll(t)
            if r[0] != PENDING and t not in outcome:
                outcome[t] = r[0]
        assert len(blocks) <= 5
    while len(outcome) < len(submitted):
        for t in list(s.running()):
            s.finish(t)
        s.step()
        for t in submitted:
            if t not in outcome:
                r = s.poll(t)
                if r[0] != PENDING:
                    outcome[t] = r[0]
    assert set(outcome.values()) <= {OK, ERR_OOM}
    order = s.order()
    for p in range(8):
        mine = [t for t in order if submitted.get(t) == p]
        assert mine == sorted(mine)
    st = s.stats()
    assert st["in_flight"] == 0 and st["queued"] == 0 and st["peak_used"] <= cap
