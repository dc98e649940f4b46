"""Host logic of the continuous-batching request loop, with a fake backend
that records what the scheduler asks of the device."""
import threading
import time

import numpy as np
import pytest

from paper_2403_05463_amd import serving as S


class FakeBackend(S.Backend):
    def __init__(self, max_members, step_time=0.0005, setup_time=0.002):
        self.max_members = max_members
        self.step_time, self.setup_time = step_time, setup_time
        self.slots = {}
        self.live_bytes = 0
        self.peak_live = 0
        self.max_slots = 0
        self.calls = []
        self.lock = threading.Lock()

    def setup(self, r):
        time.sleep(self.setup_time)
        r.nodes = r.n ** 3 * (r.P + 1) ** 3
        with self.lock:
            self.live_bytes += r.est_bytes
            self.peak_live = max(self.peak_live, self.live_bytes)
        return r

    def join(self, r):
        free = [s for s in range(self.max_members) if s not in self.slots]
        assert free, "scheduler joined more members than slots"
        self.slots[free[0]] = r
        self.max_slots = max(self.max_slots, len(self.slots))
        return free[0]

    def step(self, k):
        assert k >= 1
        self.calls.append((k, sorted(r.rid for r in self.slots.values())))
        time.sleep(self.step_time)

    def leave(self, slot, r):
        del self.slots[slot]
        with self.lock:
            self.live_bytes -= r.est_bytes
        return True


def test_request_stream_shape():
    reqs = S.make_requests(256, rate=20.0, seed=0)
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert abs(arr[-1] / 256 - 1 / 20.0) < 0.02          # mean inter-arrival ~ 1/rate
    assert {r.n for r in reqs} <= set(range(4, 25)) and {r.P for r in reqs} <= set(range(2, 7))
    assert all(0.2 <= r.frac <= 0.8 and 1e-4 <= r.nu <= 1e-2 and r.nsteps == 50 for r in reqs)
    assert S.make_requests(8, seed=3)[5].n == S.make_requests(8, seed=3)[5].n


def test_footprint_grows_with_size():
    assert S.footprint_bytes(4, 2) < S.footprint_bytes(8, 2) < S.footprint_bytes(8, 6)
    # the biggest request (24^3 elements, P = 6) stays around a gigabyte
    assert 0.5e9 < S.footprint_bytes(24, 6) < 2e9


@pytest.mark.parametrize("realtime", [False, True])
def test_admission_respects_budget_slots_and_order(realtime):
    reqs = S.make_requests(40, rate=400.0, seed=1, n_range=(3, 8), p_range=(1, 4), nsteps=7)
    budget = 3 * max(S.footprint_bytes(r.n, r.P) for r in reqs)
    be = FakeBackend(max_members=5)
    st = S.serve(reqs, be, mem_budget=budget, max_members=5, max_steps_per_call=3, realtime=realtime)
    assert len(st.requests) == 40
    assert all(r.steps_done == r.nsteps for r in st.requests)
    assert be.peak_live <= budget and st.peak_bytes <= budget
    assert be.max_slots <= 5
    by_arrival = sorted(st.requests, key=lambda r: r.arrival)
    adm = [r.t_admit for r in by_arrival]
    assert all(a <= b for a, b in zip(adm, adm[1:]))                 # first come, first admitted
    assert all(r.arrival <= r.t_admit <= r.t_join <= r.t_done for r in st.requests) if realtime else True
    # no call advances a member past its requested steps
    per = {}
    for k, members in be.calls:
        for rid in members:
            per[rid] = per.get(rid, 0) + k
    assert all(per[r.rid] == r.nsteps for r in st.requests)


def test_continuous_batching_refills_slots():
    """Requests join while others are still being stepped: the batch
    composition changes between calls, not only when it drains."""
    reqs = S.make_requests(30, rate=1e4, seed=2, n_range=(3, 5), p_range=(1, 3), nsteps=9)
    for i, r in enumerate(reqs):
        r.nsteps = 3 + 2 * (i % 5)
    be = FakeBackend(max_members=4)
    st = S.serve(reqs, be, mem_budget=10 ** 12, max_members=4, max_steps_per_call=4, realtime=False)
    overl = sum(1 for a in st.requests for b in st.requests
                if a.rid != b.rid and a.t_join < b.t_join < a.t_done)
    assert overl > 0
    comps = [tuple(m) for _, m in be.calls]
    changes = sum(1 for x, y in zip(comps, comps[1:]) if x != y and set(x) & set(y))
    assert changes > 0                    # some members stayed while others left or joined
    s = st.summary()
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


@pytest.mark.parametrize("realtime", [False, True])
def test_oversized_request_is_refused_alone(realtime):
    """A request larger than the whole budget is refused on its own; the
    requests before and after it are served."""
    reqs = S.make_requests(12, rate=500.0, seed=4, n_range=(3, 5), p_range=(1, 3), nsteps=5)
    big = reqs[5]
    big.n, big.P = 40, 7
    budget = 4 * max(S.footprint_bytes(r.n, r.P) for r in reqs if r is not big)
    assert S.footprint_bytes(big.n, big.P) > budget
    be = FakeBackend(max_members=3)
    st = S.serve(reqs, be, mem_budget=budget, max_members=3, max_steps_per_call=2, realtime=realtime)
    assert [r.rid for r in st.refused] == [big.rid] and "budget" in big.refused
    assert sorted(r.rid for r in st.requests) == sorted(r.rid for r in reqs if r is not big)
    assert all(r.steps_done == r.nsteps and not r.refused for r in st.requests)
    assert big.steps_done == 0 and big.rid not in {rid for _, m in be.calls for rid in m}
    s = st.summary()
    assert s["requests"] == 11 and s["refused"] == 1


class FailingSetup(FakeBackend):
    def setup(self, r):
        if r.rid == 2:
            raise RuntimeError("mesh rejected")
        return super().setup(r)


def test_failed_setup_is_refused_alone():
    reqs = S.make_requests(8, rate=1e4, seed=6, n_range=(3, 4), p_range=(1, 2), nsteps=4)
    budget = 2 * max(S.footprint_bytes(r.n, r.P) for r in reqs)
    be = FailingSetup(max_members=2)
    st = S.serve(reqs, be, mem_budget=budget, max_members=2, max_steps_per_call=2, realtime=False)
    assert [r.rid for r in st.refused] == [2] and "mesh rejected" in st.refused[0].refused
    assert len(st.requests) == 7 and all(r.steps_done == r.nsteps for r in st.requests)
    assert st.peak_bytes <= budget


def test_only_oversized_requests():
    r = S.make_requests(1, seed=0)[0]
    st = S.serve([r], FakeBackend(1), mem_budget=1000, max_members=1)
    assert st.requests == [] and st.refused == [r]
    assert st.summary() == {"requests": 0, "refused": 1, "wall_s": st.wall_s}
