"""Host logic of the batching server (no GPU): grouping by plan key, slot packing,
oldest-first scheduling, HBM admission with eviction, rejection of plans larger
than the budget, latency accounting and the synthetic request mix.  A recording
executor stands in for the GPU; it runs nothing."""
import time

import numpy as np
import pytest

from paper_2208_10154_amd import serve


class _Ev:
    def __init__(self, t):
        self.t = t


class _Plan:
    def __init__(self, key, slots):
        self.key, self.capacity, self.closed = key, slots, False

    def close(self):
        self.closed = True


class RecordingExecutor:
    streams = [0, 1]
    graphs_enabled = False

    def __init__(self, duration=0.0):
        self.runs, self.created = [], []
        self.duration = duration  # seconds a batch stays in flight

    def start_clock(self):
        return time.perf_counter()

    def set_origin(self, t0):
        self.t0 = t0

    def new_plan(self, nside, lmax, spin, slots):
        p = _Plan((nside, lmax, spin), slots)
        self.created.append(p)
        return p

    def plan_bytes(self, plan, slots, precision):
        return 0

    def alloc(self, shape):
        return ("buffer", shape)

    def free_plan(self, plan):
        plan.close()

    def forget_plan(self, plan):
        pass

    def run(self, plan, stream, direction, precision, reqs, n, slot_in, slot_out):
        self.runs.append(dict(plan=plan.key, stream=stream, direction=direction, precision=precision,
                              rids=[r.ticket for r in reqs], n=n, slots=slot_in is not None))
        start = max(time.perf_counter() - self.t0, getattr(self, "busy_until", 0.0))
        self.busy_until = start + self.duration
        return _Ev(self.busy_until)

    def ready(self, ev):
        return time.perf_counter() - self.t0 >= ev.t

    def event_time(self, ev):
        return ev.t


def req(nside=16, spin=0, direction="alm2map", precision="fp64", nmaps=4, arrival=0.0):
    return serve.Request(nside=nside, spin=spin, direction=direction, precision=precision, nmaps=nmaps,
                         arrival=arrival)


def test_same_key_requests_share_one_batch():
    ex = RecordingExecutor()
    s = serve.Server(1e12, max_slots=64, executor=ex)
    t = [s.submit(req(nmaps=4, arrival=0.0)) for i in range(5)]
    s.submit(req(spin=2, nmaps=2, arrival=0.0))
    s.drain()
    assert len(ex.runs) == 2
    assert ex.runs[0]["rids"] == t and ex.runs[0]["n"] == 20 and ex.runs[0]["slots"]
    assert ex.runs[1]["plan"] == (16, 47, 2)
    for r in s.tickets.values():
        assert r.status == 0 and r.done is not None and r.latency >= 0


def test_arrivals_during_a_batch_join_the_next_one():
    ex = RecordingExecutor(duration=0.05)
    s = serve.Server(1e12, max_slots=64, executor=ex, depth=1)
    t = [s.submit(req(nmaps=2, arrival=0.002 * i)) for i in range(6)]
    s.drain()
    assert [r["rids"] for r in ex.runs] == [t[:1], t[1:]]
    lat = [s.tickets[i].latency for i in t]
    assert lat[0] == pytest.approx(0.05, abs=0.02)
    assert all(x > 0.05 for x in lat[1:])  # waited for the first batch, then one batch


def test_requests_wait_for_their_arrival_time():
    ex = RecordingExecutor()
    s = serve.Server(1e12, executor=ex)
    t = s.submit(req(arrival=0.03))
    s.drain()
    r = s.tickets[t]
    assert r.done >= 0.03 and 0 <= r.latency < 0.02


def test_direction_and_precision_split_batches():
    ex = RecordingExecutor()
    s = serve.Server(1e12, max_slots=64, executor=ex)
    s.submit(req(direction="alm2map"))
    s.submit(req(direction="map2alm"))
    s.submit(req(precision="bf16x3"))
    s.submit(req(direction="alm2map"))
    s.drain()
    keys = sorted((r["direction"], r["precision"], r["n"]) for r in ex.runs)
    assert keys == [("alm2map", "bf16x3", 4), ("alm2map", "fp64", 8), ("map2alm", "fp64", 4)]
    # one plan (same nside, lmax, spin) serves all three keys
    assert len(ex.created) == 1


def test_slot_capacity_and_oversized_request():
    ex = RecordingExecutor()
    s = serve.Server(1e12, max_slots=10, executor=ex)
    a = s.submit(req(nmaps=6))
    b = s.submit(req(nmaps=6))
    c = s.submit(req(nmaps=25))
    s.drain()
    runs = {tuple(r["rids"]): r for r in ex.runs}
    assert set(runs) == {(a,), (b,), (c,)}
    assert not runs[(c,)]["slots"] and runs[(c,)]["n"] == 25  # alone, in place, chunked by the plan
    # oldest first
    assert [r["rids"][0] for r in ex.runs] == [a, b, c]


def test_oldest_waiting_key_goes_first():
    ex = RecordingExecutor()
    s = serve.Server(1e12, max_slots=64, executor=ex)
    late = s.submit(req(nside=32, arrival=0.5))
    early = s.submit(req(nside=16, arrival=0.1))
    s.drain()
    assert [r["rids"] for r in ex.runs] == [[early], [late]]


def test_admission_evicts_idle_plans_under_a_small_budget():
    ex = RecordingExecutor()
    one = serve.plan_bytes_estimate(16, 47, 0, 64)
    s = serve.Server(1.5 * one, max_slots=64, executor=ex)
    for i in range(6):
        s.submit(req(nside=16 if i % 2 == 0 else 32, nmaps=1, arrival=0.001 * i))
        s.drain()
    assert all(r.status == 0 for r in s.tickets.values())
    assert len(ex.created) == 6 and sum(p.closed for p in ex.created) == 5
    assert s.peak <= s.budget


def test_key_blocked_on_memory_does_not_stall_the_others():
    # the budget holds one plan; the oldest request needs a second plan while the
    # resident one still has queued work: that work runs first, then the resident
    # plan is evicted and the blocked request is served
    ex = RecordingExecutor(duration=0.01)
    one = serve.plan_bytes_estimate(32, 95, 0, 64)
    s = serve.Server(1.2 * one, max_slots=4, executor=ex, depth=1)
    first = s.submit(req(nside=16, nmaps=4, arrival=0.0))
    s.poll()  # plan for nside 16 resident, batch in flight
    blocked = s.submit(req(nside=32, nmaps=1, arrival=0.001))
    more = [s.submit(req(nside=16, nmaps=4, arrival=0.002)) for _ in range(3)]
    mix = []
    serve.replay(s, mix, make_io=None, stall_s=5.0)
    order = [r["rids"] for r in ex.runs]
    assert order[0] == [first] and order[-1] == [blocked]
    assert all(s.tickets[t].status == 0 for t in [first, blocked] + more)


def test_replay_reports_a_stall():
    class Stuck(RecordingExecutor):
        def ready(self, ev):
            return False
    s = serve.Server(1e12, executor=Stuck())
    with pytest.raises(RuntimeError, match="stalled"):
        serve.replay(s, [dict(arrival=0.0, nside=16, spin=0, direction="alm2map", precision="fp64", nmaps=1)],
                     make_io=lambda d: (None, None, None), stall_s=0.3)


def test_plan_larger_than_budget_is_rejected():
    ex = RecordingExecutor()
    s = serve.Server(1e6, executor=ex)
    t = s.submit(req(nside=64))
    status, lat = s.wait(t)
    assert status == serve.SHT_ERR_NOMEM and "budget" in s.tickets[t].error
    assert not ex.runs


def test_plan_estimate_grows_with_size():
    small = serve.plan_bytes_estimate(64, 191, 0, 16)
    assert serve.plan_bytes_estimate(64, 191, 2, 16) > small
    assert serve.plan_bytes_estimate(128, 383, 0, 16) > small
    # column granularity: 1..32 map sets share one tile, then multiples of 64
    assert serve.plan_bytes_estimate(64, 191, 0, 1) == serve.plan_bytes_estimate(64, 191, 0, 32)
    assert serve.plan_bytes_estimate(64, 191, 0, 33) == serve.plan_bytes_estimate(64, 191, 0, 64)
    assert serve.plan_bytes_estimate(64, 191, 0, 32) < serve.plan_bytes_estimate(64, 191, 0, 33)
    assert [serve.bucket(n) for n in (1, 32, 33, 64, 65)] == [32, 32, 64, 64, 128]


def test_request_mix_is_seeded_and_bounded():
    a = serve.request_mix(200, rate_hz=50.0, seed=3)
    b = serve.request_mix(200, rate_hz=50.0, seed=3)
    assert a == b
    arr = [r["arrival"] for r in a]
    assert all(x < y for x, y in zip(arr, arr[1:]))
    assert 2.0 < arr[-1] < 6.0  # 200 arrivals at 50 Hz
    assert {r["nside"] for r in a} == {64, 128, 256, 512, 1024}
    assert {r["spin"] for r in a} == {0, 2} and {r["precision"] for r in a} == {"fp64", "bf16x3"}
    for r in a:
        assert 1 <= r["nmaps"] <= 512
    # log-normal with median 16: some requests are far larger than the median
    assert max(r["nmaps"] for r in a) > 64
    assert abs(np.median([r["nmaps"] for r in a]) - 16) <= 4
    c = serve.request_mix(200, rate_hz=50.0, seed=3, mapset_cap_bytes=2e9)
    for r in c:
        assert serve.request_bytes(r) <= 2e9 or r["nmaps"] == 1


def test_replay_bounds_live_request_bytes():
    """Callers that hold at most max_live_bytes of request data: a request that
    would exceed it is created once earlier ones have finished, and its latency
    counts from its arrival."""
    ex = RecordingExecutor()
    ex.duration = 0.02
    s = serve.Server(1e12, max_slots=64, executor=ex)
    per = serve.mapset_bytes(16, 47, 0)
    mix = [dict(arrival=0.0 + 0.001 * k, nside=16, spin=0, direction="alm2map", precision="fp64", nmaps=4)
           for k in range(6)]
    made = []

    def make_io(d):
        made.append((s.now(), d["arrival"]))
        return None, None, None
    reqs = serve.replay(s, mix, make_io, max_live_bytes=8.5 * per, stall_s=5.0)
    assert len(reqs) == 6 and all(r.done is not None for r in reqs)
    # two requests of 4 map sets fit at a time: the later ones waited for memory
    assert sum(1 for t, a in made if t > a + 0.015) >= 3
    assert all(r.latency >= r.done - r.arrival - 1e-9 for r in reqs)
    with pytest.raises(ValueError):
        serve.replay(s, mix, make_io, max_live_bytes=2 * per)


def test_replay_small_callers_go_ahead_of_a_blocked_large_one():
    """Independent callers: while a large request waits for caller memory, a
    later small one that fits is created first; a request that has waited longer
    than bypass_age_s is not passed (no starvation); bypass_age_s=None keeps
    strict arrival order.  Requests come back in arrival order."""
    per = serve.mapset_bytes(16, 47, 0)

    def run(age):
        ex = RecordingExecutor(duration=0.05)
        s = serve.Server(1e12, max_slots=64, executor=ex)
        mix = [dict(arrival=0.001 * k, nside=16, spin=0, direction="alm2map", precision="fp64", nmaps=n)
               for k, n in enumerate((4, 8, 1))]
        made = []

        def make_io(d):
            made.append(d["nmaps"])
            return None, None, None
        reqs = serve.replay(s, mix, make_io, max_live_bytes=8.5 * per, stall_s=5.0, bypass_age_s=age)
        assert len(reqs) == 3 and all(r.done is not None for r in reqs)
        assert [r.nmaps for r in reqs] == [4, 8, 1]
        return made
    assert run(10.0) == [4, 1, 8]
    assert run(None) == [4, 8, 1]
    assert run(0.0) == [4, 8, 1]


def test_latency_stats_by_nside():
    reqs = []
    for k, (ns, lat) in enumerate(((16, 0.010), (16, 0.030), (32, 0.5))):
        r = serve.Request(nside=ns, spin=0, direction="alm2map", precision="fp64", nmaps=1)
        r.arrival, r.done = float(k), float(k) + lat
        reqs.append(r)
    st = serve.latency_stats(reqs)
    assert st["by_nside"]["16"]["requests"] == 2 and st["by_nside"]["32"]["requests"] == 1
    assert abs(st["by_nside"]["16"]["p50_ms"] - 20.0) < 1e-6 and abs(st["by_nside"]["32"]["p99_ms"] - 500.0) < 1e-6


def test_request_validation():
    with pytest.raises(ValueError):
        serve.Request(nside=16, spin=1, direction="alm2map", precision="fp64", nmaps=1)
    with pytest.raises(ValueError):
        serve.Request(nside=16, spin=0, direction="sideways", precision="fp64", nmaps=1)
    with pytest.raises(ValueError):
        serve.Request(nside=16, spin=0, direction="alm2map", precision="fp64", nmaps=0)


class StreamExecutor(RecordingExecutor):
    """Each stream runs its batches one after another; streams run side by side.
    A batch takes `cost[nside]` seconds."""

    def __init__(self, cost, nstreams=2):
        super().__init__()
        self.streams = list(range(nstreams))
        self.cost = cost
        self.until = [0.0] * nstreams

    def run(self, plan, stream, direction, precision, reqs, n, slot_in, slot_out):
        self.runs.append(dict(plan=plan.key, stream=stream, rids=[r.ticket for r in reqs], n=n))
        start = max(time.perf_counter() - self.t0, self.until[stream])
        self.until[stream] = start + self.cost[plan.key[0]]
        return _Ev(self.until[stream])


def test_small_batches_retire_behind_a_large_one():
    # a long nside-64 batch is launched first; nside-16 batches on the other stream
    # finish and retire while it runs, so their plan keeps launching (depth 1)
    ex = StreamExecutor({64: 0.3, 16: 0.01})
    s = serve.Server(1e12, max_slots=64, executor=ex, depth=1)
    big = s.submit(req(nside=64, arrival=0.0))
    small = [s.submit(req(nside=16, arrival=0.001 + 0.02 * i)) for i in range(5)]
    s.drain()
    assert [r["stream"] for r in ex.runs if r["plan"][0] == 16] == [1] * 5
    for t in small:
        assert s.tickets[t].latency < 0.05, s.tickets[t].latency
    assert s.tickets[big].latency >= 0.3


def test_idle_plan_takes_the_least_loaded_stream():
    ex = StreamExecutor({64: 0.2, 32: 0.05, 16: 0.01}, nstreams=2)
    s = serve.Server(1e12, max_slots=64, executor=ex, depth=2)
    s.submit(req(nside=64, nmaps=64, arrival=0.0))   # heavy: stream 0
    s.submit(req(nside=32, nmaps=1, arrival=0.0))    # stream 1
    s.submit(req(nside=16, nmaps=1, arrival=0.0))    # lighter load is stream 1
    s.drain()
    st = {r["plan"][0]: r["stream"] for r in ex.runs}
    assert st[64] != st[32] and st[16] == st[32]
    assert all(v == 0.0 for v in s.stream_load)



def test_serial_mode_runs_one_request_per_launch_in_arrival_order():
    ex = RecordingExecutor()
    s = serve.Server(1e12, max_slots=64, executor=ex, batching=False, depth=1)
    ts = [s.submit(req(nside=16 if k % 2 else 32, nmaps=2, arrival=0.0001 * k)) for k in range(6)]
    s.drain()
    assert [r["rids"] for r in ex.runs] == [[t] for t in ts]


def test_plan_creation_reclaims_then_evicts_on_device_out_of_memory():
    """A plan that meets a full device (memory held outside the server's account)
    first gets cached memory back, then idle plans are evicted, then it is
    created; with nothing left to free it waits instead of failing."""
    from paper_2208_10154_amd import sht

    class Tight(RecordingExecutor):
        def __init__(self):
            super().__init__()
            self.free_calls, self.fail_next = 0, 0

        def new_plan(self, nside, lmax, spin, slots):
            if self.fail_next:
                self.fail_next -= 1
                raise sht.ShtError(serve.SHT_ERR_NOMEM, "hipMalloc failed")
            return super().new_plan(nside, lmax, spin, slots)

        def reclaim(self):
            self.free_calls += 1

    ex = Tight()
    s = serve.Server(1e12, max_slots=64, executor=ex)
    s.submit(req(nside=16, arrival=0.0))
    s.drain()
    ex.fail_next = 2  # the first try and the try after reclaiming fail
    t = s.submit(req(nside=32, arrival=0.0))
    s.drain()
    assert ex.free_calls == 1
    assert (16, 47, 0) not in s.plans and (32, 95, 0) in s.plans  # the idle plan was evicted
    assert s.tickets[t].status == 0
