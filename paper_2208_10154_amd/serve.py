"""Batched transform server for one GPU: grouping, slots, HBM admission, graph replay.

The paper's throughput comes from batching: many maps of one resolution share a
single pass over the Legendre and FFT steps, which turns per-map matrix-vector
work into dense per-m products (Sec. 2.2, the batched workflow of Sec. 3.1).  A
server sees the opposite: requests of mixed resolution, spin, direction and
precision arriving at any time.  This module groups them back into batches:

* Requests with the same plan key (nside, lmax, spin, precision, direction) that
  are waiting when their plan's stream can take work are packed, oldest first,
  into the slots of one batched call (map sets concatenated along the batch
  axis); the call's chunk is the batch size rounded up to the column granularity
  of the kernels (32 map sets for small batches, then multiples of 64), so a
  small batch pays for what it holds, not for the slots.
* HBM admission: the server owns plan tables, plan workspaces and slot buffers
  and keeps their sum under a byte budget, evicting idle plans (least recently
  used) before creating new ones.  A request whose slot copy would not fit runs
  alone in place on the caller's tensors, and the plan chunks it internally; a
  request whose plan alone exceeds the budget is rejected with SHT_ERR_NOMEM.
* Batches of different plans overlap on several streams (default priority).  A
  plan's batches share its workspace, so while any is in flight the next one
  follows on the same stream; an idle plan takes the stream with the least work
  outstanding (estimated from the batch sizes), so small requests are not
  queued behind large batches of other plans.  Finished batches retire in any
  order.
* Optional graph replay: a batch bucket's launch sequence on the slot buffers is
  captured once as a HIP graph and replayed for later batches of that bucket.

Inputs and outputs stay caller-owned until the request completes; latency is
measured from the request's arrival to the GPU completion event of its batch.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import time

from . import sht

SHT_ERR_NOMEM = -2
GRANULE = 64  # map sets per column granule of the kernels beyond one small tile
SMALL = 32    # batches of up to this many map sets use a single 64-column tile


def lmax_of(nside: int) -> int:
    return 3 * nside - 1


def npix(nside: int) -> int:
    return 12 * nside * nside


def bucket(n: int) -> int:
    """Chunk width for a batch of n map sets (the kernels' column granularity)."""
    return SMALL if n <= SMALL else -(-n // GRANULE) * GRANULE


@dataclasses.dataclass
class Request:
    """One transform request.  inp/out are caller-owned contiguous float64 device
    tensors: alm [n, ncomp, (lmax+1)^2] (compact storage) and maps [n, ncomp, npix]
    (RING order); ncomp = 1 for spin 0, 3 (I, Q, U / T, E, B) for spin 2."""
    nside: int
    spin: int
    direction: str          # "alm2map" or "map2alm"
    precision: str          # "fp64", "fp32" or "bf16x3"
    nmaps: int
    inp: object = None
    out: object = None
    lmax: int = -1
    arrival: float | None = None
    ready: object = None    # optional event marking the inputs complete (the server's stream waits on it)
    # filled in by the server
    ticket: int = -1
    status: int = 0         # 0 ok, < 0 an SHT error code
    done: float | None = None
    batch: int = -1
    error: str = ""

    def __post_init__(self):
        if self.lmax < 0:
            self.lmax = lmax_of(self.nside)
        if self.direction not in ("alm2map", "map2alm"):
            raise ValueError(f"unknown direction {self.direction!r}")
        if self.spin not in (0, 2):
            raise ValueError("spin must be 0 or 2")
        if self.nmaps < 1:
            raise ValueError("nmaps must be >= 1")

    @property
    def ncomp(self) -> int:
        return 1 if self.spin == 0 else 3

    @property
    def plan_key(self):
        return (self.nside, self.lmax, self.spin)

    @property
    def key(self):
        return (self.nside, self.lmax, self.spin, self.precision, self.direction)

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


def mapset_bytes(nside: int, lmax: int, spin: int) -> int:
    """Bytes of one map set's maps plus its alm (FP64)."""
    ncomp = 1 if spin == 0 else 3
    return 8 * ncomp * (npix(nside) + (lmax + 1) ** 2)


SEG, TL = 8, 64  # Legendre seed segment and tile (rows of l), as in the library


def batch_cost(req: Request, n: int) -> float:
    """Relative GPU work of a batch of n map sets of req's key: the contraction
    dominates, columns x (lmax + 1)^2 x northern rings (the FFTs scale alike)."""
    return float(bucket(n) * req.ncomp * (req.lmax + 1) ** 2 * req.nside)


def plan_bytes_estimate(nside: int, lmax: int, spin: int, slots: int) -> int:
    """Upper estimate of a plan's device bytes before it exists: the FP64
    workspace for a chunk of `slots` map sets (m-major ring coefficients for every
    m and ring plus m-major alm rows, columns padded to the kernels' column
    granularity) and the recursion tables (seed pairs every SEG rows of l per north
    ring, coefficient rows, skip bounds); ring and FFT tables are small and covered
    by a 5% margin."""
    ncomp = 1 if spin == 0 else 3
    nring, rn = 4 * nside - 1, 2 * nside
    ldx = 2 * bucket(slots)
    ws = 8 * ncomp * ((lmax + 1) * nring + (lmax + 1) * (lmax + 2) // 2) * ldx
    tables = 0
    for s, nmu in ((0, 2), (2, 4)) if spin == 2 else ((0, 2),):
        segs = rows = 0
        for m in range(lmax + 1):
            lb = max(m, 2) if s == 2 else m
            if lb <= lmax:
                segs += (lmax - lb + SEG) // SEG
                rows += lmax + 1 - lb
        tables += segs * rn * (8 * nmu + 4) + (rows + TL) * 8 * (4 if s == 2 else 2)
        tables += (lmax + 1) * (-(-rn // 32)) * 4
    return int(1.05 * (ws + tables)) + (64 << 20)


class Executor:
    """Runs batches on the GPU through the C-ABI plans (the product path)."""

    def __init__(self, nstreams: int = 4, graphs: bool = False):
        import torch
        self.torch = torch
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self._idle = torch.cuda.Stream()  # plans are destroyed on it (it never carries work)
        self.graphs_enabled = graphs
        self._graphs = {}
        self._ref = torch.cuda.Event(enable_timing=True)
        self._ref_time = 0.0

    # --- clock: host seconds since start; GPU events are mapped onto it
    def start_clock(self) -> float:
        self.torch.cuda.synchronize()
        self._ref.record(self.streams[0])
        self._ref.synchronize()
        self._ref_time = time.perf_counter()
        return self._ref_time

    def event_time(self, ev) -> float:
        return self._ref_time - self._t0 + self._ref.elapsed_time(ev) / 1e3

    def set_origin(self, t0: float) -> None:
        self._t0 = t0

    # --- resources
    def new_plan(self, nside, lmax, spin, slots):
        return sht.Plan(nside, lmax, spin, slots)

    def plan_bytes(self, plan, slots, precision) -> int:
        plan.set_precision(precision)
        plan.set_chunk(bucket(min(slots, plan.capacity)))
        return plan.table_bytes() + plan.workspace_bytes()

    def alloc(self, shape):
        return self.torch.empty(shape, dtype=self.torch.float64, device="cuda")

    def free_plan(self, plan) -> None:
        """Release an idle plan.  The server evicts only plans whose batches have all
        retired (their completion events were seen), so none of its work is in
        flight; its stream is pointed at a stream of its own that never carries
        work, so destroying the plan waits for no other plan's batches."""
        plan.set_stream(self._idle)
        plan.close()

    def reclaim(self) -> None:
        """Return device memory cached by torch but unused (freed request and slot
        tensors) before the library allocates a plan."""
        self.torch.cuda.empty_cache()

    # --- one batch
    def run(self, plan, stream_id, direction, precision, reqs, n, slot_in, slot_out):
        torch = self.torch
        s = self.streams[stream_id]
        plan.set_stream(s)
        width = bucket(n)
        self._sized(plan, precision, width)
        with torch.cuda.stream(s):
            for r in reqs:
                if r.ready is not None:
                    s.wait_event(r.ready)
                if r.inp is not None:
                    r.inp.record_stream(s)
                    r.out.record_stream(s)
            if len(reqs) == 1 and slot_in is None:
                # alone and in place on the caller's tensors, in pieces of at most the
                # plan's capacity (contiguous views along the map axis)
                r = reqs[0]
                fn = plan.alm2map if direction == "alm2map" else plan.map2alm
                for k0 in range(0, n, plan.capacity):
                    k1 = min(n, k0 + plan.capacity)
                    plan.set_nmaps(k1 - k0)
                    fn(r.inp[k0:k1], r.out[k0:k1], stream=s)
            else:
                off = 0
                for r in reqs:
                    slot_in[off:off + r.nmaps].copy_(r.inp[:r.nmaps], non_blocking=True)
                    off += r.nmaps
                self._transform(plan, s, direction, precision, width, n, slot_in, slot_out)
                off = 0
                for r in reqs:
                    r.out[:r.nmaps].copy_(slot_out[off:off + r.nmaps], non_blocking=True)
                    off += r.nmaps
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        return ev

    def _sized(self, plan, precision, width) -> None:
        """Set the batch's precision and chunk; a workspace that grows may meet
        device memory cached by torch, which is then given back once."""
        for attempt in (0, 1):
            try:
                plan.set_precision(precision)
                plan.set_chunk(width)
                return
            except sht.ShtError as e:
                if e.code != SHT_ERR_NOMEM or attempt:
                    raise
                self.reclaim()

    def _transform(self, plan, s, direction, precision, width, n, slot_in, slot_out):
        torch = self.torch
        fn = plan.alm2map if direction == "alm2map" else plan.map2alm
        if not self.graphs_enabled:
            plan.set_nmaps(n)
            fn(slot_in, slot_out, stream=s)
            return
        # graph per (plan, direction, precision, width) over the whole bucket of
        # slots; a bucket wider than the plan's slots covers just the slots
        width = min(width, plan.capacity)
        key = (id(plan), direction, precision, width)
        g = self._graphs.get(key)
        if g is None:
            plan.set_nmaps(width)
            fn(slot_in, slot_out, stream=s)  # warm-up: work lists, workspace
            s.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                fn(slot_in, slot_out, stream=torch.cuda.current_stream())
            self._graphs[key] = g
        plan.set_stream(s)
        with torch.cuda.stream(s):
            g.replay()

    def forget_plan(self, plan) -> None:
        for k in [k for k in self._graphs if k[0] == id(plan)]:
            del self._graphs[k]

    def ready(self, ev) -> bool:
        return ev.query()

    def synchronize(self) -> None:
        self.torch.cuda.synchronize()


class _Plan:
    __slots__ = ("plan", "stream", "slots", "bytes", "last_use", "inflight", "slot_bufs")

    def __init__(self, plan, stream, slots, nbytes):
        self.plan, self.stream, self.slots, self.bytes = plan, stream, slots, nbytes
        self.last_use = 0.0
        self.inflight = 0
        self.slot_bufs = {}  # direction -> (slot_in, slot_out)


class Server:
    """Continuous-batching server.  submit() enqueues, poll() advances (retires
    finished batches, launches new ones), wait()/drain() block."""

    def __init__(self, hbm_budget_bytes: float, max_slots: int = 512, executor=None,
                 slot_bytes_per_plan: float = 8e9, depth: int = 2, batching: bool = True):
        self.budget = float(hbm_budget_bytes)
        self.batching = bool(batching)  # False: one request per launch (the serial baseline)
        self.max_slots = int(max_slots)
        self.slot_bytes_per_plan = float(slot_bytes_per_plan)
        self.depth = depth
        self.ex = executor if executor is not None else Executor()
        self.plans: dict = {}
        self.queues: dict = collections.OrderedDict()
        self.pending = []  # heap of (arrival, ticket): submitted, not yet arrived
        self.inflight = collections.deque()  # (event, plan key, [requests])
        self.used = 0.0
        self.peak = 0.0
        self.tickets = {}
        self._next_ticket = 0
        self._next_batch = 0
        self.nstreams = max(1, len(getattr(self.ex, "streams", [0])))
        self.stream_load = [0.0] * self.nstreams  # estimated work in flight per stream
        self.batches = []  # (batch id, key, maps, requests)
        self.plans_created = 0
        self.plans_evicted = 0
        self.plan_create_s = 0.0  # host seconds spent creating plans
        self.t0 = self.ex.start_clock()
        self.ex.set_origin(self.t0)

    # --- clock
    def now(self) -> float:
        return time.perf_counter() - self.t0

    # --- API
    def submit(self, req: Request) -> int:
        """Queue a request; an explicit future arrival time (server clock) holds
        it back until then (trace replay)."""
        if req.arrival is None:
            req.arrival = self.now()
        req.ticket = self._next_ticket
        self._next_ticket += 1
        self.tickets[req.ticket] = req
        heapq.heappush(self.pending, (req.arrival, req.ticket))
        return req.ticket

    def _arrivals(self) -> bool:
        now, moved = self.now(), False
        while self.pending and self.pending[0][0] <= now:
            r = self.tickets[heapq.heappop(self.pending)[1]]
            self.queues.setdefault(r.key, collections.deque()).append(r)
            moved = True
        return moved

    def wait(self, ticket: int):
        req = self.tickets[ticket]
        while req.done is None and req.status == 0:
            if not self.poll():
                time.sleep(5e-5)
        return req.status, req.latency

    def busy(self) -> bool:
        return bool(self.pending or any(self.queues.values()) or self.inflight)

    def drain(self) -> None:
        while self.pending or any(self.queues.values()) or self.inflight:
            if not self.poll():
                time.sleep(5e-5)

    # --- scheduling
    def poll(self) -> bool:
        """One scheduling round; returns True if anything changed."""
        changed = self._retire()
        changed |= self._arrivals()
        while self._launch_one():
            changed = True
        return changed

    def _retire(self) -> bool:
        """Retire every finished batch, in whatever order they finished."""
        changed, waiting = False, collections.deque()
        while self.inflight:
            item = self.inflight.popleft()
            ev, pk, reqs, sid, cost = item
            if not self.ex.ready(ev):
                waiting.append(item)
                continue
            t = self.ex.event_time(ev)
            for r in reqs:
                r.done = t
            self.plans[pk].inflight -= 1
            self.stream_load[sid] -= cost
            changed = True
        self.inflight = waiting
        return changed

    def _slots_for(self, nside, lmax, spin) -> int:
        per = mapset_bytes(nside, lmax, spin)
        return max(1, min(self.max_slots, int(self.slot_bytes_per_plan // (2 * per))))

    def _admit_plan(self, req: Request):
        """The plan of req, creating it (after evicting idle plans) if needed; None
        if it cannot be admitted now; raises MemoryError if it never can be."""
        pk = req.plan_key
        p = self.plans.get(pk)
        if p is not None:
            return p
        slots = self._slots_for(req.nside, req.lmax, req.spin)
        est = plan_bytes_estimate(req.nside, req.lmax, req.spin, slots)  # FP64 bounds the others
        if est > self.budget:
            raise MemoryError(f"plan {pk} needs about {est / 1e9:.2f} GB, budget {self.budget / 1e9:.2f} GB")
        while self.used + est > self.budget:
            idle = [(q.last_use, k) for k, q in self.plans.items()
                    if q.inflight == 0 and not any(self.queues.get(kk) for kk in self.queues if kk[:3] == k)]
            if not idle:
                return None
            self._evict(min(idle)[1])
        t0 = time.perf_counter()
        plan = self._new_plan(req, slots)
        self.plan_create_s += time.perf_counter() - t0
        if plan is None:
            return None
        self.plans_created += 1
        nbytes = max(est, self.ex.plan_bytes(plan, slots, "fp64"))
        p = _Plan(plan, 0, slots, nbytes)
        self.plans[pk] = p
        self.used += nbytes
        self.peak = max(self.peak, self.used)
        return p

    def _new_plan(self, req: Request, slots: int):
        """Create req's plan; when the device is out of memory (memory held outside
        the server's account, such as cached request tensors), give cached memory
        back and evict idle plans, then try again; None if nothing is left to free."""
        while True:
            try:
                return self.ex.new_plan(req.nside, req.lmax, req.spin, slots)
            except sht.ShtError as e:
                if e.code != SHT_ERR_NOMEM:
                    raise
            reclaim = getattr(self.ex, "reclaim", None)
            if reclaim is not None:
                reclaim()
                try:
                    return self.ex.new_plan(req.nside, req.lmax, req.spin, slots)
                except sht.ShtError as e:
                    if e.code != SHT_ERR_NOMEM:
                        raise
            idle = [(q.last_use, k) for k, q in self.plans.items() if q.inflight == 0]
            if not idle:
                return None
            self._evict(min(idle)[1])

    def _evict(self, pk) -> None:
        self.plans_evicted += 1
        p = self.plans.pop(pk)
        self.used -= p.bytes
        self.ex.forget_plan(p.plan)
        self.ex.free_plan(p.plan)

    def _slot_buffers(self, p: _Plan, req: Request):
        bufs = p.slot_bufs.get(req.direction)
        if bufs is not None:
            return bufs
        n, nc = p.slots, req.ncomp
        alm_shape, map_shape = (n, nc, (req.lmax + 1) ** 2), (n, nc, npix(req.nside))
        shapes = (alm_shape, map_shape) if req.direction == "alm2map" else (map_shape, alm_shape)
        nbytes = 8 * n * nc * ((req.lmax + 1) ** 2 + npix(req.nside))
        if self.used + nbytes > self.budget:
            return None
        bufs = (self.ex.alloc(shapes[0]), self.ex.alloc(shapes[1]))
        p.slot_bufs[req.direction] = bufs
        p.bytes += nbytes
        self.used += nbytes
        self.peak = max(self.peak, self.used)
        return bufs

    def _launch_one(self) -> bool:
        """Launch one batch: the key with the oldest waiting request whose plan's
        stream has room and whose plan is resident or can be admitted now.  A key
        blocked on memory does not hold up the others: once their queues drain,
        their plans become idle and can be evicted for it."""
        heads = sorted(((q[0].arrival, k) for k, q in self.queues.items() if q), key=lambda x: x[0])
        for _, key in heads:
            q = self.queues[key]
            head = q[0]
            p = self.plans.get(head.plan_key)
            if p is not None and p.inflight >= self.depth:
                continue
            try:
                p = self._admit_plan(head)
            except MemoryError as e:
                q.popleft()
                head.status, head.error, head.done = SHT_ERR_NOMEM, str(e), self.now()
                return True
            if p is None:
                continue
            return self._launch(key, q, p)
        return False

    def _launch(self, key, q, p) -> bool:
        head = q[0]
        reqs, n = [], 0
        while q and n + q[0].nmaps <= p.slots and (self.batching or not reqs):
            r = q.popleft()
            reqs.append(r)
            n += r.nmaps
        slot_in = slot_out = None
        if not reqs:
            reqs, n = [q.popleft()], head.nmaps  # larger than the slots: alone, in place
        elif len(reqs) > 1 or self._prefer_slots(head):
            bufs = self._slot_buffers(p, head)
            if bufs is None:
                # no room for slot buffers: run the requests one by one in place
                for r in reqs[1:][::-1]:
                    q.appendleft(r)
                reqs, n = reqs[:1], reqs[0].nmaps
            else:
                slot_in, slot_out = bufs
        bid = self._next_batch
        self._next_batch += 1
        for r in reqs:
            r.batch = bid
        if p.inflight == 0:  # free to move: the least-loaded stream
            p.stream = min(range(self.nstreams), key=lambda i: self.stream_load[i])
        cost = batch_cost(head, n)
        ev = self.ex.run(p.plan, p.stream, head.direction, head.precision, reqs, n, slot_in, slot_out)
        p.inflight += 1
        p.last_use = self.now()
        self.stream_load[p.stream] += cost
        self.inflight.append((ev, head.plan_key, reqs, p.stream, cost))
        self.batches.append((bid, key, n, len(reqs)))
        return True

    def _prefer_slots(self, head) -> bool:
        # a lone request runs in place unless slot graphs are on (graphs need fixed buffers)
        return bool(getattr(self.ex, "graphs_enabled", False))

    def close(self) -> None:
        self.drain()
        for pk in list(self.plans):
            self._evict(pk)


# ---------------------------------------------------------------------------
# synthetic request mix (config 5)
# ---------------------------------------------------------------------------
def request_mix(n: int, rate_hz: float, seed: int = 5, nsides=(64, 128, 256, 512, 1024),
                mixed: str = "bf16x3", median_maps: int = 16, sigma_ln: float = 1.0, max_maps: int = 512,
                mapset_cap_bytes: float | None = None):
    """n request descriptors (no data): Poisson arrivals at rate_hz, nside uniform
    over nsides (lmax = 3 nside - 1), T or IQU, alm2map or map2alm and FP64 or the
    mixed precision with probability 1/2 each, map count log-normal (median
    median_maps, log-sd sigma_ln) capped at max_maps (and, if given, at
    mapset_cap_bytes of maps + alm per request)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([220810154, 5, seed])))
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        nside = int(rng.choice(nsides))
        spin = 0 if rng.random() < 0.5 else 2
        direction = "alm2map" if rng.random() < 0.5 else "map2alm"
        prec = "fp64" if rng.random() < 0.5 else mixed
        k = int(round(median_maps * np.exp(sigma_ln * rng.standard_normal())))
        k = max(1, min(k, max_maps))
        if mapset_cap_bytes is not None:
            k = max(1, min(k, int(mapset_cap_bytes // mapset_bytes(nside, lmax_of(nside), spin))))
        out.append(dict(arrival=t, nside=nside, spin=spin, direction=direction, precision=prec, nmaps=k))
    return out


def request_bytes(d) -> int:
    """Device bytes of a request descriptor's input and output (maps + alm, FP64)."""
    return d["nmaps"] * mapset_bytes(d["nside"], d.get("lmax", lmax_of(d["nside"])), d["spin"])


def replay(server: Server, mix, make_io, release: bool = True, poll_sleep: float = 5e-5, stall_s: float = 60.0,
           max_live_bytes: float | None = None, bypass_age_s: float | None = 2.0):
    """Drive `server` with the request descriptors of `mix` (request_mix()
    dictionaries): each request is created with make_io(desc) -> (inp, out, ready)
    when the server clock reaches its arrival time, then submitted; finished
    requests drop their tensors when `release` is set.  With max_live_bytes the
    callers hold at most that many bytes of request inputs and outputs at a time:
    a request that would exceed it is created once earlier requests have finished,
    and its latency still counts from its arrival time.  The callers are
    independent: a later request whose buffers fit goes ahead of one that does
    not, unless that one has waited more than bypass_age_s (then it is next, so
    large requests are not starved; None keeps strict arrival order).
    Returns the requests.  Raises RuntimeError if work is waiting but nothing
    completes for stall_s."""
    order = sorted(range(len(mix)), key=lambda k: mix[k]["arrival"])
    if max_live_bytes is not None:
        if not release:
            raise ValueError("a bound on live request bytes needs release=True")
        big = max(request_bytes(d) for d in mix)
        if big > max_live_bytes:
            raise ValueError(f"a request of {big / 1e9:.1f} GB exceeds the {max_live_bytes / 1e9:.1f} GB of live requests")
    reqs, live, i, live_bytes = [], [], 0, 0
    due = []  # arrived, not yet created (arrival order)
    last_progress = time.perf_counter()
    while i < len(order) or due or server.busy():
        now = server.now()
        while i < len(order) and mix[order[i]]["arrival"] <= now:
            due.append(order[i])
            i += 1
        waiting = []
        for n_due, k in enumerate(due):
            d = mix[k]
            nb = request_bytes(d)
            if max_live_bytes is not None and live_bytes + nb > max_live_bytes:
                waiting.append(k)
                if bypass_age_s is None or now - d["arrival"] > bypass_age_s:
                    waiting.extend(due[n_due + 1:])  # nothing later goes ahead of it
                    break
                continue
            inp, out, ready = make_io(d)
            r = Request(nside=d["nside"], spin=d["spin"], direction=d["direction"], precision=d["precision"],
                        nmaps=d["nmaps"], inp=inp, out=out, arrival=d["arrival"], ready=ready)
            server.submit(r)
            reqs.append(r)
            live.append((r, nb))
            live_bytes += nb
            last_progress = time.perf_counter()
        due = waiting
        if server.poll():
            last_progress = time.perf_counter()
        else:
            time.sleep(poll_sleep)
        if (server.busy() or due) and time.perf_counter() - last_progress > stall_s:
            waiting_q = {k: len(q) for k, q in server.queues.items() if q}
            raise RuntimeError(f"server stalled: waiting {waiting_q}, {len(due)} not created, in flight "
                               f"{len(server.inflight)}, plans {list(server.plans)}, "
                               f"{server.used / 1e9:.1f} of {server.budget / 1e9:.1f} GB")
        if release and live:
            keep = []
            for r, nb in live:
                if r.done is not None or r.status != 0:
                    r.inp = r.out = r.ready = None
                    live_bytes -= nb
                else:
                    keep.append((r, nb))
            live = keep
    reqs.sort(key=lambda r: r.arrival)
    return reqs


def latency_stats(reqs) -> dict:
    import numpy as np
    lat = np.array([r.latency for r in reqs if r.latency is not None]) * 1e3
    t_end = max(r.done for r in reqs if r.done is not None)
    t_start = min(r.arrival for r in reqs)
    sets = sum(r.nmaps for r in reqs if r.status == 0)
    comp = sum(r.nmaps * r.ncomp for r in reqs if r.status == 0)
    by_nside = {}
    for ns in sorted({r.nside for r in reqs}):
        x = np.array([r.latency for r in reqs if r.nside == ns and r.latency is not None]) * 1e3
        if len(x):
            by_nside[str(ns)] = {"requests": int(len(x)), "p50_ms": round(float(np.percentile(x, 50)), 2),
                                 "p99_ms": round(float(np.percentile(x, 99)), 2)}
    return {"requests": len(reqs), "failed": sum(r.status != 0 for r in reqs),
            "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "mean_ms": round(float(lat.mean()), 2), "makespan_s": round(t_end - t_start, 3),
            "map_sets_per_s": round(sets / (t_end - t_start), 2), "maps_per_s": round(comp / (t_end - t_start), 2),
            "by_nside": by_nside}
