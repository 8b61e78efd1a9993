"""Continuous batching of kick/encounter steps over simulations kept in HBM.

A request names one simulation and asks either for one evaluation of the
step on its current state (mode "evaluate", symba_kick_encounter_batch) or
for one integrator step that advances it (mode "step", symba_step_batch).
The server keeps the simulations' states and output buffers resident in
device memory within a byte budget.  Requests arriving while calls run are
admitted into the next call; with several lanes (each a library context and
a stream of its own) a new call is issued while earlier ones still run, so
their work overlaps on the device.  The rules that keep overlapping calls
correct:
  * a simulation is in at most one call at a time: requests for a
    simulation whose call is still running wait for the next call;
  * eviction (least recently used first) never touches a simulation of a
    running call, and the device bytes of the running calls (their
    simulations and library scratch) stay reserved in the budget;
  * a call's completion is observed through an event recorded after it on
    its lane's stream; only then are its results handed out and its
    simulations released (so a step's updated state is final before another
    lane uses it), and the host waits for completions with short sleeps, not
    a busy loop.
Each step of the path runs in the library's kernels; this module only
chooses what goes into each call.

Results do not depend on batching or lanes: the library gives every problem
the tile size of a single call, so a simulation's outputs (and in step mode
its trajectory) are bit-identical whether it runs alone or with any other
simulations.
"""
from __future__ import annotations

import time
from collections import OrderedDict, deque
from contextlib import nullcontext
from dataclasses import dataclass

import numpy as np

STATE_BYTES_PER_BODY = 8 * 8           # x y z vx vy vz m rh, float64
OUTPUT_BYTES_PER_BODY = 3 * 8 + 4      # ax ay az (float64), group_id (int32)
PAIR_BYTES = 2 * 4                     # pair_i, pair_j (int32)
POLL_SLEEP_S = 20e-6                   # host pause between completion polls when there is nothing to do


def pair_capacity(n: int) -> int:
    """Output pair capacity given to a simulation of n bodies."""
    return max(4 * n, 4096)


@dataclass
class _Sim:
    state: dict            # host SoA arrays (in step mode: as of the last eviction)
    n: int
    n_m: int
    scratch: int           # library scratch in a batch (symba_scratch_bytes)
    dev: dict | None = None
    out: object | None = None
    acc: np.ndarray | None = None   # step mode: accelerations at `state`, kept while evicted
    cprob: object | None = None     # the library's problem struct while resident (pointers into dev and out)

    @property
    def resident_bytes(self) -> int:
        return self.n * (STATE_BYTES_PER_BODY + OUTPUT_BYTES_PER_BODY) + pair_capacity(self.n) * PAIR_BYTES + 16


class GpuIO:
    """The device side of the server: one library context and one stream per
    lane; uploads, evictions and calls through the binding."""

    def __init__(self, server: "Server", lanes: int):
        import torch
        from . import binding as B
        self.torch, self.B = torch, B
        self.server = server
        self.ctxs = [B.Context(max_n=server.max_batch_bodies, max_pairs=server.max_pairs) for _ in range(lanes)]
        # default-priority streams only (streams of other priorities have hung here)
        self.streams = [torch.cuda.Stream() for _ in range(lanes)]

    def scratch_bytes(self, n: int, n_m: int) -> int:
        return self.ctxs[0].scratch_bytes(n, n_m, pair_capacity(n))

    def _stream_ctx(self, stream):
        return self.torch.cuda.stream(stream) if stream is not None else nullcontext()

    def load(self, s: _Sim, lane: int, stream=None):
        """Upload simulation s for a call on `lane` (ordered on that lane's
        stream, or on `stream` when given)."""
        st = stream if stream is not None else self.streams[lane]
        with self._stream_ctx(st):
            s.dev = self.B.to_device_state(s.state, self.server.device)
            s.out = self.B.Outputs(s.n, pair_capacity(s.n), device=self.server.device)
            if self.server.mode == "step":  # a step starts from the accelerations at the current positions
                if s.acc is None:
                    self.ctxs[lane].kick_encounter(s.dev, s.n_m, abs(self.server.dt), self.server.f, out=s.out,
                                                   stream=st)
                else:
                    s.out.acc.copy_(self.torch.from_numpy(s.acc))
                s.cprob = self.B.step_problem_struct(s.dev, s.n_m, self.server.dt, self.server.f, s.out)
            else:
                s.cprob = self.B.problem_struct(s.dev, s.n_m, self.server.dt, self.server.f, s.out)

    def evict(self, s: _Sim, stream=None):
        """Drop simulation s from the device (in step mode keeping its advanced
        state and accelerations on the host).  Only called for a simulation
        whose calls have all completed."""
        with self._stream_ctx(stream):
            if self.server.mode == "step":
                s.state = {key: v.cpu().numpy() for key, v in s.dev.items()}
                s.acc = s.out.acc.cpu().numpy()
        s.dev = None
        s.out = None
        s.cprob = None

    def issue(self, lane: int, sims, stream=None):
        """Enqueue one batched call on `lane` (or on `stream`); returns the event
        recorded after it."""
        st = stream if stream is not None else self.streams[lane]
        step = self.server.mode == "step"
        arr = ((self.B.symba_step_problem if step else self.B.symba_problem) * len(sims))(*(s.cprob for s in sims))
        with self._stream_ctx(st):
            if step:
                self.ctxs[lane].step_batch_structs(arr, stream=st)
            else:
                self.ctxs[lane].kick_encounter_batch_structs(arr, stream=st)
            ev = self.torch.cuda.Event()
            ev.record(st if st is not None else self.torch.cuda.current_stream())
        return ev

    @staticmethod
    def done(token) -> bool:
        return token.query()

    def close(self):
        for c in self.ctxs:
            c.close()


class Server:
    """Serves step requests for `sims` (a list of (host state dict, n_m)).

    budget_bytes bounds the device memory the server plans for.  That covers
    the lanes' library contexts (each sized by max_batch_bodies), the resident
    simulations and the library scratch of the calls running.  A simulation
    that does not fit beside the calls' scratch waits for a later call, and
    one that cannot fit even alone is an error.  max_batch_bodies bounds the
    bodies of one call and sizes the library contexts.  lanes: calls that may
    run at once (1 = one call at a time).  io: the device side (default: the
    GPU through the library; tests may substitute one with stand-in events).
    """

    def __init__(self, sims, budget_bytes: int, dt: float, rcrit_factor: float,
                 max_batch_bodies: int | None = None, device: str = "cuda", mode: str = "evaluate",
                 lanes: int = 2, io=None):
        if mode not in ("evaluate", "step"):
            raise ValueError("mode is 'evaluate' or 'step'")
        if lanes < 1:
            raise ValueError("lanes >= 1")
        self.mode = mode
        self.device = device
        self.dt = float(dt)
        self.f = float(rcrit_factor)
        self.n_lanes = int(lanes)
        ns = [int(s["x"].size) for s, _ in sims]
        self.max_batch_bodies = int(max_batch_bodies or sum(ns) or 1)
        if ns and max(ns) > self.max_batch_bodies:
            raise ValueError("a simulation is larger than max_batch_bodies")
        # pair scratch for any batch of at most max_batch_bodies bodies
        self.max_pairs = min(4 * self.max_batch_bodies + 4096 * 64, 2**31 - 1)
        self.io = io if io is not None else GpuIO(self, self.n_lanes)
        # each lane context's own scratch, sized by max_batch_bodies and max_pairs: per
        # body the union-find, bucket and binning arrays (~96 B), per pair the
        # found and the bucket-sorted lists (24 B), plus descriptors, counters
        # and the capture arena
        self.fixed_bytes = self.n_lanes * (96 * self.max_batch_bodies + 24 * self.max_pairs + (20 << 20))
        self.sims = []
        for (state, n_m), n in zip(sims, ns):
            self.sims.append(_Sim(state=state, n=n, n_m=int(n_m), scratch=self.io.scratch_bytes(n, n_m)))
        self.budget = int(budget_bytes) - self.fixed_bytes
        self.lru: OrderedDict[int, None] = OrderedDict()   # resident sims, least recent first
        self.resident = 0
        self.uploads = 0
        self.evictions = 0
        self.busy: dict[int, int] = {}   # simulation -> lane of the running call that holds it
        self.last_progress = time.monotonic()
        for k in range(len(self.sims)):
            if self._need(k) > self.budget:
                raise ValueError(f"simulation {k} ({self.sims[k].n} bodies) does not fit the budget alone")

    @property
    def ctx(self):
        """Lane 0's library context (for plain calls beside the server)."""
        return self.io.ctxs[0]

    def close(self):
        self.io.close()

    # -- residency -----------------------------------------------------------
    def _evict(self, k: int, stream=None):
        if k in self.busy:
            raise AssertionError(f"simulation {k} is in a running call and cannot be evicted")
        s = self.sims[k]
        self.io.evict(s, stream)
        self.resident -= s.resident_bytes
        del self.lru[k]
        self.evictions += 1

    def _make_room(self, need: int, keep: set, stream=None):
        """Evicts least recently used simulations outside `keep` (and outside
        every running call) until `need` more bytes fit beside the resident
        ones."""
        for k in list(self.lru):
            if self.resident + need <= self.budget:
                return
            if k not in keep and k not in self.busy:
                self._evict(k, stream)

    def _load(self, k: int, lane: int = 0, stream=None):
        s = self.sims[k]
        self.io.load(s, lane, stream)
        self.resident += s.resident_bytes
        self.lru[k] = None
        self.uploads += 1

    def preload(self, reserve: int = 0):
        """Makes resident, in order, the simulations that fit the budget while
        `reserve` bytes stay free for the scratch of a call."""
        for k, s in enumerate(self.sims):
            if k not in self.lru and self.resident + s.resident_bytes + reserve <= self.budget:
                self._load(k)

    # -- batching ------------------------------------------------------------
    def _need(self, k: int) -> int:
        """Device bytes simulation k takes while its step runs."""
        s = self.sims[k]
        return s.resident_bytes + s.scratch

    def _prepare(self, sim_ids, lane: int, stream=None):
        """Makes the simulations of a call resident (loading on the call's lane,
        evicting others that no running call holds) and marks them recently used."""
        keep = set(sim_ids)
        scratch = sum(self.sims[k].scratch for k in keep)
        running = sum(self.sims[k].scratch for k in self.busy)
        loads = sum(self.sims[k].resident_bytes for k in keep if k not in self.lru)
        self._make_room(loads + scratch + running, keep, stream)
        for k in sim_ids:
            if k not in self.lru:
                self._load(k, lane, stream)
            else:
                self.lru.move_to_end(k)

    def run_batch(self, sim_ids, stream=None):
        """One batched call over distinct simulations on lane 0 (or on `stream`),
        loading the ones that are not resident; returns without waiting.  With
        `stream`, the evictions' copies, the uploads and the call are all
        ordered on that stream."""
        if self.busy:
            raise RuntimeError("run_batch while serve() has calls running")
        self._prepare(sim_ids, 0, stream)
        return self.io.issue(0, [self.sims[k] for k in sim_ids], stream)

    def outputs(self, k: int):
        return self.sims[k].out

    def serve(self, arrival_s, sim_ids, warmup: int = 0, on_complete=None, progress=None) -> dict:
        """Replays requests arriving at times arrival_s (seconds from the start,
        nondecreasing) for simulations sim_ids; returns latency and throughput
        statistics over the requests after the first `warmup`.  on_complete,
        if given, is called as on_complete(request_index, sim_id, outputs)
        once the call that served the request has completed, before the
        simulation can join another call.  progress, if given, is called as
        progress(served, n_requests) after each completed call.
        `last_progress` holds the monotonic time at which the loop last
        issued or completed a call or waited for an arrival with nothing
        running (a watchdog can read it)."""
        arrival_s = np.asarray(arrival_s, dtype=np.float64)
        sim_ids = np.asarray(sim_ids, dtype=np.int64)
        n_req = len(arrival_s)
        latency = np.zeros(n_req)
        done_at = np.zeros(n_req)
        pending: deque = deque()
        free_lanes = deque(range(self.n_lanes))
        running = []          # (lane, token, batch) in issue order
        nxt = served = calls = 0
        batch_sizes, overlapped = [], 0
        t0 = self.last_progress = time.monotonic()
        while served < n_req:
            now = time.monotonic() - t0
            while nxt < n_req and arrival_s[nxt] <= now:
                pending.append((nxt, int(sim_ids[nxt])))
                nxt += 1
            progressed = False
            # completions, in any order across lanes
            for call in list(running):
                lane, token, batch = call
                if not self.io.done(token):
                    continue
                t_done = time.monotonic() - t0
                for r, k in batch:
                    done_at[r] = t_done
                    latency[r] = t_done - arrival_s[r]
                    if on_complete is not None:
                        on_complete(r, k, self.sims[k].out)
                for _, k in batch:
                    del self.busy[k]
                running.remove(call)
                free_lanes.append(lane)
                served += len(batch)
                progressed = True
                if progress is not None:
                    progress(served, n_req)
            # a new call on a free lane, from the waiting requests whose
            # simulations no running call holds
            if free_lanes and pending:
                avail = self.budget - sum(self._need(k) for k in self.busy)
                batch, pending = self._pick(pending, avail)
                if batch:
                    lane = free_lanes.popleft()
                    ids = [k for _, k in batch]
                    self._prepare(ids, lane)
                    token = self.io.issue(lane, [self.sims[k] for k in ids])
                    for k in ids:
                        self.busy[k] = lane
                    if running:
                        overlapped += 1
                    running.append((lane, token, batch))
                    calls += 1
                    batch_sizes.append(len(batch))
                    progressed = True
                elif not running:
                    raise RuntimeError("no waiting request fits the budget")
            if progressed:
                self.last_progress = time.monotonic()
            else:
                if running:
                    time.sleep(POLL_SLEEP_S)
                elif nxt < n_req:
                    wait = arrival_s[nxt] - (time.monotonic() - t0)
                    if wait > 2e-4:
                        time.sleep(wait - 1e-4)
                    self.last_progress = time.monotonic()
        lat = latency[warmup:] * 1e3
        span = done_at.max() - (arrival_s[warmup] if warmup < n_req else 0.0) if n_req else 0.0
        pairs = sum(_pairs(self.sims[k]) for k in sim_ids[warmup:])
        return dict(requests=int(n_req - warmup), warmup=int(warmup), calls=calls, lanes=self.n_lanes,
                    calls_issued_while_another_ran=overlapped,
                    mean_batch=float(np.mean(batch_sizes)) if batch_sizes else 0.0,
                    latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                                    mean=float(lat.mean()), max=float(lat.max())) if lat.size else {},
                    steps_per_s=float((n_req - warmup) / span) if span > 0 else 0.0,
                    pairs_per_s=float(pairs / span) if span > 0 else 0.0,
                    uploads=self.uploads, evictions=self.evictions,
                    budget_bytes=self.budget + self.fixed_bytes)

    def _pick(self, pending: deque, budget: int):
        return pick_batch(pending, [s.n for s in self.sims], [self._need(k) for k in range(len(self.sims))],
                          budget, self.max_batch_bodies, self.max_pairs, exclude=self.busy)


def pick_batch(pending, sizes, needs, budget: int, max_bodies: int, max_pairs: int, exclude=()):
    """Splits `pending` (an iterable of (request, simulation) in arrival order)
    into the requests of the next call and the rest.  A request joins if its
    simulation is not in the call yet, is not held by a running call
    (`exclude`), and the call stays within max_bodies bodies, max_pairs of
    output pair capacity, 4096 problems and `budget` bytes of device memory
    (`needs[k]`: resident bytes plus library scratch of simulation k)."""
    batch, chosen, rest = [], set(), deque()
    bodies = need = caps = 0
    for req in pending:
        k = req[1]
        cap = pair_capacity(sizes[k])
        if (k not in chosen and k not in exclude and bodies + sizes[k] <= max_bodies and
                caps + cap <= max_pairs and len(batch) < 4096 and need + needs[k] <= budget):
            batch.append(req)
            chosen.add(k)
            bodies += sizes[k]
            caps += cap
            need += needs[k]
        else:
            rest.append(req)
    return batch, rest


def _pairs(s: _Sim) -> int:
    rows = min(s.n_m, s.n - 1)
    return rows * s.n - rows * (rows + 1) // 2
