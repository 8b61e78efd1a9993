"""Continuous batching of kick/encounter steps over simulations kept in HBM.

A request names one simulation and asks either for one evaluation of the
step on its current state (mode "evaluate", symba_kick_encounter_batch) or
for one integrator step that advances it (mode "step", symba_step_batch).
The server keeps the simulations' states and output buffers resident in
device memory within a byte budget.  When a batch needs room, it evicts the
least recently used simulations that are not in that batch (in step mode
copying back the advanced state and its accelerations, which the next step
starts from).  Whenever requests are waiting, the server runs every waiting
request whose simulation is not already in the batch as one batched library
call.  A request arriving while a call runs joins the next call.  Each step
of the path runs in the library's kernels; this module only chooses what
goes into each call.

Results do not depend on batching: the library gives every problem the
tile size of a single call, so a simulation's outputs (and in step mode its
trajectory) are bit-identical whether it runs alone or with any other
simulations.
"""
from __future__ import annotations

import time
from collections import OrderedDict, deque
from contextlib import nullcontext
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B

STATE_BYTES_PER_BODY = 8 * 8           # x y z vx vy vz m rh, float64
OUTPUT_BYTES_PER_BODY = 3 * 8 + 4      # ax ay az (float64), group_id (int32)
PAIR_BYTES = 2 * 4                     # pair_i, pair_j (int32)


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
    out: B.Outputs | None = None
    acc: np.ndarray | None = None   # step mode: accelerations at `state`, kept while evicted

    @property
    def resident_bytes(self) -> int:
        return self.n * (STATE_BYTES_PER_BODY + OUTPUT_BYTES_PER_BODY) + pair_capacity(self.n) * PAIR_BYTES + 16


class Server:
    """Serves step requests for `sims` (a list of (host state dict, n_m)).

    budget_bytes bounds the device memory the server plans for.  That covers
    the library context (sized by max_batch_bodies), the resident simulations
    and the library scratch of the batch being run.
    A simulation that does not fit beside the batch's scratch waits for a later
    batch, and one that cannot fit even alone is an error.  max_batch_bodies
    bounds the bodies of one call and sizes the library context.
    """

    def __init__(self, sims, budget_bytes: int, dt: float, rcrit_factor: float,
                 max_batch_bodies: int | None = None, device: str = "cuda", mode: str = "evaluate"):
        if mode not in ("evaluate", "step"):
            raise ValueError("mode is 'evaluate' or 'step'")
        self.mode = mode
        self.device = device
        self.dt = float(dt)
        self.f = float(rcrit_factor)
        ns = [int(s["x"].size) for s, _ in sims]
        self.max_batch_bodies = int(max_batch_bodies or sum(ns))
        if max(ns) > self.max_batch_bodies:
            raise ValueError("a simulation is larger than max_batch_bodies")
        # pair scratch for any batch of at most max_batch_bodies bodies
        self.max_pairs = min(4 * self.max_batch_bodies + 4096 * 64, 2**31 - 1)
        self.ctx = B.Context(max_n=self.max_batch_bodies, max_pairs=self.max_pairs)
        # the context's own scratch, sized by max_batch_bodies and max_pairs: per
        # body the union-find, bucket and binning arrays (~96 B), per pair the
        # found and the bucket-sorted lists (24 B), plus descriptors and counters
        self.fixed_bytes = 96 * self.max_batch_bodies + 24 * self.max_pairs + (1 << 20)
        self.sims = []
        for (state, n_m), n in zip(sims, ns):
            self.sims.append(_Sim(state=state, n=n, n_m=int(n_m),
                                  scratch=self.ctx.scratch_bytes(n, n_m, pair_capacity(n))))
        self.budget = int(budget_bytes) - self.fixed_bytes
        self.lru: OrderedDict[int, None] = OrderedDict()   # resident sims, least recent first
        self.resident = 0
        self.uploads = 0
        self.evictions = 0
        for k in range(len(self.sims)):
            if self._need(k) > self.budget:
                raise ValueError(f"simulation {k} ({self.sims[k].n} bodies) does not fit the budget alone")

    def close(self):
        self.ctx.close()

    # -- residency -----------------------------------------------------------
    def _evict(self, k: int):
        s = self.sims[k]
        if self.mode == "step":  # the simulation has moved: keep its state and accelerations
            s.state = {key: v.cpu().numpy() for key, v in s.dev.items()}
            s.acc = s.out.acc.cpu().numpy()
        s.dev = None
        s.out = None
        self.resident -= s.resident_bytes
        del self.lru[k]
        self.evictions += 1

    def _make_room(self, need: int, keep: set):
        """Evicts least recently used simulations outside `keep` until `need`
        more bytes fit beside the resident ones."""
        for k in list(self.lru):
            if self.resident + need <= self.budget:
                return
            if k not in keep:
                self._evict(k)

    def _load(self, k: int):
        s = self.sims[k]
        s.dev = B.to_device_state(s.state, self.device)
        s.out = B.Outputs(s.n, pair_capacity(s.n), device=self.device)
        if self.mode == "step":  # a step starts from the accelerations at the current positions
            if s.acc is None:
                self.ctx.kick_encounter(s.dev, s.n_m, abs(self.dt), self.f, out=s.out)
            else:
                s.out.acc.copy_(torch.from_numpy(s.acc))
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

    def _pick(self, pending: deque):
        return pick_batch(pending, [s.n for s in self.sims], [self._need(k) for k in range(len(self.sims))],
                          self.budget, self.max_batch_bodies, self.max_pairs)

    def run_batch(self, sim_ids, stream=None):
        """One batched call over distinct simulations, loading the ones that are
        not resident (evicting the least recently used others to make room).
        With `stream`, the evictions' copies, the uploads and the call are all
        ordered on that stream."""
        with torch.cuda.stream(stream) if stream is not None else nullcontext():
            keep = set(sim_ids)
            scratch = sum(self.sims[k].scratch for k in keep)
            loads = sum(self.sims[k].resident_bytes for k in keep if k not in self.lru)
            self._make_room(loads + scratch, keep)
            for k in sim_ids:
                if k not in self.lru:
                    self._load(k)
                else:
                    self.lru.move_to_end(k)
            probs = [(self.sims[k].dev, self.sims[k].n_m, self.dt, self.f, self.sims[k].out) for k in sim_ids]
            if self.mode == "step":
                self.ctx.step_batch(probs)
            else:
                self.ctx.kick_encounter_batch(probs)

    def outputs(self, k: int) -> B.Outputs:
        return self.sims[k].out

    def serve(self, arrival_s, sim_ids, warmup: int = 0, on_complete=None) -> dict:
        """Replays requests arriving at times arrival_s (seconds from the start,
        nondecreasing) for simulations sim_ids; returns latency and throughput
        statistics over the requests after the first `warmup`.  on_complete,
        if given, is called as on_complete(request_index, sim_id, outputs)
        right after the call that served the request has finished."""
        arrival_s = np.asarray(arrival_s, dtype=np.float64)
        sim_ids = np.asarray(sim_ids, dtype=np.int64)
        n_req = len(arrival_s)
        latency = np.zeros(n_req)
        done_at = np.zeros(n_req)
        pending: deque = deque()
        nxt = served = calls = 0
        batch_sizes = []
        t0 = time.monotonic()
        while served < n_req:
            now = time.monotonic() - t0
            while nxt < n_req and arrival_s[nxt] <= now:
                pending.append((nxt, int(sim_ids[nxt])))
                nxt += 1
            if not pending:
                wait = arrival_s[nxt] - (time.monotonic() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
                continue
            batch, pending = self._pick(pending)
            if not batch:
                raise RuntimeError("no waiting request fits the budget")
            ids = [k for _, k in batch]
            self.run_batch(ids)
            torch.cuda.synchronize()
            t_done = time.monotonic() - t0
            calls += 1
            batch_sizes.append(len(batch))
            for r, k in batch:
                done_at[r] = t_done
                latency[r] = t_done - arrival_s[r]
                if on_complete is not None:
                    on_complete(r, k, self.sims[k].out)
            served += len(batch)
        lat = latency[warmup:] * 1e3
        span = done_at[-1] - (arrival_s[warmup] if warmup < n_req else 0.0)
        pairs = sum(_pairs(self.sims[k]) for k in sim_ids[warmup:])
        return dict(requests=int(n_req - warmup), warmup=int(warmup), calls=calls,
                    mean_batch=float(np.mean(batch_sizes)) if batch_sizes else 0.0,
                    latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                                    mean=float(lat.mean()), max=float(lat.max())),
                    steps_per_s=float((n_req - warmup) / span) if span > 0 else 0.0,
                    pairs_per_s=float(pairs / span) if span > 0 else 0.0,
                    uploads=self.uploads, evictions=self.evictions,
                    budget_bytes=self.budget + self.fixed_bytes)


def pick_batch(pending, sizes, needs, budget: int, max_bodies: int, max_pairs: int):
    """Splits `pending` (an iterable of (request, simulation) in arrival order)
    into the requests of the next call and the rest.  A request joins if its
    simulation is not in the call yet and the call stays within max_bodies
    bodies, max_pairs of output pair capacity, 4096 problems and `budget`
    bytes of device memory (`needs[k]`: resident bytes plus library scratch
    of simulation k)."""
    batch, chosen, rest = [], set(), deque()
    bodies = need = caps = 0
    for req in pending:
        k = req[1]
        cap = pair_capacity(sizes[k])
        if (k not in chosen and bodies + sizes[k] <= max_bodies and caps + cap <= max_pairs and
                len(batch) < 4096 and need + needs[k] <= budget):
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
