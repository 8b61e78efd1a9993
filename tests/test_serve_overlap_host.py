"""The serving loop with several calls in flight, driven on the CPU through a
stand-in for the device side whose calls complete at random later times.

The stand-in keeps its own record of which simulations each running call
holds and fails the test if the server evicts or reloads such a simulation,
puts it into a second call, or hands out a result before its call completed.
"""
import time

import numpy as np
import pytest

from paper_2304_07325_amd import serve as S


class _Token:
    def __init__(self, ready_at, ids):
        self.ready_at = ready_at
        self.ids = ids


class FakeIO:
    """Device side with calls that take `min_s`..`max_s` seconds of wall time."""

    def __init__(self, seed, min_s=2e-4, max_s=3e-3):
        self.rng = np.random.default_rng(seed)
        self.min_s, self.max_s = min_s, max_s
        self.inflight = {}        # token id -> set of simulation ids
        self.resident = set()
        self.max_inflight = 0
        self.evicted_busy = self.reloaded_busy = self.rebatched = 0
        self.polls = 0
        self.loads = self.evicts = 0
        self.completed = set()    # token ids observed complete

    def _busy(self):
        return set().union(*self.inflight.values()) if self.inflight else set()

    def scratch_bytes(self, n, n_m):
        return 40 * n + 4096

    def load(self, s, lane, stream=None):
        if id(s) in self._busy():
            self.reloaded_busy += 1
        assert id(s) not in self.resident
        self.resident.add(id(s))
        self.loads += 1
        s.dev, s.out = {"sim": id(s)}, {"calls": 0}

    def evict(self, s, stream=None):
        if id(s) in self._busy():
            self.evicted_busy += 1
        self.resident.discard(id(s))
        self.evicts += 1
        s.dev = s.out = None

    def issue(self, lane, sims, stream=None):
        ids = {id(s) for s in sims}
        assert all(i in self.resident for i in ids), "a simulation of the call is not resident"
        if ids & self._busy():
            self.rebatched += 1
        for s in sims:
            s.out["calls"] += 1
        tok = _Token(time.monotonic() + self.rng.uniform(self.min_s, self.max_s), ids)
        self.inflight[id(tok)] = ids
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        return tok

    def done(self, tok):
        self.polls += 1
        if time.monotonic() >= tok.ready_at:
            self.inflight.pop(id(tok), None)
            self.completed.add(id(tok))
            return True
        return False

    def close(self):
        pass


def _sims(sizes):
    return [({"x": np.zeros(n)}, n) for n in sizes]


def _server(io, sizes, budget, lanes=2, mode="evaluate"):
    return S.Server(_sims(sizes), budget, 1.0, 3.5, max_batch_bodies=max(sizes) * 4, mode=mode, lanes=lanes, io=io)


def _replay(srv, io, n_req, rate, seed):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_req))
    ids = rng.integers(0, len(srv.sims), n_req)
    served = []

    def on_complete(r, k, out):
        # the call that served r has completed (its token was observed done),
        # and the simulation is still held by it
        assert k in srv.busy
        assert not any(id(srv.sims[k]) in held for held in io.inflight.values())
        served.append((r, k))

    t0 = time.monotonic()
    stats = srv.serve(t, ids, on_complete=on_complete)
    return stats, served, ids, time.monotonic() - t0


@pytest.mark.parametrize("lanes", [2, 3])
def test_running_calls_hold_their_simulations(lanes):
    sizes = [int(x) for x in np.random.default_rng(1).integers(50, 400, 24)]
    io = FakeIO(seed=2)
    probe = _server(FakeIO(0), sizes, 1 << 40, lanes=lanes)
    # room for a few simulations only: evictions happen while other calls run
    budget = probe.fixed_bytes + 4 * max(probe._need(k) for k in range(len(sizes)))
    srv = _server(io, sizes, budget, lanes=lanes)
    stats, served, ids, _ = _replay(srv, io, 600, rate=4000.0, seed=3)
    assert io.evicted_busy == 0 and io.reloaded_busy == 0 and io.rebatched == 0
    assert stats["evictions"] > 0
    assert io.max_inflight >= 2 and stats["calls_issued_while_another_ran"] > 0
    assert io.max_inflight <= lanes
    # every request served exactly once, and a simulation's requests in arrival order
    assert sorted(r for r, _ in served) == list(range(len(ids)))
    assert all(ids[r] == k for r, k in served)
    for k in range(len(sizes)):
        mine = [r for r, kk in served if kk == k]
        assert mine == sorted(mine)
    assert not srv.busy and not io.inflight


def test_budget_reserves_running_calls():
    """With a budget that holds one call's simulations only, a second call
    waits for the first: nothing the first holds is evicted for it."""
    sizes = [300] * 6
    io = FakeIO(seed=5)
    probe = _server(FakeIO(0), sizes, 1 << 40)
    budget = probe.fixed_bytes + probe._need(0) + 10
    srv = _server(io, sizes, budget)
    stats, served, ids, _ = _replay(srv, io, 200, rate=3000.0, seed=6)
    assert io.max_inflight == 1 and io.evicted_busy == 0 and io.rebatched == 0
    assert sorted(r for r, _ in served) == list(range(len(ids)))
    assert stats["calls"] == len(ids)    # one simulation per call: nothing else fits


def test_polling_is_paced():
    """Waiting for completions sleeps between polls: polls stay within the
    number of loop passes that the sleeps allow, far below a busy loop."""
    sizes = [200] * 4
    io = FakeIO(seed=8, min_s=2e-3, max_s=4e-3)
    srv = _server(io, sizes, 1 << 40)
    stats, served, ids, elapsed = _replay(srv, io, 120, rate=500.0, seed=9)
    passes_with_work = 2 * stats["calls"] + len(ids)
    assert io.polls <= srv.n_lanes * (passes_with_work + elapsed / S.POLL_SLEEP_S)
    assert len(served) == len(ids)


def test_one_lane_runs_one_call_at_a_time():
    sizes = [100, 150, 200, 250]
    io = FakeIO(seed=11)
    srv = _server(io, sizes, 1 << 40, lanes=1)
    stats, served, ids, _ = _replay(srv, io, 150, rate=5000.0, seed=12)
    assert io.max_inflight == 1 and stats["calls_issued_while_another_ran"] == 0
    assert sorted(r for r, _ in served) == list(range(len(ids)))


def test_pick_batch_skips_running_simulations():
    from collections import deque
    pending = deque([(0, 1), (1, 2), (2, 3), (3, 1)])
    batch, rest = S.pick_batch(pending, [10] * 4, [1] * 4, 10**9, 10**9, 10**9, exclude={1, 3})
    assert batch == [(1, 2)] and list(rest) == [(0, 1), (2, 3), (3, 1)]


def test_evicting_a_running_simulation_is_refused():
    io = FakeIO(seed=0)
    srv = _server(io, [100, 100], 1 << 40)
    srv._prepare([0], 0)
    srv.busy[0] = 0
    with pytest.raises(AssertionError):
        srv._evict(0)
    srv._make_room(1 << 50, keep=set())   # cannot make room: the running simulation stays
    assert 0 in srv.lru and io.evicts == 0
