"""Continuous batching over resident simulations (GPU): every request's
outputs are bit-identical to a single call on that simulation alone, with a
budget that holds everything and with one that forces evictions."""
import numpy as np
import pytest

import oracle
from paper_2304_07325_amd import diskgen as dg
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

DT = dg.DT_HALF_YEAR
F = dg.RCRIT_FACTOR


def _population():
    specs = [(300, 299, 41, 2.0), (1200, 1199, 42, 4.0), (2500, 250, 43, 4.0), (700, 699, 44, 1.5),
             (4200, 4199, 45, 6.0), (64, 63, 46, 0.5), (1800, 1799, 47, 3.0), (900, 90, 48, 3.0)]
    return [(G.dense_state(n, seed=s, box=b, n_m=nm), nm) for (n, nm, s, b) in specs]


def _alone(sims):
    from paper_2304_07325_amd import binding as B
    ctx = B.Context(max_n=max(s["x"].size for s, _ in sims), max_pairs=1 << 16)
    out = [G.run_gpu(ctx, s, nm, DT, F, pair_cap=max(4 * s["x"].size, 4096)) for s, nm in sims]
    ctx.close()
    return out


@pytest.mark.parametrize("budget", ["roomy", "tight"])
def test_served_outputs_match_single_calls(budget):
    from paper_2304_07325_amd.serve import Server
    sims = _population()
    ref = _alone(sims)
    ora = oracle.default()
    for (s, nm), r in zip(sims[:3], ref[:3]):
        G.check_pairs_groups(r, ora.kick_encounter(s, nm, DT, F))
    if budget == "roomy":
        limit = 1 << 34
    else:   # room for the largest simulation's step and little more: forces evictions
        probe = Server(sims, 1 << 34, DT, F)
        limit = probe.fixed_bytes + max(probe._need(k) for k in range(len(sims))) + 100_000
        probe.close()
    server = Server(sims, limit, DT, F)
    rng = np.random.default_rng(7)
    ids = rng.integers(0, len(sims), 60)
    t = np.sort(rng.uniform(0.0, 0.05, len(ids)))
    G.say("serve", budget, "budget", limit, "requests", len(ids))
    seen = {}

    def check(r, k, out):
        got = out.to_host()
        want = ref[k]
        assert got["acc"].tobytes() == want["acc"].tobytes(), f"request {r} (sim {k}): acc differs"
        assert np.array_equal(got["pair_i"], want["pair_i"]) and np.array_equal(got["pair_j"], want["pair_j"])
        assert np.array_equal(got["group_id"], want["group_id"]) and got["n_groups"] == want["n_groups"]
        assert got["status"] == want["status"]
        seen[r] = k

    stats = server.serve(t, ids, warmup=5, on_complete=check)
    assert len(seen) == len(ids)
    assert stats["requests"] == len(ids) - 5 and stats["latency_ms"]["p99"] >= stats["latency_ms"]["p50"] > 0
    if budget == "tight":
        assert stats["evictions"] > 0
    print(budget, stats)
    server.close()


def test_served_steps_match_stepping_alone():
    """Step mode under a budget that forces evictions: after the c-th request
    for a simulation, its state and accelerations are the same bits as after c
    steps of that simulation alone (evicted simulations are copied back and
    resume where they stopped)."""
    import torch
    from paper_2304_07325_amd import binding as B
    from paper_2304_07325_amd.serve import Server, pair_capacity
    specs = [(700, 699, 0.5), (300, 30, 0.2), (1500, 1499, 0.1), (65, 64, 1.0), (2000, 200, 0.3), (1100, 1099, 0.4)]
    sims = [(dg.make_disk(n, nm, "hot", 60 + k).state(0), nm) for k, (n, nm, _) in enumerate(specs)]
    h = 0.25 * dg.YEAR
    rng = np.random.default_rng(9)
    ids = rng.integers(0, len(sims), 40)
    t = np.sort(rng.uniform(0.0, 0.03, len(ids)))
    counts = np.bincount(ids, minlength=len(sims))
    G.say("serve step mode, requests", len(ids))
    # every simulation stepped alone, the states after 1..counts[k] steps kept
    want = []
    ctx = B.Context(max_n=max(n for n, _, _ in specs), max_pairs=1 << 16)
    for (s, nm), c in zip(sims, counts):
        st = B.to_device_state(s)
        out = B.Outputs(s["x"].size, pair_capacity(s["x"].size))
        ctx.kick_encounter(st, nm, h, F, out=out)
        seq = []
        for _ in range(c):
            ctx.step(st, nm, h, F, out)
            torch.cuda.synchronize()
            seq.append(({k: v.cpu().numpy() for k, v in st.items()}, out.to_host()))
        want.append(seq)
    ctx.close()
    probe = Server(sims, 1 << 34, h, F, mode="step")
    limit = probe.fixed_bytes + max(probe._need(k) for k in range(len(sims))) + 100_000
    probe.close()
    server = Server(sims, limit, h, F, mode="step")
    done = np.zeros(len(sims), dtype=int)

    def check(r, k, out):
        st, ref = want[k][done[k]]
        got = {key: v.cpu().numpy() for key, v in server.sims[k].dev.items()}
        for key in ("x", "y", "z", "vx", "vy", "vz"):
            assert got[key].tobytes() == st[key].tobytes(), f"request {r} (sim {k}, step {done[k] + 1}): {key}"
        g = out.to_host()
        assert g["acc"].tobytes() == ref["acc"].tobytes(), f"request {r}: acc differs"
        assert np.array_equal(g["pair_i"], ref["pair_i"]) and np.array_equal(g["group_id"], ref["group_id"])
        done[k] += 1

    stats = server.serve(t, ids, on_complete=check)
    assert (done == counts).all() and stats["evictions"] > 0
    print(stats)
    server.close()


def test_run_batch_on_a_side_stream():
    """Step mode driven through run_batch on a stream of its own, under a
    budget that evicts a simulation on every call and with no host
    synchronisation between calls: the evictions' copies, the uploads and the
    steps are ordered on that stream, so each simulation ends where stepping
    it alone ends."""
    import torch
    from paper_2304_07325_amd import binding as B
    from paper_2304_07325_amd.serve import Server, pair_capacity
    specs = [(600, 599), (300, 30), (900, 899), (450, 449)]
    sims = [(dg.make_disk(n, nm, "hot", 80 + k).state(0), nm) for k, (n, nm) in enumerate(specs)]
    h = 0.3 * dg.YEAR
    order = [0, 1, 2, 3, 0, 2, 1, 3, 3, 0, 2, 1, 0]
    G.say("run_batch on a side stream", len(order))
    want = []
    ctx = B.Context(max_n=max(n for n, _ in specs), max_pairs=1 << 16)
    for k, (s, nm) in enumerate(sims):
        st = B.to_device_state(s)
        out = B.Outputs(s["x"].size, pair_capacity(s["x"].size))
        ctx.kick_encounter(st, nm, h, F, out=out)
        for _ in range(order.count(k)):
            ctx.step(st, nm, h, F, out)
        torch.cuda.synchronize()
        want.append({key: v.cpu().numpy() for key, v in st.items()})
    ctx.close()
    probe = Server(sims, 1 << 34, h, F, mode="step")
    limit = probe.fixed_bytes + max(probe._need(k) for k in range(len(sims))) + 1000
    probe.close()
    server = Server(sims, limit, h, F, mode="step")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for k in order:
        server.run_batch([k], stream=side)
    torch.cuda.synchronize()
    assert server.evictions >= len(order) // 2   # most calls evict another simulation
    for k in range(len(sims)):
        if server.sims[k].dev is not None:
            got = {key: v.cpu().numpy() for key, v in server.sims[k].dev.items()}
        else:
            got = server.sims[k].state
        for key in ("x", "y", "z", "vx", "vy", "vz"):
            assert got[key].tobytes() == want[k][key].tobytes(), (k, key)
    server.close()


def test_overlapped_calls_match_single_calls():
    """Two calls in flight: a large simulation's call is running when
    requests for small ones arrive, so they go out on the second lane at
    once; a second request for the large simulation waits for its first call.
    Every output is the same bits as a single call on that simulation alone."""
    from paper_2304_07325_amd.serve import Server
    specs = [(30000, 29999, "cold", 90), (500, 499, "hot", 91), (800, 80, "cold", 92), (1200, 1199, "hot", 93),
             (300, 299, "cold", 94)]
    sims = [(dg.make_disk(n, nm, kind, seed).state(0), nm) for (n, nm, kind, seed) in specs]
    ref = _alone(sims)
    ids = [0, 1, 2, 3, 0, 4, 1, 0, 2, 3]
    t = [0.0, 1e-4, 2e-4, 3e-4, 4e-4, 5e-4, 6e-4, 7e-4, 8e-4, 9e-4]
    G.say("overlapped serving, requests", len(ids))
    server = Server(sims, 1 << 34, DT, F, lanes=2)
    server.preload()
    import torch
    torch.cuda.synchronize()
    seen = []

    def check(r, k, out):
        got = out.to_host()
        want = ref[k]
        assert got["acc"].tobytes() == want["acc"].tobytes(), f"request {r} (sim {k}): acc differs"
        assert np.array_equal(got["pair_i"], want["pair_i"]) and np.array_equal(got["pair_j"], want["pair_j"])
        assert np.array_equal(got["group_id"], want["group_id"]) and got["n_groups"] == want["n_groups"]
        seen.append(r)

    stats = server.serve(t, ids, on_complete=check)
    print(stats)
    assert sorted(seen) == list(range(len(ids)))
    assert stats["calls_issued_while_another_ran"] >= 1
    big = [r for r in seen if ids[r] == 0]
    assert big == sorted(big)
    server.close()
