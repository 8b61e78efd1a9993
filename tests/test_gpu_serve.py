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
