"""HIP path vs oracle, element by element (GPU).

Pairs, group labels and group counts must be bit-identical; accelerations
agree per body within 1e-12 normwise relative (conditioning-limited bodies
are checked against the exactly summed value instead, and counted).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2304_07325_amd import diskgen as dg
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

DT = dg.DT_HALF_YEAR
F = dg.RCRIT_FACTOR


@pytest.fixture(scope="module", params=["auto", "binned"])
def ctx(request):
    """A context with the default choice of spatial binning (by problem size)
    and one that bins every problem."""
    from paper_2304_07325_amd import binding as B
    c = B.Context(max_n=100_000, max_pairs=1 << 20)
    if request.param == "binned":
        c.set_option(B.OPT_BIN, 2)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


def compare(ctx, ora, s, n_m, dt=DT, f=F, label=""):
    n = s["x"].size
    G.say(label, f"n={n} n_m={n_m} dt={dt} f={f}")
    gpu = G.run_gpu(ctx, s, n_m, dt, f)
    ref = ora.kick_encounter(s, n_m, dt, f)
    G.check_pairs_groups(gpu, ref)
    err, limited = G.check_acc(s, n_m, gpu["acc"], ref["acc"])
    return gpu, ref, err, limited


@pytest.mark.parametrize("n,n_m", [(1, 0), (1, 1), (2, 1), (2, 2), (3, 0), (3, 1), (63, 62), (64, 64),
                                   (65, 64), (127, 126), (129, 40), (200, 199), (257, 256), (300, 1),
                                   (513, 100), (700, 699)])
def test_small_dense(ctx, ora, n, n_m):
    s = G.dense_state(n, seed=1000 + n + n_m, n_m=n_m)
    gpu, ref, err, lim = compare(ctx, ora, s, n_m, label="small_dense")
    if n > 50 and min(n_m, n - 1) > 1:
        assert len(ref["pair_i"]) > 0


@pytest.mark.parametrize("rows", [1, 2, 4])
@pytest.mark.parametrize("field_rows", [1, 2])
def test_tile_options(ctx, ora, rows, field_rows):
    from paper_2304_07325_amd import binding as B
    ctx.set_option(B.OPT_TILE_ROWS, rows)
    ctx.set_option(B.OPT_FIELD_ROWS, field_rows)
    try:
        for n, n_m in ((777, 776), (1100, 300), (530, 530)):
            if rows > 1 and n == 777:  # this case runs split block pairs (tile-pair tasks) at the end
                assert (B.plan_tasks(n, n_m, rows, field_rows)[:, 0] == 2).any()
            s = G.dense_state(n, seed=7 * n + rows, box=3.0, n_m=n_m)
            compare(ctx, ora, s, n_m, label=f"rows={rows} field_rows={field_rows}")
    finally:
        ctx.set_option(B.OPT_TILE_ROWS, 0)
        ctx.set_option(B.OPT_FIELD_ROWS, 0)


@pytest.mark.parametrize("k", [0, 1, 7, 19])
def test_disk1k(ctx, ora, k):
    w = dg.WORKLOADS["disk1k"]
    d = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    compare(ctx, ora, d.state(k), w["n_massive"], label=f"disk1k eval {k}")


@pytest.mark.parametrize("k", [0, 50])
def test_disk10k(ctx, ora, k):
    w = dg.WORKLOADS["disk10k"]
    d = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    gpu, ref, err, lim = compare(ctx, ora, d.state(k), w["n_massive"], label=f"disk10k eval {k}")
    print(f"disk10k eval {k}: max rel err {err:.2e}, conditioning-limited {lim}, pairs {gpu['n_pairs']}")


def test_field100k(ctx, ora):
    w = dg.WORKLOADS["field100k"]
    d = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    gpu, ref, err, lim = compare(ctx, ora, d.state(3), w["n_massive"], label="field100k")
    print(f"field100k: max rel err {err:.2e}, limited {lim}, pairs {gpu['n_pairs']}")


def test_repeat_is_bit_identical(ctx):
    w = dg.WORKLOADS["disk10k"]
    s = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"]).state(2)
    G.say("determinism disk10k")
    a = G.run_gpu(ctx, s, w["n_massive"], DT, F)
    for _ in range(3):
        b = G.run_gpu(ctx, s, w["n_massive"], DT, F)
        assert a["acc"].tobytes() == b["acc"].tobytes()
        assert np.array_equal(a["pair_i"], b["pair_i"]) and np.array_equal(a["group_id"], b["group_id"])


def test_capacity_overflow_keeps_groups(ctx, ora):
    s = G.dense_state(600, seed=5, box=1.0)
    ref = ora.kick_encounter(s, 599, DT, F)
    npairs = len(ref["pair_i"])
    assert npairs > 20
    G.say("capacity overflow", npairs)
    gpu = G.run_gpu(ctx, s, 599, DT, F, pair_cap=npairs - 1)
    assert gpu["status"] & 1
    assert gpu["n_pairs"] == npairs
    assert np.array_equal(gpu["group_id"], ref["group_id"]) and gpu["n_groups"] == ref["n_groups"]
    G.check_acc(s, 599, gpu["acc"], ref["acc"])
    ok = G.run_gpu(ctx, s, 599, DT, F, pair_cap=npairs)   # a retry with room succeeds
    G.check_pairs_groups(ok, ref)


def test_coincident_bodies_flag_nonfinite(ctx, ora):
    s = G.dense_state(100, seed=9)
    for c in ("x", "y", "z"):
        s[c][40] = s[c][7]
    G.say("coincident bodies")
    gpu = G.run_gpu(ctx, s, 99, DT, F)
    ref = ora.kick_encounter(s, 99, DT, F)
    assert gpu["status"] & 2
    assert np.array_equal(gpu["pair_i"], ref["pair_i"]) and np.array_equal(gpu["group_id"], ref["group_id"])
    ok = np.ones(100, bool)
    ok[[7, 40]] = False
    assert not np.isfinite(gpu["acc"][~ok]).all() and not np.isfinite(ref["acc"][~ok]).all()
    G.check_acc(s, 99, gpu["acc"][ok], ref["acc"][ok], bodies=np.nonzero(ok)[0])


def _near_threshold_pairs(n_pairs, seed, dt):
    """Pairs placed a few ulp either side of the encounter threshold in each
    regime (start, end of step, interior closest approach)."""
    rng = np.random.default_rng(seed)
    xs, vs, rhs = [], [], []
    for k in range(n_pairs):
        rh = rng.uniform(0.01, 0.05)
        rc = 3.0 * rh + 3.0 * rh
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        p = rng.normal(size=3); p -= p.dot(u) * u; p /= np.linalg.norm(p)
        regime = k % 3
        scale = 1.0 + rng.integers(-6, 7) * 2.0 ** -52
        if regime == 0:
            d = rc * scale * u
            w = 0.01 * u
        elif regime == 1:
            end = rc * scale * u
            w = rng.uniform(0.001, 0.05) * (-u + 0.3 * p)
            d = end - w * dt
        else:
            speed = rng.uniform(0.001, 0.1)
            d = rc * scale * p + speed * dt * rng.uniform(0.1, 0.9) * u
            w = -speed * u
        base = rng.uniform(-15, 15, 3)
        xs += [base, base + d]
        vs += [np.zeros(3), w]
        rhs += [rh, rh]
    X, V = np.array(xs), np.array(vs)
    return dict(x=X[:, 0].copy(), y=X[:, 1].copy(), z=X[:, 2].copy(), vx=V[:, 0].copy(),
                vy=V[:, 1].copy(), vz=V[:, 2].copy(), m=np.full(len(xs), 1e-9), rh=np.array(rhs))


def test_near_threshold_flags_exact(ctx, ora):
    s = _near_threshold_pairs(1500, seed=77, dt=DT)
    n = s["x"].size
    G.say("near-threshold pairs", n)
    gpu = G.run_gpu(ctx, s, n - 1, DT, F)
    ref = ora.kick_encounter(s, n - 1, DT, F)
    G.check_pairs_groups(gpu, ref)
    near = sum(1 for i, j in zip(ref["pair_i"], ref["pair_j"]) if j == i + 1 and i % 2 == 0)
    assert 200 < near < 1400, near   # a mix of flagged and unflagged threshold pairs


def test_accuracy_disk(ctx, ora):
    d = dg.make_accuracy_disk()
    for k in (0, 10):
        compare(ctx, ora, d.state(k), d.n_massive, dt=d.dt, f=F, label=f"accuracy disk {k}")


def _batch_specs():
    # (n, n_m, seed): all-massive and field-heavy problems, ragged sizes
    return [(1, 0, 1), (2, 1, 2), (65, 64, 3), (700, 699, 4), (300, 30, 5), (1500, 1499, 6),
            (129, 129, 7), (2000, 200, 8), (513, 512, 9), (64, 10, 10), (3001, 3000, 11), (900, 1, 12)]


@pytest.mark.parametrize("rows,binning", [(0, 0), (2, 0), (0, 2)])
def test_batch_matches_plain_and_oracle(ora, rows, binning):
    import torch
    from paper_2304_07325_amd import binding as B
    specs = _batch_specs()
    states = [G.dense_state(n, seed=s, box=4.0, n_m=nm) for (n, nm, s) in specs]
    total = sum(n for n, _, _ in specs)
    G.say("batch", len(specs), "problems", total, "bodies", "rows", rows, "binning", binning)
    ctx = B.Context(max_n=total, max_pairs=sum(max(4 * n, 4096) for n, _, _ in specs))
    ctx.set_option(B.OPT_TILE_ROWS, rows)
    ctx.set_option(B.OPT_BIN, binning)
    dev = [B.to_device_state(s) for s in states]
    outs = [B.Outputs(n, max(4 * n, 4096)) for n, _, _ in specs]
    probs = [(d, nm, DT, F, o) for d, (n, nm, _), o in zip(dev, specs, outs)]
    for rep in range(2):           # the second call reuses the uploaded descriptors
        ctx.kick_encounter_batch(probs)
        torch.cuda.synchronize()
        got = [o.to_host() for o in outs]
        for (n, nm, _), s, g in zip(specs, states, got):
            ref = ora.kick_encounter(s, nm, DT, F)
            G.check_pairs_groups(g, ref)
            G.check_acc(s, nm, g["acc"], ref["acc"])
    # every problem gets the tile size a single call gives it, so its results
    # are bit-identical to the plain call's whatever else is in the batch
    plain_ctx = B.Context(max_n=max(n for n, _, _ in specs), max_pairs=1 << 16)
    plain_ctx.set_option(B.OPT_TILE_ROWS, rows)
    plain_ctx.set_option(B.OPT_BIN, binning)
    for (n, nm, _), d, g in zip(specs, dev, got):
        p = G.run_gpu(plain_ctx, {k: v.cpu().numpy() for k, v in d.items()}, nm, DT, F)
        assert p["acc"].tobytes() == g["acc"].tobytes(), "batched acc differs from the plain call"
    plain_ctx.close()
    ctx.close()


def test_batch_graph_replays_match_eager(ora):
    """A batched step captured in a HIP graph: every replay, with eager calls
    in between, gives the eager call's outputs bit for bit."""
    import torch
    from paper_2304_07325_amd import binding as B
    specs = [(900, 899, 31), (1500, 150, 32), (4100, 4099, 33), (300, 299, 34)]
    states = [G.dense_state(n, seed=s, box=4.0, n_m=nm) for (n, nm, s) in specs]
    total = sum(n for n, _, _ in specs)
    G.say("graph replay of a batch", specs)
    ctx = B.Context(max_n=total, max_pairs=1 << 18)
    dev = [B.to_device_state(s) for s in states]
    outs = [B.Outputs(n, 1 << 15) for n, _, _ in specs]
    probs = [(d, nm, DT, F, o) for d, (n, nm, _), o in zip(dev, specs, outs)]
    ctx.kick_encounter_batch(probs)
    torch.cuda.synchronize()
    eager = [o.to_host() for o in outs]
    for (n, nm, _), s, e in zip(specs, states, eager):
        G.check_pairs_groups(e, ora.kick_encounter(s, nm, DT, F))
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        ctx.kick_encounter_batch(probs, stream=stream)
    for rep in range(3):
        for o in outs:
            o.acc.zero_()
            o.group_id.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        for e, o in zip(eager, outs):
            g = o.to_host()
            assert g["acc"].tobytes() == e["acc"].tobytes(), f"replay {rep}: acc differs"
            assert np.array_equal(g["pair_i"], e["pair_i"]) and np.array_equal(g["pair_j"], e["pair_j"])
            assert np.array_equal(g["group_id"], e["group_id"]) and g["n_groups"] == e["n_groups"]
            assert g["status"] == e["status"]
        ctx.kick_encounter_batch(probs)   # eager work between replays
        torch.cuda.synchronize()
    ctx.close()


def _tight_screen_pairs(n_pairs, seed, dt, vscale):
    """Head-on pairs for which the screen's reach bound is tight
    (rc_i = rc_j = |w| dt / 2), the end-of-step separation a few ulp either
    side of rc, all moving with a common velocity up to `vscale` (the screen's
    expanded velocity term cancels there)."""
    rng = np.random.default_rng(seed)
    xs, vs, rhs = [], [], []
    for k in range(n_pairs):
        rh = rng.uniform(0.01, 0.05)
        c = F * rh
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        speed = 2.0 * c / dt
        s = 1.0 + rng.integers(-8, 9) * 2.0 ** -50
        d = -(2.0 * c * s + speed * dt) * u
        common = rng.normal(size=3) * vscale
        base = rng.uniform(-15, 15, 3)
        xs += [base, base + d]
        vs += [common, common + speed * u]
        rhs += [rh, rh]
    X, V = np.array(xs), np.array(vs)
    return dict(x=X[:, 0].copy(), y=X[:, 1].copy(), z=X[:, 2].copy(), vx=V[:, 0].copy(),
                vy=V[:, 1].copy(), vz=V[:, 2].copy(), m=np.full(len(xs), 1e-9), rh=np.array(rhs))


@pytest.mark.parametrize("vscale", [0.0, 0.5, 1e3])
def test_tight_screen_moving_frame(ctx, ora, vscale):
    s = _tight_screen_pairs(1200, seed=91, dt=DT, vscale=vscale)
    n = s["x"].size
    G.say("tight-screen pairs", n, "common velocity scale", vscale)
    gpu = G.run_gpu(ctx, s, n - 1, DT, F)
    ref = ora.kick_encounter(s, n - 1, DT, F)
    G.check_pairs_groups(gpu, ref)
    near = sum(1 for i, j in zip(ref["pair_i"], ref["pair_j"]) if j == i + 1 and i % 2 == 0)
    assert 100 < near < 1100, near


def test_batch_crowded_problems(ora):
    """Crowded problems in a batch: tens of thousands of flagged pairs, so the
    per-wave candidate queues fill up and are drained inside the tasks, and
    one encounter group spans almost every body."""
    import torch
    from paper_2304_07325_amd import binding as B
    specs = [(400, 399, 21, 0.3), (500, 50, 22, 4.0), (300, 299, 23, 0.2)]
    states = [G.dense_state(n, seed=s, box=b, n_m=nm) for (n, nm, s, b) in specs]
    total = sum(n for n, _, _, _ in specs)
    refs = [ora.kick_encounter(s, nm, DT, F) for s, (n, nm, _, _) in zip(states, specs)]
    assert len(refs[0]["pair_i"]) > 20000
    G.say("batch of crowded problems", [len(r["pair_i"]) for r in refs])
    ctx = B.Context(max_n=total, max_pairs=1 << 18)
    dev = [B.to_device_state(s) for s in states]
    outs = [B.Outputs(n, 1 << 16) for n, _, _, _ in specs]
    ctx.kick_encounter_batch([(d, nm, DT, F, o) for d, (n, nm, _, _), o in zip(dev, specs, outs)])
    torch.cuda.synchronize()
    for (n, nm, _, _), s, o, ref in zip(specs, states, outs, refs):
        g = o.to_host()
        G.check_pairs_groups(g, ref)
        G.check_acc(s, nm, g["acc"], ref["acc"])
    ctx.close()


@pytest.fixture(scope="module")
def hot50k_ref(ora):
    """The oracle's whole step on one state of the 50k-body hot disk (every
    one of the 1.25e9 pairs: accelerations, pair list, groups), computed once
    for both contexts."""
    w = dg.WORKLOADS["hot50k"]
    d = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    s = d.state(3)
    return s, ora.kick_encounter(s, w["n_massive"], DT, F, cap=1 << 20)


def test_hot50k_full_size(ctx, hot50k_ref):
    """The 50k-body hot disk at full size, as the library runs it: the pair
    list compared entry by entry with the oracle's, the groups with the
    oracle's connected components of that list, and every one of the 50000
    accelerations with the oracle's (per body, normwise, 1e-12)."""
    w = dg.WORKLOADS["hot50k"]
    s, ref = hot50k_ref
    n, n_m = w["n"], w["n_massive"]
    G.say("hot50k full size")
    gpu = G.run_gpu(ctx, s, n_m, DT, F, pair_cap=1 << 20)
    G.check_pairs_groups(gpu, ref)
    err, lim = G.check_acc(s, n_m, gpu["acc"], ref["acc"])
    rel = np.linalg.norm(gpu["acc"] - ref["acc"], axis=1) / np.linalg.norm(ref["acc"], axis=1)
    print(f"hot50k: pairs {len(ref['pair_i'])}, groups {ref['n_groups']}, acc rel err max {err:.2e} "
          f"p99 {np.percentile(rel, 99):.2e} median {np.median(rel):.2e}, conditioning-limited {lim}")


def test_autotune_chooses_a_size_and_stays_exact(ora):
    """The autotuner times every tile size and tail split, keeps one plan for
    the size class, and the outputs of its final call and of a later call of
    the same size are bit-identical and match the oracle."""
    from paper_2304_07325_amd import binding as B
    s = G.dense_state(3000, seed=61, box=6.0)
    G.say("autotune n=3000")
    ctx = B.Context(max_n=4096, max_pairs=1 << 16)
    dev = B.to_device_state(s)
    out = B.Outputs(3000, 1 << 15)
    rows = ctx.autotune(dev, 2999, DT, F, out=out)
    assert rows in (1, 2, 4)
    plan_rows, split = ctx.plan_for(3000, 2999)
    assert plan_rows == rows and 0 <= split <= 3 and (rows > 1 or split == 0)
    assert ctx.plan_for(2500, 2499) == (rows, split)     # the same size class
    tuned = out.to_host()
    ref = ora.kick_encounter(s, 2999, DT, F)
    G.check_pairs_groups(tuned, ref)
    G.check_acc(s, 2999, tuned["acc"], ref["acc"])
    again = G.run_gpu(ctx, s, 2999, DT, F, pair_cap=1 << 15)
    assert again["acc"].tobytes() == tuned["acc"].tobytes()
    forced = B.Context(max_n=4096, max_pairs=1 << 16)
    forced.set_option(B.OPT_TILE_ROWS, rows)
    forced.set_option(B.OPT_SPLIT, split)
    assert G.run_gpu(forced, s, 2999, DT, F, pair_cap=1 << 15)["acc"].tobytes() == tuned["acc"].tobytes()
    forced.close()
    ctx.close()


@pytest.mark.parametrize("rows", [2, 4])
def test_every_tail_split_is_exact(ora, rows):
    """The fold schedule with 0 to 3 split diagonals (SYMBA_OPT_SPLIT): the
    plan reports what the fold allows, every schedule matches the oracle, and
    a batch with the same forced schedule gives each problem its single
    call's bits."""
    import torch
    from paper_2304_07325_amd import binding as B
    s = G.dense_state(3000, seed=62, box=6.0)
    s2 = G.dense_state(1400, seed=63, box=4.0)
    ref = ora.kick_encounter(s, 2999, DT, F)
    for D in range(4):
        G.say("tail split", rows, D)
        ctx = B.Context(max_n=4400, max_pairs=1 << 16)
        ctx.set_option(B.OPT_TILE_ROWS, rows)
        ctx.set_option(B.OPT_SPLIT, D)
        assert ctx.plan_for(3000, 2999) == (rows, D)
        got = G.run_gpu(ctx, s, 2999, DT, F, pair_cap=1 << 14)
        G.check_pairs_groups(got, ref)
        G.check_acc(s, 2999, got["acc"], ref["acc"])
        alone2 = G.run_gpu(ctx, s2, 1399, DT, F, pair_cap=1 << 14)
        sts = [B.to_device_state(s), B.to_device_state(s2)]
        outs = [B.Outputs(3000, 1 << 14), B.Outputs(1400, 1 << 14)]
        ctx.kick_encounter_batch([(sts[0], 2999, DT, F, outs[0]), (sts[1], 1399, DT, F, outs[1])])
        torch.cuda.synchronize()
        assert outs[0].to_host()["acc"].tobytes() == got["acc"].tobytes()
        assert outs[1].to_host()["acc"].tobytes() == alone2["acc"].tobytes()
        ctx.close()
    ctx = B.Context(max_n=64)
    for bad in (-2, 9):
        with pytest.raises(Exception):
            ctx.set_option(B.OPT_SPLIT, bad)
    ctx.close()


def test_screen_statistics(ctx):
    """symba_read_stats: the screen passes at least every flagged pair, and the
    counts cover the problems evaluated since the last read."""
    w = dg.WORKLOADS["disk1k"]
    s = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"]).state(4)
    G.say("screen statistics disk1k")
    ctx.read_stats()
    res = [G.run_gpu(ctx, s, w["n_massive"], DT, F) for _ in range(3)]
    cands, flagged, probs = ctx.read_stats()
    assert probs == 3
    assert flagged == 3 * res[0]["n_pairs"]
    assert cands >= flagged
    assert ctx.read_stats() == (0, 0, 0)


def test_nonfinite_inputs_match_oracle(ctx, ora):
    """A field body at an infinite position, a massive body with a NaN
    velocity and one with an infinite Hill radius: the flagged pairs and
    groups still match the oracle exactly (the screen passes non-finite pairs
    on to the exact test), the status reports the non-finite acceleration
    (the infinite field body's), and every finite acceleration is exact."""
    s = G.dense_state(400, seed=17, box=2.0, n_m=300)
    s["x"][350] = np.inf
    s["vy"][77] = np.nan
    s["rh"][200] = np.inf
    G.say("non-finite inputs")
    gpu = G.run_gpu(ctx, s, 300, DT, F)
    ref = ora.kick_encounter(s, 300, DT, F)
    assert gpu["status"] & 2
    assert np.array_equal(gpu["pair_i"], ref["pair_i"]) and np.array_equal(gpu["pair_j"], ref["pair_j"])
    assert np.array_equal(gpu["group_id"], ref["group_id"]) and gpu["n_groups"] == ref["n_groups"]
    fin = np.isfinite(ref["acc"]).all(axis=1)
    assert fin.sum() == 399 and not np.isfinite(gpu["acc"][350]).all()
    G.check_acc(s, 300, gpu["acc"][fin], ref["acc"][fin], bodies=np.nonzero(fin)[0])
