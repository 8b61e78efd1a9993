"""The FP32 and FP64 pair screens (SYMBA_OPT_SCREEN) against the oracle (GPU).

The screen only decides which pairs get the exact FP64 encounter test, so
with either screen the pair list, the groups and the status must match the
oracle bit for bit, and the accelerations (which the screen never touches)
must be the same bits as with the FP64 screen.  The FP32 screen rejects only
pairs that the FP64 screen rejects too, so it passes at least as many
candidates.
"""
import numpy as np
import pytest

import oracle
from paper_2304_07325_amd import diskgen as dg
from tests import gpu_util as G
from tests.test_gpu_parity import _near_threshold_pairs, _tight_screen_pairs

pytestmark = pytest.mark.gpu

DT = dg.DT_HALF_YEAR
F = dg.RCRIT_FACTOR


@pytest.fixture(scope="module", params=["auto", "binned"])
def ctxs(request):
    """Two contexts with the same binning choice: FP64 screen and FP32 screen."""
    from paper_2304_07325_amd import binding as B
    c64 = B.Context(max_n=100_000, max_pairs=1 << 20)
    c32 = B.Context(max_n=100_000, max_pairs=1 << 20)
    c64.set_option(B.OPT_SCREEN, B.SCREEN_FP64)
    c32.set_option(B.OPT_SCREEN, B.SCREEN_FP32)
    if request.param == "binned":
        c64.set_option(B.OPT_BIN, 2)
        c32.set_option(B.OPT_BIN, 2)
    yield c64, c32
    c64.close()
    c32.close()


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


def both(ctxs, ora, s, n_m, label, pair_cap=None):
    """Runs the problem with both screens: the FP32 run must match the oracle
    exactly and carry the FP64 run's accelerations bit for bit."""
    c64, c32 = ctxs
    G.say("screen32", label, f"n={s['x'].size} n_m={n_m}")
    g64 = G.run_gpu(c64, s, n_m, DT, F, pair_cap=pair_cap)
    g32 = G.run_gpu(c32, s, n_m, DT, F, pair_cap=pair_cap)
    ref = ora.kick_encounter(s, n_m, DT, F)
    G.check_pairs_groups(g32, ref)
    G.check_pairs_groups(g64, ref)
    assert g32["acc"].tobytes() == g64["acc"].tobytes(), "the screen changed an acceleration"
    return g32, ref


@pytest.mark.parametrize("n,n_m", [(1, 0), (2, 2), (3, 1), (65, 64), (129, 40), (257, 256), (513, 100),
                                   (700, 699)])
def test_small_dense(ctxs, ora, n, n_m):
    both(ctxs, ora, G.dense_state(n, seed=2000 + n + n_m, n_m=n_m), n_m, "small dense")


@pytest.mark.parametrize("rows", [1, 2, 4])
def test_tile_sizes(ctxs, ora, rows):
    from paper_2304_07325_amd import binding as B
    for c in ctxs:
        c.set_option(B.OPT_TILE_ROWS, rows)
    try:
        for n, n_m in ((777, 776), (1100, 300)):
            both(ctxs, ora, G.dense_state(n, seed=11 * n + rows, box=3.0, n_m=n_m), n_m, f"rows={rows}")
    finally:
        for c in ctxs:
            c.set_option(B.OPT_TILE_ROWS, 0)


def test_near_threshold(ctxs, ora):
    s = _near_threshold_pairs(1500, seed=78, dt=DT)
    both(ctxs, ora, s, s["x"].size - 1, "near-threshold pairs")


@pytest.mark.parametrize("vscale", [0.0, 0.5, 1e3])
def test_tight_screen_moving_frame(ctxs, ora, vscale):
    """Pairs just outside the screen's reach in frames moving at up to 1e3
    times their relative speed: the expanded form cancels, and FP32 keeps far
    fewer digits than FP64, so this is where a missing margin would show."""
    s = _tight_screen_pairs(1200, seed=92, dt=DT, vscale=vscale)
    both(ctxs, ora, s, s["x"].size - 1, f"tight screen, frame speed x{vscale}")


@pytest.mark.parametrize("k", [0, 13])
def test_disk1k(ctxs, ora, k):
    w = dg.WORKLOADS["disk1k"]
    d = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    both(ctxs, ora, d.state(k), w["n_massive"], f"disk1k state {k}")


def test_disk10k(ctxs, ora):
    w = dg.WORKLOADS["disk10k"]
    d = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    both(ctxs, ora, d.state(7), w["n_massive"], "disk10k state 7")


def test_nonfinite_inputs(ctxs, ora):
    """Non-finite inputs make their pairs candidates under both screens."""
    s = G.dense_state(400, seed=18, box=2.0, n_m=300)
    s["x"][350] = np.inf
    s["vy"][77] = np.nan
    s["rh"][200] = np.inf
    s["vx"][120] = 1e300   # far beyond the FP32 range: its pairs must still be tested
    c64, c32 = ctxs
    G.say("screen32 non-finite and huge inputs")
    g64 = G.run_gpu(c64, s, 300, DT, F)
    g32 = G.run_gpu(c32, s, 300, DT, F)
    ref = ora.kick_encounter(s, 300, DT, F)
    for g in (g32, g64):
        assert g["status"] & 2
        assert np.array_equal(g["pair_i"], ref["pair_i"]) and np.array_equal(g["pair_j"], ref["pair_j"])
        assert np.array_equal(g["group_id"], ref["group_id"]) and g["n_groups"] == ref["n_groups"]
    assert g32["status"] == g64["status"]
    assert g32["acc"].tobytes() == g64["acc"].tobytes()


def test_fp32_screen_passes_a_superset(ctxs):
    """Candidates of the FP32 screen >= those of the FP64 screen (it rejects
    only what the FP64 screen rejects), and both cover every flagged pair."""
    c64, c32 = ctxs
    w = dg.WORKLOADS["disk10k"]
    s = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"]).state(2)
    G.say("screen32 candidate counts disk10k")
    c64.read_stats()
    c32.read_stats()
    r = G.run_gpu(c64, s, w["n_massive"], DT, F)
    G.run_gpu(c32, s, w["n_massive"], DT, F)
    cand64, flag64, _ = c64.read_stats()
    cand32, flag32, _ = c32.read_stats()
    assert flag64 == flag32 == r["n_pairs"]
    assert cand32 >= cand64 >= flag64
    print(f"disk10k candidates: FP64 screen {cand64}, FP32 screen {cand32}, flagged {flag64}")


def test_hot50k_full_size(ora):
    """The 50k hot disk with the FP32 screen (binned, as the library runs it
    at this size): every one of the 1.25e9 pairs tested by the oracle, the
    pair list and groups compared exactly."""
    from paper_2304_07325_amd import binding as B
    w = dg.WORKLOADS["hot50k"]
    d = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    s = d.state(5)
    n, n_m = w["n"], w["n_massive"]
    G.say("screen32 hot50k full size")
    c32 = B.Context(max_n=n, max_pairs=1 << 20)
    c32.set_option(B.OPT_SCREEN, B.SCREEN_FP32)
    gpu = G.run_gpu(c32, s, n_m, DT, F, pair_cap=1 << 20)
    c32.close()
    pi, pj = ora.pairs(s, n_m, DT, F)
    gid, ng = ora.groups(n, pi, pj)
    G.check_pairs_groups(gpu, dict(pair_i=pi, pair_j=pj, group_id=gid, n_groups=ng))
