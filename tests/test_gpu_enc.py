"""symba_step_enc (GPU) against the encounter-step oracle: one step at a time
from the oracle's own inputs (state, level-0 accelerations, flagged pairs),
so rounding differences cannot grow over many steps, on a fast flyby through
several shells, three separate flybys (three groups in parallel), a
crowded cluster (a group of 89 pairs) and a cold disk with nothing flagged (bit-identical to symba_step); the status bit
and the plain step for a group over the size limit; time reversal on the
device."""
import math

import numpy as np
import pytest

import oracle
from oracle import symba_enc as E
from paper_2304_07325_amd import diskgen as dg
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

F = 3.0
KEYS = ("x", "y", "z", "vx", "vy", "vz")
# One step's positions and velocities agree to 1e-11 of their scale: both
# sides compute in FP64, the device with fused multiply-adds and its own
# Kepler solver (Laguerre-Conway on Danby's variable against Newton on
# Curtis' universal anomaly, each converged to ~1e-15), through up to a few
# hundred substeps, each a few ulp, amplified by the encounter's shear.
STATE_TOL = 1e-11
ACC_TOL = 1e-11


def _state(x, v_helio, m):
    x, v, m = (np.asarray(a, dtype=np.float64) for a in (x, v_helio, m))
    vb = v - (m[:, None] * v).sum(0) / (1.0 + m.sum())
    rh = (m / 3.0) ** (1.0 / 3.0) * np.linalg.norm(x, axis=1)
    return dict(x=x[:, 0].copy(), y=x[:, 1].copy(), z=x[:, 2].copy(), vx=vb[:, 0].copy(), vy=vb[:, 1].copy(),
                vz=vb[:, 2].copy(), m=m.copy(), rh=rh)


def _flyby(phase=0.0, b=0.003, vrel=0.3, sep=0.3, mA=1e-4, mB=3e-5):
    c, s = math.cos(phase), math.sin(phase)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    x = np.array([[1.0, 0.0, 0.0], [1.0 + b, -sep, 0.0]]) @ rot.T
    v = np.array([[0.0, 1.0, 0.0], [0.0, 1.0 + vrel, 0.0]]) @ rot.T
    return x, v, np.array([mA, mB])


class Dev:
    """A device state and outputs on one context."""

    def __init__(self, n, pair_cap=None):
        import torch
        from paper_2304_07325_amd import binding as B
        self.B, self.torch, self.n = B, torch, n
        self.ctx = B.Context(max_n=max(n, 64), max_pairs=1 << 16)
        self.out = B.Outputs(n, pair_cap or max(4 * n, 4096))

    def load(self, s, acc=None, pairs=None, ora=None):
        """Uploads state s; with acc and pairs, also the outputs a step reads
        (level-0 accelerations, pairs, their groups, status 0)."""
        t = self.torch
        self.st = self.B.to_device_state(s)
        if acc is not None:
            pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
            gid, ng = ora.groups(self.n, pairs[:, 0], pairs[:, 1])
            self.out.acc.copy_(t.from_numpy(np.ascontiguousarray(acc.T)))
            k = len(pairs)
            self.out.pair_i[:k].copy_(t.from_numpy(pairs[:, 0].astype(np.int32)))
            self.out.pair_j[:k].copy_(t.from_numpy(pairs[:, 1].astype(np.int32)))
            self.out.scalars64.fill_(k)
            self.out.group_id.copy_(t.from_numpy(gid))
            self.out.scalars32.copy_(t.tensor([ng, 0], dtype=t.int32))

    def state(self):
        self.torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in self.st.items()}

    def close(self):
        self.ctx.close()


def _compare_step(dev, ora, s, n_m, h, acc, pairs):
    """One device step from the oracle's inputs against the oracle's step."""
    want, acc_w, pairs_w = E.step(s, n_m, h, F, acc, pairs, ora=ora)
    dev.load(s, acc, pairs, ora)
    dev.ctx.step_enc(dev.st, n_m, h, F, dev.out)
    got = dev.state()
    out = dev.out.to_host()
    # each vector measured against its own size (a thin disk's z components
    # are far smaller than its in-plane ones)
    pscale = max(np.abs(want[k]).max() for k in ("x", "y", "z")) + 1.0
    vscale = max(np.abs(want[k]).max() for k in ("vx", "vy", "vz"))
    for k in KEYS:
        scale = pscale if k in ("x", "y", "z") else vscale
        assert np.abs(got[k] - want[k]).max() <= STATE_TOL * scale, (k, np.abs(got[k] - want[k]).max())
    assert out["status"] == 0
    assert np.array_equal(np.stack([out["pair_i"], out["pair_j"]], 1), pairs_w)
    # measured against the Newtonian sums: deep inside R_0 the level-0 force
    # of a pair is zero, and its accelerations cancel to rounding
    scale = np.abs(ora.accel(want, n_m)).max()
    assert np.abs(out["acc"] - acc_w).max() <= ACC_TOL * scale
    return want, acc_w, pairs_w


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


def test_flyby_step_by_step(ora):
    x, v, m = _flyby()
    s = _state(x, v, m)
    h = 0.025
    acc, pairs = E.prepare(s, 2, h, F, ora=ora)
    dev = Dev(2)
    G.say("flyby, 40 steps")
    deepest = 0
    for k in range(40):
        s, acc, pairs = _compare_step(dev, ora, s, 2, h, acc, pairs)
        d = np.linalg.norm([s["x"][1] - s["x"][0], s["y"][1] - s["y"][0]])
        r0 = F * s["rh"].sum()
        while deepest < E.L_MAX and d < E.shell_radius(r0, deepest + 1):
            deepest += 1
    assert deepest >= 3   # the flyby went through several shells
    dev.close()


def test_three_groups_in_parallel(ora):
    xs, vs, ms = zip(*(_flyby(phase=p, sep=0.15) for p in (0.0, 2.1, 4.2)))
    s = _state(np.concatenate(xs), np.concatenate(vs), np.concatenate(ms))
    h = 0.025
    acc, pairs = E.prepare(s, 6, h, F, ora=ora)
    dev = Dev(6)
    G.say("three flybys, 16 steps")
    for _ in range(16):
        assert len(pairs) == 3
        s, acc, pairs = _compare_step(dev, ora, s, 6, h, acc, pairs)
    dev.close()


def _cluster(n=40, spread=0.08, seed=12):
    """A crowded patch of Earth-mass bodies near 1 AU: 90 flagged pairs in a
    group of 89 pairs and one of 1."""
    rng = np.random.default_rng(seed)
    x = np.c_[1.0 + rng.normal(0, spread, n), rng.normal(0, spread, n), rng.normal(0, spread / 5, n)]
    r = np.linalg.norm(x[:, :2], axis=1)
    v = np.c_[-x[:, 1], x[:, 0], np.zeros(n)] / r[:, None] ** 1.5 + rng.normal(0, 0.01, (n, 3))
    return _state(x, v, np.full(n, 3e-6))


def test_crowded_cluster(ora):
    """Groups of many pairs (89 and 1), each resolved by one workgroup."""
    s = _cluster()
    n = s["x"].size
    h = 0.01
    acc, pairs = E.prepare(s, n, h, F, ora=ora)
    assert len(pairs) >= 60
    dev = Dev(n)
    G.say("crowded cluster, 5 steps")
    for _ in range(5):
        s, acc, pairs = _compare_step(dev, ora, s, n, h, acc, pairs)
    dev.close()


def test_prepare_matches_the_oracle(ora):
    s = _cluster()
    n = s["x"].size
    h = 0.01
    acc, pairs = E.prepare(s, n, h, F, ora=ora)
    dev = Dev(n)
    dev.load(s)
    dev.ctx.enc_prepare(dev.st, n, h, F, dev.out)
    out = dev.out.to_host()
    assert np.array_equal(np.stack([out["pair_i"], out["pair_j"]], 1), pairs)
    assert np.abs(out["acc"] - acc).max() <= ACC_TOL * np.abs(ora.accel(s, n)).max()
    assert out["status"] == 0
    # the reweighting changed what the plain evaluation gives
    plain = ora.kick_encounter(s, n, h, F)["acc"]
    assert np.abs(out["acc"] - plain).max() > 1e-6 * np.abs(plain).max()
    dev.close()


def _cold_ring(n=60, seed=5):
    rng = np.random.default_rng(seed)
    a = np.sort(rng.uniform(5.0, 20.0, n))
    th = rng.uniform(0, 2 * np.pi, n)
    x = np.c_[a * np.cos(th), a * np.sin(th), np.zeros(n)]
    v = np.c_[-np.sin(th), np.cos(th), np.zeros(n)] / np.sqrt(a)[:, None]
    return _state(x, v, np.full(n, 1e-9))


def test_nothing_flagged_is_the_plain_step_bitwise():
    s = _cold_ring()
    n = s["x"].size
    h = 0.5 * dg.YEAR
    plain, enc = Dev(n), Dev(n)
    plain.load(s)
    enc.load(s)
    plain.ctx.kick_encounter(plain.st, n, abs(h), F, out=plain.out)
    enc.ctx.enc_prepare(enc.st, n, h, F, enc.out)
    G.say("cold ring, 4 steps, plain vs encounter step")
    for _ in range(4):
        plain.ctx.step(plain.st, n, h, F, plain.out)
        enc.ctx.step_enc(enc.st, n, h, F, enc.out)
        a, b = plain.state(), enc.state()
        assert plain.out.to_host()["n_pairs"] == 0 and enc.out.to_host()["n_pairs"] == 0
        for k in KEYS:
            assert a[k].tobytes() == b[k].tobytes(), k
        assert plain.out.to_host()["acc"].tobytes() == enc.out.to_host()["acc"].tobytes()
    plain.close()
    enc.close()


def test_group_over_the_limit_takes_the_plain_step():
    """A tight cluster whose one group has more than 255 pairs: the status
    reports it and the step is the plain step, bit for bit."""
    rng = np.random.default_rng(11)
    n = 40
    x = np.c_[1.0 + rng.normal(0, 0.01, n), rng.normal(0, 0.01, n), rng.normal(0, 0.002, n)]
    v = np.c_[-x[:, 1], x[:, 0], np.zeros(n)]
    s = _state(x, v, np.full(n, 3e-6))
    h = 0.01
    plain, enc = Dev(n), Dev(n)
    plain.load(s)
    enc.load(s)
    plain.ctx.kick_encounter(plain.st, n, abs(h), F, out=plain.out)
    enc.ctx.enc_prepare(enc.st, n, h, F, enc.out)
    first = enc.out.to_host()
    assert first["n_pairs"] > 255 and first["n_groups"] == 1
    assert first["status"] & enc.B.STATUS_ENC_SKIPPED
    plain.ctx.step(plain.st, n, h, F, plain.out)
    enc.ctx.step_enc(enc.st, n, h, F, enc.out)
    a, b = plain.state(), enc.state()
    for k in KEYS:
        assert a[k].tobytes() == b[k].tobytes(), k
    assert enc.out.to_host()["status"] & enc.B.STATUS_ENC_SKIPPED
    plain.close()
    enc.close()


def test_time_reversal_on_the_device():
    x, v, m = _flyby(sep=0.12)
    s = _state(x, v, m)
    h = 0.025
    dev = Dev(2)
    dev.load(s)
    dev.ctx.enc_prepare(dev.st, 2, h, F, dev.out)
    for _ in range(20):
        dev.ctx.step_enc(dev.st, 2, h, F, dev.out)
    mid = dev.state()
    for k in ("vx", "vy", "vz"):
        dev.st[k].neg_()
    dev.ctx.enc_prepare(dev.st, 2, h, F, dev.out)
    for _ in range(20):
        dev.ctx.step_enc(dev.st, 2, h, F, dev.out)
    back = dev.state()
    assert np.abs(mid["x"] - s["x"]).max() > 0.05   # it moved
    for k in ("x", "y", "z"):
        assert np.abs(back[k] - s[k]).max() < 1e-11, k
    for k in ("vx", "vy", "vz"):
        assert np.abs(-back[k] - s[k]).max() < 1e-11, k
    dev.close()


def test_graph_replays_match_eager_steps():
    """Encounter steps captured into a graph: each replay gives the bits of the
    same number of eager steps (run on a second context and state), with
    eager work on the captured context between the replays."""
    import torch
    x, v, m = _flyby(sep=0.15)   # inside the critical radius for all nine steps
    s = _state(x, v, m)
    h = 0.025
    eager, graphed = Dev(2), Dev(2)
    eager.load(s)
    graphed.load(s)
    eager.ctx.enc_prepare(eager.st, 2, h, F, eager.out)
    graphed.ctx.enc_prepare(graphed.st, 2, h, F, graphed.out)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for _ in range(3):
            graphed.ctx.step_enc(graphed.st, 2, h, F, graphed.out, stream=side)
    torch.cuda.synchronize()
    other = Dev(2)
    for rep in range(3):
        graph.replay()
        for _ in range(3):
            eager.ctx.step_enc(eager.st, 2, h, F, eager.out)
        # eager work on the captured context in between
        other.load(s)
        graphed.ctx.enc_prepare(other.st, 2, h, F, other.out)
        torch.cuda.synchronize()
        a, b = eager.state(), graphed.state()
        for k in KEYS:
            assert a[k].tobytes() == b[k].tobytes(), (rep, k)
        ea, ga = eager.out.to_host(), graphed.out.to_host()
        assert ea["acc"].tobytes() == ga["acc"].tobytes() and ea["n_pairs"] == ga["n_pairs"] == 1
    for d in (eager, graphed, other):
        d.close()


def test_cluster_with_field_bodies(ora):
    """Massless field bodies in the groups (N_m < N - 1): they feel the massive
    bodies and pull nothing."""
    s = _cluster(n=40, spread=0.08, seed=12)
    n, n_m = 40, 28
    h = 0.01
    acc, pairs = E.prepare(s, n_m, h, F, ora=ora)
    assert (pairs[:, 1] >= n_m).any()   # some flagged pairs have a field body
    dev = Dev(n)
    G.say("cluster with 12 field bodies, 4 steps")
    for _ in range(4):
        s, acc, pairs = _compare_step(dev, ora, s, n_m, h, acc, pairs)
    dev.close()


def test_binned_problem_groups(ora):
    """A problem large enough to be binned (20,000 massive bodies): the table is
    built from caller indices, so the groups and their integration are the
    same as unbinned; one step from the oracle's inputs."""
    from paper_2304_07325_amd import diskgen as dgen
    d = dgen.make_disk(20000, 19999, "hot", 77)
    s = d.state(0)
    n = s["x"].size
    h = dgen.DT_HALF_YEAR
    acc, pairs = E.prepare(s, n, h, F, ora=ora)
    assert 0 < len(pairs) <= 8192
    dev = Dev(n)
    G.say("binned 20k hot disk, 1 step,", len(pairs), "pairs")
    _compare_step(dev, ora, s, n, h, acc, pairs)
    dev.close()


def test_flyby_backwards_step_by_step(ora):
    """Negative steps (h < 0): the level tests run on the reversed motion on
    both sides; the flyby integrated backwards from inside the critical
    radius, through closest approach."""
    x, v, m = _flyby(sep=0.15)
    s = _state(x, v, m)
    s = dict(s, vx=-s["vx"], vy=-s["vy"], vz=-s["vz"])   # run the flyby in reverse
    h = -0.025
    acc, pairs = E.prepare(s, 2, h, F, ora=ora)
    dev = Dev(2)
    G.say("flyby backwards, 12 steps")
    for _ in range(12):
        s, acc, pairs = _compare_step(dev, ora, s, 2, h, acc, pairs)
    dev.close()


@pytest.mark.parametrize("n,n_m", [(1, 1), (2, 0), (3, 1), (70, 0)])
def test_degenerate_problems_are_the_plain_step(n, n_m):
    """One body, or no massive body, or one massive row: no pair can be
    flagged and the encounter step is symba_step bit for bit."""
    rng = np.random.default_rng(n)
    a = rng.uniform(1.0, 3.0, n)
    th = rng.uniform(0, 2 * np.pi, n)
    x = np.c_[a * np.cos(th), a * np.sin(th), rng.normal(0, 0.01, n)]
    v = np.c_[-np.sin(th), np.cos(th), np.zeros(n)] / np.sqrt(a)[:, None]
    s = _state(x, v, np.full(n, 1e-9))
    h = 0.05
    plain, enc = Dev(n), Dev(n)
    plain.load(s)
    enc.load(s)
    plain.ctx.kick_encounter(plain.st, n_m, abs(h), F, out=plain.out)
    enc.ctx.enc_prepare(enc.st, n_m, h, F, enc.out)
    for _ in range(3):
        plain.ctx.step(plain.st, n_m, h, F, plain.out)
        enc.ctx.step_enc(enc.st, n_m, h, F, enc.out)
    a_, b_ = plain.state(), enc.state()
    for k in KEYS:
        assert a_[k].tobytes() == b_[k].tobytes(), k
    assert enc.out.to_host()["status"] == 0
    plain.close()
    enc.close()


@pytest.mark.parametrize("case", ["cluster", "flyby", "field", "binary", "triple"])
def test_fused_small_problem_launches_are_bit_identical(case):
    """Problems of one block run the encounter step in two fused launches;
    the general launches (SYMBA_OPT_ENC_FUSE = 0) give the same bits.  The
    fused launch compiles the register forms of the group integration into
    itself, the general group kernel calls them as functions: the tight
    binary and triple (every substep at the deepest level) compare the two
    through tens of thousands of substeps."""
    from paper_2304_07325_amd import binding as B
    if case == "flyby":
        x, v, m = _flyby(sep=0.15)
        s, n_m, h = _state(x, v, m), 2, 0.025
    elif case in ("binary", "triple"):
        s = _binary() if case == "binary" else _triple()
        n_m, h = s["x"].size, 0.05
    else:
        s, h = _cluster(), 0.01
        n_m = 40 if case == "cluster" else 28
    n = s["x"].size
    fused, plain = Dev(n), Dev(n)
    plain.ctx.set_option(B.OPT_ENC_FUSE, 0)
    for d in (fused, plain):
        d.load(s)
        d.ctx.enc_prepare(d.st, n_m, h, F, d.out)
    G.say("fused vs general launches,", case)
    for step in range(6):
        for d in (fused, plain):
            d.ctx.step_enc(d.st, n_m, h, F, d.out)
        a, b = fused.state(), plain.state()
        for k in KEYS:
            assert a[k].tobytes() == b[k].tobytes(), (step, k)
        fa, pa = fused.out.to_host(), plain.out.to_host()
        assert fa["acc"].tobytes() == pa["acc"].tobytes()
        assert np.array_equal(fa["pair_i"], pa["pair_i"]) and fa["status"] == pa["status"]
    fused.close()
    plain.close()


def _binary(extra=0):
    """A tight binary (two 3e-8 solar-mass bodies 2e-5 AU apart on a mutual
    circular orbit, well inside the deepest shell) on a 10 AU orbit, plus
    `extra` far-apart bodies on a wide ring: the pair stays at level 8 for
    the whole step (4^8 substeps at that level)."""
    m, a, sep = 3e-8, 10.0, 2e-5
    vc, vb = math.sqrt(1.0 / a), math.sqrt(2 * m / sep) / 2
    x = [[a - sep / 2, 0.0, 0.0], [a + sep / 2, 0.0, 0.0]]
    v = [[0.0, vc - vb, 0.0], [0.0, vc + vb, 0.0]]
    for k in range(extra):
        th, r = 2 * math.pi * (k + 1) / (extra + 2), 6.0 + 10.0 * k / max(extra, 1)
        x.append([r * math.cos(th), r * math.sin(th), 0.0])
        v.append([-math.sin(th) / math.sqrt(r), math.cos(th) / math.sqrt(r), 0.0])
    return _state(x, v, [m] * (2 + extra))


def _triple():
    """The tight binary with a third body 1.5e-4 AU from its centre on a
    circular orbit about it: a group of three pairs, all in the deepest shell."""
    s = _binary()
    m, a, d = 3e-8, 10.0, 1.5e-4
    vc, v3 = math.sqrt(1.0 / a), math.sqrt(2 * m / d)
    x = np.stack([s["x"], s["y"], s["z"]], 1).tolist() + [[a, d, 0.0]]
    v = [[0.0, vc - math.sqrt(2 * m / 2e-5) / 2, 0.0], [0.0, vc + math.sqrt(2 * m / 2e-5) / 2, 0.0],
         [-v3, vc, 0.0]]
    return _state(x, v, [m, m, m])


@pytest.mark.parametrize("case", ["flyby", "binary", "binary_wide", "triple", "cluster", "cluster_small", "disk1k"])
def test_small_groups_in_registers_are_bit_identical(case):
    """Groups of at most 64 bodies and 64 pairs run in registers (one pair:
    the two bodies in two lanes; more: a lane per body and a lane per pair),
    SYMBA_OPT_ENC_REGS = 1; the routines for groups of any size, which keep
    them in LDS (SYMBA_OPT_ENC_REGS = 0), give the same bits: a fast flyby, a
    tight binary at the deepest level for the whole step (one block, and 300
    bodies through the general launches), a tight triple, a crowded cluster
    (one group over the limit of the register path next to a smaller one), a
    small cluster (one group of many pairs in registers) and 20 steps of the
    paper's 1k disk."""
    from paper_2304_07325_amd import binding as B
    if case == "flyby":
        x, v, m = _flyby(sep=0.15)
        s, n_m, h, steps = _state(x, v, m), 2, 0.025, 6
    elif case == "binary":
        s, n_m, h, steps = _binary(), 2, dg.DT_HALF_YEAR, 1
    elif case == "binary_wide":
        s, n_m, h, steps = _binary(298), 300, dg.DT_HALF_YEAR, 1
    elif case == "triple":
        s, n_m, h, steps = _triple(), 3, 0.05, 2
    elif case == "cluster":
        s, h, steps = _cluster(), 0.01, 4
        n_m = 40
    elif case == "cluster_small":
        s, h, steps = _cluster(n=16, spread=0.05), 0.01, 4
        n_m = 16
    else:
        w = dg.WORKLOADS["disk1k"]
        s = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"]).state(0)
        n_m, h, steps = w["n_massive"], dg.DT_HALF_YEAR, 20
    n = s["x"].size
    regs, lds = Dev(n), Dev(n)
    lds.ctx.set_option(B.OPT_ENC_REGS, 0)
    for d in (regs, lds):
        d.load(s)
        d.ctx.enc_prepare(d.st, n_m, h, F, d.out)
    G.say("small groups in registers vs LDS,", case)
    for step in range(steps):
        for d in (regs, lds):
            d.ctx.step_enc(d.st, n_m, h, F, d.out)
        a, b = regs.state(), lds.state()
        for k in KEYS:
            assert a[k].tobytes() == b[k].tobytes(), (step, k)
        ra, la = regs.out.to_host(), lds.out.to_host()
        assert ra["acc"].tobytes() == la["acc"].tobytes()
        assert ra["status"] == la["status"] == 0
        assert np.array_equal(ra["pair_i"], la["pair_i"]) and np.array_equal(ra["pair_j"], la["pair_j"])
    if case.startswith("binary"):
        assert regs.out.to_host()["n_pairs"] >= 1   # still a pair, deep in the shells
    regs.close()
    lds.close()


def test_paper_disk1k_trajectory_tracks_the_oracle():
    """90 encounter steps of the paper's 1k benchmark disk (Sec. 3) on the
    device against the oracle's own 90 steps (stored by
    tests/golden/make_enc_paper_disk1k.py): every 10 steps the relative energy
    error, the smallest separation and the number of flagged pairs agree.  The
    two sides round differently from the first step on, so this checks that the
    whole integrator (groups through the shells, evaluation, level-0
    reweighting) follows the same trajectory over many steps, not only one step
    from shared inputs."""
    import json
    import os
    import torch
    from paper_2304_07325_amd import binding as B
    from tests.golden.make_enc_paper_disk1k import split_energy
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "enc_paper_disk1k.json")))
    w = dg.WORKLOADS[gold["disk"]]
    disk = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    s0 = disk.state(0)
    n, n_m, h, f = gold["n"], gold["n_massive"], gold["h"], gold["rcrit_factor"]
    e0, _ = split_energy(s0)
    st = B.to_device_state(s0)
    ctx = B.Context(max_n=n, max_pairs=1 << 14)
    out = B.Outputs(n, 1 << 12)
    G.say("paper disk1k, 90 encounter steps")
    ctx.enc_prepare(st, n_m, h, f, out)
    want = {c["step"]: c for c in gold["checkpoints"]}
    for k in range(1, max(want) + 1):
        ctx.step_enc(st, n_m, h, f, out)
        if k in want:
            torch.cuda.synchronize()
            o = out.to_host()
            s = {key: v.cpu().numpy() for key, v in st.items()}
            e, rmin = split_energy(s)
            err = abs(e - e0) / abs(e0)
            c = want[k]
            assert o["status"] == 0 and o["n_pairs"] == c["n_pairs"], (k, o["status"], o["n_pairs"], c)
            # energy errors of 1e-11 .. 2e-9 of |E|: 5 % of the value plus the
            # rounding of E itself (about 1e-12 of |E| over 500k pair terms)
            assert abs(err - c["energy_rel_err"]) <= 0.05 * c["energy_rel_err"] + 1e-12, (k, err, c)
            assert abs(rmin - c["min_separation"]) <= 1e-6 * c["min_separation"], (k, rmin, c)
    ctx.close()


@pytest.mark.parametrize("case", ["binary", "triple"])
def test_deepest_level_step_matches_the_oracle(case, ora):
    """One step of a tight binary and of a tight triple that stay inside the
    deepest shell for the whole step (every substep down to level 8: 87,380
    for the binary, its short arcs drifted by the f and g series, its groups
    in the register forms) against the oracle's step, stored by
    tests/golden/make_enc_deep.py, from the oracle's own inputs.  Such a step
    is ill-conditioned (the binary turns about 1,400 times), so each
    coordinate is held to 30 times the spread that moving one input
    coordinate by one ulp gives the oracle's own step (the device rounds
    differently in every operation, not in one input: about ten times that
    spread measured), plus the usual tolerance; the pairs must be the same."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "enc_deep.json")))["cases"][case]
    s = {"binary": _binary, "triple": _triple}[case]()
    n_m, h = gold["n_m"], gold["h"]
    acc, pairs = E.prepare(s, n_m, h, F, ora=ora)
    dev = Dev(s["x"].size)
    G.say("deepest level, one step,", case)
    dev.load(s, acc, pairs, ora)
    dev.ctx.step_enc(dev.st, n_m, h, F, dev.out)
    got = dev.state()
    out = dev.out.to_host()
    want = dict(s)
    want.update({k: np.asarray(v, dtype=np.float64) for k, v in gold["state"].items()})
    pscale = max(np.abs(want[k]).max() for k in ("x", "y", "z")) + 1.0
    vscale = max(np.abs(want[k]).max() for k in ("vx", "vy", "vz"))
    for k in KEYS:
        scale = pscale if k in ("x", "y", "z") else vscale
        tol = 30.0 * gold["spread"][k] + STATE_TOL * scale
        assert np.abs(got[k] - want[k]).max() <= tol, (k, np.abs(got[k] - want[k]).max(), tol)
    assert out["status"] == 0
    assert np.array_equal(np.stack([out["pair_i"], out["pair_j"]], 1), np.asarray(gold["pairs"]).reshape(-1, 2))
    scale = np.abs(ora.accel(want, n_m)).max()
    assert np.abs(out["acc"] - np.asarray(gold["acc"])).max() <= 30.0 * gold["acc_spread"] + ACC_TOL * scale
    dev.close()
