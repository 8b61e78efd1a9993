"""symba_step (GPU) against the step oracle: the state after one and after
many steps, the evaluation at the new positions, time reversal, and the
energy of the paper's accuracy-test kind of system."""
import numpy as np
import pytest

import oracle
from oracle import dh_step as S
from paper_2304_07325_amd import diskgen as dg
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

F = dg.RCRIT_FACTOR
KEYS = ("x", "y", "z", "vx", "vy", "vz")


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


class Runner:
    """A device state with its outputs, stepped by symba_step."""

    def __init__(self, s, n_m, h, screen=None, binned=False):
        import torch
        from paper_2304_07325_amd import binding as B
        self.B, self.torch = B, torch
        self.n, self.n_m, self.h = s["x"].size, n_m, h
        self.ctx = B.Context(max_n=max(self.n, 64), max_pairs=1 << 16)
        if screen is not None:
            self.ctx.set_option(B.OPT_SCREEN, screen)
        if binned:   # the evaluation in the binned order, whose final kick maps positions back
            self.ctx.set_option(B.OPT_BIN, 2)
        self.st = B.to_device_state(s)
        self.out = B.Outputs(self.n, 1 << 15)
        self.ctx.kick_encounter(self.st, n_m, abs(h), F, out=self.out)

    def step(self, k=1, h=None):
        for _ in range(k):
            self.ctx.step(self.st, self.n_m, self.h if h is None else h, F, self.out)
        self.torch.cuda.synchronize()

    def state(self):
        return {k: v.cpu().numpy() for k, v in self.st.items()}

    def close(self):
        self.ctx.close()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _compare_state(got, want, tol):
    for k in KEYS:
        assert _rel(got[k], want[k]) < tol, (k, _rel(got[k], want[k]))


@pytest.mark.parametrize("binned", [False, True])
@pytest.mark.parametrize("which", ["disk1k", "dense_field"])
def test_one_step_matches_oracle(ora, which, binned):
    if which == "disk1k":
        w = dg.WORKLOADS["disk1k"]
        s = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"]).state(0)
        n_m, h = w["n_massive"], dg.DT_HALF_YEAR
    else:   # massive and field bodies on bound orbits, closer together
        d = dg.make_disk(900, 300, "hot", 77)
        s, n_m, h = d.state(0), 300, 0.1 * dg.YEAR
    G.say("step", which, "binned" if binned else "")
    r = Runner(s, n_m, h, binned=binned)
    r.step()
    got = r.state()
    want, acc_want = S.step(s, n_m, h, ora=ora)
    _compare_state(got, want, 1e-13)
    # the evaluation at the new positions is the path's, exactly as for a plain call
    ev = r.out.to_host()
    ref = ora.kick_encounter(got, n_m, abs(h), F)
    G.check_pairs_groups(ev, ref)
    G.check_acc(got, n_m, ev["acc"], ref["acc"])
    r.close()


def test_many_steps_track_oracle(ora):
    d = dg.make_disk(600, 599, "hot", 31)
    s, n_m, h = d.state(0), 599, 0.2 * dg.YEAR
    G.say("step x40 hot 600")
    r = Runner(s, n_m, h)
    r.step(40)
    got = r.state()
    acc = None
    want = s
    for _ in range(40):
        want, acc = S.step(want, n_m, h, acc=acc, ora=ora)
    _compare_state(got, want, 1e-11)
    r.close()


def test_step_reverses(ora):
    """A step of -h after a step of h returns to the start."""
    d = dg.make_accuracy_disk(n=100)
    s = d.state(0)
    G.say("step reversal")
    r = Runner(s, d.n_massive, d.dt)
    r.step(5)
    r.step(5, h=-d.dt)
    back = r.state()
    for k in KEYS:
        assert _rel(back[k], s[k]) < 1e-13, (k, _rel(back[k], s[k]))
    r.close()


@pytest.mark.parametrize("screen", [1, 2])
def test_energy_of_the_accuracy_disk(ora, screen):
    """100 equal planetesimals 5 Hill radii apart from 5 AU, 0.1-year steps
    (the paper's accuracy test, Sec. 3) for 200 years: the relative energy
    error stays below 1e-8 and is the same with either screen."""
    d = dg.make_accuracy_disk(n=100)
    s = d.state(0)
    G.say("accuracy disk energy, screen", screen)
    r = Runner(s, d.n_massive, d.dt, screen=screen)
    e0 = S.energy(s, d.n_massive)
    worst = 0.0
    for _ in range(10):
        r.step(200)
        worst = max(worst, abs(S.energy(r.state(), d.n_massive) - e0) / abs(e0))
    assert worst < 1e-8, worst
    r.close()


def test_kepler_drift_of_every_conic(ora):
    """Massless bodies (no kick, no Sun drift) on ellipses up to e = 0.95,
    near-parabolic and hyperbolic orbits, over arcs from a small fraction of
    an orbit to several orbits: the device's Kepler drift (Danby's universal
    variable, Laguerre-Conway) against the oracle's (Curtis' universal
    anomaly, Newton)."""
    rng = np.random.default_rng(11)
    n = 640
    x = rng.normal(size=(n, 3))
    x *= (rng.uniform(0.5, 30.0, n) / np.linalg.norm(x, axis=1))[:, None]
    r = np.linalg.norm(x, axis=1)
    v = rng.normal(size=(n, 3))
    # speeds from deep ellipses through the parabola (sqrt(2/r)) to hyperbolae
    v *= (np.sqrt(2.0 / r) * rng.uniform(0.2, 2.5, n) / np.linalg.norm(v, axis=1))[:, None]
    v[:40] *= (np.sqrt(2.0 / r[:40]) / np.linalg.norm(v[:40], axis=1))[:, None] * (1 + rng.uniform(-1e-9, 1e-9, 40))[:, None]
    s = dict(x=x[:, 0].copy(), y=x[:, 1].copy(), z=x[:, 2].copy(), vx=v[:, 0].copy(), vy=v[:, 1].copy(),
             vz=v[:, 2].copy(), m=np.zeros(n), rh=np.zeros(n))
    for h in (0.05, 7.0, 300.0, -40.0):
        G.say("kepler drift conics h", h)
        rr = Runner(s, 0, h)
        rr.step()
        got = rr.state()
        rr.close()
        xw, vw = S.kepler_drift(x, v, h)
        gx = np.stack([got["x"], got["y"], got["z"]], 1)
        gv = np.stack([got["vx"], got["vy"], got["vz"]], 1)
        ex = np.linalg.norm(gx - xw, axis=1) / np.linalg.norm(xw, axis=1)
        ev = np.linalg.norm(gv - vw, axis=1) / np.linalg.norm(vw, axis=1)
        assert ex.max() < 1e-11 and ev.max() < 1e-11, (h, ex.max(), ev.max())


@pytest.mark.parametrize("binned", [False, True])
def test_step_batch_matches_single_steps(ora, binned):
    """Simulations of uneven size, all-massive and field-heavy, stepped
    together by symba_step_batch (with their own steps h) for several
    rounds: every state, acceleration and pair list is the same bits as
    stepping each alone with symba_step (also with every problem binned,
    where each closing kick maps binned positions back)."""
    from paper_2304_07325_amd import binding as B
    import torch
    specs = [(700, 699, 0.5), (300, 30, 0.2), (1500, 1499, 0.1), (65, 64, 1.0), (2000, 200, 0.3)]
    sims = [dg.make_disk(n, nm, "hot", 40 + k).state(0) for k, (n, nm, _) in enumerate(specs)]
    G.say("step batch", len(specs), "binned" if binned else "")
    alone = []
    for (n, nm, yr), s in zip(specs, sims):
        r = Runner(s, nm, yr * dg.YEAR, binned=binned)
        r.step(3)
        alone.append((r.state(), r.out.to_host()))
        r.close()
    total = sum(n for n, _, _ in specs)
    ctx = B.Context(max_n=total, max_pairs=1 << 17)
    if binned:
        ctx.set_option(B.OPT_BIN, 2)
    sts = [B.to_device_state(s) for s in sims]
    outs = [B.Outputs(n, 1 << 13) for n, _, _ in specs]   # the pair scratch of the context is shared out
    for (n, nm, yr), st, o in zip(specs, sts, outs):
        ctx.kick_encounter(st, nm, yr * dg.YEAR, F, out=o)
    probs = [(st, nm, yr * dg.YEAR, F, o) for (n, nm, yr), st, o in zip(specs, sts, outs)]
    for _ in range(3):
        ctx.step_batch(probs)
    torch.cuda.synchronize()
    for (want_s, want_o), st, o in zip(alone, sts, outs):
        got = {k: v.cpu().numpy() for k, v in st.items()}
        for k in KEYS:
            assert got[k].tobytes() == want_s[k].tobytes(), k
        g = o.to_host()
        assert g["status"] == want_o["status"] == 0
        assert g["acc"].tobytes() == want_o["acc"].tobytes()
        assert np.array_equal(g["pair_i"], want_o["pair_i"]) and np.array_equal(g["pair_j"], want_o["pair_j"])
        assert np.array_equal(g["group_id"], want_o["group_id"])
    ctx.close()


def test_step_graph_replays_match_eager():
    """Twenty steps of the accuracy disk captured in a HIP graph and replayed
    three times, with eager steps and synchronisations between the replays:
    every replay leaves the state and accelerations of twenty eager steps,
    bit for bit (the step allocates nothing and records no memset)."""
    import torch
    d = dg.make_accuracy_disk(n=100)
    s, nm, h = d.state(0), d.n_massive, d.dt
    G.say("step graph replays")
    eager = Runner(s, nm, h)
    graphed = Runner(s, nm, h)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for _ in range(20):
            graphed.ctx.step(graphed.st, nm, h, F, graphed.out, stream=side)
    torch.cuda.synchronize()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        eager.step(20)
        got, want = graphed.state(), eager.state()
        for k in KEYS:
            assert got[k].tobytes() == want[k].tobytes(), (rep, k)
        assert graphed.out.to_host()["acc"].tobytes() == eager.out.to_host()["acc"].tobytes(), rep
    eager.close()
    graphed.close()
