"""The full heliocentric output (option SYMBA_OPT_ACC = SYMBA_ACC_HELIO)
against the oracle's: the interaction sum plus the Sun's pull and the
indirect term of the heliocentric frame, within 1e-12 per body; pairs and
groups as without the option; a batch gives each problem the bits of its
single call; the step ignores the option."""
import numpy as np
import pytest

import oracle
from paper_2304_07325_amd import diskgen as dg
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

DT = dg.DT_HALF_YEAR
F = dg.RCRIT_FACTOR
RTOL = 1e-12


@pytest.fixture(scope="module")
def ora():
    return oracle.default()


def _case(which):
    if which == "disk1k":
        w = dg.WORKLOADS["disk1k"]
        return dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"]).state(0), w["n_massive"]
    if which in ("field", "field_binned"):
        return dg.make_disk(3000, 300, "hot", 5).state(0), 300
    if which == "massless":   # no massive body: the Sun's pull alone
        return dg.make_disk(700, 0, "hot", 6).state(0), 0
    return dg.make_disk(1, 1, "hot", 7).state(0), 1   # one body


def _ctx(n, binned=False):
    from paper_2304_07325_amd import binding as B
    ctx = B.Context(max_n=max(n, 64), max_pairs=1 << 16)
    ctx.set_option(B.OPT_ACC, B.ACC_HELIO)
    if binned:
        ctx.set_option(B.OPT_BIN, 2)
    return ctx


def _rel(got, want):
    num = np.linalg.norm(got - want, axis=1)
    den = np.linalg.norm(want, axis=1)
    return float((num / den).max())


@pytest.mark.parametrize("which", ["disk1k", "field", "field_binned", "massless", "single"])
def test_helio_matches_oracle(ora, which):
    s, n_m = _case(which)
    n = s["x"].size
    G.say("helio", which, n, n_m)
    ctx = _ctx(n, binned=which == "field_binned")
    got = G.run_gpu(ctx, s, n_m, DT, F)
    ctx.close()
    ref = ora.kick_encounter(s, n_m, DT, F)
    G.check_pairs_groups(got, ref)
    want = ora.helio(s, n_m, ref["acc"])
    assert _rel(got["acc"], want) < RTOL, _rel(got["acc"], want)


def test_helio_batch_matches_single_calls(ora):
    from paper_2304_07325_amd import binding as B
    import torch
    sims = [_case("disk1k"), _case("field"), (dg.make_disk(500, 499, "cold", 8).state(0), 499), _case("massless")]
    G.say("helio batch", len(sims))
    total = sum(s["x"].size for s, _ in sims)
    single = []
    for s, n_m in sims:
        ctx = _ctx(s["x"].size)
        single.append(G.run_gpu(ctx, s, n_m, DT, F, pair_cap=1 << 13))
        ctx.close()
    ctx = _ctx(total)
    sts = [B.to_device_state(s) for s, _ in sims]
    outs = [B.Outputs(s["x"].size, 1 << 13) for s, _ in sims]
    ctx.kick_encounter_batch([(st, n_m, DT, F, o) for st, (_, n_m), o in zip(sts, sims, outs)])
    torch.cuda.synchronize()
    for (s, n_m), o, one in zip(sims, outs, single):
        g = o.to_host()
        assert g["status"] == 0
        assert g["acc"].tobytes() == one["acc"].tobytes()
        assert np.array_equal(g["pair_i"], one["pair_i"]) and np.array_equal(g["group_id"], one["group_id"])
        ref = ora.kick_encounter(s, n_m, DT, F)
        assert _rel(g["acc"], ora.helio(s, n_m, ref["acc"])) < RTOL
    ctx.close()


def test_step_ignores_the_option():
    """The step kicks with the interaction term whatever the option says."""
    from paper_2304_07325_amd import binding as B
    import torch
    s, n_m = _case("disk1k")
    n = s["x"].size
    h = 0.2 * dg.YEAR
    G.say("helio option and the step")
    runs = []
    for helio in (False, True):
        ctx = B.Context(max_n=n, max_pairs=1 << 16)
        st = B.to_device_state(s)
        out = B.Outputs(n, 1 << 13)
        ctx.kick_encounter(st, n_m, h, F, out=out)   # interaction term: what a step starts from
        if helio:
            ctx.set_option(B.OPT_ACC, B.ACC_HELIO)
        for _ in range(3):
            ctx.step(st, n_m, h, F, out)
        torch.cuda.synchronize()
        runs.append(({k: v.cpu().numpy() for k, v in st.items()}, out.to_host()))
        ctx.close()
    (s0, o0), (s1, o1) = runs
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert s0[k].tobytes() == s1[k].tobytes(), k
    assert o0["acc"].tobytes() == o1["acc"].tobytes()


def test_option_values_are_checked():
    from paper_2304_07325_amd import binding as B
    ctx = B.Context(max_n=64)
    for opt, bad in ((B.OPT_ACC, 2), (B.OPT_ACC, -1), (B.OPT_TIMING, 2)):
        with pytest.raises(Exception):
            ctx.set_option(opt, bad)
    ctx.set_option(B.OPT_ACC, B.ACC_INTERACTION)
    ctx.close()
