"""Graph capture on a context is independent of later calls (GPU): a batch,
a step batch and a single call are captured, eager calls with other, larger
problems follow on the same context (its partial-sum buffer grows, so the one
the graph uses must be kept, and the eager descriptor staging is rewritten),
and every replay still gives the eager outputs of the captured problems bit
for bit."""
import numpy as np
import pytest

from paper_2304_07325_amd import diskgen as dg
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

DT = dg.DT_HALF_YEAR
F = dg.RCRIT_FACTOR


@pytest.fixture(scope="module")
def ora():
    import oracle
    return oracle.default()


def _same(g, e, what):
    assert g["acc"].tobytes() == e["acc"].tobytes(), f"{what}: acc differs"
    assert np.array_equal(g["pair_i"], e["pair_i"]) and np.array_equal(g["pair_j"], e["pair_j"]), what
    assert np.array_equal(g["group_id"], e["group_id"]) and g["n_groups"] == e["n_groups"], what
    assert g["status"] == e["status"] == 0, what


def _problems(B, specs, seed0, box):
    states = [G.dense_state(n, seed=seed0 + k, box=box, n_m=nm) for k, (n, nm) in enumerate(specs)]
    dev = [B.to_device_state(s) for s in states]
    outs = [B.Outputs(n, 1 << 15) for n, _ in specs]
    return states, dev, outs, [(d, nm, DT, F, o) for d, (n, nm), o in zip(dev, specs, outs)]


def test_captured_batch_unaffected_by_later_calls(ora):
    import torch
    from paper_2304_07325_amd import binding as B
    spec_a = [(900, 899), (1500, 150), (2100, 2099)]
    spec_b = [(6000, 5999), (300, 299), (4000, 400), (2500, 2499)]   # other sizes, more partial sums
    ctx = B.Context(max_n=sum(n for n, _ in spec_b) + 16, max_pairs=1 << 18)
    sa, da, oa, pa = _problems(B, spec_a, 100, 4.0)
    sb, db, ob, pb = _problems(B, spec_b, 200, 6.0)
    G.say("capture batch A, eager batch B, replay A")
    ctx.kick_encounter_batch(pa)
    torch.cuda.synchronize()
    eager_a = [o.to_host() for o in oa]
    for (n, nm), s, e in zip(spec_a, sa, eager_a):
        G.check_pairs_groups(e, ora.kick_encounter(s, nm, DT, F))
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        ctx.kick_encounter_batch(pa, stream=stream)
    torch.cuda.synchronize()
    for rep in range(3):
        ctx.kick_encounter_batch(pb)          # other problems, eager, same context
        torch.cuda.synchronize()
        eager_b = [o.to_host() for o in ob]
        for o in oa:
            o.acc.zero_()
            o.group_id.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, (e, o) in enumerate(zip(eager_a, oa)):
            _same(o.to_host(), e, f"replay {rep} problem {k}")
        if rep == 0:
            for (n, nm), s, e in zip(spec_b, sb, eager_b):
                G.check_pairs_groups(e, ora.kick_encounter(s, nm, DT, F))
    ctx.close()


def test_captured_single_call_unaffected_by_later_calls(ora):
    import torch
    from paper_2304_07325_amd import binding as B
    ctx = B.Context(max_n=8192, max_pairs=1 << 16)
    sa, da, oa, pa = _problems(B, [(1200, 1199)], 300, 4.0)
    sb, db, ob, pb = _problems(B, [(8000, 7999)], 301, 8.0)
    G.say("capture a single call, eager larger call, replay")
    ctx.kick_encounter(da[0], 1199, DT, F, out=oa[0])
    torch.cuda.synchronize()
    eager = oa[0].to_host()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        ctx.kick_encounter(da[0], 1199, DT, F, out=oa[0], stream=stream)
    torch.cuda.synchronize()
    for rep in range(2):
        ctx.kick_encounter(db[0], 7999, DT, F, out=ob[0])
        torch.cuda.synchronize()
        oa[0].acc.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _same(oa[0].to_host(), eager, f"replay {rep}")
    G.check_pairs_groups(ob[0].to_host(), ora.kick_encounter(sb[0], 7999, DT, F))
    ctx.close()


def test_captured_step_batch_unaffected_by_later_calls():
    import torch
    from paper_2304_07325_amd import binding as B
    wa = [dg.make_disk(n, nm, "hot", 400 + n) for n, nm in ((700, 699), (1300, 1299))]
    wb = [dg.make_disk(n, nm, "cold", 500 + n) for n, nm in ((5000, 4999), (900, 899), (3000, 2999))]
    ctx = B.Context(max_n=sum(w.n for w in wb) + 16, max_pairs=1 << 16)
    h = dg.DT_HALF_YEAR

    def setup(ws):
        sts = [B.to_device_state(w.state(0)) for w in ws]
        outs = [B.Outputs(w.n, 1 << 14) for w in ws]
        for w, st, o in zip(ws, sts, outs):
            ctx.kick_encounter(st, w.n_massive, h, F, out=o)
        torch.cuda.synchronize()
        return sts, outs

    sa, oa = setup(wa)
    sb, ob = setup(wb)
    init_a = [{k: v.clone() for k, v in st.items()} for st in sa]
    init_acc = [o.acc.clone() for o in oa]
    steps_a = [(st, w.n_massive, h, F, o) for st, w, o in zip(sa, wa, oa)]
    steps_b = [(st, w.n_massive, h, F, o) for st, w, o in zip(sb, wb, ob)]
    G.say("capture step batch A, eager step batch B, replay A")
    ctx.step_batch(steps_a)
    torch.cuda.synchronize()
    eager_x = [{k: v.cpu().numpy().copy() for k, v in st.items()} for st in sa]
    eager_o = [o.to_host() for o in oa]

    def restore():
        for st, ini in zip(sa, init_a):
            for k in st:
                st[k].copy_(ini[k])
        for o, a in zip(oa, init_acc):
            o.acc.copy_(a)
        torch.cuda.synchronize()

    restore()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        ctx.step_batch(steps_a, stream=stream)
    torch.cuda.synchronize()
    for rep in range(2):
        ctx.step_batch(steps_b)
        torch.cuda.synchronize()
        restore()
        graph.replay()
        torch.cuda.synchronize()
        for k, (st, ex, eo, o) in enumerate(zip(sa, eager_x, eager_o, oa)):
            for key in ("x", "y", "z", "vx", "vy", "vz"):
                assert st[key].cpu().numpy().tobytes() == ex[key].tobytes(), f"replay {rep} sim {k}: {key}"
            _same(o.to_host(), eo, f"replay {rep} sim {k}")
    ctx.close()
