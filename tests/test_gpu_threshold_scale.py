"""Near-threshold encounter pairs at scale (GPU): 10^8 pairs placed within a
few ulp of the critical radius, in each regime of the predicate (separation
at the start of the step, at its end, at an interior closest approach) and
in frames moving at up to 100 times the pairs' relative speed, run through
the library with its default screen (FP32, conservative, every candidate
confirmed in FP64).  The flags must be the oracle's on every pair, no other
pair may be flagged, and each flagged partner must join its owner's group:
a screen that dropped one candidate would show as a missing pair."""
import numpy as np
import pytest

import oracle
from paper_2304_07325_amd import diskgen as dg
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

DT = dg.DT_HALF_YEAR
F = dg.RCRIT_FACTOR
TARGET_PAIRS = 100_000_000


def _unit(rng, k):
    u = rng.normal(size=(k, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _geometry(rng, n_own, per, massive_partners):
    """Owners on a grid (far enough apart that no cross pair can come near),
    each with `per` partners: the partner offsets d and relative velocities w
    place every pair within a few ulp of its critical radius, a third in each
    regime of the predicate."""
    g = int(np.ceil(n_own ** (1.0 / 3.0)))
    spacing = 2.0 if massive_partners else 1.0   # partners of neighbouring owners never meet either
    o = np.arange(n_own)
    centres = spacing * (np.stack([o % g, (o // g) % g, o // (g * g)], 1).astype(np.float64) - g / 2)
    rh_own = rng.uniform(0.01, 0.05, n_own)
    k = n_own * per
    owner = np.repeat(o, per)
    rc = F * rh_own[owner] * (2.0 if massive_partners else 1.0)   # f (rh_i + rh_j)
    u = _unit(rng, k)
    p = _unit(rng, k)
    p -= np.sum(p * u, 1, keepdims=True) * u
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    scale = 1.0 + rng.integers(-6, 7, k) * 2.0 ** -52
    regime = np.arange(k) % 3
    d = np.empty((k, 3))
    w = np.empty((k, 3))
    r0 = regime == 0   # separation at the start of the step, receding
    d[r0] = (rc * scale)[r0, None] * u[r0]
    w[r0] = 0.01 * u[r0]
    r1 = regime == 1   # separation at the end of the step, approaching
    w[r1] = rng.uniform(0.001, 0.05, (r1.sum(), 1)) * (-u[r1] + 0.3 * p[r1])
    d[r1] = (rc * scale)[r1, None] * u[r1] - w[r1] * DT
    r2 = regime == 2   # closest approach inside the step
    speed = rng.uniform(0.001, 0.1, (r2.sum(), 1))
    d[r2] = (rc * scale)[r2, None] * p[r2] + speed * DT * rng.uniform(0.1, 0.9, (r2.sum(), 1)) * u[r2]
    w[r2] = -speed * u[r2]
    return dict(centres=centres, rh_own=rh_own, owner=owner, d=d, w=w, massive=massive_partners)


def _system(rng, geo, vframe):
    """One evaluation's state: the geometry under a random rotation (the
    separations stay within a rounding of where they were put) in a frame
    moving at vframe.  Returns (state, n_m, owner of each pair, partner)."""
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    rot = q * np.sign(np.diag(r))
    d, w = geo["d"] @ rot.T, geo["w"] @ rot.T
    centres, rh_own, owner = geo["centres"], geo["rh_own"], geo["owner"]
    n_own, k = centres.shape[0], owner.size
    frame = vframe * _unit(rng, 1)[0]
    if geo["massive"]:   # owner 2q, partner 2q + 1, all massive
        n = 2 * n_own
        X = np.empty((n, 3))
        V = np.empty((n, 3))
        X[0::2], X[1::2] = centres, centres + d
        V[0::2], V[1::2] = frame, frame + w
        rh = np.repeat(rh_own, 2)
        pi, pj, n_m = 2 * owner, 2 * owner + 1, n
    else:                # owners massive [0, n_own), partners field after them
        n = n_own + k
        X = np.concatenate([centres, centres[owner] + d])
        V = np.concatenate([np.broadcast_to(frame, (n_own, 3)), frame + w])
        rh = np.concatenate([rh_own, np.zeros(k)])
        pi, pj, n_m = owner, n_own + np.arange(k), n_own
    m = np.where(np.arange(n) < n_m, 1e-9, 0.0)
    s = dict(x=X[:, 0].copy(), y=X[:, 1].copy(), z=X[:, 2].copy(), vx=V[:, 0].copy(), vy=V[:, 1].copy(),
             vz=V[:, 2].copy(), m=m, rh=rh)
    return s, n_m, pi.astype(np.int32), pj.astype(np.int32)


def test_near_threshold_pairs_at_scale():
    from paper_2304_07325_amd import binding as B
    import torch
    ora = oracle.default()
    rng = np.random.default_rng(2024)
    # geometries: 1000 massive owners with 100 field partners each (the
    # massive x field tasks), and 50000 isolated pairs of massive bodies (the
    # folded triangle); a few of each, rotated anew for every evaluation
    geos = [[_geometry(rng, 1000, 100, False) for _ in range(3)],
            [_geometry(rng, 50_000, 1, True) for _ in range(3)]]
    max_n = 101_000
    ctxs = {}
    for name, opt in (("auto", 0), ("binned", 2), ("unbinned", 1)):
        ctxs[name] = B.Context(max_n=max_n, max_pairs=1 << 18)
        ctxs[name].set_option(B.OPT_BIN, opt)
    done = flagged = evals = 0
    while done < TARGET_PAIRS:
        kind = evals % 2
        vframe = (0.0, 0.5, 100.0)[evals % 3]
        s, n_m, pi, pj = _system(rng, geos[kind][(evals // 2) % 3], vframe)
        n = s["x"].size
        # stars binned or not; the massive pairs binned (the default at this size) or not
        c = ctxs[("binned", "auto", "auto", "unbinned")[evals % 4]]
        if evals % 100 == 0:
            G.say(f"near-threshold scale: evaluation {evals}, pairs so far {done}, flagged {flagged}")
        st = B.to_device_state(s)
        o = B.Outputs(n, 1 << 18)
        c.kick_encounter(st, n_m, DT, F, out=o)
        torch.cuda.synchronize()
        g = o.to_host()
        want = ora.encounter_list(s, pi, pj, DT, F)
        assert g["status"] == 0, (evals, g["status"])
        assert g["n_pairs"] == int(want.sum()), (evals, g["n_pairs"], int(want.sum()))
        assert np.array_equal(g["pair_i"], pi[want]) and np.array_equal(g["pair_j"], pj[want]), evals
        assert np.array_equal(g["group_id"][pj[want]], pi[want]), evals
        done += pi.size
        flagged += int(want.sum())
        evals += 1
    # the pairs sit at the threshold: both outcomes in bulk
    assert 0.2 * done < flagged < 0.8 * done, (flagged, done)
    print(f"{done} near-threshold pairs in {evals} evaluations, {flagged} flagged, all as the oracle")
    for c in ctxs.values():
        c.close()
