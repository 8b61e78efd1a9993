"""Pins of the oracle against facts that do not come from the oracle itself.

Each check_* function takes an `oracle.Oracle` and raises AssertionError when
the oracle disagrees with the fact it pins.  They are run against the real
oracle (test_oracle_pins.py) and against deliberately broken builds of it
(test_oracle_mutants.py), which must each fail at least one check.

What pins what (paper: Lau & Lee, Sec. 2 pair loop / encounter check / grouping):
  force      -- 50-digit brute force over the physical definition (every body
                feels every massive body), two-body exact dyadic closed form,
                ring closed form, momentum invariant (with and without the
                Sun's indirect term), Kepler limit N=1, exact translation and
                mass-scaling invariances, massive/field semantics of Sec. 2;
  encounter  -- exact rational minimum of |d + w t|^2 over [0, dt] away from
                the threshold, hand-built special cases, strict inequality at
                dyadic equality, enumeration of the trapezoid and its order;
  groups     -- scipy's connected components relabelled by minimum index,
                hand-built graphs.
"""
from __future__ import annotations

import math
from fractions import Fraction

import mpmath
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

EPS = np.finfo(np.float64).eps


# ----------------------------------------------------------------------------
# small input builders (random but seeded; no method arithmetic)
# ----------------------------------------------------------------------------
def random_state(n, seed, spread=10.0, vscale=0.3, field_mass=0.0, n_m=None):
    rng = np.random.default_rng(seed)
    s = dict(
        x=rng.uniform(-spread, spread, n), y=rng.uniform(-spread, spread, n),
        z=rng.uniform(-spread / 10, spread / 10, n),
        vx=rng.normal(0, vscale, n), vy=rng.normal(0, vscale, n), vz=rng.normal(0, vscale / 10, n),
        m=rng.uniform(1e-9, 1e-5, n), rh=rng.uniform(0.0, 0.5, n))
    if n_m is not None and n_m < n - 1:
        s["m"][n_m:] = field_mass
        s["rh"][n_m:] = 0.0
    return s


def massive_count(n, n_m):
    return n if n_m >= n - 1 else n_m


def rows_count(n, n_m):
    return min(n_m, n - 1)


# ----------------------------------------------------------------------------
# force pins
# ----------------------------------------------------------------------------
def brute_force_accel(s, n_m, dps=50):
    """a_k = sum over massive j != k of m_j (x_j - x_k)/|x_j - x_k|^3, in 50 digits."""
    n = len(s["x"])
    nmass = massive_count(n, n_m)
    out = np.zeros((n, 3))
    if rows_count(n, n_m) <= 0:
        return out
    with mpmath.workdps(dps):
        P = [[mpmath.mpf(float(s[c][k])) for c in ("x", "y", "z")] for k in range(n)]
        M = [mpmath.mpf(float(s["m"][k])) for k in range(n)]
        for k in range(n):
            acc = [mpmath.mpf(0)] * 3
            for j in range(nmass):
                if j == k:
                    continue
                d = [P[j][c] - P[k][c] for c in range(3)]
                r = mpmath.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
                for c in range(3):
                    acc[c] += M[j] * d[c] / r ** 3
            out[k] = [float(a) for a in acc]
    return out


def check_force_brute(o):
    cases = [(2, 1, 0), (3, 2, 1), (5, 4, 2), (7, 7, 3), (9, 3, 4), (12, 11, 5), (12, 0, 6),
             (10, 1, 7), (11, 5, 8)]
    for n, n_m, seed in cases:
        s = random_state(n, seed, n_m=n_m, field_mass=0.0)
        ref = brute_force_accel(s, n_m)
        got = o.accel(s, n_m)
        for k in range(n):
            nr = np.linalg.norm(ref[k])
            err = np.linalg.norm(got[k] - ref[k])
            assert err <= 1e-13 * max(nr, 1e-300) or (nr == 0 and err == 0), \
                f"brute force n={n} n_m={n_m} body {k}: {got[k]} vs {ref[k]}"
        # the fused step must give the same accelerations
        fused = o.kick_encounter(s, n_m, 0.5, 1.0)["acc"]
        assert np.array_equal(fused, got), "fused step differs from the force loop"


def check_two_body_exact(o):
    for k in (-3, 0, 2, 5):
        for axis in range(3):
            d = 2.0 ** k
            s = {c: np.zeros(2) for c in ("x", "y", "z", "vx", "vy", "vz", "rh")}
            s["m"] = np.array([3.0e-6, 5.0e-7])
            s[("x", "y", "z")[axis]][1] = d
            s["x"] += 1.5  # a dyadic common offset keeps the difference exact
            a = o.accel(s, 1)
            exp0 = np.zeros(3); exp0[axis] = s["m"][1] / d ** 2
            exp1 = np.zeros(3); exp1[axis] = -s["m"][0] / d ** 2
            assert np.array_equal(a[0], exp0) and np.array_equal(a[1], exp1), \
                f"two-body closed form failed at |d|=2^{k} axis {axis}: {a}"
            s2 = {c: v.copy() for c, v in s.items()}  # N_m = N gives the same result
            assert np.array_equal(o.accel(s2, 2), a)


def check_ring(o):
    for n, R in ((5, 7.25), (16, 11.0), (33, 5.5)):
        m = 2.5e-6
        th = 2 * np.pi * np.arange(n) / n + 0.3
        tilt = 0.4
        x = R * np.cos(th)
        y = R * np.sin(th) * np.cos(tilt)
        z = R * np.sin(th) * np.sin(tilt)
        s = dict(x=x, y=y, z=z, m=np.full(n, m))
        a = o.accel(s, n - 1)
        mag = m / (4 * R * R) * sum(1.0 / math.sin(math.pi * k / n) for k in range(1, n))
        pos = np.stack([x, y, z], axis=1)
        expected = -mag * pos / R
        err = np.abs(a - expected).max() / mag
        assert err < 1e-13, f"ring n={n}: relative error {err}"


def check_momentum(o):
    for n, n_m, seed in ((50, 49, 11), (80, 30, 12), (64, 64, 13)):
        s = random_state(n, seed, n_m=n_m)
        a = o.accel(s, n_m)
        nmass = massive_count(n, n_m)
        m = s["m"][:nmass]
        total = (m[:, None] * a[:nmass]).sum(axis=0)
        pos = np.stack([s["x"], s["y"], s["z"]], axis=1)[:nmass]
        d = pos[None, :, :] - pos[:, None, :]
        r2 = (d ** 2).sum(-1) + np.eye(nmass)
        scale = (m[:, None] * m[None, :] / r2).sum()
        assert np.all(np.abs(total) <= 8 * nmass * EPS * scale), f"momentum {total} scale {scale}"
        # with the Sun's indirect term: sum m_i a_hel_i + (1 + sum m_i) A0 = 0
        h = o.helio(s, n_m, a)
        r3 = (pos ** 2).sum(-1) ** 1.5
        A0 = (m[:, None] * pos / r3[:, None]).sum(axis=0)
        resid = (m[:, None] * h[:nmass]).sum(axis=0) + (1.0 + m.sum()) * A0
        sc = scale + (m[:, None] * np.abs(pos) / r3[:, None]).sum() * (2 + m.sum())
        assert np.all(np.abs(resid) <= 16 * nmass * EPS * sc), f"indirect-term momentum {resid}"


def check_kepler_limit(o):
    for x0, y0, z0, m in ((1.0, 0.0, 0.0, 3e-6), (0.0, -4.0, 0.0, 1e-3), (2.0, 3.0, -1.0, 0.0)):
        s = dict(x=np.array([x0]), y=np.array([y0]), z=np.array([z0]), m=np.array([m]))
        a = o.accel(s, 0)
        assert np.all(a == 0.0)
        h = o.helio(s, 0, a)
        r = math.sqrt(x0 * x0 + y0 * y0 + z0 * z0)
        exp = -(1.0 + m) * np.array([x0, y0, z0]) / r ** 3
        assert np.allclose(h[0], exp, rtol=2e-15, atol=0), f"Kepler limit {h[0]} vs {exp}"


def check_invariances(o):
    rng = np.random.default_rng(21)
    n = 24
    grid = 2.0 ** -20
    s = dict(x=rng.integers(-2 ** 22, 2 ** 22, n) * grid, y=rng.integers(-2 ** 22, 2 ** 22, n) * grid,
             z=rng.integers(-2 ** 18, 2 ** 18, n) * grid, m=rng.uniform(1e-8, 1e-5, n))
    a = o.accel(s, n - 1)
    t = dict(s, x=s["x"] + 32.0, y=s["y"] - 8.0, z=s["z"] + 0.5)
    assert np.array_equal(o.accel(t, n - 1), a), "translation by a dyadic shift changed the result"
    u = dict(s, m=s["m"] * 2.0 ** 7)
    assert np.array_equal(o.accel(u, n - 1), a * 2.0 ** 7), "mass scaling by 2^7 is not exact"


def check_massive_field_semantics(o):
    n, n_m = 20, 6
    s = random_state(n, 31, n_m=n_m, field_mass=0.0)
    a = o.accel(s, n_m)
    # field particles exert no force: their masses are never used
    s2 = dict(s, m=s["m"].copy())
    s2["m"][n_m:] = np.random.default_rng(3).uniform(1e-4, 1e-3, n - n_m)
    assert np.array_equal(o.accel(s2, n_m), a), "field-particle masses changed the result"
    # field-field pairs never interact: moving one field body leaves other field bodies alone
    s3 = dict(s, x=s["x"].copy())
    s3["x"][n - 1] += 0.25
    a3 = o.accel(s3, n_m)
    assert np.array_equal(a3[n_m:n - 1], a[n_m:n - 1]), "field bodies interacted"
    assert np.array_equal(a3[:n_m], a[:n_m]), "a field particle pulled a massive body"
    assert not np.array_equal(a3[n - 1], a[n - 1])
    # N_m = N - 1 and N_m = N are the same (all massive)
    s4 = random_state(15, 32)
    assert np.array_equal(o.accel(s4, 14), o.accel(s4, 15))
    # every body feels exactly the massive bodies (brute force, field masses nonzero)
    ref = brute_force_accel(dict(s2, m=np.where(np.arange(n) < n_m, s2["m"], 0.0)), n_m)
    got = o.accel(s2, n_m)
    assert np.allclose(got, ref, rtol=1e-13, atol=0)
    # body-by-body sums agree with the loop nest
    for k in (0, n_m - 1, n_m, n - 1):
        assert np.allclose(o.accel_body(s2, n_m, k), got[k], rtol=1e-13, atol=1e-30)


# ----------------------------------------------------------------------------
# encounter pins
# ----------------------------------------------------------------------------
def exact_min_sep2(d, w, dt):
    """min over t in [0, dt] of |d + w t|^2 in exact rationals."""
    d = [Fraction(v) for v in d]
    w = [Fraction(v) for v in w]
    dt = Fraction(dt)
    v2 = sum(c * c for c in w)
    vr = sum(a * b for a, b in zip(d, w))
    if v2 == 0:
        t = Fraction(0)
    else:
        t = min(max(-vr / v2, Fraction(0)), dt)
    return sum((a + b * t) ** 2 for a, b in zip(d, w)), t


def _pair_case(d, w, rhi, rhj):
    bi = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0, rhi)
    bj = (d[0], d[1], d[2], w[0], w[1], w[2], rhj)
    return bi, bj


def check_encounter_exact(o, n_cases=3000, seed=41):
    rng = np.random.default_rng(seed)
    dt = 0.5 * 2 * math.pi
    f = 3.0
    seen = {("start", True): 0, ("start", False): 0, ("end", True): 0, ("end", False): 0,
            ("interior", True): 0, ("interior", False): 0}
    for _ in range(n_cases):
        rhi, rhj = rng.uniform(0.005, 0.05, 2)
        rc = Fraction(float(f * rhi)) + Fraction(float(f * rhj))
        rcf = float(rc)
        regime = rng.integers(3)
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        p = rng.normal(size=3); p -= p.dot(u) * u; p /= np.linalg.norm(p)
        target = rcf * rng.uniform(0.6, 1.4)
        if regime == 0:      # receding: closest at the start
            d = target * u
            w = rng.uniform(0.001, 0.1) * (u + 0.5 * rng.normal(size=3) * 0.2)
            if d.dot(w) < 0:
                w = -w
        elif regime == 1:    # still approaching at the end: the closest point is the end
            end = target * u
            w = rng.uniform(0.001, 0.1) * (-u + 0.3 * p)
            d = end - w * dt
        else:                # closest approach inside the step
            b = target
            speed = rng.uniform(0.001, 0.2)
            t_star = dt * rng.uniform(0.05, 0.95)
            w = -speed * u
            d = b * p + speed * t_star * u
        d = [float(v) for v in d]
        w = [float(v) for v in w]
        m2, t = exact_min_sep2(d, w, dt)
        ratio = m2 / (rc * rc)
        if abs(ratio - 1) < Fraction(1, 10 ** 9):
            continue
        expect = ratio < 1
        bi, bj = _pair_case(d, w, rhi, rhj)
        got = o.encounter(bi, bj, dt, f)
        assert got == expect, f"encounter d={d} w={w} exact ratio {float(ratio)} got {got}"
        assert o.encounter(bj, bi, dt, f) == got, "encounter test is not symmetric"
        kind = "start" if t == 0 else ("end" if t == Fraction(dt) else "interior")
        seen[(kind, expect)] += 1
    assert all(v > 20 for v in seen.values()), f"regimes not all exercised: {seen}"


def check_encounter_special(o):
    dt, f = math.pi, 2.0
    rh = 0.25                       # rc = 2*0.25 + 2*0.25 = 1 exactly
    # stationary pair: flagged iff r < rc, strict at equality
    for r, exp in ((0.5, True), (0.999, True), (1.0, False), (1.0000001, False)):
        bi, bj = _pair_case((r, 0.0, 0.0), (0.0, 0.0, 0.0), rh, rh)
        assert o.encounter(bi, bj, dt, f) == exp, f"stationary r={r}"
    # receding from exactly rc: not flagged (strict)
    bi, bj = _pair_case((1.0, 0.0, 0.0), (0.25, 0.0, 0.0), rh, rh)
    assert not o.encounter(bi, bj, dt, f)
    # head-on approach that gets inside rc within dt
    bi, bj = _pair_case((4.0, 0.0, 0.0), (-1.0, 0.0, 0.0), rh, rh)
    assert o.encounter(bi, bj, dt, f)
    # head-on approach that reaches exactly rc at the end of a dyadic step: not flagged
    bi, bj = _pair_case((2.0, 0.0, 0.0), (-0.5, 0.0, 0.0), rh, rh)
    assert not o.encounter(bi, bj, 2.0, f)
    assert o.encounter(bi, bj, 2.0 + 2.0 ** -40, f)
    # fly-by passing inside rc mid-step, outside at both ends
    bi, bj = _pair_case((-3.0, 0.5, 0.0), (6.0 / dt, 0.0, 0.0), rh, rh)
    assert o.encounter(bi, bj, dt, f)
    # same geometry but slower: closest approach after the step, end point outside
    bi, bj = _pair_case((-3.0, 0.5, 0.0), (0.5 / dt, 0.0, 0.0), rh, rh)
    assert not o.encounter(bi, bj, dt, f)
    # fly-by missing by more than rc
    bi, bj = _pair_case((-3.0, 1.5, 0.0), (6.0 / dt, 0.0, 0.0), rh, rh)
    assert not o.encounter(bi, bj, dt, f)
    # dt = 0 keeps only the start-of-step test
    bi, bj = _pair_case((1.5, 0.0, 0.0), (-10.0, 0.0, 0.0), rh, rh)
    assert not o.encounter(bi, bj, 0.0, f)
    assert o.encounter(bi, bj, dt, f)
    # coincident bodies are flagged; a massless pair with rh = 0 never is
    bi, bj = _pair_case((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), rh, rh)
    assert o.encounter(bi, bj, dt, f)
    bi, bj = _pair_case((1e-9, 0.0, 0.0), (0.0, 0.0, 0.0), 0.0, 0.0)
    assert not o.encounter(bi, bj, dt, f)
    # the critical radius is the sum of both bodies' f * R_H
    bi, bj = _pair_case((0.7, 0.0, 0.0), (0.0, 0.0, 0.0), 0.25, 0.125)
    assert o.encounter(bi, bj, dt, f)           # rc = 0.75
    bi, bj = _pair_case((0.8, 0.0, 0.0), (0.0, 0.0, 0.0), 0.25, 0.125)
    assert not o.encounter(bi, bj, dt, f)


def check_pair_enumeration(o):
    """Pairs come from the trapezoid only, each once, in lexicographic order."""
    for n, n_m, seed in ((30, 29, 51), (40, 12, 52), (25, 25, 53), (18, 0, 54), (22, 1, 55)):
        s = random_state(n, seed, spread=2.0, n_m=n_m)
        s["rh"][:] = np.where(np.arange(n) < massive_count(n, n_m), 0.2, 0.0)
        dt, f = 0.7, 1.5
        pi, pj = o.pairs(s, n_m, dt, f)
        expect = []
        for i in range(rows_count(n, n_m)):
            for j in range(i + 1, n):
                bi = tuple(s[c][i] for c in ("x", "y", "z", "vx", "vy", "vz", "rh"))
                bj = tuple(s[c][j] for c in ("x", "y", "z", "vx", "vy", "vz", "rh"))
                m2, _ = exact_min_sep2([bj[c] - bi[c] for c in range(3)],
                                       [bj[c] - bi[c] for c in range(3, 6)], dt)
                rc = Fraction(float(f * bi[6])) + Fraction(float(f * bj[6]))
                if m2 < rc * rc:
                    expect.append((i, j))
        got = list(zip(pi.tolist(), pj.tolist()))
        assert got == expect, f"pairs n={n} n_m={n_m}: {got[:10]} vs {expect[:10]}"
        # the predicate over a list of pairs: the same decisions, pair by pair
        ii = np.array([i for i in range(rows_count(n, n_m)) for j in range(i + 1, n)], np.int32)
        jj = np.array([j for i in range(rows_count(n, n_m)) for j in range(i + 1, n)], np.int32)
        flags = o.encounter_list(s, ii, jj, dt, f)
        assert list(zip(ii[flags].tolist(), jj[flags].tolist())) == expect
        assert len(set(got)) == len(got)
        fused = o.kick_encounter(s, n_m, dt, f)
        assert np.array_equal(fused["pair_i"], pi) and np.array_equal(fused["pair_j"], pj)
        for i in (0, n - 1, n // 2):
            partners = o.partners(s, n_m, i, dt, f)
            exp = sorted([b for a, b in got if a == i] + [a for a, b in got if b == i])
            assert partners.tolist() == exp


# ----------------------------------------------------------------------------
# grouping pins
# ----------------------------------------------------------------------------
def reference_groups(n, pi, pj):
    g = sp.coo_matrix((np.ones(len(pi)), (pi, pj)), shape=(n, n))
    ncomp, lab = connected_components(g, directed=False)
    first = np.full(ncomp, n)
    np.minimum.at(first, lab, np.arange(n))
    sizes = np.bincount(lab, minlength=ncomp)
    return first[lab].astype(np.int32), int((sizes >= 2).sum())


def check_groups(o):
    rng = np.random.default_rng(61)
    for n, e in ((1, 0), (10, 0), (10, 3), (50, 30), (200, 150), (300, 600), (64, 2000)):
        if n > 1 and e:
            a = rng.integers(0, n, e)
            b = rng.integers(0, n, e)
            keep = a != b
            a, b = a[keep], b[keep]
            pi, pj = np.minimum(a, b), np.maximum(a, b)
        else:
            pi = pj = np.zeros(0, np.int64)
        gid, ng = o.groups(n, pi, pj)
        ref, rng_ng = reference_groups(n, pi, pj)
        assert np.array_equal(gid, ref), f"groups n={n} e={e}"
        assert ng == rng_ng
    # hand-built: a chain joined at its far end, a star and an isolated body
    pi = np.array([5, 6, 7, 0, 0, 0], np.int32)
    pj = np.array([6, 7, 8, 8, 2, 3], np.int32)
    gid, ng = o.groups(10, pi, pj)
    assert gid.tolist() == [0, 1, 0, 0, 4, 0, 0, 0, 0, 9] and ng == 1
    gid, ng = o.groups(6, np.array([3, 1], np.int32), np.array([4, 2], np.int32))
    assert gid.tolist() == [0, 1, 1, 3, 3, 5] and ng == 2


ALL_CHECKS = [check_two_body_exact, check_ring, check_momentum, check_kepler_limit,
              check_invariances, check_massive_field_semantics, check_force_brute,
              check_encounter_special, check_encounter_exact, check_pair_enumeration,
              check_groups]
