"""Pins of the encounter-step oracle (oracle/symba_enc.py) against what the
mathematics fixes: the partition function's smoothness and the exact split
of the pair potential into levels, the level forces as gradients of their
potentials, a close flyby against a high-accuracy solution of the equations
of motion (and its energy and angular momentum), exact time reversal, the
plain step when nothing is flagged, and independence of the group order.
Planted mistakes in the oracle fail these pins (the last tests)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from oracle import dh_step as S
from oracle import symba_enc as E

F = 3.0


def _state(x, v_helio, m, n_m=None):
    """State dict from heliocentric positions and velocities (barycentric
    velocities: the Sun's velocity, -sum m v / (1 + sum m), added)."""
    x, v, m = (np.asarray(a, dtype=np.float64) for a in (x, v_helio, m))
    vb = v - (m[:, None] * v).sum(0) / (1.0 + m.sum())
    rh = (m / 3.0) ** (1.0 / 3.0) * np.linalg.norm(x, axis=1)
    return dict(x=x[:, 0].copy(), y=x[:, 1].copy(), z=x[:, 2].copy(), vx=vb[:, 0].copy(), vy=vb[:, 1].copy(),
                vz=vb[:, 2].copy(), m=m.copy(), rh=rh)


def _flyby(phase=0.0, b=0.003, vrel=0.3, sep=0.3, mA=1e-4, mB=3e-5):
    """Body B overtakes body A (circular orbit at 1 AU) from `sep` behind with
    relative speed vrel and impact parameter b: a fast flyby much closer than
    the critical radius, through several shells.  Rotated by `phase`."""
    c, s = math.cos(phase), math.sin(phase)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    x = np.array([[1.0, 0.0, 0.0], [1.0 + b, -sep, 0.0]]) @ rot.T
    v = np.array([[0.0, 1.0, 0.0], [0.0, 1.0 + vrel, 0.0]]) @ rot.T
    return x, v, np.array([mA, mB])


def _xs(s):
    return np.stack([s["x"], s["y"], s["z"]], axis=1)


def _vs(s):
    return np.stack([s["vx"], s["vy"], s["vz"]], axis=1)


def _ang_mom(s):
    return (s["m"][:, None] * np.cross(_xs(s), _vs(s))).sum(0)


def _exact_positions(s, t):
    """Heliocentric equations of motion (Sun's mass 1, G = 1, indirect term
    included) solved by an 8th-order Runge-Kutta method at tolerance 1e-13."""
    m = s["m"]
    n = m.size
    u = _vs(s) + (m[:, None] * _vs(s)).sum(0)   # heliocentric velocities

    def rhs(_, y):
        X = y[:3 * n].reshape(n, 3)
        A = -(1.0 + m)[:, None] * X / np.linalg.norm(X, axis=1)[:, None] ** 3
        ind = (m[:, None] * X / np.linalg.norm(X, axis=1)[:, None] ** 3)
        for i in range(n):
            for j in range(n):
                if i != j:
                    d = X[j] - X[i]
                    A[i] += m[j] * d / np.linalg.norm(d) ** 3 - ind[j]
        return np.concatenate([y[3 * n:], A.ravel()])

    sol = solve_ivp(rhs, (0.0, t), np.concatenate([_xs(s).ravel(), u.ravel()]), method="DOP853",
                    rtol=1e-13, atol=1e-16)
    return sol.y[:3 * n, -1].reshape(n, 3)


def _run_enc(s, n_m, h, steps):
    acc, pairs = E.prepare(s, n_m, h, F)
    r_min, flagged = np.inf, 0
    for _ in range(steps):
        s, acc, pairs = E.step(s, n_m, h, F, acc, pairs)
        x = _xs(s)
        r_min = min(r_min, float(np.linalg.norm(x[1] - x[0])))
        flagged += len(pairs) > 0
    return s, r_min, flagged


def _run_plain(s, n_m, h, steps):
    acc = oracle.default().accel(s, n_m)
    for _ in range(steps):
        s, acc = S.step(s, n_m, h, acc)
    return s


# --- the partition and the split of the potential ---------------------------

def test_partition_is_the_c3_smoothstep():
    """f_3 is a polynomial of degree 7 (a degree-7 fit through 40 samples is
    exact), 0 at 0 and 1 at 1, with derivatives 1..3 zero at both ends and the
    4th not; the returned derivative is the polynomial's."""
    xs = np.linspace(0.0, 1.0, 40)
    f, df = E.partition(xs)
    p = np.polynomial.Polynomial.fit(xs, f, 7).convert()
    assert np.abs(p(xs) - f).max() < 1e-13
    assert abs(p(0.0)) < 1e-12 and abs(p(1.0) - 1.0) < 1e-12
    for k in (1, 2, 3):
        d = p.deriv(k)
        assert abs(d(0.0)) < 1e-9 and abs(d(1.0)) < 1e-9, k
    assert abs(p.deriv(4)(0.0)) > 100.0
    assert np.abs(p.deriv(1)(xs) - df).max() < 1e-9
    assert np.all(np.diff(f) > 0)
    assert np.array_equal(E.partition(np.array([-0.5, 1.5]))[0], [0.0, 1.0])


def test_levels_split_the_potential_exactly():
    """sum_k W_k = 1 and sum_k W_k' = 0 at every separation: the levels'
    potentials add up to the Newtonian one."""
    r0 = 0.17
    r = np.concatenate([np.geomspace(1e-5, 2.0, 4000), np.array([E.shell_radius(r0, k) for k in range(9)]) * (1 + 1e-9)])
    w = sum(E.weight(k, r, r0)[0] for k in range(E.L_MAX + 1))
    dw = sum(E.weight(k, r, r0)[1] for k in range(E.L_MAX + 1))
    assert np.abs(w - 1.0).max() < 1e-14
    assert np.abs(dw).max() < 1e-9 * np.abs(E.weight(1, r, r0)[1]).max()
    # outside R_0 only level 0 acts, fully; deep inside only the deepest level
    out = r > r0
    assert np.all(E.weight(0, r[out], r0)[0] == 1.0)
    deep = r < E.shell_radius(r0, E.L_MAX)
    assert np.all(E.weight(E.L_MAX, r[deep], r0)[0] == 1.0)


@pytest.mark.parametrize("k", [0, 1, 3, E.L_MAX])
def test_level_force_is_the_gradient(k):
    """m_j (W - r W') / r^2, the radial pull of level k on body i, is
    d/dr(-W(r) / r) per unit masses: checked against central differences of
    the level's potential."""
    r0 = 0.2
    lo = E.shell_radius(r0, min(k + 1, E.L_MAX)) * 0.5
    r = np.linspace(lo, r0 * 1.2, 3001)[1:-1]
    eps = 1e-7 * r

    def pot(rr):
        return -E.weight(k, rr, r0)[0] / rr

    fd = (pot(r + eps) - pot(r - eps)) / (2 * eps)
    g = E.force_factor(k, r, r0) / r ** 2
    assert np.abs(fd - g).max() < 1e-6 * np.abs(g).max() + 1e-6


def test_level0_acceleration_by_its_definition():
    """Newtonian accelerations plus the correction over the flagged pairs are
    the level-0 accelerations summed directly over every pair with its W_0
    weight (pairs inside R_0 are always flagged)."""
    rng = np.random.default_rng(3)
    n = 40
    x = np.c_[rng.uniform(0.95, 1.05, n), rng.uniform(-0.05, 0.05, n), rng.uniform(-0.01, 0.01, n)]
    v = np.c_[-x[:, 1], x[:, 0], np.zeros(n)] + rng.normal(0, 0.01, (n, 3))
    m = rng.uniform(1e-7, 1e-5, n)
    for n_m in (n, 25):
        s = _state(x, v, m)
        ev = oracle.default().kick_encounter(s, n_m, 0.01, F)
        inside = 0
        for i, j in zip(ev["pair_i"], ev["pair_j"]):
            inside += np.linalg.norm(x[j] - x[i]) < F * (s["rh"][i] + s["rh"][j])
        assert inside > 20
        got = ev["acc"] + E.level0_correction(s, n_m, F, ev["pair_i"], ev["pair_j"])
        want = E.accel_level0(s, n_m, F)
        assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()
        assert np.abs(got - ev["acc"]).max() > 1e-3 * np.abs(want).max()   # the weighting matters here


# --- the step --------------------------------------------------------------

@pytest.fixture(scope="module")
def flyby_runs():
    x, v, m = _flyby()
    s0 = _state(x, v, m)
    h, T = 0.025, 2.0
    steps = int(round(T / h))
    enc, r_min, flagged = _run_enc(s0, 2, h, steps)
    plain = _run_plain(s0, 2, h, steps)
    return dict(s0=s0, enc=enc, plain=plain, exact=_exact_positions(s0, T), r_min=r_min, flagged=flagged)


def test_flyby_matches_the_equations_of_motion(flyby_runs):
    """A flyby to 0.07 of the critical radius, resolved by the shells, ends
    within 1e-6 of a high-accuracy solution; the plain step (every pair a
    full-strength kick at the outer step) misses by 100 times more."""
    r = flyby_runs
    r0 = F * r["s0"]["rh"].sum()
    assert r["r_min"] < 0.1 * r0 and r["flagged"] > 10
    err_enc = np.abs(_xs(r["enc"]) - r["exact"]).max()
    err_plain = np.abs(_xs(r["plain"]) - r["exact"]).max()
    assert err_enc < 1e-6, err_enc
    assert err_plain > 100 * err_enc, (err_plain, err_enc)


def test_flyby_energy_and_angular_momentum(flyby_runs):
    """Energy is kept to 1e-6 through the flyby, 100 times better than the
    plain step; angular momentum, which every sub-map conserves exactly, to
    rounding."""
    r = flyby_runs
    e0 = S.energy(r["s0"], 2)
    de = abs(S.energy(r["enc"], 2) - e0) / abs(e0)
    de_plain = abs(S.energy(r["plain"], 2) - e0) / abs(e0)
    assert de < 1e-6 and de_plain > 100 * de, (de, de_plain)
    l0 = _ang_mom(r["s0"])
    assert np.abs(_ang_mom(r["enc"]) - l0).max() < 1e-13 * np.abs(l0).max()


def test_time_reversal():
    """Steps forward, velocities reversed, as many steps again, velocities
    reversed: back at the start to rounding (the window stays inside R_0, so
    the outer flag is the same in both directions)."""
    x, v, m = _flyby(sep=0.12)
    s0 = _state(x, v, m)
    h, steps = 0.025, 20
    acc, pairs = E.prepare(s0, 2, h, F)
    s = s0
    r0 = F * s0["rh"].sum()
    for _ in range(steps):
        s, acc, pairs = E.step(s, 2, h, F, acc, pairs)
        assert len(pairs) == 1 and np.linalg.norm(_xs(s)[1] - _xs(s)[0]) < r0
    back = dict(s, vx=-s["vx"], vy=-s["vy"], vz=-s["vz"])
    acc, pairs = E.prepare(back, 2, h, F)
    for _ in range(steps):
        back, acc, pairs = E.step(back, 2, h, F, acc, pairs)
    assert np.abs(_xs(back) - _xs(s0)).max() < 1e-11
    assert np.abs(-_vs(back) - _vs(s0)).max() < 1e-11


def test_no_flagged_pair_is_the_plain_step():
    """With no pair flagged anywhere, the step is the non-encounter step,
    bit for bit."""
    rng = np.random.default_rng(5)
    n = 60
    a = np.sort(rng.uniform(5.0, 20.0, n))
    th = rng.uniform(0, 2 * np.pi, n)
    x = np.c_[a * np.cos(th), a * np.sin(th), np.zeros(n)]
    v = np.c_[-np.sin(th), np.cos(th), np.zeros(n)] / np.sqrt(a)[:, None]
    s = _state(x, v, np.full(n, 1e-9))
    h = 0.5 * 2 * np.pi
    acc, pairs = E.prepare(s, n, h, F)
    assert len(pairs) == 0
    plain_acc = oracle.default().accel(s, n)
    assert acc.tobytes() == plain_acc.tobytes()
    se, sp = s, s
    for _ in range(3):
        se, acc, pairs = E.step(se, n, h, F, acc, pairs)
        sp, plain_acc = S.step(sp, n, h, plain_acc)
        assert len(pairs) == 0
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert se[k].tobytes() == sp[k].tobytes(), k


def test_group_order_does_not_matter():
    """Three independent flybys around the orbit (three groups): integrating
    the groups in any order gives the same bits."""
    xs, vs, ms = zip(*(_flyby(phase=p, sep=0.1) for p in (0.0, 2.1, 4.2)))
    s = _state(np.concatenate(xs), np.concatenate(vs), np.concatenate(ms))
    h = 0.025
    acc, pairs = E.prepare(s, 6, h, F)
    assert len(pairs) == 3
    ref = E.step(s, 6, h, F, acc, pairs)
    for order in ([2, 1, 0], [1, 2, 0]):
        got = E.step(s, 6, h, F, acc, pairs, group_order=order)
        for k in ("x", "y", "z", "vx", "vy", "vz"):
            assert got[0][k].tobytes() == ref[0][k].tobytes(), (order, k)


# --- planted mistakes --------------------------------------------------------

def _flyby_errors():
    x, v, m = _flyby()
    s0 = _state(x, v, m)
    h, T = 0.025, 2.0
    enc, _, _ = _run_enc(s0, 2, h, int(round(T / h)))
    err = np.abs(_xs(enc) - _exact_positions(s0, T)).max()
    de = abs(S.energy(enc, 2) - S.energy(s0, 2)) / abs(S.energy(s0, 2))
    return err, de


def test_unplanted_oracle_passes_the_short_flyby():
    err, de = _flyby_errors()
    assert err < 1e-6 and de < 1e-6, (err, de)


@pytest.mark.parametrize("mistake", ["derivative_sign", "no_recursion", "own_mass", "weight_level_off"])
def test_planted_mistakes_fail_a_pin(monkeypatch, mistake):
    """Each planted mistake fails the level-force gradient pin or the flyby
    pin (accuracy against the equations of motion, or energy)."""
    if mistake == "derivative_sign":
        def bad(k, r, r0):
            w, dw = E.weight(k, r, r0)
            return w + r * dw
        monkeypatch.setattr(E, "force_factor", bad)
    elif mistake == "no_recursion":
        monkeypatch.setattr(E, "encounter", lambda *a: False)
    elif mistake == "own_mass":
        orig = E._Group.kick

        def bad_kick(self, k, dt, active):
            m = self.m
            self.m = m[::-1].copy()
            try:
                orig(self, k, dt, active)
            finally:
                self.m = m
        monkeypatch.setattr(E._Group, "kick", bad_kick)
    elif mistake == "weight_level_off":
        orig_w = E.weight
        monkeypatch.setattr(E, "weight", lambda k, r, r0: orig_w(min(k + 1, E.L_MAX), r, r0) if k > 0
                            else orig_w(k, r, r0))
    gradient_ok = True
    for k in (0, 1, 3, E.L_MAX):
        try:
            test_level_force_is_the_gradient(k)
        except AssertionError:
            gradient_ok = False
    err, de = _flyby_errors()
    assert not gradient_ok or err > 1e-6 or de > 1e-6, (mistake, err, de)


def test_negative_substeps_test_the_reversed_motion():
    """Over a negative interval the test looks backwards: a pair that
    approaches (will meet within tau) has receded over -tau, and the test
    over -tau of the motion equals the test over tau of the reversed motion."""
    dx = np.array([1.0, 0.0, 0.0])
    dv = np.array([-1.0, 0.0, 0.0])   # closing at unit speed
    assert E.encounter(dx, dv, 0.5, 0.8)        # inside 0.5 within 0.8 ahead
    assert not E.encounter(dx, dv, 0.5, -0.8)   # was farther apart before
    assert E.encounter(dx, -dv, 0.5, -0.8)      # receding pair met in the past
    rng = np.random.default_rng(4)
    for _ in range(200):
        a, w = rng.normal(size=3), rng.normal(size=3)
        rad, tau = rng.uniform(0.1, 2.0), rng.uniform(0.01, 2.0)
        assert E.encounter(a, w, rad, -tau) == E.encounter(a, -w, rad, tau)
