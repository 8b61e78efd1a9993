"""Pins of the step oracle (oracle/dh_step.py) against what the mathematics
fixes: Kepler orbits from their elements, the circle's rotation, exact time
reversal of the symmetric map, conservation of the energy it approximately
conserves, and the massless limit."""
import math

import numpy as np
import pytest

import oracle
from oracle import dh_step as S
from paper_2304_07325_amd import diskgen as dg


def _orbits(n, seed, emax):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 30.0, n)
    e = rng.uniform(0.0, emax, n)
    inc = rng.uniform(0.0, math.pi, n)
    Om, om, M = (rng.uniform(0.0, 2 * math.pi, n) for _ in range(3))
    return a, e, inc, Om, om, M


@pytest.mark.parametrize("emax", [0.0, 0.3, 0.7])
def test_kepler_drift_matches_elements(emax):
    """Drifting a state for h equals the state built from its elements with the
    mean anomaly advanced by n h (an independent route: eccentric anomaly from
    Kepler's equation), over arcs from a tiny fraction to several periods."""
    a, e, inc, Om, om, M = _orbits(200, 5, emax)
    pos, vel = dg.elements_to_cartesian(a, e, inc, Om, om, M, 1.0)
    x0, v0 = np.stack(pos, 1), np.stack(vel, 1)
    for h in (1e-3, 0.7, 25.0, -13.0):
        x, v = S.kepler_drift(x0, v0, h)
        nmot = np.sqrt(1.0 / a ** 3)
        pos1, vel1 = dg.elements_to_cartesian(a, e, inc, Om, om, np.mod(M + nmot * h, 2 * math.pi), 1.0)
        x1, v1 = np.stack(pos1, 1), np.stack(vel1, 1)
        np.testing.assert_allclose(x, x1, rtol=0, atol=1e-11 * np.abs(x1).max())
        np.testing.assert_allclose(v, v1, rtol=0, atol=1e-11 * np.abs(v1).max())


def test_kepler_drift_circle_is_a_rotation():
    r, w = 4.0, 4.0 ** -1.5
    for h in (0.1, 3.0, 100.0):
        x, v = S.kepler_drift(np.array([[r, 0.0, 0.0]]), np.array([[0.0, r * w, 0.0]]), h)
        np.testing.assert_allclose(x[0], [r * math.cos(w * h), r * math.sin(w * h), 0.0], atol=1e-13)
        np.testing.assert_allclose(v[0], [-r * w * math.sin(w * h), r * w * math.cos(w * h), 0.0], atol=1e-14)


def test_kepler_drift_hyperbolic_conserves_and_reverses():
    """Unbound orbits: energy and angular momentum kept, and drifting back
    returns the start."""
    rng = np.random.default_rng(3)
    x0 = rng.normal(size=(50, 3)) * 5
    v0 = rng.normal(size=(50, 3))
    r0 = np.linalg.norm(x0, axis=1)
    v0 *= (np.sqrt(2.0 / r0) * rng.uniform(1.1, 3.0, 50) / np.linalg.norm(v0, axis=1))[:, None]
    x, v = S.kepler_drift(x0, v0, 40.0)
    en = lambda x, v: 0.5 * np.sum(v * v, 1) - 1.0 / np.linalg.norm(x, axis=1)
    np.testing.assert_allclose(en(x, v), en(x0, v0), rtol=1e-12)
    np.testing.assert_allclose(np.cross(x, v), np.cross(x0, v0), rtol=0, atol=1e-11 * np.abs(np.cross(x0, v0)).max())
    xb, vb = S.kepler_drift(x, v, -40.0)
    np.testing.assert_allclose(xb, x0, atol=1e-10)
    np.testing.assert_allclose(vb, v0, atol=1e-12)


def _system(n=12, seed=4):
    d = dg.make_accuracy_disk(n=n, seed=seed)
    return d.state(0), d.n_massive, d.dt


def test_step_is_time_reversible():
    """The map is a symmetric composition, so a step of -h undoes a step of h."""
    s0, n_m, h = _system()
    s1, _ = S.step(s0, n_m, h)
    s2, _ = S.step(s1, n_m, -h)
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(s2[k], s0[k], rtol=0, atol=1e-12)
    for k in ("vx", "vy", "vz"):
        np.testing.assert_allclose(s2[k], s0[k], rtol=0, atol=1e-14)


def test_step_conserves_energy():
    """The paper's accuracy-test kind of system (equal planetesimals 5 Hill
    radii apart, 0.1-year steps): the energy error stays small and bounded,
    and a step that pushed the bodies the wrong way (a sign slip in the kick)
    would not keep it."""
    s, n_m, h = _system(n=10)
    e0 = S.energy(s, n_m)
    acc = None
    errs = []
    for _ in range(400):
        s, acc = S.step(s, n_m, h, acc=acc)
        errs.append(abs(S.energy(s, n_m) - e0) / abs(e0))
    assert max(errs) < 1e-9, max(errs)
    # a sign slip of the interaction term shows up at once
    s, n_m, h = _system(n=10)
    bad = dict(s)
    ora = oracle.default()
    s1, _ = S.step(bad, n_m, h, acc=-ora.accel(bad, n_m))
    assert abs(S.energy(s1, n_m) - e0) / abs(e0) > 10 * max(errs)


def test_massless_step_is_the_kepler_drift():
    """With every mass zero there is no kick and no Sun drift."""
    s, n_m, h = _system()
    s = dict(s, m=np.zeros_like(s["m"]))
    s1, acc = S.step(s, n_m, h)
    x0 = np.stack([s["x"], s["y"], s["z"]], 1)
    v0 = np.stack([s["vx"], s["vy"], s["vz"]], 1)
    x, v = S.kepler_drift(x0, v0, h)
    assert not acc.any()
    np.testing.assert_array_equal(np.stack([s1["x"], s1["y"], s1["z"]], 1), x)
    np.testing.assert_array_equal(np.stack([s1["vx"], s1["vy"], s1["vz"]], 1), v)


def test_kepler_drift_every_conic_keeps_invariants():
    """Ellipses, near-parabolae and hyperbolae over short and very long arcs:
    the drift keeps each orbit's energy and angular momentum."""
    rng = np.random.default_rng(11)
    n = 400
    x = rng.normal(size=(n, 3))
    x *= (rng.uniform(0.5, 30.0, n) / np.linalg.norm(x, axis=1))[:, None]
    r = np.linalg.norm(x, axis=1)
    v = rng.normal(size=(n, 3))
    v *= (np.sqrt(2.0 / r) * rng.uniform(0.2, 2.5, n) / np.linalg.norm(v, axis=1))[:, None]
    v[:30] *= (np.sqrt(2.0 / r[:30]) / np.linalg.norm(v[:30], axis=1))[:, None]
    en = lambda x, v: 0.5 * np.sum(v * v, 1) - 1 / np.linalg.norm(x, axis=1)
    scale = 1 / np.linalg.norm(x, axis=1)
    for h in (0.05, 7.0, 300.0, -40.0):
        xn, vn = S.kepler_drift(x, v, h)
        assert np.isfinite(xn).all() and np.isfinite(vn).all()
        assert (np.abs(en(xn, vn) - en(x, v)) / scale).max() < 1e-11
        np.testing.assert_allclose(np.cross(xn, vn), np.cross(x, v), rtol=0, atol=1e-10)
