"""Oracle of one SyMBA step with its close encounters resolved -- test
infrastructure only (tests, the smoke check and the benchmark's CPU baseline
may use it; the GPU library never does).

The paper (Sec. 2, last paragraph; Sec. 3) integrates the encounter groups
found by the close-encounter check in parallel, the pairs of one group one
after the other, with SyMBA's multiple time step scheme (Duncan, Levison &
Lee 1998): M = 4 substeps per level, adjacent shell radii in the ratio 2.08,
and the partition function f_l with l = 3 (Brasser et al. 2015).  The paper
names these but does not define them, so this module states one reading of
them, derived from the mathematics of a force split into smooth shells:

Shells.  A pair (i, j) has the critical radius R_0 = f (rh_i + rh_j) of the
encounter check (f the critical-radius factor, rh Hill radii) and the inner
radii R_k = R_{k-1} / 2.08.

Partition.  f_3 is the polynomial of degree 7 that rises from 0 at x = 0 to 1
at x = 1 with its first three derivatives zero at both ends:
    f_3(x) = 35 x^4 - 84 x^5 + 70 x^6 - 20 x^7,   f_3'(x) = 140 x^3 (1 - x)^3.
F_k(r) = f_3((r - R_{k+1}) / (R_k - R_{k+1})), clipped to 0 below R_{k+1} and
to 1 above R_k; F_{-1} = 0.  The pair potential V = -m_i m_j / r is split as
    V = sum_{k=0}^{L} V^(k),  V^(k) = V W_k,  W_k = F_k - F_{k-1} (k < L),
    W_L = 1 - F_{L-1}  (everything left at the deepest level L = 8).
The force of V W on body i is m_j (W - r W') (x_j - x_i) / r^3: the exact
gradient, derivative of the weight included, so every kick is the exact flow
of a potential and the map stays symplectic.

Step (time step h; heliocentric positions x, barycentric velocities v, the
Sun's mass 1, G = 1):
    v += (h/2) a0;  x += (h/2) P;  drift;  x += (h/2) P;  evaluate;  v += (h/2) a0,
with a0 the level-0 acceleration (every pair weighted by W_0 = F_0, which is
1 outside R_0) and P = sum of m v over the massive bodies.  The drift moves
every body in no flagged pair along its Kepler orbit for h.  The flagged
pairs (those the close-encounter check of the evaluation at the step's start
found, screened |h| ahead) form the encounter groups (connected components);
each group is integrated on its own, its pairs in their lexicographic order,
by M substeps of level 1.  A substep of level k >= 1 and length tau is
    kick_k(tau/2);  check;  drift;  kick_k(tau/2),
where kick_k applies the forces of V^(k) of the pairs at level k, the check
applies the close-encounter test with radius R_k over tau to those pairs (the
flagged ones form level k + 1), the bodies of no flagged pair drift along
their Kepler orbits for tau, and the others take M substeps of level k + 1
of length tau / M.  At level L there is no check: its bodies drift for tau.
The evaluation at the step's end gives the Newtonian accelerations, the
pairs flagged for the next step (with the velocities before the closing
kick) and their groups; the accelerations of flagged pairs inside R_0 are
then re-weighted to level 0.

Plain float64 numpy and Python loops, slow and direct: groups are small.
"""
from __future__ import annotations

import numpy as np

from . import default as _default
from .dh_step import kepler_drift, sun_momentum

M_SUB = 4             # substeps per level (the paper's Sec. 3)
SHELL_RATIO = 2.08    # R_k / R_{k+1} (the paper's Sec. 3)
L_MAX = 8             # deepest level (a reading: the paper gives none)


def partition(x):
    """f_3 on [0, 1] (clipped outside) and its derivative."""
    x = np.clip(np.asarray(x, dtype=np.float64), 0.0, 1.0)
    f = x ** 4 * (35.0 - 84.0 * x + 70.0 * x ** 2 - 20.0 * x ** 3)
    df = 140.0 * x ** 3 * (1.0 - x) ** 3
    return f, df


def shell_radius(r0, k):
    """R_k = R_0 / 2.08^k, by k successive divisions."""
    r = np.asarray(r0, dtype=np.float64)
    for _ in range(k):
        r = r / SHELL_RATIO
    return r


def changeover(k, r, r0):
    """F_k(r) and dF_k/dr for a pair of critical radius r0 (F_{-1} = 0)."""
    r = np.asarray(r, dtype=np.float64)
    if k < 0:
        return np.zeros_like(r), np.zeros_like(r)
    hi, lo = shell_radius(r0, k), shell_radius(r0, k + 1)
    f, df = partition((r - lo) / (hi - lo))
    return f, df / (hi - lo)


def weight(k, r, r0):
    """W_k(r) and W_k'(r) of level k (0 <= k <= L_MAX)."""
    if k == L_MAX:
        f, df = changeover(k - 1, r, r0)
        return 1.0 - f, -df
    fa, dfa = changeover(k, r, r0)
    fb, dfb = changeover(k - 1, r, r0)
    return fa - fb, dfa - dfb


def force_factor(k, r, r0):
    """W - r W': the factor on the Newtonian pair force of level k."""
    w, dw = weight(k, r, r0)
    return w - r * dw


def encounter(dx, dv, radius, tau):
    """The close-encounter test with radius `radius` over an interval tau:
    inside now, inside at the linearly extrapolated end, or a closest
    approach within the interval that is inside.  A negative tau (a step
    backwards in time) tests the reversed motion over |tau|."""
    if tau < 0.0:
        dv, tau = -dv, -tau
    r2 = float(dx @ dx)
    v2 = float(dv @ dv)
    vr = float(dx @ dv)
    rc2 = radius * radius
    if r2 < rc2:
        return True
    if r2 + 2.0 * vr * tau + v2 * tau * tau < rc2:
        return True
    if vr < 0.0 and -vr < v2 * tau:
        return r2 * v2 - vr * vr < rc2 * v2
    return False


def _groups(pairs):
    """Connected components of the pair graph: lists of pair indices, each in
    the pairs' order, the components ordered by their smallest body."""
    parent = {}

    def find(a):
        while parent.setdefault(a, a) != a:
            a = parent[a]
        return a

    for i, j in pairs:
        a, b = find(int(i)), find(int(j))
        if a != b:
            parent[max(a, b)] = min(a, b)
    comp = {}
    for p, (i, _) in enumerate(pairs):
        comp.setdefault(find(int(i)), []).append(p)
    return [comp[k] for k in sorted(comp)]


class _Group:
    """One encounter group: its bodies' positions and velocities (rows of X,
    V), masses (0 for field bodies), critical radii and pairs (local
    indices, the pairs' order)."""

    def __init__(self, X, V, m, rc, pairs):
        self.X, self.V, self.m, self.rc = X, V, m, rc
        self.pairs = pairs

    def kick(self, k, dt, active):
        a = np.zeros_like(self.V)
        for p in active:
            i, j = self.pairs[p]
            d = self.X[j] - self.X[i]
            r = float(np.sqrt(d @ d))
            g = float(force_factor(k, r, self.rc[i] + self.rc[j])) / (r * r * r)
            a[i] += (self.m[j] * g) * d
            a[j] -= (self.m[i] * g) * d
        for b in sorted({b for p in active for b in self.pairs[p]}):
            self.V[b] = self.V[b] + dt * a[b]

    def drift(self, bodies, tau):
        if bodies:
            idx = sorted(bodies)
            x, v = kepler_drift(self.X[idx], self.V[idx], tau)
            self.X[idx], self.V[idx] = x, v

    def substep(self, k, tau, active):
        self.kick(k, tau / 2, active)
        bodies = {b for p in active for b in self.pairs[p]}
        if k == L_MAX:
            self.drift(bodies, tau)
        else:
            flagged = []
            for p in active:
                i, j = self.pairs[p]
                if encounter(self.X[j] - self.X[i], self.V[j] - self.V[i],
                             float(shell_radius(self.rc[i] + self.rc[j], k)), tau):
                    flagged.append(p)
            deeper = {b for p in flagged for b in self.pairs[p]}
            self.drift(bodies - deeper, tau)
            for _ in range(M_SUB):
                if flagged:
                    self.substep(k + 1, tau / M_SUB, flagged)
        self.kick(k, tau / 2, active)

    def integrate(self, h):
        everything = list(range(len(self.pairs)))
        for _ in range(M_SUB):
            self.substep(1, h / M_SUB, everything)


def _xv(s):
    x = np.stack([s["x"], s["y"], s["z"]], axis=1).astype(np.float64)
    v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1).astype(np.float64)
    return x, v


def _masses(s, n_m):
    m = np.asarray(s["m"], dtype=np.float64).copy()
    n = m.size
    n_tri = n if n_m >= n - 1 else n_m
    m[n_tri:] = 0.0
    return m


def level0_correction(s, n_m, f, pair_i, pair_j):
    """What turns the Newtonian accelerations of state s into level-0 ones:
    for every listed pair inside R_0, m (F_0 - r F_0' - 1) (x_j - x_i) / r^3
    on i and its opposite (with m_i) on j, summed in the pairs' order."""
    x, _ = _xv(s)
    m = _masses(s, n_m)
    rc = f * np.asarray(s["rh"], dtype=np.float64)
    da = np.zeros_like(x)
    for i, j in zip(pair_i, pair_j):
        d = x[j] - x[i]
        r = float(np.sqrt(d @ d))
        r0 = rc[i] + rc[j]
        if r >= r0:
            continue
        g = (float(force_factor(0, r, r0)) - 1.0) / (r * r * r)
        da[i] += (m[j] * g) * d
        da[j] -= (m[i] * g) * d
    return da


def accel_level0(s, n_m, f):
    """The level-0 acceleration by its definition: every pair of the
    trapezoid with its force weighted by W_0 - r W_0' (massive bodies pull),
    O(N^2) numpy."""
    x, _ = _xv(s)
    m = _masses(s, n_m)
    rc = f * np.asarray(s["rh"], dtype=np.float64)
    n = len(x)
    a = np.zeros_like(x)
    for i in range(n):
        d = x - x[i]
        r = np.sqrt(np.sum(d * d, axis=1))
        r[i] = 1.0
        g = force_factor(0, r, rc[i] + rc) / r ** 3
        g[i] = 0.0
        a[i] = np.sum((m * g)[:, None] * d, axis=0)
    return a


def prepare(s, n_m, h, f, ora=None):
    """The step's inputs for state s: level-0 accelerations and the pairs the
    check flags |h| ahead."""
    ora = ora if ora is not None else _default()
    ev = ora.kick_encounter(s, n_m, abs(h), f)
    acc = ev["acc"] + level0_correction(s, n_m, f, ev["pair_i"], ev["pair_j"])
    return acc, np.stack([ev["pair_i"], ev["pair_j"]], axis=1)


def step(s, n_m, h, f, acc, pairs, ora=None, group_order=None):
    """One step of state s (dict x y z vx vy vz m rh) with level-0
    accelerations acc ([n, 3]) and flagged pairs ([p, 2], lexicographic)
    at s.  Returns (new state, level-0 accelerations, flagged pairs) at the
    new positions.  group_order, if given, is the order in which the groups
    are integrated (a permutation of their indices): groups are independent,
    so it must not change any bit."""
    ora = ora if ora is not None else _default()
    x, v = _xv(s)
    m = np.asarray(s["m"], dtype=np.float64)
    ms = _masses(s, n_m)
    rc = f * np.asarray(s["rh"], dtype=np.float64)
    v = v + (h / 2) * acc
    x = x + (h / 2) * sun_momentum(v, m, n_m)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    in_pair = np.zeros(len(x), dtype=bool)
    in_pair[pairs.ravel()] = True
    free = np.flatnonzero(~in_pair)
    if free.size:
        x[free], v[free] = kepler_drift(x[free], v[free], h)
    groups = _groups(pairs)
    order = range(len(groups)) if group_order is None else group_order
    for g in order:
        gp = pairs[groups[g]]
        bodies = np.unique(gp)
        local = {int(b): k for k, b in enumerate(bodies)}
        G = _Group(x[bodies].copy(), v[bodies].copy(), ms[bodies], rc[bodies],
                   [(local[int(i)], local[int(j)]) for i, j in gp])
        G.integrate(h)
        x[bodies], v[bodies] = G.X, G.V
    x = x + (h / 2) * sun_momentum(v, m, n_m)
    new = dict(s)
    new.update(x=x[:, 0].copy(), y=x[:, 1].copy(), z=x[:, 2].copy(),
               vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy())
    ev = ora.kick_encounter(new, n_m, abs(h), f)
    acc_new = ev["acc"] + level0_correction(new, n_m, f, ev["pair_i"], ev["pair_j"])
    v = v + (h / 2) * acc_new
    new.update(vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy())
    return new, acc_new, np.stack([ev["pair_i"], ev["pair_j"]], axis=1)
