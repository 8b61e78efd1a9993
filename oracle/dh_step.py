"""Oracle of one non-encounter step of SyMBA's democratic heliocentric map --
test infrastructure only (tests, the smoke check and the benchmark's CPU
baseline may use it; the GPU library never does).

SyMBA (the paper's Sec. 1: Duncan, Levison & Lee 1998, a variant of the
Wisdom-Holman map) splits the Hamiltonian, in heliocentric positions x and
barycentric velocities v with G = 1 and the Sun's mass 1, into
  H_Kep = sum_i (m_i |v_i|^2 / 2 - m_i / |x_i|)       each body on its Kepler orbit,
  H_Sun = |sum_i m_i v_i|^2 / 2                       a linear drift of every position,
  H_int = -sum_{i<j} m_i m_j / |x_i - x_j|            the pair interactions (the path),
and one step of length h is the symmetric product
  kick(h/2) . Sun drift(h/2) . Kepler drift(h) . Sun drift(h/2) . kick(h/2),
the kicks applying v_i += (h/2) a_i with a_i the interaction acceleration
of the trapezoid (massive bodies pull every body; field bodies, m = 0, pull
nothing and add nothing to the Sun drift's momentum).  This is the step
outside close encounters: the partition-weighted kick inside rc and the
recursive sub-steps of encounter groups are not computed (their weighting
function is not given).

Plain float64 numpy, slow and direct: the Kepler drift solves the universal
Kepler equation for the universal anomaly chi (Curtis, Orbital Mechanics for
Engineering Students, Sec. 3.7) by bracketed Newton iterations to full
convergence and applies the Lagrange f and g coefficients.
"""
from __future__ import annotations

import numpy as np

from . import default as _default


def stumpff_c(z):
    """C(z) = (1 - cos sqrt z) / z, continued to z <= 0 (series near 0)."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 1e-3
    pos = (z > 0) & ~small
    neg = (z < 0) & ~small
    zs = z[small]
    out[small] = 1 / 2 - zs / 24 + zs ** 2 / 720 - zs ** 3 / 40320
    out[pos] = (1 - np.cos(np.sqrt(z[pos]))) / z[pos]
    out[neg] = (np.cosh(np.sqrt(-z[neg])) - 1) / -z[neg]
    return out


def stumpff_s(z):
    """S(z) = (sqrt z - sin sqrt z) / sqrt(z)^3, continued to z <= 0 (series near 0)."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 1e-3
    pos = (z > 0) & ~small
    neg = (z < 0) & ~small
    zs = z[small]
    out[small] = 1 / 6 - zs / 120 + zs ** 2 / 5040 - zs ** 3 / 362880
    sp = np.sqrt(z[pos])
    out[pos] = (sp - np.sin(sp)) / sp ** 3
    sn = np.sqrt(-z[neg])
    out[neg] = (np.sinh(sn) - sn) / sn ** 3
    return out


def _universal_f(chi, r0, vr0, alpha, smu, h):
    """Curtis' universal Kepler equation F(chi) and F'(chi) = r (> 0, so F rises
    monotonically from -inf to +inf); overflow of the hyperbolic functions is
    mapped to the sign the monotone F must have there."""
    with np.errstate(over="ignore", invalid="ignore"):
        z = alpha * chi * chi
        C, S = stumpff_c(z), stumpff_s(z)
        F = r0 * vr0 / smu * chi * chi * C + (1 - alpha * r0) * chi ** 3 * S + r0 * chi - smu * h
        dF = r0 * vr0 / smu * chi * (1 - z * S) + (1 - alpha * r0) * chi * chi * C + r0
    bad = ~np.isfinite(F)
    F = np.where(bad, np.where(chi > 0, np.inf, -np.inf), F)
    return F, dF


def kepler_drift(x, v, h, mu=1.0, max_iter=400):
    """Each row of x, v (shape [n, 3]) moved along its two-body orbit about a
    fixed centre of gravitational parameter mu for a time h.  The universal
    anomaly is found by Newton's method kept inside a bracket of the root
    (bisection whenever a Newton step would leave it), which converges for
    every conic and arc length."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    r0 = np.sqrt(np.sum(x * x, axis=1))
    v0sq = np.sum(v * v, axis=1)
    vr0 = np.sum(x * v, axis=1) / r0
    alpha = 2.0 / r0 - v0sq / mu                  # reciprocal semimajor axis
    smu = np.sqrt(mu)
    h = np.full(len(x), float(h)) if np.ndim(h) == 0 else np.asarray(h, dtype=np.float64)
    # bracket [lo, hi] with F(lo) <= 0 <= F(hi), grown geometrically from 0
    lo, hi = np.minimum(0.0, smu * h / r0), np.maximum(0.0, smu * h / r0)
    for _ in range(200):
        Flo, _ = _universal_f(lo, r0, vr0, alpha, smu, h)
        Fhi, _ = _universal_f(hi, r0, vr0, alpha, smu, h)
        grow_lo, grow_hi = Flo > 0, Fhi < 0
        if not (grow_lo.any() or grow_hi.any()):
            break
        lo = np.where(grow_lo, 2 * lo - 1.0, lo)
        hi = np.where(grow_hi, 2 * hi + 1.0, hi)
    # first guesses: exact for a circle; for a hyperbola the anomaly grows like
    # the logarithm of the time (r ~ v_inf t far out)
    vinf2 = np.maximum(-alpha * mu, 1e-300)
    with np.errstate(invalid="ignore"):
        hyp = np.sign(h) * smu * np.log1p(np.sqrt(vinf2) * np.abs(h) / r0) / np.sqrt(vinf2)
    chi = np.where(alpha > 0, smu * alpha * h, np.where(alpha < 0, hyp, smu * h / r0))
    chi = np.clip(chi, lo, hi)
    dx_old = hi - lo
    for _ in range(max_iter):
        F, dF = _universal_f(chi, r0, vr0, alpha, smu, h)
        lo = np.where(F <= 0, chi, lo)
        hi = np.where(F >= 0, chi, hi)
        with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
            newton = chi - F / dF
            # bisect when Newton leaves the bracket or shrinks it too slowly
            slow = np.abs(2 * F) > np.abs(dx_old * dF)
        inside = np.isfinite(newton) & (newton > lo) & (newton < hi) & ~slow
        new = np.where(inside, newton, 0.5 * (lo + hi))
        dx_old = np.abs(new - chi)
        done = (np.abs(new - chi) <= 1e-15 * np.abs(new)) | (F == 0)
        chi = new
        if done.all():
            break
    z = alpha * chi * chi
    C, S = stumpff_c(z), stumpff_s(z)
    f = 1 - chi * chi / r0 * C
    g = h - chi ** 3 / smu * S
    xn = f[:, None] * x + g[:, None] * v
    r = np.sqrt(np.sum(xn * xn, axis=1))
    fdot = smu / (r * r0) * (alpha * chi ** 3 * S - chi)
    gdot = 1 - chi * chi / r * C
    vn = fdot[:, None] * x + gdot[:, None] * v
    return xn, vn


def _xv(s):
    x = np.stack([s["x"], s["y"], s["z"]], axis=1).astype(np.float64)
    v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1).astype(np.float64)
    return x, v


def _massive(n, n_m):
    return n if n_m >= n - 1 else n_m


def sun_momentum(v, m, n_m):
    """sum over the massive bodies of m_i v_i (the Sun drift's velocity, Sun mass 1)."""
    k = _massive(len(v), n_m)
    return (m[:k, None] * v[:k]).sum(axis=0)


def step(s, n_m, h, acc=None, ora=None):
    """One step of the map above on state s (dict of float64 arrays x y z vx vy
    vz m rh).  acc: the interaction accelerations at the current positions
    ([n, 3]; computed when not given).  Returns (new state, accelerations at
    the new positions)."""
    ora = ora if ora is not None else _default()
    x, v = _xv(s)
    m = np.asarray(s["m"], dtype=np.float64)
    if acc is None:
        acc = ora.accel(s, n_m)
    v = v + (h / 2) * acc
    x = x + (h / 2) * sun_momentum(v, m, n_m)
    x, v = kepler_drift(x, v, h)
    x = x + (h / 2) * sun_momentum(v, m, n_m)
    new = dict(s)
    new.update(x=x[:, 0].copy(), y=x[:, 1].copy(), z=x[:, 2].copy())
    acc_new = ora.accel(new, n_m)
    v = v + (h / 2) * acc_new
    new.update(vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy())
    return new, acc_new


def energy(s, n_m):
    """H_Kep + H_Sun + H_int of the massive bodies (field bodies carry no energy)."""
    x, v = _xv(s)
    m = np.asarray(s["m"], dtype=np.float64)
    k = _massive(len(x), n_m)
    x, v, m = x[:k], v[:k], m[:k]
    r = np.sqrt(np.sum(x * x, axis=1))
    e = np.sum(0.5 * m * np.sum(v * v, axis=1) - m / r)
    p = (m[:, None] * v).sum(axis=0)
    e += 0.5 * np.dot(p, p)
    for i in range(k - 1):
        d = x[i + 1:] - x[i]
        e -= np.sum(m[i] * m[i + 1:] / np.sqrt(np.sum(d * d, axis=1)))
    return e
