"""Seeded synthetic planetesimal disks: the inputs of the kick/encounter path.

This module only builds inputs. It holds none of the path's arithmetic (no
pair force, no encounter test, no grouping), so the oracle and the HIP path
can both be fed from it without sharing any of the method's code.

Recipe (Sec. 3 of the paper, "Benchmarking & Tests"):
  * masses drawn from the cumulative number N(>m) = C m^-0.3 exp(-m/m0) with
    m0 = 1e-2 Earth masses and a floor m_min = 1e-3 Earth masses;
  * bulk density 2 g/cm^3 gives the physical radius (carried, unused on the path);
  * semimajor axis uniform in 5-20 AU; eccentricity and inclination Rayleigh
    with scales 1e-6 and 5e-7 ("cold"); the three angles uniform in [0, 2pi).
A "hot" variant (scales 0.05 and 0.025) makes encounter lists non-empty.

Units: G = 1, masses in solar masses, lengths in AU, time in yr/(2 pi), so
one year is 2 pi and the paper's 0.5 yr step is exactly pi.  The Sun is the
implicit central mass 1; bodies exclude it.  Heliocentric Cartesian states
come from the orbital elements through Kepler's equation with mu = 1 + m.
Evaluation k of a run sees every body advanced along its unperturbed Kepler
orbit to t = k * dt, so neighbours and encounter lists change with k while
the host still produces identical bytes for every consumer.

The Hill radius R_H = a (m/3)^(1/3) is computed here, once, from the initial
semimajor axis, and handed to both consumers as an input array; field
particles (massless) get m = 0 and R_H = 0.

All randomness: numpy Generator(PCG64(SeedSequence(seed))), drawn in a fixed
order (m, a, e, i, Omega, omega, M) so that a seed fixes the disk bit for bit.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Physical constants (IAU 2015 nominal values; the paper states none).
M_EARTH = 3.0034896149e-6          # GM_earth / GM_sun
AU_CM = 1.495978707e13             # cm
M_SUN_G = 1.988409870698051e33     # g
RHO_CGS = 2.0                      # g cm^-3, bulk density of the paper's disk
RHO_CODE = RHO_CGS * AU_CM ** 3 / M_SUN_G   # in M_sun / AU^3  (~3.367e6)

YEAR = 2.0 * math.pi               # one year in code units (G = M_sun = 1, AU)
DT_HALF_YEAR = 0.5 * YEAR          # the paper's step, exactly pi

# Mass function parameters (paper, Sec. 3).
M0 = 1e-2 * M_EARTH
M_MIN = 1e-3 * M_EARTH
MASS_SLOPE = 0.3

COLD = (1e-6, 5e-7)                # Rayleigh scales (e, i) of the paper's disk
HOT = (0.05, 0.025)                # dynamically hot disk


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed))))


def mass_survival(m):
    """Fraction of bodies heavier than m: (m/m_min)^-0.3 exp(-(m - m_min)/m0)."""
    m = np.asarray(m, dtype=np.float64)
    return (m / M_MIN) ** (-MASS_SLOPE) * np.exp(-(m - M_MIN) / M0)


def sample_masses(rng: np.random.Generator, n: int) -> np.ndarray:
    """Inverse-CDF draw from N(>m) by 80 bisection steps in log m."""
    u = 1.0 - rng.random(n)                      # u in (0, 1]
    lo = np.full(n, math.log(M_MIN))
    hi = np.full(n, math.log(M_MIN * 1e4))       # survival ~1e-430 there
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        s = mass_survival(np.exp(mid))
        above = s > u                            # survival still too large: go heavier
        lo = np.where(above, mid, lo)
        hi = np.where(above, hi, mid)
    return np.exp(0.5 * (lo + hi))


def rayleigh(rng: np.random.Generator, scale: float, n: int) -> np.ndarray:
    u = rng.random(n)
    return scale * np.sqrt(-2.0 * np.log1p(-u))


def solve_kepler(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly E with E - e sin E = M (Newton, elliptic orbits)."""
    if np.any(e >= 1.0):
        raise ValueError("elliptic orbits only")
    M = np.mod(M, 2.0 * math.pi)
    E = M + e * np.sin(M)
    for _ in range(60):
        f = E - e * np.sin(E) - M
        E_new = E - f / (1.0 - e * np.cos(E))
        if np.all(np.abs(E_new - E) <= 1e-15 * np.maximum(1.0, np.abs(E))):
            E = E_new
            break
        E = E_new
    return E


def elements_to_cartesian(a, e, inc, Om, om, M, mu):
    """Heliocentric position and velocity from Keplerian elements (textbook)."""
    E = solve_kepler(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = np.sqrt(1.0 - e * e)
    n = np.sqrt(mu / a ** 3)
    Edot = n / (1.0 - e * cE)
    xp, yp = a * (cE - e), a * b * sE
    vxp, vyp = -a * sE * Edot, a * b * cE * Edot
    cO, sO = np.cos(Om), np.sin(Om)
    co, so = np.cos(om), np.sin(om)
    ci, si = np.cos(inc), np.sin(inc)
    P = (cO * co - sO * so * ci, sO * co + cO * so * ci, so * si)
    Q = (-cO * so - sO * co * ci, -sO * so + cO * co * ci, co * si)
    pos = [xp * P[k] + yp * Q[k] for k in range(3)]
    vel = [vxp * P[k] + vyp * Q[k] for k in range(3)]
    return pos, vel


@dataclasses.dataclass
class Disk:
    """Orbital elements of one disk; `state(k)` gives the inputs of evaluation k.

    Massive bodies occupy [0, n_massive) and field particles [n_massive, n).
    n_massive = n - 1 or n means every body is massive.
    """
    n: int
    n_massive: int
    kind: str
    seed: int
    m: np.ndarray
    radius: np.ndarray
    rh: np.ndarray
    a: np.ndarray
    e: np.ndarray
    inc: np.ndarray
    Om: np.ndarray
    om: np.ndarray
    M: np.ndarray
    dt: float = DT_HALF_YEAR

    def state(self, k: int = 0) -> dict:
        mu = 1.0 + self.m
        n_mean = np.sqrt(mu / self.a ** 3)
        Mk = self.M + n_mean * (k * self.dt)
        (x, y, z), (vx, vy, vz) = elements_to_cartesian(
            self.a, self.e, self.inc, self.Om, self.om, Mk, mu)
        out = dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, m=self.m.copy(), rh=self.rh.copy())
        return {key: np.ascontiguousarray(v, dtype=np.float64) for key, v in out.items()}


def make_disk(n: int, n_massive: int | None = None, kind: str = "cold", seed: int = 0,
              dt: float = DT_HALF_YEAR, a_range=(5.0, 20.0)) -> Disk:
    """A seeded disk with the paper's distributions (massive bodies first)."""
    if n < 1:
        raise ValueError("n >= 1")
    if n_massive is None:
        n_massive = n - 1
    if not 0 <= n_massive <= n:
        raise ValueError("0 <= n_massive <= n")
    scales = {"cold": COLD, "hot": HOT}[kind]
    rng = _rng(seed)
    n_mass = n if n_massive >= n - 1 else n_massive   # bodies that carry mass
    m = np.zeros(n)
    m[:n_mass] = sample_masses(rng, n_mass)
    a = rng.uniform(a_range[0], a_range[1], n)
    e = rayleigh(rng, scales[0], n)
    inc = rayleigh(rng, scales[1], n)
    Om = rng.uniform(0.0, 2.0 * math.pi, n)
    om = rng.uniform(0.0, 2.0 * math.pi, n)
    M = rng.uniform(0.0, 2.0 * math.pi, n)
    radius = np.cbrt(3.0 * m / (4.0 * math.pi * RHO_CODE))
    rh = a * np.cbrt(m / 3.0)
    return Disk(n=n, n_massive=n_massive, kind=kind, seed=seed, m=m, radius=radius, rh=rh,
                a=a, e=e, inc=inc, Om=Om, om=om, M=M, dt=dt)


def make_accuracy_disk(n: int = 100, seed: int = 60, spacing_hill: float = 5.0,
                       a_inner: float = 5.0, mass_earth: float = 1e-2) -> Disk:
    """The paper's accuracy-test disk (Sec. 3): n equal planetesimals of 1e-2
    Earth masses, neighbours `spacing_hill` Hill radii apart from 5 AU out, with
    the cold Rayleigh e and i.  Spacing uses each inner neighbour's Hill radius."""
    rng = _rng(seed)
    mm = mass_earth * M_EARTH
    hill = (mm / 3.0) ** (1.0 / 3.0)
    a = np.empty(n)
    a[0] = a_inner
    for k in range(1, n):
        a[k] = a[k - 1] * (1.0 + spacing_hill * hill)
    m = np.full(n, mm)
    e = rayleigh(rng, COLD[0], n)
    inc = rayleigh(rng, COLD[1], n)
    Om = rng.uniform(0.0, 2.0 * math.pi, n)
    om = rng.uniform(0.0, 2.0 * math.pi, n)
    M = rng.uniform(0.0, 2.0 * math.pi, n)
    radius = np.cbrt(3.0 * m / (4.0 * math.pi * RHO_CODE))
    rh = a * np.cbrt(m / 3.0)
    return Disk(n=n, n_massive=n - 1, kind="cold", seed=seed, m=m, radius=radius, rh=rh,
                a=a, e=e, inc=inc, Om=Om, om=om, M=M, dt=0.1 * YEAR)


def pair_count(n: int, n_massive: int) -> int:
    """Pairs in the trapezoid {(i, j): i < min(N_m, N-1), i < j < N}."""
    rows = min(n_massive, n - 1)
    return rows * n - rows * (rows + 1) // 2


# --------------------------------------------------------------------------
# Workloads (sizes, mixes and seeds of the five benchmark configurations)
# --------------------------------------------------------------------------
RCRIT_FACTOR = 3.0      # critical radius in Hill radii

WORKLOADS = {
    "disk1k": dict(n=1000, n_massive=999, kind="cold", evals=20, seed=1001),
    "disk2k": dict(n=2000, n_massive=1999, kind="cold", evals=20, seed=1010),
    "disk5k": dict(n=5000, n_massive=4999, kind="cold", evals=20, seed=1011),
    "disk10k": dict(n=10000, n_massive=9999, kind="cold", evals=100, seed=1002),
    "field100k": dict(n=100000, n_massive=1000, kind="cold", evals=100, seed=1003),
    "hot50k": dict(n=50000, n_massive=49999, kind="hot", evals=10, seed=1004),
}


def batch_sizes(n_disks: int = 64, seed: int = 1005, lo: int = 1000, hi: int = 20000):
    """(N, N_m, seed) of each disk of the 64-disk batch: N log-uniform in
    [lo, hi]; N_m = N - 1 for even k and N // 10 for odd k."""
    rng = _rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_disks))).astype(int)
    out = []
    for k, n in enumerate(ns):
        n = int(n)
        nm = n - 1 if k % 2 == 0 else n // 10
        out.append((n, nm, seed * 1000 + k))
    return out


def serving_population(n_sims: int = 256, seed: int = 1006, lo: int = 500, hi: int = 50000):
    """(N, N_m, kind, seed) of each resident simulation: N log-uniform in
    [lo, hi], all massive; even ids cold, odd ids hot."""
    rng = _rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_sims))).astype(int)
    return [(int(n), int(n) - 1, "cold" if k % 2 == 0 else "hot", seed * 1000 + k)
            for k, n in enumerate(ns)]


def poisson_arrivals(rate_hz: float, n: int, n_sims: int, seed: int = 1007):
    """Arrival times (s) of n step requests at `rate_hz` and the simulation each names."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n)
    sims = rng.integers(0, n_sims, n)
    return np.cumsum(gaps), sims
