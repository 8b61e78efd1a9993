"""The synthetic disks follow the paper's recipe (Sec. 3) and are reproducible."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2304_07325_amd import diskgen as dg


def test_seed_fixes_every_byte():
    a = dg.make_disk(500, 499, "cold", 7).state(3)
    b = dg.make_disk(500, 499, "cold", 7).state(3)
    for k in a:
        assert a[k].tobytes() == b[k].tobytes()
    c = dg.make_disk(500, 499, "cold", 8).state(3)
    assert c["x"].tobytes() != a["x"].tobytes()


def test_mass_function_ks():
    d = dg.make_disk(20000, 19999, "cold", 11)
    cdf = lambda m: 1.0 - dg.mass_survival(m)  # noqa: E731
    assert d.m.min() >= dg.M_MIN * (1 - 1e-12)
    assert stats.kstest(d.m, cdf).pvalue > 1e-3


def test_elements_ks():
    d = dg.make_disk(20000, 19999, "hot", 12)
    assert stats.kstest(d.a, stats.uniform(5.0, 15.0).cdf).pvalue > 1e-3
    assert stats.kstest(d.e, stats.rayleigh(scale=0.05).cdf).pvalue > 1e-3
    assert stats.kstest(d.inc, stats.rayleigh(scale=0.025).cdf).pvalue > 1e-3
    for ang in (d.Om, d.om, d.M):
        assert stats.kstest(ang, stats.uniform(0, 2 * math.pi).cdf).pvalue > 1e-3
    c = dg.make_disk(5000, 4999, "cold", 13)
    assert stats.kstest(c.e, stats.rayleigh(scale=1e-6).cdf).pvalue > 1e-3
    assert stats.kstest(c.inc, stats.rayleigh(scale=5e-7).cdf).pvalue > 1e-3


@pytest.mark.parametrize("k", [0, 1, 17])
def test_states_lie_on_their_orbits(k):
    d = dg.make_disk(2000, 1999, "hot", 14)
    s = d.state(k)
    mu = 1.0 + d.m
    r = np.sqrt(s["x"] ** 2 + s["y"] ** 2 + s["z"] ** 2)
    v2 = s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2
    a = 1.0 / (2.0 / r - v2 / mu)                     # vis-viva
    assert np.allclose(a, d.a, rtol=1e-12)
    h = np.cross(np.stack([s["x"], s["y"], s["z"]], 1), np.stack([s["vx"], s["vy"], s["vz"]], 1))
    inc = np.arccos(h[:, 2] / np.linalg.norm(h, axis=1))
    assert np.allclose(inc, d.inc, atol=1e-9)


def test_field_particles_and_hill_radius():
    d = dg.make_disk(3000, 300, "cold", 15)
    assert np.all(d.m[300:] == 0) and np.all(d.rh[300:] == 0)
    assert np.all(d.m[:300] > 0)
    assert np.allclose(d.rh[:300], d.a[:300] * (d.m[:300] / 3) ** (1 / 3), rtol=1e-14)
    assert dg.pair_count(3000, 300) == 300 * 3000 - 300 * 301 // 2
    assert dg.pair_count(10000, 9999) == 49995000 == dg.pair_count(10000, 10000)
    assert dg.pair_count(100000, 1000) == 99499500


def test_units_and_step():
    assert dg.DT_HALF_YEAR == math.pi
    assert abs(dg.RHO_CODE - 3.3674e6) / 3.3674e6 < 1e-3


def test_batch_and_serving_mixes():
    b = dg.batch_sizes()
    assert len(b) == 64
    assert all(1000 <= n <= 20000 for n, _, _ in b)
    assert all(nm == (n - 1 if k % 2 == 0 else n // 10) for k, (n, nm, _) in enumerate(b))
    pop = dg.serving_population()
    assert len(pop) == 256 and all(500 <= n <= 50000 for n, _, _, _ in pop)
    t, sims = dg.poisson_arrivals(2000.0, 5000, 256)
    assert np.all(np.diff(t) > 0) and abs(5000 / t[-1] - 2000) < 150


def test_generator_matches_paper_parameters():
    import json
    import os
    p = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))
    mf = p["mass_function"]
    assert dg.MASS_SLOPE == mf["slope"]
    assert dg.M0 == mf["m0_earth"] * dg.M_EARTH and dg.M_MIN == mf["m_min_earth"] * dg.M_EARTH
    assert dg.RHO_CGS == p["bulk_density_g_cm3"]
    assert dg.COLD == (p["rayleigh_scale_e"], p["rayleigh_scale_i"])
    assert dg.DT_HALF_YEAR == p["time_step_years"] * dg.YEAR
    d = dg.make_accuracy_disk()
    acc = p["accuracy_test"]
    assert d.n == acc["N"] and d.a[0] == acc["inner_au"]
    assert np.allclose(d.m, acc["mass_earth"] * dg.M_EARTH)
    assert d.dt == acc["time_step_years"] * dg.YEAR
    w = dg.WORKLOADS
    # the paper's benchmark sizes (Sec. 3), all-massive cold disks
    assert sorted(w[k]["n"] for k in ("disk1k", "disk2k", "disk5k", "disk10k")) == sorted(p["benchmark_N"])
    for k in ("disk1k", "disk2k", "disk5k", "disk10k"):
        assert w[k]["kind"] == "cold" and w[k]["n_massive"] == w[k]["n"] - 1
