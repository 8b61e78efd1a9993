"""The all-core oracle build (the benchmark's CPU context; the paper's Sec. 2
scheme: folded rows, thread-private accumulators summed in thread order)
against the single-thread oracle: the same pairs and groups, accelerations
that differ only by the order of the additions."""
import numpy as np
import pytest

import oracle
from paper_2304_07325_amd import diskgen as dg


@pytest.fixture(scope="module")
def both():
    return oracle.default(), oracle.Oracle(oracle.load_omp())


@pytest.mark.parametrize("n,n_m,kind,seed", [(1, 0, "cold", 3), (2, 1, "cold", 4), (257, 256, "cold", 5),
                                             (1000, 999, "cold", 1001), (3000, 300, "cold", 7),
                                             (2000, 1999, "hot", 8), (777, 0, "cold", 9)])
def test_omp_matches_single_thread(both, n, n_m, kind, seed):
    one, omp = both
    s = dg.make_disk(n, n_m, kind, seed).state(2)
    a = one.kick_encounter(s, n_m, dg.DT_HALF_YEAR, dg.RCRIT_FACTOR)
    b = omp.kick_encounter_omp(s, n_m, dg.DT_HALF_YEAR, dg.RCRIT_FACTOR)
    assert b["threads"] >= 1
    assert np.array_equal(a["pair_i"], b["pair_i"]) and np.array_equal(a["pair_j"], b["pair_j"])
    assert np.array_equal(a["group_id"], b["group_id"]) and a["n_groups"] == b["n_groups"]
    den = np.linalg.norm(a["acc"], axis=1)
    num = np.linalg.norm(a["acc"] - b["acc"], axis=1)
    rel = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    assert rel.max() < 1e-12, rel.max()


def test_omp_crowded_matches(both):
    """A crowded state (thousands of pairs, one group spanning most bodies):
    the per-thread pair lists are merged into the same lexicographic list."""
    one, omp = both
    rng = np.random.default_rng(11)
    n = 600
    s = dict(x=rng.uniform(9, 10, n), y=rng.uniform(-0.5, 0.5, n), z=rng.uniform(-0.1, 0.1, n),
             vx=rng.normal(0, 0.05, n), vy=rng.normal(0, 0.05, n), vz=rng.normal(0, 0.01, n),
             m=rng.uniform(1e-10, 1e-6, n), rh=rng.uniform(0.01, 0.05, n))
    a = one.kick_encounter(s, n - 1, dg.DT_HALF_YEAR, dg.RCRIT_FACTOR)
    b = omp.kick_encounter_omp(s, n - 1, dg.DT_HALF_YEAR, dg.RCRIT_FACTOR)
    assert len(a["pair_i"]) > 5000
    assert np.array_equal(a["pair_i"], b["pair_i"]) and np.array_equal(a["pair_j"], b["pair_j"])
    assert np.array_equal(a["group_id"], b["group_id"])
