"""Batch selection of the serving loop (host logic only, no GPU)."""
import pytest
from collections import deque

from paper_2304_07325_amd.serve import pair_capacity, pick_batch


def test_distinct_simulations_in_arrival_order():
    pending = deque([(0, 3), (1, 1), (2, 3), (3, 2), (4, 1)])
    batch, rest = pick_batch(pending, sizes=[100] * 4, needs=[10] * 4, budget=10**9, max_bodies=10**9,
                             max_pairs=10**9)
    assert batch == [(0, 3), (1, 1), (3, 2)]
    assert list(rest) == [(2, 3), (4, 1)]


def test_budget_and_body_bounds():
    sizes = [1000, 2000, 3000]
    needs = [100, 200, 300]
    pending = deque([(0, 0), (1, 1), (2, 2)])
    batch, rest = pick_batch(pending, sizes, needs, budget=350, max_bodies=10**9, max_pairs=10**9)
    assert batch == [(0, 0), (1, 1)] and list(rest) == [(2, 2)]
    batch, rest = pick_batch(pending, sizes, needs, budget=10**9, max_bodies=3500, max_pairs=10**9)
    assert batch == [(0, 0), (1, 1)]
    cap = pair_capacity(1000) + pair_capacity(2000)
    batch, rest = pick_batch(pending, sizes, needs, budget=10**9, max_bodies=10**9, max_pairs=cap)
    assert batch == [(0, 0), (1, 1)]


def test_later_small_request_fills_room_left():
    # a large request that does not fit is skipped, a later small one still joins
    batch, rest = pick_batch(deque([(0, 0), (1, 1), (2, 2)]), [10, 10**6, 10], [5, 10**9, 5], budget=100,
                             max_bodies=10**9, max_pairs=10**9)
    assert batch == [(0, 0), (2, 2)] and list(rest) == [(1, 1)]


def test_server_rejects_unknown_mode():
    from paper_2304_07325_amd.serve import Server
    with pytest.raises(ValueError):
        Server([], 1 << 30, 1.0, 3.5, mode="drift")
