"""The C-ABI library loads, exports what include/symba.h declares, rejects bad
arguments before touching a device, and its folded task plan covers the
paper's trapezoid exactly once (CPU only: no device call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2304_07325_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "symba.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(symba_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = declared_functions()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), f"{name} declared in symba.h but not exported"
    assert set(names) == set(B.EXPORTS)


def test_errors_before_any_device_work():
    lib = B.lib()
    assert lib.symba_ctx_create(None, 0, 100, 0, 0) == B.SYMBA_EINVAL
    h = ctypes.c_void_p()
    assert lib.symba_ctx_create(ctypes.byref(h), 0, 0, 0, 0) == B.SYMBA_EINVAL
    assert lib.symba_ctx_create(ctypes.byref(h), 0, 100, -1, 0) == B.SYMBA_EINVAL
    assert lib.symba_ctx_create(ctypes.byref(h), 0, 100, 0, 7) == B.SYMBA_EINVAL
    assert h.value is None
    assert lib.symba_ctx_destroy(None) == B.SYMBA_EINVAL
    assert lib.symba_set_option(None, B.OPT_TILE_ROWS, 2) == B.SYMBA_EINVAL
    st = B.symba_state()
    out = B.symba_out()
    assert lib.symba_kick_encounter(None, ctypes.byref(st), 10, 9, 1.0, 3.0, ctypes.byref(out), None) \
        == B.SYMBA_EINVAL
    assert lib.symba_kick_encounter_batch(None, None, 1, None) == B.SYMBA_EINVAL
    mst = B.symba_mstate()
    assert lib.symba_step(None, ctypes.byref(mst), 10, 9, 1.0, 3.0, ctypes.byref(out), None) == B.SYMBA_EINVAL
    assert lib.symba_step(None, None, 10, 9, float("nan"), 3.0, None, None) == B.SYMBA_EINVAL
    assert lib.symba_step_batch(None, None, 1, None) == B.SYMBA_EINVAL
    assert lib.symba_strerror(B.SYMBA_ETOOBIG).decode().startswith("problem larger")
    assert lib.symba_plan_tasks(0, 0, 1, 1, None, 0) == -1
    assert lib.symba_plan_tasks(10, 11, 1, 1, None, 0) == -1
    assert lib.symba_plan_tasks(10, 5, 3, 1, None, 0) == -1
    # the no-allocation entry point: argument checks, and sizes beyond its
    # fixed scratch, are refused before the device is touched (the pointers
    # below are never dereferenced on the host)
    assert lib.symba_kick_encounter_noalloc(None, 10, 9, 1.0, 3.0, None, None) == B.SYMBA_EINVAL
    fake = B.symba_state(*([8] * 8))
    fo = B.symba_out(8, 8, 8, 8, 8, 16, 8, 8, 8, 8)
    n_big = B.NOALLOC_MAX_N + 1
    assert lib.symba_kick_encounter_noalloc(ctypes.byref(fake), n_big, n_big - 1, 1.0, 3.0, ctypes.byref(fo),
                                            None) == B.SYMBA_ETOOBIG
    assert lib.symba_kick_encounter_noalloc(ctypes.byref(fake), 10, 11, 1.0, 3.0, ctypes.byref(fo),
                                            None) == B.SYMBA_EINVAL
    assert lib.symba_kick_encounter_noalloc(ctypes.byref(fake), 10, 9, -1.0, 3.0, ctypes.byref(fo),
                                            None) == B.SYMBA_EINVAL


def expand(tasks, n, n_m, rows, field_rows):
    """Pairs covered by a task list, as a sorted array of i * n + j (i < j)."""
    n_rows = min(n_m, n - 1)
    n_tri = n if n_m >= n - 1 else n_m
    S, F = 64 * rows, 64 * field_rows
    keys = []
    for kind, a, b in tasks:
        if kind in (0, 2):
            T = S if kind == 0 else 64
            bi = np.arange(a * T, min(a * T + T, n_tri))
            bj = np.arange(b * T, min(b * T + T, n_tri))
            I, J = np.meshgrid(bi, bj, indexing="ij")
            I, J = I.ravel(), J.ravel()
            if a == b:
                keep = I < J
                I, J = I[keep], J[keep]
            lo, hi = np.minimum(I, J), np.maximum(I, J)
            keys.append(lo * n + hi)
        else:  # field block a against segment b of the massive rows
            f = np.arange(n_tri + a * F, min(n_tri + a * F + F, n))
            rows_seg = np.arange(b * B.FIELD_SEG_ROWS, min((b + 1) * B.FIELD_SEG_ROWS, n_rows))
            I, J = np.meshgrid(rows_seg, f, indexing="ij")
            keys.append(I.ravel() * n + J.ravel())
    return np.sort(np.concatenate(keys)) if keys else np.zeros(0, np.int64)


def trapezoid(n, n_m):
    rows = min(n_m, n - 1)
    out = [i * n + j for i in range(rows) for j in range(i + 1, n)]
    return np.array(sorted(out), dtype=np.int64)


@pytest.mark.parametrize("n,n_m", [(1, 0), (1, 1), (2, 1), (2, 2), (5, 0), (64, 63), (65, 64), (130, 130),
                                   (300, 299), (257, 256), (700, 699), (400, 90), (333, 1), (200, 64),
                                   (1000, 999), (900, 128), (1200, 500), (700, 385)])
@pytest.mark.parametrize("rows,field_rows", [(1, 1), (2, 1), (4, 2)])
def test_plan_covers_trapezoid_once(n, n_m, rows, field_rows):
    tasks = B.plan_tasks(n, n_m, rows, field_rows)
    got = expand(tasks, n, n_m, rows, field_rows)
    exp = trapezoid(n, n_m)
    assert got.size == exp.size, "a pair is covered twice or not at all"
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("n", [64 * 5, 64 * 6, 64 * 7 + 3, 64 * 40])
def test_fold_balances_block_rows(n):
    """Every block row of the folded triangle gets the same number of tasks
    (the triangle mapped onto a rectangle), up to the one extra task per row
    of the first half when the block count is even."""
    tasks = B.plan_tasks(n, n - 1, 1, 1)
    blocks = (n + 63) // 64
    per_row = np.bincount(tasks[tasks[:, 0] == 0][:, 1], minlength=blocks)
    assert per_row.max() - per_row.min() <= 1
    assert len(tasks) == blocks * (blocks + 1) // 2


@pytest.mark.parametrize("n,n_m,rows", [(64 * 9, 64 * 9, 1), (3000, 500, 2), (900, 128, 1), (1, 0, 1)])
def test_launch_order_puts_field_tasks_first(n, n_m, rows):
    """Field tasks (the long ones when the massive rows are many) are
    launched before the triangle's block pairs."""
    tasks = B.plan_tasks(n, n_m, rows, 1)
    kinds = tasks[:, 0] if len(tasks) else np.zeros(0)
    n_field = int((kinds == 1).sum())
    n_whole = int((kinds == 0).sum())
    assert (kinds[:n_field] == 1).all() and (kinds[n_field:n_field + n_whole] == 0).all()
    assert (kinds[n_field + n_whole:] == 2).all()


@pytest.mark.parametrize("n,rows", [(64 * 2 * 9, 2), (10000, 2), (64 * 4 * 12 + 5, 4), (64 * 2 * 3, 2)])
def test_tail_split_tile_pairs(n, rows):
    """The block pairs at the smallest nonzero fold offsets run as 64 x 64
    tile pairs at the end of the launch: every block is the stationary block
    of exactly one split pair per split offset and the streamed block of
    exactly one, and every tile pair of a split block pair appears once."""
    tasks = B.plan_tasks(n, n - 1, rows, 1)
    split = tasks[tasks[:, 0] == 2]
    blocks = -(-n // (64 * rows))
    assert len(split) % (rows * rows * blocks) == 0 and len(split) > 0
    D = len(split) // (rows * rows * blocks)
    assert D <= (blocks - 1) // 2
    bi, bj = split[:, 1] // rows, split[:, 2] // rows
    off = (bj - bi) % blocks
    assert set(off.tolist()) == set(range(1, D + 1))
    for k in range(1, D + 1):
        sel = off == k
        assert np.array_equal(np.sort(np.unique(bi[sel])), np.arange(blocks))
        tiles = split[sel][:, 1:]
        assert len(np.unique(tiles[:, 0] * 10**6 + tiles[:, 1])) == len(tiles) == blocks * rows * rows
    whole = tasks[tasks[:, 0] == 0]
    woff = (whole[:, 2] - whole[:, 1]) % blocks
    assert not np.isin(woff, np.arange(1, D + 1)).any()


@pytest.mark.parametrize("n,rows", [(50000, 4), (30000, 2)])
def test_deep_launches_keep_block_pairs_whole(n, rows):
    """A triangle many workgroup rounds deep has no split block pairs: its
    ragged end is a small part of the kernel, so the split would only add
    per-task overhead."""
    tasks = B.plan_tasks(n, n - 1, rows, 1)
    assert (tasks[:, 0] != 2).all()
    blocks = -(-n // (64 * rows))
    assert len(tasks) == blocks * ((blocks - 1) // 2 + 1) + (blocks // 2 if blocks % 2 == 0 else 0)


def test_binding_constants_match_header():
    """The binding's option and status constants are the header's values."""
    import re
    text = open(os.path.join(ROOT, "include", "symba.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define SYMBA_(\w+)\s+(-?\d+)", text)}
    for name in ("OPT_TILE_ROWS", "OPT_FIELD_ROWS", "OPT_SCREEN", "OPT_TIMING", "OPT_BIN", "OPT_ACC", "OPT_SPLIT",
                 "SCREEN_AUTO", "SCREEN_FP32", "SCREEN_FP64", "ACC_INTERACTION", "ACC_HELIO",
                 "NOALLOC_MAX_N", "NOALLOC_MAX_PAIRS"):
        assert getattr(B, name) == defs[name], name


def test_binding_rejects_mismatched_sizes():
    """The binding refuses, before anything reaches the library, a state
    whose arrays differ in length and outputs smaller than the state (the
    library takes every array to hold len(x) bodies)."""
    import torch
    s = {k: torch.zeros(10, dtype=torch.float64) for k in B.STATE_KEYS}
    s["m"] = torch.zeros(9, dtype=torch.float64)
    with pytest.raises(ValueError, match="elements"):
        B._state_struct(s)
    s["m"] = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="outputs hold"):
        B._state_struct(s, B.Outputs(8, 16, device="cpu"))
    with pytest.raises(ValueError, match="device tensor"):   # host tensors never reach the library
        B._state_struct(s, B.Outputs(10, 16, device="cpu"))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits at once with a message."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2 and "one GPU only" in r.stderr
