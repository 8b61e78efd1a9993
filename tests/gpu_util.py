"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle element by element."""
from __future__ import annotations

import math
import sys

import numpy as np

EPS = np.finfo(np.float64).eps
ACC_RTOL = 1e-12          # per-body normwise relative tolerance on accelerations


def say(*msg):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print("[gpu-case]", *msg, file=sys.stderr, flush=True)


def run_gpu(ctx, state, n_m, dt, f, pair_cap=None, stream=None):
    import torch
    from paper_2304_07325_amd import binding as B
    st = B.to_device_state(state)
    n = state["x"].size
    out = B.Outputs(n, pair_cap if pair_cap is not None else max(4 * n, 4096))
    ctx.kick_encounter(st, n_m, dt, f, out=out, stream=stream)
    torch.cuda.synchronize()
    return out.to_host()


def term_magnitudes(state, n_m, k):
    """S_k = sum over massive j != k of m_j / |x_j - x_k|^2 (scale of body k's sum)."""
    n = state["x"].size
    nmass = n if n_m >= n - 1 else n_m
    if min(n_m, n - 1) <= 0:
        return 0.0
    j = np.arange(nmass)
    j = j[j != k]
    d = np.stack([state[c][j] - state[c][k] for c in ("x", "y", "z")], 1)
    return float((state["m"][j] / (d ** 2).sum(1)).sum())


def exact_sum_accel(state, n_m, k):
    """Body k's acceleration with the float64 pair terms summed exactly (fsum)."""
    n = state["x"].size
    nmass = n if n_m >= n - 1 else n_m
    out = np.zeros(3)
    if min(n_m, n - 1) <= 0:
        return out
    j = np.arange(nmass)
    j = j[j != k]
    d = np.stack([state[c][j] - state[c][k] for c in ("x", "y", "z")], 1)
    r2 = (d ** 2).sum(1)
    q = state["m"][j] / (r2 * np.sqrt(r2))
    for c in range(3):
        out[c] = math.fsum((q * d[:, c]).tolist())
    return out


def check_acc(state, n_m, gpu_acc, ref_acc, rtol=ACC_RTOL, bodies=None):
    """Normwise per-body check.  A body whose relative error exceeds rtol only
    passes as conditioning-limited: both results within 4 sqrt(N) eps S_k of
    the exactly summed value, S_k the sum of its term magnitudes.
    Returns (max relative error, number of conditioning-limited bodies)."""
    n = state["x"].size
    idx = np.arange(len(gpu_acc)) if bodies is None else np.asarray(bodies)
    num = np.linalg.norm(gpu_acc - ref_acc, axis=1)
    den = np.linalg.norm(ref_acc, axis=1)
    assert np.all(np.isfinite(gpu_acc)), "non-finite GPU acceleration"
    rel = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num == 0, 0.0, np.inf))
    limited = 0
    for pos in np.nonzero(rel > rtol)[0]:
        k = int(idx[pos])
        S = term_magnitudes(state, n_m, k)
        exact = exact_sum_accel(state, n_m, k)
        bound = 4.0 * math.sqrt(n) * EPS * S
        eg = np.linalg.norm(gpu_acc[pos] - exact)
        er = np.linalg.norm(ref_acc[pos] - exact)
        assert eg <= bound and er <= bound, (
            f"body {k}: rel err {rel[pos]:.3e}, |gpu-exact| {eg:.3e}, |ref-exact| {er:.3e}, bound {bound:.3e}")
        limited += 1
    return float(rel.max()) if rel.size else 0.0, limited


def check_pairs_groups(gpu, ref):
    assert gpu["status"] == 0, f"status {gpu['status']}"
    assert gpu["n_pairs"] == len(ref["pair_i"]), f"n_pairs {gpu['n_pairs']} vs {len(ref['pair_i'])}"
    assert np.array_equal(gpu["pair_i"], ref["pair_i"]), "pair_i differs"
    assert np.array_equal(gpu["pair_j"], ref["pair_j"]), "pair_j differs"
    assert np.array_equal(gpu["group_id"], ref["group_id"]), "group_id differs"
    assert gpu["n_groups"] == ref["n_groups"], f"n_groups {gpu['n_groups']} vs {ref['n_groups']}"


def dense_state(n, seed, box=1.5, rh=(0.01, 0.06), vscale=0.05, n_m=None):
    """A crowded random state with many encounters (long union-find chains)."""
    rng = np.random.default_rng(seed)
    s = dict(x=rng.uniform(-box, box, n), y=rng.uniform(-box, box, n), z=rng.uniform(-box / 4, box / 4, n),
             vx=rng.normal(0, vscale, n), vy=rng.normal(0, vscale, n), vz=rng.normal(0, vscale / 4, n),
             m=rng.uniform(1e-10, 1e-6, n), rh=rng.uniform(rh[0], rh[1], n))
    if n_m is not None and n_m < n - 1:
        s["m"][n_m:] = 0.0
        s["rh"][n_m:] = 0.0
    s["x"] = s["x"] + 10.0  # away from the Sun, as in a disk
    return s
