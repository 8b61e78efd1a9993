#!/usr/bin/env python3
"""Benchmark of the SyMBA kick/encounter step on one MI355X.

Headline: FP64 pair-interactions per second on the 10k cold planetesimal disk
(N = 10000 all massive, the paper's Sec. 3 recipe, dt = 0.5 yr, critical
radius 3 Hill radii), one step = one kick/encounter evaluation (pair forces
over the trapezoid, encounter test over the same pairs, grouping).  The 100
Kepler-advanced input states are resident in HBM before timing starts.

Also reported: p50/p99 step latency (plain calls, one at a time), the
64-disk batch (plain per-disk calls vs one batched launch vs the batched
launch replayed from a captured graph), the FP64 roofline of the tile
kernel (HIP events around it, live), and the CPU oracle timed on a bounded
sample of the same workload.

Prints one JSON line.  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR_MM = 41      # fused massive-massive pair: 25 force + 16 encounter test
FLOP_PER_PAIR_MF = 34      # fused massive-field pair
PEAK_FP64_VECTOR = 78.6    # TFLOP/s, MI355X: 256 CU x 128 FP64 FLOP/clk x 2.4 GHz
PEAK_HBM = 8000.0          # GB/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def percentiles(xs):
    import numpy as np
    a = np.asarray(xs, dtype=float)
    return dict(p50=float(np.percentile(a, 50)), p99=float(np.percentile(a, 99)), samples=int(a.size))


def kernel_source_hash():
    h = hashlib.sha256()
    for p in ("paper_2304_07325_amd/csrc/symba_kernels.hip", "paper_2304_07325_amd/csrc/symba_internal.h"):
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload, rows):
    """HBM bytes per tile-kernel launch from the committed rocprofv3 PMC summary,
    only if it was taken on the current kernel source, for this workload and
    with the tile size this run uses."""
    if workload != "disk10k":
        return None
    p = os.path.join(ROOT, "profiles", "traffic_k_tiles_disk10k.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    m = re.search(r"k_tiles<(\d+)", t.get("kernel", ""))
    if not m or int(m.group(1)) != rows:
        return None
    return t.get("hbm_bytes_per_launch")


HOT_CHECK = {}   # a GPU evaluation of the 50k hot disk, checked against the oracle in the CPU leg


def hot_oracle_check(o, c):
    """The kept 50k hot-disk evaluation against the oracle's whole step (all
    1.25e9 pairs): every pair and label, every acceleration (per body,
    normwise relative error)."""
    import numpy as np
    g, n, n_m = c["gpu"], c["n"], c["n_m"]
    t0 = time.perf_counter()
    ref = o.kick_encounter(c["state"], n_m, c["dt"], c["f"], cap=1 << 20)
    el = time.perf_counter() - t0
    pi, pj = ref["pair_i"], ref["pair_j"]
    same_len = len(pi) == len(g["pair_i"])
    mism = int(len(pi) != len(g["pair_i"])) if not same_len else int(
        np.count_nonzero((pi != g["pair_i"]) | (pj != g["pair_j"])))
    missed = len(set(zip(pi.tolist(), pj.tolist())) - set(zip(g["pair_i"].tolist(), g["pair_j"].tolist())))
    rel = np.linalg.norm(g["acc"] - ref["acc"], axis=1) / np.linalg.norm(ref["acc"], axis=1)
    return dict(state=c["state_index"], pairs=len(pi), pair_mismatches=mism, false_negatives=missed,
                label_mismatches=int(np.count_nonzero(ref["group_id"] != g["group_id"])), groups=ref["n_groups"],
                groups_gpu=g["n_groups"], oracle_seconds=el,
                acc_rel_err=dict(bodies=int(n), max=float(rel.max()), p99=float(np.percentile(rel, 99)),
                                 median=float(np.median(rel)), above_1e12=int(np.count_nonzero(rel > 1e-12))))


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), affinity_cores=len(os.sched_getaffinity(0)))


def cpu_baseline(disk, n_m, dt, f, budget_s=15.0):
    """The CPU leg: the single-thread oracle (the parity reference) pinned to
    one core and timed on a bounded sample of the headline workload; for
    context, the all-core build of the same loop nest (the paper's Sec. 2
    scheme) on the same sample; and the oracle check of the kept 50k
    hot-disk evaluation."""
    import oracle
    from paper_2304_07325_amd import diskgen as dg
    o = oracle.default()
    if HOT_CHECK:
        HOT_CHECK["row"]["oracle_check"] = chk = hot_oracle_check(o, HOT_CHECK)
        log(f"hot50k oracle check {chk}")
    pairs = dg.pair_count(disk.n, n_m)
    affinity = os.sched_getaffinity(0)
    core = min(affinity)
    os.sched_setaffinity(0, {core})
    try:
        done, t0 = 0, time.perf_counter()
        while True:
            o.kick_encounter(disk.state(done), n_m, dt, f)
            done += 1
            if time.perf_counter() - t0 >= budget_s or done >= 100:
                break
        el = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, affinity)
    omp = oracle.Oracle(oracle.load_omp())
    done_p, t0 = 0, time.perf_counter()
    threads = None
    while True:
        threads = omp.kick_encounter_omp(disk.state(done_p), n_m, dt, f)["threads"]
        done_p += 1
        if time.perf_counter() - t0 >= budget_s / 3 or done_p >= 100:
            break
    el_p = time.perf_counter() - t0
    # the encounter step's oracle (numpy, one thread) on the paper's 100-body
    # accuracy disk, for the GPU's steps/s on the same disk
    from oracle import symba_enc
    acc_disk = dg.make_accuracy_disk(n=100)
    s_e, h_e = acc_disk.state(0), acc_disk.dt
    acc_e, pairs_e = symba_enc.prepare(s_e, acc_disk.n_massive, h_e, f, ora=o)
    done_e, flagged_e, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s / 5 and done_e < 20000:
        s_e, acc_e, pairs_e = symba_enc.step(s_e, acc_disk.n_massive, h_e, f, acc_e, pairs_e, ora=o)
        done_e += 1
        flagged_e += len(pairs_e)
    el_e = time.perf_counter() - t0
    info = cpu_info()
    return dict(value=pairs * done / el, unit="pair-interactions/s", cores=1, kind="oracle",
                sample=f"{done} evaluations of the 10k disk (states 0..{done - 1}), single thread pinned to core "
                       f"{core}, {el:.1f} s",
                **info,
                all_cores={"value": pairs * done_p / el_p, "unit": "pair-interactions/s", "threads": threads,
                           "sample": f"{done_p} evaluations of the 10k disk (states 0..{done_p - 1}), {el_p:.1f} s",
                           "kind": "oracle loop nest built with OpenMP: folded rows, thread-private "
                                   "accumulators summed in thread order (context, not the parity reference)"},
                encounter_step={"value": done_e / el_e, "unit": "steps/s", "kind": "oracle (encounter step, numpy)",
                                "sample": f"the first {done_e} 0.1-year steps of the 100-body accuracy disk, "
                                          f"{flagged_e} flagged pairs in all, {el_e:.1f} s"})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-steps", type=int, default=300)
    ap.add_argument("--batch-rounds", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--workload", default="disk10k")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-others", action="store_true", help="skip the 1k, 100k-field and 50k-hot disks")
    ap.add_argument("--no-step", action="store_true", help="skip the full-step (drifts + evaluation) legs")
    ap.add_argument("--accuracy-years", type=float, default=1e4,
                    help="length of the accuracy-disk integration of the step leg")
    ap.add_argument("--paper-steps", type=int, default=200,
                    help="encounter steps on each of the paper's 1k, 2k, 5k and 10k disks (0: skip)")
    ap.add_argument("--paper-budget-s", type=float, default=8.0,
                    help="wall-time cap per disk of those runs")
    ap.add_argument("--no-hot-check", action="store_true",
                    help="skip the oracle check of one 50k hot-disk evaluation (about 20 s of host time)")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-warmup", type=int, default=1000)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-lanes", type=int, default=2, help="serving calls in flight at once")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run one plain device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2304_07325_amd import binding as B
    from paper_2304_07325_amd import diskgen as dg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes read, {nbytes} bytes written")
        return
    w = dg.WORKLOADS[args.workload]
    n, n_m, dt, f = w["n"], w["n_massive"], dg.DT_HALF_YEAR, dg.RCRIT_FACTOR
    disk = dg.make_disk(n, n_m, w["kind"], w["seed"])
    evals = w["evals"]
    log(f"workload {args.workload}: n={n} n_m={n_m} evals={evals}")
    states = [B.to_device_state(disk.state(k)) for k in range(evals)]
    pairs = dg.pair_count(n, n_m)
    n_rows = min(n_m, n - 1)
    n_tri = n if n_m >= n - 1 else n_m
    mm = n_tri * (n_tri - 1) // 2 if n_m >= n - 1 else n_rows * (n_rows - 1) // 2
    flop = FLOP_PER_PAIR_MM * mm + FLOP_PER_PAIR_MF * (pairs - mm)

    ctx = B.Context(max_n=max(n, 1), max_pairs=max(16 * n, 1 << 16))
    outs = [B.Outputs(n, max(16 * n, 1 << 16)) for _ in range(2)]
    stream = torch.cuda.current_stream()
    plan = ctx.plan_for(n, n_m)   # tile rows and split diagonals the library picks for this size

    for s in range(args.warmup):
        ctx.kick_encounter(states[s % evals], n_m, dt, f, out=outs[s % 2])
    torch.cuda.synchronize()
    chk = outs[(args.warmup - 1) % 2].to_host() if args.warmup else None
    if chk is not None:
        assert chk["status"] == 0, f"status {chk['status']}"

    # ---- throughput: K steps back to back, no instrumentation ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.kick_encounter(states[s % evals], n_m, dt, f, out=outs[s % 2])
    enqueued = time.perf_counter() - t0
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = pairs * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    # ---- kernel times: a separate pass with HIP events recorded on the call's
    # stream around the tile kernel and around the two closing kernels ----
    kpass = max(args.steps, 100)
    ctx.set_option(B.OPT_TIMING, 1)
    ctx.read_timing()
    for s in range(kpass):
        ctx.kick_encounter(states[s % evals], n_m, dt, f, out=outs[s % 2])
    torch.cuda.synchronize()
    tiles_ms, fin_ms, calls = ctx.read_timing()
    ctx.set_option(B.OPT_TIMING, 0)
    tile_ms = tiles_ms / max(calls, 1)
    post_ms = fin_ms / max(calls, 1)
    achieved = flop / (tile_ms * 1e-3) / 1e12
    log(f"throughput {value:.4e} pairs/s, {ms_per_step:.4f} ms/step (host enqueue {1e3 * enqueued / args.steps:.4f} "
        f"ms/call); tile kernel {tile_ms * 1e3:.1f} us, closing kernels {post_ms * 1e3:.1f} us ({calls} timed calls)")

    # ---- latency: one step at a time ----
    lat = []
    for s in range(args.latency_steps):
        t = time.perf_counter()
        ctx.kick_encounter(states[s % evals], n_m, dt, f, out=outs[0])
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - t))
    latency = percentiles(lat)
    log(f"latency p50 {latency['p50']:.4f} ms p99 {latency['p99']:.4f} ms")

    batched = None
    if not args.no_batch:
        batched = bench_batch(args, B, dg, torch)
    served = None
    if not args.no_serve:
        served = bench_serve(args, dg, torch)
    others = None
    if not args.no_others:
        others = bench_other_workloads(args, B, dg, torch)
    step = None
    if not args.no_step:
        step = bench_step(args, B, dg, torch)

    result = {
        "metric": "FP64 pair-interactions/s (10k disk) + p50/p99 step latency, batched vs plain",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "screen": "f32 (conservative pair screen; every candidate gets the exact f64 test)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: cold planetesimal disk (Sec. 3 recipe), N={n}, N_m={n_m}, "
                               f"dt=0.5 yr, rcrit=3 Hill radii, {evals} Kepler-advanced states resident in HBM",
                   "pairs_per_step": pairs, "parallelism": "single GPU",
                   "plan": dict(zip(("rows", "split"), plan))},
        "latency_ms": latency,
        "step_breakdown_us": {"tile_kernel": tile_ms * 1e3, "closing_kernels": post_ms * 1e3,
                              "wall_per_step": ms_per_step * 1e3,
                              "host_enqueue_per_call": 1e6 * enqueued / args.steps,
                              "kernel_pass_calls": calls},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VECTOR, "traffic": traffic_from_profiles(args.workload, plan[0]),
                     "kernel": "k_tiles", "kernel_us": tile_ms * 1e3, "flop_per_launch": flop},
        "batched": batched,
        "served": served,
        "other_workloads": others,
        "step": step,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(disk, n_m, dt, f)
    print(json.dumps(result), flush=True)
    ctx.close()


def bench_step(args, B, dg, torch):
    """symba_step, the non-encounter step around the path: steps/s on the 10k
    disk, and the paper's accuracy test (Sec. 3: 100 equal planetesimals 5
    Hill radii apart, 0.1-year steps, 1e4 years) with its relative energy and
    angular-momentum errors.  Every pair gets its full force (no encounter
    sub-steps), so the steps with flagged encounter pairs are counted too."""
    import numpy as np
    f = dg.RCRIT_FACTOR
    res = {}
    w = dg.WORKLOADS[args.workload]
    n, n_m = w["n"], w["n_massive"]
    disk = dg.make_disk(n, n_m, w["kind"], w["seed"])
    st = B.to_device_state(disk.state(0))
    ctx = B.Context(max_n=n, max_pairs=max(16 * n, 1 << 16))
    out = B.Outputs(n, max(16 * n, 1 << 16))
    h = dg.DT_HALF_YEAR
    ctx.kick_encounter(st, n_m, h, f, out=out)
    for _ in range(5):
        ctx.step(st, n_m, h, f, out)
    torch.cuda.synchronize()
    steps = 100
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(st, n_m, h, f, out)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    res[args.workload] = {"steps_per_s": 1.0 / sec, "ms_per_step": sec * 1e3,
                          "pairs_per_s": dg.pair_count(n, n_m) / sec, "steps": steps}
    log(f"step {args.workload}: {1.0 / sec:.0f} steps/s, {sec * 1e3:.4f} ms/step")
    ctx.close()
    # the accuracy test, with the plain step and with the encounter step
    acc_disk = dg.make_accuracy_disk(n=100)
    res["accuracy_disk"] = accuracy_run(args, B, dg, torch, acc_disk, encounters=False)
    res["accuracy_disk_enc"] = accuracy_run(args, B, dg, torch, acc_disk, encounters=True)
    if args.paper_steps > 0:
        res["paper_disks_enc"] = paper_disk_runs(args, B, dg, torch)
    return res


def split_energy(st, torch):
    """Energy of the split Hamiltonian (Kepler + Sun + interaction terms,
    heliocentric positions, barycentric velocities) and angular momentum of a
    device state, in FP64 on the GPU (the pair sum in row blocks)."""
    x = torch.stack([st["x"], st["y"], st["z"]], 1)
    v = torch.stack([st["vx"], st["vy"], st["vz"]], 1)
    m = st["m"]
    p = (m[:, None] * v).sum(0)
    e = float((0.5 * m * (v * v).sum(1) - m / x.norm(dim=1)).sum() + 0.5 * (p @ p))
    n = x.shape[0]
    idx = torch.arange(n, device=x.device)
    pot = 0.0
    for i0 in range(0, n, 1024):
        i1 = min(i0 + 1024, n)
        r = (x[i0:i1, None, :] - x[None, :, :]).norm(dim=2)
        upper = idx[None, :] > idx[i0:i1, None]
        mm = m[i0:i1, None] * m[None, :]
        pot += float(torch.where(upper, mm / torch.where(upper, r, torch.ones_like(r)), torch.zeros_like(r)).sum())
    L = (m[:, None] * torch.linalg.cross(x, v)).sum(0)
    return e - pot, L


def paper_disk_runs(args, B, dg, torch):
    """The encounter step (symba_step_enc) on the paper's four benchmark
    disks (Sec. 3: 1k, 2k, 5k and 10k cold planetesimal disks, 0.5-year
    steps): `--paper-steps` steps of each (or `--paper-budget-s` seconds),
    each step timed on its own, since a step lasts as long as its deepest
    encounter group's chain of substeps.  Reported with the projected time of
    the paper's 1e4-year runs (20,000 steps) at the measured mean."""
    import numpy as np
    f, h = dg.RCRIT_FACTOR, dg.DT_HALF_YEAR
    res = {}
    for name in ("disk1k", "disk2k", "disk5k", "disk10k"):
        w = dg.WORKLOADS[name]
        n, n_m = w["n"], w["n_massive"]
        disk = dg.make_disk(n, n_m, w["kind"], w["seed"])
        st = B.to_device_state(disk.state(0))
        ctx = B.Context(max_n=n, max_pairs=1 << 16)
        out = B.Outputs(n, 1 << 14)
        e0, L0 = split_energy(st, torch)
        ctx.enc_prepare(st, n_m, h, f, out)
        torch.cuda.synchronize()
        ctx.read_stats()
        ts, skipped = [], 0
        t_start = time.perf_counter()
        for _ in range(args.paper_steps):
            t0 = time.perf_counter()
            ctx.step_enc(st, n_m, h, f, out)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            skipped += bool(int(out.scalars32[1].item()) & B.STATUS_ENC_SKIPPED)
            if time.perf_counter() - t_start > args.paper_budget_s:
                break
        _, flagged, calls = ctx.read_stats()
        e1, L1 = split_energy(st, torch)
        ms = np.array(ts) * 1e3
        r = {"n": n, "n_m": n_m, "steps": len(ts), "years": len(ts) * h / dg.YEAR,
             "steps_per_s": len(ts) / float(np.sum(ts)), "ms_per_step": percentiles(ms),
             "ms_per_step_mean": float(ms.mean()),
             "projected_s_for_1e4_years": float(ms.mean()) * 1e-3 * round(1e4 * dg.YEAR / h),
             "encounter_pairs_per_step": flagged / max(calls, 1), "steps_with_unresolved_pairs": skipped,
             "energy_rel_err_end": abs(e1 - e0) / abs(e0),
             "angmom_rel_err_end": float((L1 - L0).norm() / L0.norm())}
        res[name] = r
        log(f"paper disk {name}, encounter step: {len(ts)} steps, {r['steps_per_s']:.1f} steps/s, mean "
            f"{r['ms_per_step_mean']:.2f} ms (p50 {r['ms_per_step']['p50']:.2f}, p99 {r['ms_per_step']['p99']:.2f}), "
            f"{r['encounter_pairs_per_step']:.0f} flagged pairs/step, 1e4 yr projected "
            f"{r['projected_s_for_1e4_years']:.0f} s, energy err {r['energy_rel_err_end']:.2e}")
        ctx.close()
    return res


def accuracy_run(args, B, dg, torch, acc_disk, encounters):
    """The paper's accuracy test (Sec. 3): the 100-body disk integrated for
    `--accuracy-years` in 0.1-year steps, with the relative energy and
    angular-momentum errors at 50 checkpoints.  encounters: the encounter
    step (symba_step_enc: groups through the shells) instead of the plain
    step (every pair a full-strength kick)."""
    import numpy as np
    f = dg.RCRIT_FACTOR
    s0 = acc_disk.state(0)
    nm, h = acc_disk.n_massive, acc_disk.dt
    total = int(round(args.accuracy_years * dg.YEAR / h))
    label = "encounter step" if encounters else "plain step"

    def start(st, ctx, out):
        if encounters:
            ctx.enc_prepare(st, nm, h, f, out)
        else:
            ctx.kick_encounter(st, nm, h, f, out=out)

    def step(st, ctx, out, stream=None):
        if encounters:
            ctx.step_enc(st, nm, h, f, out, stream=stream)
        else:
            ctx.step(st, nm, h, f, out, stream=stream)

    def invariants(s):
        """Energy of the split Hamiltonian (Kepler + Sun + interaction terms,
        heliocentric positions, barycentric velocities), angular momentum and
        the smallest pair separation."""
        x = np.stack([s["x"], s["y"], s["z"]], 1)
        v = np.stack([s["vx"], s["vy"], s["vz"]], 1)
        m = s["m"]
        p = (m[:, None] * v).sum(0)
        e = float(np.sum(0.5 * m * np.sum(v * v, 1) - m / np.linalg.norm(x, axis=1)) + 0.5 * p @ p)
        d = x[:, None, :] - x[None, :, :]
        r = np.sqrt(np.sum(d * d, -1))
        iu = np.triu_indices(len(m), 1)
        e -= float(np.sum((m[:, None] * m[None, :])[iu] / r[iu]))
        L = (m[:, None] * np.cross(x, v)).sum(0)
        return e, L, float(r[iu].min())

    # eager steps on a copy, for the launch cost the graphs below remove
    chunks = 50
    per = max(total // chunks, 1)
    eager_n = per
    st_e = B.to_device_state(s0)
    ctx_e = B.Context(max_n=128, max_pairs=1 << 14)
    out_e = B.Outputs(100, 1 << 13)
    start(st_e, ctx_e, out_e)
    for _ in range(20):
        step(st_e, ctx_e, out_e)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(eager_n):
        step(st_e, ctx_e, out_e)
    torch.cuda.synchronize()
    eager_rate = eager_n / (time.perf_counter() - t0)
    ctx_e.close()
    # the run itself: graphs of graph_steps steps (the same bits as eager
    # steps), the remainder of each chunk eager
    st = B.to_device_state(s0)
    ctx = B.Context(max_n=128, max_pairs=1 << 14)
    out = B.Outputs(100, 1 << 13)
    start(st, ctx, out)   # also sizes the context's scratch for the captured steps
    torch.cuda.synchronize()
    ctx.read_stats()
    graph_steps = 100
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()   # capturing runs nothing: the run starts at s0
    with torch.cuda.graph(graph, stream=side):
        for _ in range(graph_steps):
            step(st, ctx, out, stream=side)
    torch.cuda.synchronize()
    e0, L0, _ = invariants(s0)
    worst_e, worst_l, skipped = 0.0, 0.0, 0
    # the invariants after every graph of steps (outside the timed time): an
    # approach closer than the deepest shell resolves (a collision, which the
    # paper's code would merge) shows as a jump of the energy error
    jump_at, worst_before, rmin = None, 0.0, float("inf")
    wall, done, first_rate = 0.0, 0, None
    while done < total:
        k = min(graph_steps, total - done)
        t0 = time.perf_counter()
        if k == graph_steps:
            graph.replay()
        else:
            for _ in range(k):
                step(st, ctx, out)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        done += k
        if first_rate is None and done >= per:
            # the same steps as the eager timing above (the cost of a step
            # depends on how deep its encounters go, which changes over the run)
            first_rate = done / wall
        cur = {key: v.cpu().numpy() for key, v in st.items()}
        e, L, rm = invariants(cur)
        err = abs(e - e0) / abs(e0)
        if jump_at is None and err > 1e-6:
            jump_at = done
        if jump_at is None:
            worst_before = max(worst_before, err)
        rmin = min(rmin, rm)
        worst_e = max(worst_e, err)
        worst_l = max(worst_l, float(np.linalg.norm(L - L0) / np.linalg.norm(L0)))
        skipped += bool(int(out.scalars32[1].item()) & B.STATUS_ENC_SKIPPED)
    _, flagged, calls = ctx.read_stats()
    r = {"n": 100, "step_years": h / dg.YEAR, "years": done * h / dg.YEAR, "steps": done,
         "stepper": "symba_step_enc" if encounters else "symba_step",
         "energy_rel_err_max": worst_e, "energy_rel_err_end": abs(e - e0) / abs(e0),
         "angmom_rel_err_max": worst_l, "checkpoints": -(-total // graph_steps), "checkpoint_steps": graph_steps,
         "first_energy_jump_above_1e-6": None if jump_at is None else
         {"by_step": jump_at, "years": jump_at * h / dg.YEAR, "energy_rel_err_max_before": worst_before},
         "closest_sampled_separation_au": rmin,
         "encounter_pairs_per_step": flagged / max(calls, 1), "wall_s": wall,
         "steps_per_s": done / wall, "graph_steps": graph_steps,
         "first_steps": {"steps": per, "graph_steps_per_s": first_rate, "eager_steps_per_s": eager_rate}}
    if encounters:
        r["checkpoints_with_unresolved_pairs"] = skipped
    log(f"accuracy disk, {label}: {done} steps ({done * h / dg.YEAR:.0f} yr) in {wall:.1f} s ({done / wall:.0f} "
        f"steps/s in graphs of {graph_steps}; first {per} steps {first_rate:.0f} steps/s in graphs, "
        f"{eager_rate:.0f} eager), energy err max "
        f"{worst_e:.2e}, angular momentum err max {worst_l:.2e}" +
        ("" if jump_at is None else f"; energy error first above 1e-6 by step {jump_at} "
         f"({jump_at * h / dg.YEAR:.0f} yr), at most {worst_before:.2e} before"))
    ctx.close()
    return r


def bench_other_workloads(args, B, dg, torch):
    """The paper's other benchmark sizes (1k, 2k and 5k cold disks), the
    100k-body field disk (1000 massive) and the 50k-body hot disk: throughput
    over their Kepler-advanced states, and for the hot
    disk the screen's candidates vs confirmed pairs and one evaluation checked
    against the oracle (every pair and label, 600 sampled accelerations)."""
    import numpy as np
    res = {}
    dt, f = dg.DT_HALF_YEAR, dg.RCRIT_FACTOR
    for name in ("disk1k", "disk2k", "disk5k", "field100k", "hot50k"):
        w = dg.WORKLOADS[name]
        n, n_m, evals = w["n"], w["n_massive"], w["evals"]
        disk = dg.make_disk(n, n_m, w["kind"], w["seed"])
        host = [disk.state(k) for k in range(evals)]
        states = [B.to_device_state(h) for h in host]
        ctx = B.Context(max_n=n, max_pairs=max(16 * n, 1 << 16))
        out = B.Outputs(n, max(16 * n, 1 << 16))
        for k in range(min(3, evals)):
            ctx.kick_encounter(states[k], n_m, dt, f, out=out)
        torch.cuda.synchronize()
        ctx.read_stats()
        ctx.set_option(B.OPT_TIMING, 1)
        ctx.read_timing()
        steps = max(evals, 20)
        t0 = time.perf_counter()
        for k in range(steps):
            ctx.kick_encounter(states[k % evals], n_m, dt, f, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tiles_ms, fin_ms, calls = ctx.read_timing()
        ctx.set_option(B.OPT_TIMING, 0)
        cands, flagged, probs = ctx.read_stats()
        pairs = dg.pair_count(n, n_m)
        r = dict(n=n, n_m=n_m, kind=w["kind"], steps=steps, pairs_per_step=pairs,
                 pairs_per_s=pairs * steps / el, ms_per_step=1e3 * el / steps,
                 tile_kernel_us=1e3 * tiles_ms / max(calls, 1), post_kernels_us=1e3 * fin_ms / max(calls, 1),
                 screen=dict(candidates_per_step=cands / max(probs, 1), flagged_per_step=flagged / max(probs, 1),
                             pass_rate=cands / max(probs, 1) / pairs,
                             confirmed_fraction=flagged / cands if cands else None))
        if name == "hot50k" and not args.no_hot_check:
            # one evaluation kept for the CPU leg, which checks it against the oracle
            k = 3
            ctx.kick_encounter(states[k], n_m, dt, f, out=out)
            torch.cuda.synchronize()
            HOT_CHECK.update(state_index=k, state=host[k], n=n, n_m=n_m, dt=dt, f=f, gpu=out.to_host(), row=r)
        ctx.close()
        res[name] = r
        log(f"{name}: {r['pairs_per_s']:.3e} pairs/s, {r['ms_per_step']:.3f} ms/step, "
            f"screen pass rate {r['screen']['pass_rate']:.2e}")
    return res


class _ServeWatchdog:
    """Ends the process with a non-zero status (and a line naming the run)
    when a serving loop has neither issued nor completed a call for
    `limit_s` seconds: a stalled run stops at once instead of going silent."""

    def __init__(self, srv, limit_s: float, what: str):
        import threading
        self.srv, self.limit_s, self.what = srv, limit_s, what
        self.served = 0
        self.stop = threading.Event()
        self.thread = threading.Thread(target=self._run, daemon=True)

    def progress(self, served, n_req):
        step = max(n_req // 4, 1)
        if served // step > self.served // step:
            log(f"  {self.what}: {served}/{n_req} requests served")
        self.served = served

    def _run(self):
        while not self.stop.wait(0.5):
            idle = time.monotonic() - self.srv.last_progress
            if idle > self.limit_s:
                print(f"serving watchdog: {self.what} made no progress for {idle:.1f} s "
                      f"({self.served} requests served, {len(self.srv.busy)} simulations in running calls)",
                      file=sys.stderr, flush=True)
                os._exit(3)

    def __enter__(self):
        self.thread.start()
        return self

    def __exit__(self, *exc):
        self.stop.set()
        self.thread.join()


def bench_serve(args, dg, torch):
    """256 resident simulations (N log-uniform in [500, 50000], all massive,
    even ids cold and odd ids hot), step requests arriving as a Poisson stream
    that names a uniformly random simulation, served by continuous batching
    with `--serve-lanes` calls in flight: latency from arrival to completion
    (host monotonic clock).  Run with a 200 GB device budget (nothing is
    evicted), again with one call in flight, and with 0.5 GB, which keeps only
    part of the population resident.  Then at saturation (every request
    waiting from the start): served steps/s with one and with several calls
    in flight against the same requests as plain per-simulation calls.  Each
    serving loop runs under a watchdog that ends the process at its first
    stall."""
    from paper_2304_07325_amd.serve import Server
    dt, f = dg.DT_HALF_YEAR, dg.RCRIT_FACTOR
    lanes = args.serve_lanes
    pop = dg.serving_population()
    sims = [(dg.make_disk(n, nm, kind, seed).state(0), nm) for (n, nm, kind, seed) in pop]
    total = sum(n for n, _, _, _ in pop)
    res = {"simulations": len(sims), "bodies": total, "rate_hz": args.serve_rate, "lanes": lanes}
    runs = (("budget_200GB", 200 << 30, None, args.serve_requests, args.serve_warmup, lanes),
            ("budget_200GB_one_call_in_flight", 200 << 30, None, args.serve_requests // 4,
             args.serve_warmup // 4, 1),
            ("budget_0.5GB", 512 << 20, 100_000, args.serve_requests // 5, args.serve_warmup // 5, lanes))
    for name, budget, max_bodies, n_req, warm, n_lanes in runs:
        t, ids = dg.poisson_arrivals(args.serve_rate, n_req + warm, len(sims))
        srv = Server(sims, budget, dt, f, max_batch_bodies=max_bodies, lanes=n_lanes)
        srv.preload(reserve=n_lanes * max(srv._need(k) - srv.sims[k].resident_bytes for k in range(len(sims))))
        torch.cuda.synchronize()
        log(f"serve {name}: {n_req + warm} requests at {args.serve_rate:.0f}/s, {n_lanes} lane(s)")
        with _ServeWatchdog(srv, 20.0, f"serve {name}") as wd:
            stats = srv.serve(t, ids, warmup=warm, progress=wd.progress)
        srv.close()
        res[name] = stats
        log(f"serve {name}: p50 {stats['latency_ms']['p50']:.3f} ms p99 {stats['latency_ms']['p99']:.3f} ms, "
            f"{stats['steps_per_s']:.0f} steps/s, mean batch {stats['mean_batch']:.1f}, "
            f"calls issued while another ran {stats['calls_issued_while_another_ran']}/{stats['calls']}, "
            f"uploads {stats['uploads']}, evictions {stats['evictions']}")
    # saturation: every request already waiting at t = 0, served by continuous
    # batching, against the same requests in the same order as plain
    # per-simulation calls on the same resident simulations
    import numpy as np
    n_sat = max(args.serve_requests // 10, 1)
    _, ids = dg.poisson_arrivals(args.serve_rate, n_sat, len(sims))
    sat = {"requests": n_sat}
    for n_lanes in sorted({1, lanes}):
        srv = Server(sims, 200 << 30, dt, f, lanes=n_lanes)
        srv.preload()
        torch.cuda.synchronize()
        with _ServeWatchdog(srv, 20.0, f"serve saturated, {n_lanes} lane(s)") as wd:
            stats = srv.serve(np.zeros(n_sat), ids, progress=wd.progress)
        sat[f"lanes_{n_lanes}"] = {"served_steps_per_s": stats["steps_per_s"],
                                   "served_pairs_per_s": stats["pairs_per_s"], "mean_batch": stats["mean_batch"],
                                   "calls": stats["calls"],
                                   "calls_issued_while_another_ran": stats["calls_issued_while_another_ran"]}
        log(f"serve saturated, {n_lanes} lane(s): {stats['steps_per_s']:.0f} steps/s "
            f"(mean batch {stats['mean_batch']:.1f}, {stats['calls']} calls)")
        if n_lanes == lanes:
            for k in ids[:20]:   # warm the plain path
                srv.ctx.kick_encounter(srv.sims[k].dev, srv.sims[k].n_m, dt, f, out=srv.sims[k].out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in ids:
                srv.ctx.kick_encounter(srv.sims[k].dev, srv.sims[k].n_m, dt, f, out=srv.sims[k].out)
            torch.cuda.synchronize()
            plain_s = time.perf_counter() - t0
            pairs = stats["pairs_per_s"] * n_sat / stats["steps_per_s"]
            sat.update(plain_steps_per_s=n_sat / plain_s, plain_pairs_per_s=pairs / plain_s)
        srv.close()
    res["saturated"] = sat
    log(f"serve saturated: {sat[f'lanes_{lanes}']['served_steps_per_s']:.0f} steps/s served with {lanes} lane(s) "
        f"vs {sat['plain_steps_per_s']:.0f} steps/s as plain calls")
    return res


def bench_batch(args, B, dg, torch):
    """64 disks (N log-uniform in [1000, 20000], N_m = N-1 or N/10): 64 plain
    calls per round vs one batched launch vs the batched launch replayed from
    a captured graph."""
    import numpy as np
    specs = dg.batch_sizes()
    dt, f = dg.DT_HALF_YEAR, dg.RCRIT_FACTOR
    states, outs = [], []
    total_n, total_pairs = 0, 0
    for (n, nm, seed) in specs:
        d = dg.make_disk(n, nm, "cold", seed)
        states.append(B.to_device_state(d.state(0)))
        outs.append(B.Outputs(n, max(8 * n, 4096)))
        total_n += n
        total_pairs += dg.pair_count(n, nm)
    cap = sum(o.pair_cap for o in outs)
    ctx = B.Context(max_n=total_n, max_pairs=cap)
    probs = [(st, nm, dt, f, o) for st, (n, nm, _), o in zip(states, specs, outs)]
    # autotune: one representative problem per size class (power of two of n_tri)
    tuned = {}
    for st, (n, nm, _), o in zip(states, specs, outs):
        n_tri = n if nm >= n - 1 else nm
        cls = n_tri.bit_length() - 1
        if cls not in tuned:
            ctx.autotune(st, nm, dt, f, out=o)
            tuned[cls] = ctx.plan_for(n, nm)   # (bodies per lane, split diagonals)
    log("autotuned (bodies per lane, split diagonals) by size class 2^k: " +
        ", ".join(f"{k}:{v}" for k, v in sorted(tuned.items())))
    rounds = args.batch_rounds

    def plain_round():
        for st, nm, _, _, o in probs:
            ctx.kick_encounter(st, nm, dt, f, out=o)

    def batch_round():
        ctx.kick_encounter_batch(probs)

    res = {"disks": len(specs), "bodies": total_n, "pairs_per_round": total_pairs,
           "autotuned_plan": {f"2^{k}": {"rows": v[0], "split": v[1]} for k, v in sorted(tuned.items())}}
    for name, fn in (("plain", plain_round), ("batched", batch_round)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(rounds):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            lat.append(1e3 * (time.perf_counter() - t))
        el = time.perf_counter() - t0
        res[name] = dict(disk_steps_per_s=len(specs) * rounds / el, pairs_per_s=total_pairs * rounds / el,
                         round_latency_ms=percentiles(lat))
        log(f"batch {name}: {res[name]['disk_steps_per_s']:.1f} disk-steps/s")
    # graph-captured batched launch
    try:
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            batch_round()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            ctx.kick_encounter_batch(probs, stream=s)
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(rounds):
            t = time.perf_counter()
            g.replay()
            torch.cuda.synchronize()
            lat.append(1e3 * (time.perf_counter() - t))
        el = time.perf_counter() - t0
        res["batched_graph"] = dict(disk_steps_per_s=len(specs) * rounds / el,
                                    pairs_per_s=total_pairs * rounds / el, round_latency_ms=percentiles(lat))
        log(f"batch graph: {res['batched_graph']['disk_steps_per_s']:.1f} disk-steps/s")
    except Exception as exc:  # reported, not hidden
        res["batched_graph"] = {"error": repr(exc)}
    ctx.close()
    return res


if __name__ == "__main__":
    main()
