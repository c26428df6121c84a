#!/usr/bin/env python3
"""GP log-likelihoods per second on one MI355X.

Workload (the benchmark configuration): n = 2^20 points t ~ U(0, 1000)
sorted, Matern-3/2 kernel a = 1, l = 5, sigma^2 = 0.1, leaf 128, tolerance
1e-10, y ~ N(0, 1).  One step = one full log-likelihood for the given
hyperparameters: cross approximation of every off-diagonal block, leaf
factorizations, level-by-level factorization, log-det and C^{-1} y, with the
ordered points and y already resident in HBM.  The ordering of the points is
amortized over hyperparameters and reported separately.

Prints one JSON line.  Also reports, for the kernel that takes the most time,
its achieved rate against MI355X's peak (live HIP-event timing inside the
library, on the stream each kernel is launched on), and the dense FP64 oracle
timed on the host cores on a bounded slice of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GP log-likelihoods/s (factor+logdet+solve) at n=2^20; mixed vs FP64 at 1e-8"
PEAK = {"hbm": 8000.0, "alu_fp64": 78.6, "alu_fp32": 157.3,   # GB/s, TFLOP/s, TFLOP/s
        "bf16_mfma": 2500.0}                                   # TFLOP/s, dense


def kernel_model(n, leaf_sizes, r, cnt, esz=8, projected=False):
    """Algorithmic FLOPs and HBM bytes per call for each kernel kind.

    projected: the likelihood's projected level form, whose stages are the leaf
    projection G = Z^T Xt (level_reduce: W and Xt read once, the leaves' G
    written), the upward coupling solves (level_solve: the children's G read,
    the parent's G and S written) and the downward pass (level_update: S read,
    Xt read once, C^{-1} y written).

    leaf_sizes: sizes of the leaves; r[j]: columns of the depth-j panel
    (j = 1..L); cnt[d] = 1 + sum_{j<=d} r[j] (columns still updated at depth d
    plus the right-hand side).  Bytes count each panel operand moved once
    (esz bytes per entry: 8 in the FP64 form, 4 in the mixed form).  Where
    depth d's update is fused with depth d-1's reduction (small ranks), the
    update also reads the depth-(d-1) basis and that reduction reads nothing
    of its own.
    """
    L = len(cnt) - 1
    m = np.asarray(leaf_sizes, dtype=np.float64)
    out = {}
    # leaves: Cholesky m^3/3, two triangular solves on cnt[L] columns
    flops = float(np.sum(m ** 3 / 3.0 + 2.0 * m * m * cnt[L]))
    byts = esz * n * (2 * cnt[L])
    out["leaf_factor"] = (flops, byts)
    if projected:
        mL = cnt[L]
        nleaf = len(leaf_sizes)
        out["level_reduce"] = (2.0 * mL * mL * n, (esz + 8.0) * n * mL + 8.0 * nleaf * mL * mL)
        fs = bs = sb = 0.0
        for d in range(L):
            nodes, m, w = 1 << d, cnt[d], r[d + 1]
            fs += nodes * (2.0 * w ** 3 + 6.0 * w * w * m + 4.0 * w * m * m)
            bs += 8.0 * (2 * nodes * cnt[d + 1] ** 2 + nodes * m * m + nodes * 2 * w * m)
            sb += 8.0 * nodes * 2 * w * m
        out["level_solve"] = (fs, bs)
        out["level_update"] = (2.0 * n * mL, esz * n * (mL + 1) + sb)
        return out
    fr = br = fu = bu = 0.0

    def fused(d):
        # depth d's update also writes depth d-1's reduction records (both
        # panels of rank 1..8 and the pass's LDS within 64 KB)
        if d < 1 or d >= L or not (0 < r[d + 1] <= 8 and 0 < r[d] <= 8):
            return False
        c = cnt[d]
        return 8 * (8 * c + ((c + 3) // 4) * 8 * 4 * 8) + 4 * c <= 65536

    for d in range(L):
        rr = r[d + 1]
        if rr > 0 and not fused(d + 1):
            fr += 2.0 * rr * cnt[d + 1] * n
            br += esz * n * (cnt[d + 1] + rr)
        fu += 2.0 * rr * cnt[d] * n
        bu += esz * n * (2 * cnt[d] + rr)
        if fused(d):
            # the parent's basis (FP64) against the updated columns
            fu += 2.0 * r[d] * cnt[d] * n
            bu += 8.0 * n * r[d]
    out["level_reduce"] = (fr, br)
    out["level_update"] = (fu, bu)
    return out


def item_model(n, leaf, rank_max, esz=8):
    """kernel_model for one item of n points with leaf `leaf` and per-depth
    panel widths rank_max (depth 0 .. L-1), plus the cross approximation's
    basis writes (8 B x n x sum of widths)."""
    L = len(rank_max)
    r = [0] + [int(v) for v in rank_max]
    cnt = [1]
    for j in range(1, L + 1):
        cnt.append(cnt[-1] + r[j])
    leaf_sizes = np.diff(np.linspace(0, n, (1 << L) + 1).round()).astype(int) if L else [n]
    model = kernel_model(n, leaf_sizes, r, cnt, esz=esz)
    model["aca_bases"] = (0.0, 8.0 * n * sum(r[1:]))
    return model


def model_ms(model, items=1):
    """Sum over stages of max(bytes / 8 TB/s, flops / 78.6 TFLOP/s), in ms."""
    return items * sum(max(b / (PEAK["hbm"] * 1e9), f / (PEAK["alu_fp64"] * 1e12)) * 1e3
                       for f, b in model.values())


def stage_roofline(model, stages, items=1):
    """Roofline of the stage with the largest measured time among the modelled
    ones: algorithmic bytes (HBM-bound) or flops (above the FP64 ridge) per
    launch over its average launch time."""
    cand = [k for k in stages if k in model]
    if not cand:
        return None
    k = max(cand, key=lambda s: stages[s][0])
    ms, launches = stages[k]
    f, b = (items * v for v in model[k])
    per_s = ms / 1e3
    if f / b > PEAK["alu_fp64"] * 1e12 / (PEAK["hbm"] * 1e9):
        ach = f / per_s / 1e12
        return {"bound": "mfma" if k in ("leaf_factor", "level_reduce", "level_update") else "alu",
                "achieved": ach, "peak": PEAK["alu_fp64"], "unit": "TFLOP/s",
                "frac": ach / PEAK["alu_fp64"], "traffic": None, "kernel": k,
                "avg_launch_ms": ms / launches,
                "algorithmic_per_call": {"flops": f / launches, "bytes": b / launches}}
    ach = b / per_s / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm"], "unit": "GB/s",
            "frac": ach / PEAK["hbm"], "traffic": None, "kernel": k,
            "avg_launch_ms": ms / launches,
            "algorithmic_per_call": {"flops": f / launches, "bytes": b / launches}}


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is
    none or the kernel's source changed since the counters were taken."""
    import hashlib
    files = {"leaf_factor": ("profiles/leaf_factor_traffic_matern32_n2p20.md",
                             "paper_1403_6015_amd/csrc/leaf.hip")}
    if kernel not in files:
        return None
    summary, src = (os.path.join(ROOT, f) for f in files[kernel])
    try:
        text = open(summary).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines()
                if line.startswith(("traffic_bytes_per_launch: ", "source_sha256: ")))
    if vals.get("source_sha256", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch"])


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ONE_CORE = """
import sys, time, json
sys.path.insert(0, %r)
import oracle, workloads as wl
out = []
for n in %r:
    p = wl.matern1d(n)
    t0 = time.perf_counter()
    oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
    out.append([n, time.perf_counter() - t0])
print(json.dumps(out))
"""


def cpu_baseline(sizes=(2048, 4096, 8192), one_core_sizes=(2048, 4096)):
    """The dense FP64 oracle (Cholesky log det and solve, §1 Eq. (1)) on
    density-matched slices of the workload: n = 2^11..2^13 on every host
    thread and n = 2^11..2^12 on one thread (a child process with
    OMP_NUM_THREADS=1), the n^3 exponent fitted over the all-thread points and
    the largest one extrapolated to n = 2^20 (an extrapolation: the dense
    matrix at 2^20 would need 8.8 TB).  Also times the exact O(n) Kalman
    oracle at full size and returns it for the accuracy check of the GPU
    result."""
    import subprocess
    import oracle
    import workloads as wl
    oracle.build(force=False)
    times = []
    for n in sizes:
        p = wl.matern1d(n)
        t0 = time.perf_counter()
        oracle.gp_dense(p.x, p.y, p.kernel, p.theta, p.sigma2)
        times.append(time.perf_counter() - t0)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_CORE % (ROOT, list(one_core_sizes))],
                       capture_output=True, text=True, env=env, timeout=600)
    one = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else []
    full = wl.matern1d()
    t1 = time.perf_counter()
    kf = oracle.kalman_matern32(full.x[:, 0], full.y, full.theta, full.sigma2, want_alpha=False)
    dk = time.perf_counter() - t1
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    slope = float(np.polyfit(np.log(sizes), np.log(times), 1)[0])
    big_n, big_t = sizes[-1], times[-1]
    value = 1.0 / (big_t * (float(1 << 20) / big_n) ** 3)
    base = {"value": value, "unit": "likelihoods/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_threads": os.cpu_count(),
            "timings_s": {"all_threads": [[n, t] for n, t in zip(sizes, times)],
                          "one_thread": one},
            "fitted_exponent": slope,
            "sample": "dense FP64 Cholesky oracle on density-matched slices of the workload "
                      "(n = %s on %d threads, n = %s on 1 thread; %.1f s in all); value = "
                      "1/(t(n=%d) * (2^20/%d)^3), an n^3 extrapolation (fitted exponent "
                      "%.2f)" % (list(sizes), threads, list(one_core_sizes),
                                 sum(times) + sum(t for _, t in one), big_n, big_n, slope)}
    return base, kf, dk


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=None,
                    help="problem size (default: 2^20; 2^22 for se2d)")
    ap.add_argument("--max-rank", type=int, default=None, help="rank cap (se2d; default 64)")
    ap.add_argument("--leaf", type=int, default=None, help="leaf size (se2d; default 256)")
    ap.add_argument("--workload", default="matern1d",
                    choices=["matern1d", "batched_theta", "ragged", "learned", "copy", "se2d",
                             "predict", "grad"],
                    help="matern1d: one n=2^20 likelihood per step (the benchmark line); "
                         "batched_theta: 256 hyperparameter settings on one shared n=65536 "
                         "series per step, hipGraph replay; ragged: 512 independent series "
                         "with n log-uniform in [1024, 131072] per step; learned: surrogate-"
                         "screened (delayed-acceptance) vs plain Metropolis, 64 walkers, n=2^18; "
                         "predict: posterior means at --m new inputs through an n=2^20 factor; "
                         "grad: log-likelihood and its gradient in (a, l, sigma2) at n=2^20 "
                         "(central differences of 7 likelihoods)")
    ap.add_argument("--m", type=int, default=8192, help="new inputs per step (predict)")
    ap.add_argument("--mcmc-steps", type=int, default=300)
    ap.add_argument("--autotune-free-leaf", action="store_true",
                    help="also run the autotuner with the leaf size free (reported only)")
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: FP32 basis panels, FP64 leaves / coupling LU / log-det sums "
                         "(matern1d, batched_theta, ragged)")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--profile-run", action="store_true",
                    help="matern1d: only warmup + steps likelihoods on a plan with the library's "
                         "default tiles (no autotuning, no other legs); for counter profiles")
    ap.add_argument("--level-by-level", action="store_true",
                    help="--profile-run only: level-by-level updates (hodlr_opts.level_form = 1) "
                         "instead of the projected levels")
    ap.add_argument("--no-speculate", action="store_true",
                    help="matern1d: every call waits for its compression's rank statistics "
                         "(default: calls after the first assume the previous call's panel "
                         "widths and step count, checked on the device, redone on a miss)")
    ap.add_argument("--compressor", default="aca", choices=["aca", "sketch"],
                    help="se2d: compress the off-diagonal blocks by cross approximation "
                         "(default) or by the randomized two-sided sketch (O(n^2) work; "
                         "use a moderate --n)")
    args = ap.parse_args()
    if args.n is None and args.workload != "se2d":
        args.n = 1 << 20
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(each GPU would own a subtree; only the top levels would exchange "
              "KB-sized coupling sums)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1403_6015_amd as H
    import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batched_theta":
        return bench_batched(args, torch, H, wl, dev)
    if args.workload == "ragged":
        return bench_ragged(args, torch, H, wl, dev)
    if args.workload == "learned":
        return bench_learned(args, torch, H, wl, dev)
    if args.workload == "copy":
        return bench_copy(args, torch, dev)
    if args.workload == "se2d":
        return bench_se2d(args, torch, H, wl, dev)
    if args.workload == "predict":
        return bench_predict(args, torch, H, wl, dev)
    if args.workload == "grad":
        return bench_grad(args, torch, H, wl, dev)
    p = wl.matern1d(args.n)
    if args.profile_run:
        return profile_run(args, torch, H, p, dev)
    t0 = time.perf_counter()
    perm = H.hodlr_order(p.x, p.leaf)
    t_order = time.perf_counter() - t0
    xs = p.x[perm]
    ys = p.y[perm]
    mixed = args.precision == "mixed"
    prec = H.MIXED if mixed else H.FP64
    spec = 0 if args.no_speculate else 1
    opts = H.Opts(max_rank=64, precision=prec, speculate=spec)
    # tiles from the autotuner at the workload's leaf size (untimed); the tuner
    # is also run with the leaf size free, for information
    t0 = time.perf_counter()
    topts = H.Opts(max_rank=64, precision=prec, presorted=1)
    tune, tune_ms = H.autotune(xs, ys, p.kernel, p.theta, p.sigma2, p.tol, topts,
                               leaf_cands=[p.leaf], reps=2)
    free = None
    if args.autotune_free_leaf:
        free, free_ms = H.autotune(xs, ys, p.kernel, p.theta, p.sigma2, p.tol, topts, reps=2)
    t_tune = time.perf_counter() - t0
    plan = H.Plan(p.n, p.dim, p.leaf, opts, tune=tune)
    d_x = torch.from_numpy(np.ascontiguousarray(xs.T)).to(dev)
    d_y = torch.from_numpy(np.ascontiguousarray(ys)).to(dev)
    work = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    out = torch.zeros(8, dtype=torch.float64, device=dev)
    z = torch.empty(p.n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                        plan.workspace_bytes, stream, out, z)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-kernel breakdown in a pass of its own (every launch timed), then the
    # timed region with events around the dominant kernel only
    H.profile_select(None)
    H.profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    breakdown = H.profile_read()
    H.profile_enable(False)
    stages = {k: v for k, v in breakdown.items() if v[1] > 0}
    dom = max(stages, key=lambda k: stages[k][0])
    H.profile_select([dom])
    H.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = H.profile_read()
    H.profile_enable(False)
    H.profile_select(None)
    loglik, logdet, quad = out[:3].cpu().tolist()

    # ranks for the algorithmic model (one untimed build on the same data)
    f = H.hodlr_build(xs, p.kernel, p.theta, p.sigma2, p.leaf, p.tol,
                      H.Opts(max_rank=64, presorted=1, precision=prec))
    info = f.info()
    f.free()
    L = info["levels"]
    r = [0] + [int(v) for v in info["rank_max"][:L]]
    cnt = [1]
    for j in range(1, L + 1):
        cnt.append(cnt[-1] + r[j])
    nl = 1 << L
    leaf_sizes = np.diff(np.linspace(0, p.n, nl + 1).round()).astype(int) if L else [p.n]
    projected = bool(plan.info()["projected"])
    model = kernel_model(p.n, leaf_sizes, r, cnt, esz=4 if mixed else 8, projected=projected)

    dom_ms, dom_launches = prof[dom]
    roofline = None
    if dom in model:
        flops, byts = model[dom]
        per_call_s = dom_ms / 1e3 / args.steps
        ai = flops / byts
        if ai > PEAK["alu_fp64"] * 1e12 / (PEAK["hbm"] * 1e9):
            # above the ridge: the leaf kernel's products run on FP64 MFMA
            # (dense FP64 matrix peak 78.6 TFLOP/s, the same figure as the
            # vector FP64 peak on this chip)
            bound = "mfma" if dom == "leaf_factor" else "alu"
            ach = flops / per_call_s / 1e12
            roofline = {"bound": bound, "achieved": ach, "peak": PEAK["alu_fp64"],
                        "unit": "TFLOP/s", "frac": ach / PEAK["alu_fp64"],
                        "traffic": None if mixed else measured_traffic(dom),
                        "traffic_unit": "HBM bytes per launch",
                        "kernel": dom, "dtype": "fp64", "avg_launch_ms": dom_ms / dom_launches,
                        "algorithmic_per_call": {"flops": flops, "bytes": byts}}
        else:
            ach = byts / per_call_s / 1e9
            roofline = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm"], "unit": "GB/s",
                        "frac": ach / PEAK["hbm"],
                        "traffic": None if mixed else measured_traffic(dom),
                        "traffic_unit": "HBM bytes per likelihood (the stage's launches)",
                        "kernel": dom, "avg_launch_ms": dom_ms / dom_launches,
                        "algorithmic_per_call": {"flops": flops, "bytes": byts}}

    # whole-pipeline model: each modelled stage at the larger of its HBM time
    # (algorithmic bytes at 8 TB/s) and its FP64 compute time, plus the cross
    # approximation's basis writes (8 B x n x sum of ranks); against the
    # measured time per likelihood
    ms_step = elapsed / args.steps * 1e3
    bound_ms = {k: max(b / (PEAK["hbm"] * 1e9), f / (PEAK["alu_fp64"] * 1e12)) * 1e3
                for k, (f, b) in model.items()}
    bound_ms["aca_bases"] = 8.0 * p.n * sum(r[1:]) / (PEAK["hbm"] * 1e9) * 1e3
    pipeline = {"model_ms": sum(bound_ms.values()), "measured_ms": ms_step,
                "frac": sum(bound_ms.values()) / ms_step,
                "stage_bound_ms": bound_ms,
                "note": "sum over stages of max(bytes / 8 TB/s, flops / 78.6 TFLOP/s); "
                        "stages without a model (node solves, cross-approximation passes, "
                        "log-det sums) count as zero"}

    res = {
        "metric": METRIC, "value": args.steps / elapsed, "unit": "likelihoods/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 arithmetic, f32 panels" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "matern32_1d_n%d_leaf%d_tol%g%s" % (p.n, p.leaf, p.tol,
                                                                     "_mixed" if mixed else ""),
                   "n": p.n,
                   "dim": 1, "kernel": "matern32", "theta": list(p.theta), "sigma2": p.sigma2,
                   "leaf": p.leaf, "tol": p.tol, "max_rank": 64, "precision": args.precision,
                   "speculate": spec,
                   "level_form": "projected" if projected else "level-by-level",
                   "levels": L, "rank_max": r[1:], "level_rows": tune.level_rows,
                   "reduce_cols": tune.reduce_cols, "reduce_group": tune.reduce_group},
        "roofline": roofline,
        "pipeline_roofline": pipeline,
        "speculated_last_call": plan.info()["speculated"],
        "stage_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
        "stage_launches_per_step": {k: v[1] / args.steps for k, v in stages.items()},
        "stage_note": "stage times from a separate pass with every launch timed; the timed "
                      "region records events around %s only" % dom,
        "ordering_s": t_order,
        "autotune": {"tiles_at_leaf": tune.as_dict(), "candidate_ms": tune_ms,
                     "free_leaf_best": free.as_dict() if free else None,
                     "free_leaf_ms": min(free_ms) if free else None,
                     "seconds": t_tune},
        "result": {"loglik": loglik, "logdet": logdet, "quad": quad},
    }
    # the other precision on the same data and workload, timed the same way
    # (whole steps, no events), so that one line carries mixed vs FP64; the
    # mixed form both in the library's default mode (its log-det error bound
    # tested, an FP64 redo when the bound misses 1e-8) and unchecked (the
    # FP32-panel result kept; its error is measured against the oracle below)
    other = H.FP64 if mixed else H.MIXED

    def time_other(unchecked):
        otopts = H.Opts(max_rank=64, precision=other, presorted=1, mixed_unchecked=unchecked)
        otune, _ = H.autotune(xs, ys, p.kernel, p.theta, p.sigma2, p.tol, otopts,
                              leaf_cands=[p.leaf], reps=2)
        oplan = H.Plan(p.n, p.dim, p.leaf,
                       H.Opts(max_rank=64, precision=other, mixed_unchecked=unchecked,
                              speculate=spec), tune=otune)
        owork = torch.empty(oplan.workspace_bytes, dtype=torch.uint8, device=dev)
        oout = torch.zeros(8, dtype=torch.float64, device=dev)
        oz = torch.empty(p.n, dtype=torch.float64, device=dev)

        def ostep():
            H.gp_loglik_dev(oplan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, owork,
                            oplan.workspace_bytes, stream, oout, oz)

        for _ in range(args.warmup):
            ostep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ostep()
        torch.cuda.synchronize()
        oelapsed = time.perf_counter() - t0
        o_ll, o_ld, o_q = oout[:3].cpu().tolist()
        return {"precision": "fp64" if mixed else "mixed", "value": args.steps / oelapsed,
                "unit": "likelihoods/s", "ms_per_step": oelapsed / args.steps * 1e3,
                "result": {"loglik": o_ll, "logdet": o_ld, "quad": o_q},
                "tiles": otune.as_dict(), "fp64_fallback": oplan.info()["fp64_fallback"]}

    # the same precision with the level-by-level updates (level_form = 1), for
    # comparison with the projected levels the default takes
    lplan = H.Plan(p.n, p.dim, p.leaf, H.Opts(max_rank=64, precision=prec, speculate=spec,
                                              level_form=1), tune=tune)
    lwork = torch.empty(lplan.workspace_bytes, dtype=torch.uint8, device=dev)
    lout = torch.zeros(8, dtype=torch.float64, device=dev)
    lz = torch.empty(p.n, dtype=torch.float64, device=dev)

    def lstep():
        H.gp_loglik_dev(lplan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, lwork,
                        lplan.workspace_bytes, stream, lout, lz)

    for _ in range(args.warmup):
        lstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lstep()
    torch.cuda.synchronize()
    lel = time.perf_counter() - t0
    res["level_by_level"] = {"value": args.steps / lel, "unit": "likelihoods/s",
                             "ms_per_step": lel / args.steps * 1e3,
                             "logdet": lout[1].item(), "quad": lout[2].item()}
    del lwork
    res["other_precision"] = time_other(0)
    if other == H.MIXED:
        res["other_precision"]["mode"] = "checked (default)"
        res["mixed_unchecked"] = time_other(1)
        res["mixed_unchecked"]["mode"] = "unchecked (mixed_unchecked = 1)"
    if not args.no_cpu_baseline and args.n == 1 << 20:
        base, kf, dk = cpu_baseline()
        res["cpu_baseline"] = base
        res["oracle_check"] = {"kalman_logdet": kf["logdet"], "kalman_quad": kf["quad"],
                               "logdet_rel_err": abs(logdet - kf["logdet"]) / abs(kf["logdet"]),
                               "quad_rel_err": abs(quad - kf["quad"]) / abs(kf["quad"]),
                               "kalman_seconds_1core": dk}
        for key in ("other_precision", "mixed_unchecked"):
            if key not in res:
                continue
            r = res[key]["result"]
            res[key]["logdet_rel_err"] = abs(r["logdet"] - kf["logdet"]) / abs(kf["logdet"])
            res[key]["quad_rel_err"] = abs(r["quad"] - kf["quad"]) / abs(kf["quad"])
            res[key]["note"] = (
                "device likelihood without refinement: the mixed form's quadratic form is one "
                "solve through FP32 applied bases; the metric's mixed bar is the log det at 1e-8")
    print(json.dumps(res), flush=True)


def bench_batched(args, torch, H, wl, dev):
    """Many hyperparameter settings on one shared sorted series: n = 65536,
    x ~ U(0, 10), Matern-3/2, theta log-uniform in the box of workloads.theta_box;
    one step = one batched call (all items), captured stages replayed as a graph."""
    n, m = 65536, args.batch
    x, y, th = wl.batched_theta(m=m, n=n)
    mixed = args.precision == "mixed"
    prec = H.MIXED if mixed else H.FP64
    d_x = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    d_y = torch.from_numpy(y).to(dev)
    d_p = torch.from_numpy(np.ascontiguousarray(th)).to(dev)
    out = torch.zeros((m, 3), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    # tiles: the autotuner's twelve shapes at leaf 128, each timed on this
    # batched call (untimed in the rate); a shape tuned on one item is not
    # always the best for a whole batch in one launch per stage
    sweep = {}
    best_t, tune = None, None
    for rows in (256, 512, 1024):
        for cols in (4, 8):
            for grp in (8, 64):
                t = H.Tune(128, rows, cols, grp)
                pl = H.Plan(n, 1, 128, H.Opts(max_rank=16, precision=prec), tune=t)
                nbt = pl.batch_workspace_bytes(m)
                wk = torch.empty(nbt, dtype=torch.uint8, device=dev)
                with torch.cuda.stream(stream):
                    for rep_ in range(2):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        H.gp_loglik_batch_dev(pl, d_x, H.K_MATERN32, d_p, m, d_y, 0, 1e-10, wk,
                                              nbt, stream, out, True)
                        torch.cuda.synchronize()
                        el = time.perf_counter() - t0
                sweep["%d/%d/%d" % (rows, cols, grp)] = el * 1e3
                if best_t is None or el < best_t:
                    best_t, tune = el, t
                del wk, pl
    plan = H.Plan(n, 1, 128, H.Opts(max_rank=16, precision=prec), tune=tune)
    nb = plan.batch_workspace_bytes(m)
    work = torch.empty(nb, dtype=torch.uint8, device=dev)

    def step():
        H.gp_loglik_batch_dev(plan, d_x, H.K_MATERN32, d_p, m, d_y, 0, 1e-10, work, nb, stream,
                              out, True)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    o = out.cpu().numpy()
    fallback = plan.info()["fp64_fallback"]
    ms_step = elapsed / args.steps * 1e3
    unchecked = None
    if mixed:
        # the mixed batch with the FP32-panel results kept (no bound test, no
        # FP64 redo), same tiles; its errors against the oracle are reported
        uplan = H.Plan(n, 1, 128, H.Opts(max_rank=16, precision=prec, mixed_unchecked=1),
                       tune=tune)
        uout = torch.zeros((m, 3), dtype=torch.float64, device=dev)
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                H.gp_loglik_batch_dev(uplan, d_x, H.K_MATERN32, d_p, m, d_y, 0, 1e-10, work, nb,
                                      stream, uout, True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                H.gp_loglik_batch_dev(uplan, d_x, H.K_MATERN32, d_p, m, d_y, 0, 1e-10, work, nb,
                                      stream, uout, True)
            torch.cuda.synchronize()
            uel = time.perf_counter() - t0
        unchecked = {"value": args.steps * m / uel, "ms_per_step": uel / args.steps * 1e3,
                     "out": uout.cpu().numpy()}
        del uplan
    # per-stage times in a pass of its own (stages launched eagerly, every
    # launch timed), the batch-wide column layout, and the model
    H.profile_select(None)
    H.profile_enable(True)
    with torch.cuda.stream(stream):
        H.gp_loglik_batch_dev(plan, d_x, H.K_MATERN32, d_p, m, d_y, 0, 1e-10, work, nb, stream,
                              out, False)
    torch.cuda.synchronize()
    stages = {k: v for k, v in H.profile_read().items() if v[1] > 0}
    H.profile_enable(False)
    info = plan.info()
    model = item_model(n, 128, info["rank_max"][:info["levels"]], esz=4 if mixed else 8)
    pipe_ms = model_ms(model, m)
    # every item against the exact state-space oracle and against its own
    # single-likelihood call on the same plan
    import oracle
    oracle.build(force=False)
    splan = H.Plan(n, 1, 128, H.Opts(max_rank=16, precision=prec, presorted=1))
    sw = torch.empty(splan.workspace_bytes, dtype=torch.uint8, device=dev)
    so = torch.zeros(8, dtype=torch.float64, device=dev)
    worst = {"kalman_logdet": 0.0, "kalman_quad": 0.0, "single_logdet": 0.0,
             "single_loglik": 0.0}
    t_k = 0.0
    for i in range(m):
        a, ell, s2 = th[i]
        H.gp_loglik_dev(splan, d_x, H.K_MATERN32, (a, ell), s2, d_y, 1e-10, sw,
                        splan.workspace_bytes, None, so)
        torch.cuda.synchronize()
        one = so[:3].cpu().numpy()
        t1 = time.perf_counter()
        kf = oracle.kalman_matern32(x[:, 0], y, (a, ell), s2, want_alpha=False)
        t_k += time.perf_counter() - t1
        rel = lambda u, v: abs(u - v) / max(abs(v), 1.0)
        worst["kalman_logdet"] = max(worst["kalman_logdet"], rel(o[i, 1], kf["logdet"]))
        worst["kalman_quad"] = max(worst["kalman_quad"], rel(o[i, 2], kf["quad"]))
        worst["single_logdet"] = max(worst["single_logdet"], rel(o[i, 1], one[1]))
        worst["single_loglik"] = max(worst["single_loglik"], rel(o[i, 0], one[0]))
        if unchecked is not None:
            uo = unchecked["out"]
            eu = rel(uo[i, 1], kf["logdet"])
            worst["unchecked_kalman_logdet"] = max(worst.get("unchecked_kalman_logdet", 0.0), eu)
            unchecked["over"] = unchecked.get("over", 0) + int(eu > 1e-8)
    del sw, splan
    if unchecked is not None:
        unchecked.pop("out")
        unchecked["logdet_max_rel_err_vs_kalman"] = worst.pop("unchecked_kalman_logdet")
        unchecked["items_over_1e-8"] = unchecked.pop("over", 0)
    res = {"metric": "GP log-likelihoods/s, batched hyperparameters (n=65536 shared series)",
           "value": args.steps * m / elapsed, "unit": "likelihoods/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 arithmetic, f32 panels" if mixed else "f64",
           "data": "synthetic",
           "config": {"workload": "batched_theta_m%d_n%d%s" % (m, n, "_mixed" if mixed else ""),
                      "n": n, "items": m,
                      "kernel": "matern32", "leaf": 128, "tol": 1e-10, "max_rank": 16,
                      "graph": True, "precision": args.precision, "tiles": tune.as_dict()},
           "tile_sweep_ms": sweep,
           "finite_items": int(np.isfinite(o[:, 0]).sum()),
           "ranks": {"batch_rank_max": info["rank_max"][:info["levels"]],
                     "capped_blocks": info["capped_blocks"]},
           "roofline": stage_roofline(model, stages, m),
           "pipeline_roofline": {"model_ms": pipe_ms, "measured_ms": ms_step,
                                 "frac": pipe_ms / ms_step,
                                 "note": "the per-point model of the single likelihood (each "
                                         "modelled stage at the larger of bytes / 8 TB/s and "
                                         "flops / 78.6 TFLOP/s, plus the basis writes) for "
                                         "every item at the batch-wide panel widths"},
           "stage_ms_per_step": {k: v[0] for k, v in stages.items()},
           "stage_note": "stage times from an eager (no graph) pass with every launch timed",
           "fp64_fallback": fallback,
           "mixed_unchecked": unchecked,
           "oracle_check": {"items": m, "max_rel_err": worst, "kalman_seconds_1core": t_k,
                            "note": "every item: log det and quadratic form against the exact "
                                    "Kalman oracle; log det and log-likelihood against the "
                                    "item's own gp_loglik_dev call (relative to max(|v|, 1))"}}
    print(json.dumps(res), flush=True)


def bench_grad(args, torch, H, wl, dev):
    """The Matern-3/2 workload of the benchmark line (n = 2^20, leaf 128, tol
    1e-10): one step = gp_loglik_grad_dev, the log-likelihood and its central
    difference gradient in (a, l, sigma2) from 7 likelihoods (the two sigma2
    items on the point's compression).  Checked against the same difference of the exact Kalman
    likelihood; the single-likelihood time on the same plan is reported for
    the cost ratio."""
    p = wl.matern1d(args.n)
    mixed = args.precision == "mixed"
    prec = H.MIXED if mixed else H.FP64
    plan = H.Plan(p.n, 1, p.leaf, H.Opts(max_rank=64, presorted=1, precision=prec))
    d_x = torch.from_numpy(np.ascontiguousarray(p.x.T)).to(dev)
    d_y = torch.from_numpy(p.y).to(dev)
    nb = plan.grad_workspace_bytes
    work = torch.empty(nb, dtype=torch.uint8, device=dev)
    out = torch.zeros(6, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()

    def step():
        H.gp_loglik_grad_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, 0.0, work, nb,
                             stream, out)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        # one likelihood on the same plan and workspace, for the cost ratio
        o1 = torch.zeros(8, dtype=torch.float64, device=dev)
        for _ in range(args.warmup):
            H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                            plan.workspace_bytes, stream, o1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                            plan.workspace_bytes, stream, o1)
        torch.cuda.synchronize()
        single = time.perf_counter() - t1
    o = out.cpu().numpy()
    info = plan.info()
    model = item_model(p.n, p.leaf, info["rank_max"][:info["levels"]], esz=4 if mixed else 8)
    ms_step = elapsed / args.steps * 1e3
    pipe_ms = model_ms(model, 7)
    import oracle
    oracle.build(force=False)
    base = [p.theta[0], p.theta[1], p.sigma2]
    h = 1e-3 if mixed else 1e-4
    L0 = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2, want_alpha=False)["loglik"]
    errs = []
    for j in range(3):
        up, dn = list(base), list(base)
        up[j] = base[j] * (1.0 + h)
        dn[j] = base[j] * (1.0 - h)
        Lu = oracle.kalman_matern32(p.x[:, 0], p.y, up[:2], up[2], want_alpha=False)["loglik"]
        Ld = oracle.kalman_matern32(p.x[:, 0], p.y, dn[:2], dn[2], want_alpha=False)["loglik"]
        gk = (Lu - Ld) / (up[j] - dn[j])
        errs.append({"grad": float(o[3 + j]), "kalman_difference": gk,
                     "err_over_L_per_p": abs(o[3 + j] - gk) / (abs(L0) / base[j])})
    res = {"metric": "GP log-likelihood gradients/s (value + dL/d(a, l, sigma2)) at n=2^20",
           "value": args.steps / elapsed, "unit": "gradients/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 arithmetic, f32 panels" if mixed else "f64", "data": "synthetic",
           "config": {"workload": "grad_matern32_1d_n%d_leaf%d_tol%g%s"
                                  % (p.n, p.leaf, p.tol, "_mixed" if mixed else ""),
                      "n": p.n, "kernel": "matern32", "theta": list(p.theta), "sigma2": p.sigma2,
                      "leaf": p.leaf, "tol": p.tol, "likelihoods_per_gradient": 7,
                      "rel_step": h, "precision": args.precision},
           "single_likelihood_ms": single / args.steps * 1e3,
           "cost_vs_one_likelihood": ms_step / (single / args.steps * 1e3),
           "pipeline_roofline": {"model_ms": pipe_ms, "measured_ms": ms_step,
                                 "frac": pipe_ms / ms_step,
                                 "note": "the per-point model of one likelihood (each modelled "
                                         "stage at the larger of bytes / 8 TB/s and flops / "
                                         "78.6 TFLOP/s) times the 7 likelihoods"},
           "result": {"loglik": float(o[0]), "grad": [float(v) for v in o[3:6]]},
           "oracle_check": {"loglik_rel_err_vs_kalman": abs(o[0] - L0) / abs(L0),
                            "components": errs,
                            "note": "each component against the same central difference of "
                                    "the exact Kalman likelihood at the same 7 points, error "
                                    "relative to |L| / p"}}
    print(json.dumps(res), flush=True)


def bench_ragged(args, torch, H, wl, dev):
    """Many independent series of uneven size: 512 items, n log-uniform in
    [1024, 131072], x ~ U(0, 10) sorted, y ~ N(0, 1), Matern-3/2, theta from
    the box of workloads.theta_box.  One step = one gp_loglik_ragged call over
    all items (host arrays in, host results out: the transfers of points and
    observations are inside the timed region)."""
    m = 512
    xs, ys, th = wl.batched_ragged(m=m)
    mixed = args.precision == "mixed"
    prec = H.MIXED if mixed else H.FP64
    opts = H.Opts(max_rank=16, precision=prec)
    # autotune the tiles once per size class (first item of each class,
    # untimed); the workers take them from the tuner's cache
    tuned = {}
    for i in range(m):
        cls = int(np.ceil(np.log2(len(xs[i]))))
        if cls not in tuned:
            t, _ = H.autotune(xs[i], ys[i], H.K_MATERN32, th[i, :2], th[i, 2], 1e-10,
                              H.Opts(max_rank=16, precision=prec, presorted=1),
                              leaf_cands=[128], reps=1)
            tuned[cls] = t.as_dict()

    def step():
        return H.gp_loglik_ragged(xs, ys, H.K_MATERN32, th, 128, 1e-10, opts, args.workers)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        o = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ntot = int(sum(len(x) for x in xs))
    # untimed: every item against the exact Kalman oracle and against a single
    # gp_loglik_dev call on its own plan, whose ranks feed the per-point model
    import oracle
    oracle.build(force=False)
    worst = {"kalman_logdet": 0.0, "kalman_quad": 0.0, "single_logdet": 0.0,
             "single_loglik": 0.0}
    pipe_ms = 0.0
    so = torch.zeros(8, dtype=torch.float64, device=dev)
    for i in range(m):
        ni = len(xs[i])
        a, ell, s2 = th[i]
        kf = oracle.kalman_matern32(xs[i][:, 0], ys[i], (a, ell), s2, want_alpha=False)
        pl = H.Plan(ni, 1, 128, H.Opts(max_rank=16, precision=prec, presorted=1))
        wk = torch.empty(pl.workspace_bytes, dtype=torch.uint8, device=dev)
        dx = torch.from_numpy(np.ascontiguousarray(xs[i][:, 0])).to(dev)
        dy = torch.from_numpy(np.ascontiguousarray(ys[i])).to(dev)
        H.gp_loglik_dev(pl, dx, H.K_MATERN32, (a, ell), s2, dy, 1e-10, wk, pl.workspace_bytes,
                        None, so)
        torch.cuda.synchronize()
        one = so[:3].cpu().numpy()
        inf = pl.info()
        pipe_ms += model_ms(item_model(ni, 128, inf["rank_max"][:inf["levels"]],
                                       esz=4 if mixed else 8))
        rel = lambda u, v: abs(u - v) / max(abs(v), 1.0)
        worst["kalman_logdet"] = max(worst["kalman_logdet"], rel(o[i, 1], kf["logdet"]))
        worst["kalman_quad"] = max(worst["kalman_quad"], rel(o[i, 2], kf["quad"]))
        worst["single_logdet"] = max(worst["single_logdet"], rel(o[i, 1], one[1]))
        worst["single_loglik"] = max(worst["single_loglik"], rel(o[i, 0], one[0]))
        del wk, pl
    res = {"metric": "GP log-likelihoods/s, independent series of uneven size",
           "value": args.steps * m / elapsed, "unit": "likelihoods/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 arithmetic, f32 panels" if mixed else "f64",
           "data": "synthetic",
           "config": {"workload": "ragged_m%d_n1024to131072%s" % (m, "_mixed" if mixed else ""),
                      "items": m, "precision": args.precision,
                      "total_points": ntot, "kernel": "matern32", "leaf": 128, "tol": 1e-10,
                      "max_rank": 16, "workers": args.workers, "host_buffers": True,
                      "tiles_per_size_class": {str(k): v for k, v in sorted(tuned.items())}},
           "points_per_s": args.steps * ntot / elapsed,
           "finite_items": int(np.isfinite(o[:, 0]).sum()),
           "pipeline_roofline": {"model_ms": pipe_ms, "measured_ms": elapsed / args.steps * 1e3,
                                 "frac": pipe_ms / (elapsed / args.steps * 1e3),
                                 "note": "sum over items of the per-point model at each item's "
                                         "own ranks; the measured time includes the host "
                                         "transfers, so the fraction is a lower bound"},
           "oracle_check": {"items": m, "max_rel_err": worst,
                            "note": "every item: log det and quadratic form against the exact "
                                    "Kalman oracle; log det and log-likelihood against a single "
                                    "gp_loglik_dev call on its own plan (relative to "
                                    "max(|v|, 1))"}}
    print(json.dumps(res), flush=True)


def bench_learned(args, torch, H, wl, dev):
    """Surrogate-screened sampling of log theta for n = 2^18 Matern-3/2 data
    drawn at theta = (1, 5, 0.1): Laplace scale from exact likelihoods,
    20000 exact training likelihoods around the mode, device training, then
    64 walkers of plain and of delayed-acceptance Metropolis with the same
    proposal; value = effective samples per second of the delayed form."""
    from paper_1403_6015_amd import learned as LR
    p = wl.learned(1 << 18)
    gp = LR.ExactGP(p.x, p.y, kernel=p.kernel, leaf=p.leaf, tol=p.tol, max_rank=16, chunk=256)
    t_true = np.log([p.theta[0], p.theta[1], p.sigma2])
    t0 = time.perf_counter()
    mode, cov = LR.laplace(gp, t_true, 0.05)
    t_laplace = time.perf_counter() - t0
    t0 = time.perf_counter()
    X, T = LR.training_set(gp, mode, cov, n=20000)
    t_data = time.perf_counter() - t0
    nval = 2000
    sur = LR.Surrogate(seed=0)
    t0 = time.perf_counter()
    hist = sur.fit(X[nval:], T[nval:], epochs=150, batch=256, lr=2e-3)
    t_train = time.perf_counter() - t0
    pred = sur.predict(X[:nval])
    rmse = float(np.sqrt(np.mean((pred - T[:nval]) ** 2)))
    # the network's kernels: flops of one training pass (forward and backward
    # on each minibatch sample: 2 x (3*128 + 128*128 + 128) multiply-adds
    # forward, twice that backward) over the fit's wall time, against the BF16
    # matrix peak (the products of the two 128-wide layers run on BF16 MFMA);
    # latency-bound at width 128, reported as achieved, not as a bound
    fl = 3.0 * 2.0 * (3 * 128 + 128 * 128 + 128) * (len(T) - nval) * 150
    mlp_tf = fl / t_train / 1e12
    rmse_bulk, nbulk = LR.bulk_rmse(pred, T[:nval], gp.loglik(mode[None])[0])
    sd = np.sqrt(np.diag(cov))
    lo, hi = mode - 12 * sd, mode + 12 * sd
    W = 64
    rng = np.random.default_rng(5)
    start = mode + 2.0 * rng.standard_normal((W, 3)) @ np.linalg.cholesky(cov).T
    start = np.clip(start, lo, hi)
    chol = 2.38 / np.sqrt(3.0) * np.linalg.cholesky(cov)
    steps, burn = args.mcmc_steps, args.mcmc_steps // 5
    res_runs = {}
    for name, s in (("plain", None), ("delayed", sur)):
        chain, tal, secs = LR.sample(gp, start, chol, lo, hi, steps, surrogate=s, seed=7)
        e = LR.chain_ess(chain, burn)
        post = chain[burn:].reshape(-1, 3)
        res_runs[name] = {"seconds": secs, "ess": e, "ess_per_s": e / secs,
                          "exact_evals": tal["exact_evals"], "survivors": tal["survivors"],
                          "accepted": tal["accepted"], "proposals": tal["proposals"],
                          "acceptance": tal["accepted"] / tal["proposals"],
                          "post_mean_log_theta": post.mean(axis=0).tolist(),
                          "post_sd_log_theta": post.std(axis=0).tolist()}
    da, pm = res_runs["delayed"], res_runs["plain"]
    res = {"metric": "effective samples/s of surrogate-screened (delayed-acceptance) Metropolis",
           "value": da["ess_per_s"], "unit": "effective samples/s", "n_gpus": 1,
           "steps": steps, "warmup": 0, "ms_per_step": da["seconds"] / steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "learned_damh_n262144_w64", "n": p.n, "walkers": W,
                      "kernel": "matern32", "theta_true": list(map(float, [p.theta[0], p.theta[1],
                                                                           p.sigma2])),
                      "training_pairs": int(len(T) - nval), "validation_pairs": nval,
                      "network": "3-128-128-1 tanh, bf16 weights, fp32 accumulation",
                      "burn_in": burn},
           "gain_vs_plain_mh": da["ess_per_s"] / pm["ess_per_s"],
           "plain_mh": pm, "delayed_acceptance": da,
           "surrogate": {"validation_rmse_nats": rmse, "validation_rmse_bulk_nats": rmse_bulk,
                         "validation_bulk_points": nbulk, "final_train_loss": float(hist[-50:].mean()),
                         "train_seconds": t_train, "data_seconds": t_data,
                         "laplace_seconds": t_laplace},
           "laplace": {"mode_log_theta": mode.tolist(), "sd_log_theta": sd.tolist()},
           "ess_per_s_including_training": da["ess"] / (da["seconds"] + t_train + t_data)}
    res["roofline"] = {"bound": "latency", "achieved": mlp_tf, "peak": PEAK["bf16_mfma"],
                       "unit": "TFLOP/s", "frac": mlp_tf / PEAK["bf16_mfma"], "traffic": None,
                       "kernel": "mlp_tile_kernel + mlp_update_kernel (one fit)",
                       "note": "width-128 network: the fit is bound by launch and barrier "
                               "latency, far below the BF16 matrix peak"}
    # the exact stage (the judge of the surrogate) against the exact
    # state-space oracle at the Laplace mode and at the last states of the
    # delayed chains
    import oracle
    oracle.build(force=False)
    pts = np.vstack([mode[None], chain[-1][:7]])
    ex = gp.loglik(pts)
    errs = []
    for q, e in zip(pts, ex):
        a, ell, s2 = np.exp(q)
        kf = oracle.kalman_matern32(p.x[:, 0], p.y, (a, ell), s2, want_alpha=False)
        errs.append(abs(e - kf["loglik"]) / abs(kf["loglik"]))
    res["oracle_check"] = {"points": int(len(pts)), "max_rel_err_loglik": float(max(errs)),
                           "note": "batched exact HODLR log-likelihoods (the second stage) "
                                   "against the Kalman oracle at the Laplace mode and seven "
                                   "chain states"}
    print(json.dumps(res), flush=True)


def bench_se2d(args, torch, H, wl, dev):
    """The 2-D configuration: n = 2^22 points ~ U([0,1]^2) (smaller --n keeps
    the density on a sub-square), k-d ordered, SE a = 1, l = 0.05,
    sigma^2 = 1e-2, leaf 256, off-diagonal ranks capped at --max-rank (64 as
    configured; a larger cap is the measured-cap variant), tolerance 1e-10.
    Timed: the device likelihood (compression, factorization, log det and one
    solve through the factor) with the ordered points resident in HBM.
    Untimed, beside it: the relative residual ||y - C z|| / ||y|| of the
    factor's solve z with C applied exactly (one O(n^2) FP64 product on the
    GPU, whose time is the cost of one refinement step), and for the level
    products on FP64 MFMA their achieved rate against the matrix peak."""
    n = args.n or (1 << 22)
    cap = args.max_rank if args.max_rank is not None else 64
    leaf = args.leaf or 256
    p = wl.se2d(n)
    mixed = args.precision == "mixed"
    prec = H.MIXED if mixed else H.FP64
    t0 = time.perf_counter()
    perm = H.hodlr_order(p.x, leaf)
    t_order = time.perf_counter() - t0
    xs = np.ascontiguousarray(p.x[perm])
    ys = np.ascontiguousarray(p.y[perm])
    sketch = args.compressor == "sketch"
    comp = H.COMPRESS_SKETCH if sketch else H.COMPRESS_ACA
    plan = H.Plan(n, 2, leaf, H.Opts(max_rank=cap, precision=prec, compressor=comp))
    d_x = torch.from_numpy(np.ascontiguousarray(xs.T)).to(dev)
    d_y = torch.from_numpy(ys).to(dev)
    work = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    out = torch.zeros(8, dtype=torch.float64, device=dev)
    z = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                        plan.workspace_bytes, stream, out, z)

    config = {"workload": "se2d_n%d_leaf%d_cap%d%s%s" % (n, leaf, cap, "_mixed" if mixed else "",
                                                       "_sketch" if sketch else ""),
              "n": n, "dim": 2, "kernel": "se", "theta": list(p.theta), "sigma2": p.sigma2,
              "side": p.meta["side"], "leaf": leaf, "max_rank": cap, "tol": p.tol,
              "precision": args.precision, "compressor": args.compressor,
              "workspace_bytes": plan.workspace_bytes}
    res = {"metric": "GP log-likelihoods/s, 2-D SE (n=2^22 unit square at full size)",
           "unit": "likelihoods/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 arithmetic, f32 panels" if mixed else "f64", "data": "synthetic",
           "config": config, "ordering_s": t_order}
    try:
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    except H.HodlrError as e:
        # the configured cap can be too coarse for this kernel and noise level:
        # the library then reports a coupling matrix that is not positive
        res.update({"value": None, "ms_per_step": None, "status": e.name, "error": str(e)})
        print(json.dumps(res), flush=True)
        return
    loglik, logdet, quad = out[:3].cpu().tolist()
    info = plan.info()
    # per-stage breakdown in a pass of its own (every launch timed)
    H.profile_select(None)
    H.profile_enable(True)
    step()
    torch.cuda.synchronize()
    stages = {k: v for k, v in H.profile_read().items() if v[1] > 0}
    H.profile_enable(False)
    # exact residual of the factor's solve
    cz = torch.empty_like(z)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    H.hodlr_matvec_dev(n, 2, d_x, p.kernel, p.theta, p.sigma2, z, cz, stream)
    torch.cuda.synchronize()
    t_mv = time.perf_counter() - t1
    resid = float(torch.linalg.vector_norm(d_y - cz) / torch.linalg.vector_norm(d_y))
    L = info["levels"]
    r = [0] + [int(v) for v in info["rank_max"][:L]]
    cnt = [1]
    for j in range(1, L + 1):
        cnt.append(cnt[-1] + r[j])
    leaf_sizes = np.diff(np.linspace(0, n, (1 << L) + 1).round()).astype(int)
    model = kernel_model(n, leaf_sizes, r, cnt, esz=4 if mixed else 8)
    mfma = {}
    for k in ("level_reduce", "level_update", "leaf_factor"):
        if k in stages and k in model:
            fl, by = model[k]
            ms = stages[k][0]
            ach = fl / (ms / 1e3) / 1e12
            mfma[k] = {"achieved": ach, "frac": ach / PEAK["alu_fp64"], "ms": ms,
                       "launches": stages[k][1], "flops": fl, "bytes": by}
    dom = max(("level_reduce", "level_update", "leaf_factor"),
              key=lambda k: mfma[k]["ms"] if k in mfma else -1.0)
    roofline = None
    if dom in mfma:
        d = mfma[dom]
        roofline = {"bound": "mfma", "achieved": d["achieved"], "peak": PEAK["alu_fp64"],
                    "unit": "TFLOP/s", "frac": d["frac"], "traffic": None, "kernel": dom,
                    "dtype": "fp64", "avg_launch_ms": d["ms"] / d["launches"],
                    "algorithmic_per_call": {"flops": d["flops"] / d["launches"],
                                             "bytes": d["bytes"] / d["launches"]}}
    sketch_info = None
    if sketch:
        # the sketch stage on FP64 MFMA: per node, A X and A^T Y (2 m nb (s + s')
        # flops) and the partial cores (2 m s' s), with the widths the library uses
        fl = 0.0
        sizes = [n]
        for d in range(L):
            nxt = []
            for sz in sizes:
                m_, nb_ = sz // 2, sz - sz // 2
                s_ = min(cap + 16, m_, nb_)
                sp_ = min(s_ + 8, m_) if s_ > 0 else 0
                fl += 2.0 * m_ * nb_ * (s_ + sp_) + 2.0 * m_ * sp_ * s_
                nxt += [m_, nb_]
            sizes = nxt
        ms_sk = stages.get("sketch", (float("nan"), 0))[0]
        ach = fl / (ms_sk / 1e3) / 1e12
        sketch_info = {"flops": fl, "ms": ms_sk, "achieved_tflops": ach,
                       "frac": ach / PEAK["alu_fp64"], "launches": stages.get("sketch", (0, 0))[1],
                       "note": "the sketch products' flops over the sketch kernels' summed "
                               "event time, against the FP64 matrix peak"}
        # the same likelihood with cross approximation, untimed, for comparison
        aplan = H.Plan(n, 2, leaf, H.Opts(max_rank=cap, precision=prec))
        aw = torch.empty(aplan.workspace_bytes, dtype=torch.uint8, device=dev)
        ao = torch.zeros(8, dtype=torch.float64, device=dev)
        try:
            H.gp_loglik_dev(aplan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, aw,
                            aplan.workspace_bytes, stream, ao)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for _ in range(args.steps):
                H.gp_loglik_dev(aplan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, aw,
                                aplan.workspace_bytes, stream, ao)
            torch.cuda.synchronize()
            aco = ao[:3].cpu().tolist()
            sketch_info["aca_same_problem"] = {
                "ms_per_likelihood": (time.perf_counter() - t2) / args.steps * 1e3,
                "logdet": aco[1], "logdet_rel_diff": abs(aco[1] - logdet) / abs(logdet),
                "rank_max": aplan.info()["rank_max"][:L]}
        except H.HodlrError as e:
            sketch_info["aca_same_problem"] = {"status": e.name}
        del aw, aplan
    res.update({"value": args.steps / el, "ms_per_step": el / args.steps * 1e3, "status": "OK",
                "sketch": sketch_info,
                "ranks": {"rank_max": info["rank_max"], "rank_mean": info["rank_mean"],
                          "capped_blocks": info["capped_blocks"]},
                "roofline": roofline, "mfma_level_kernels": mfma,
                "stage_ms_per_step": {k: v[0] for k, v in stages.items()},
                "stage_launches_per_step": {k: v[1] for k, v in stages.items()},
                "result": {"loglik": loglik, "logdet": logdet, "quad": quad},
                "oracle_check": {"relative_residual": resid, "exact_product_seconds": t_mv,
                                 "note": "||y - C z|| / ||y|| for the factor's unrefined solve "
                                         "z, C applied entry by entry in FP64 on the GPU "
                                         "(hodlr_matvec_dev); no dense oracle exists at this "
                                         "size"}})
    print(json.dumps(res), flush=True)


# VALU instructions per kernel evaluation in the inner loop of the 1-D
# Matern-3/2 product kernel (gfx950 assembly, -O3: 109 instructions per
# unrolled iteration of 4 evaluations: subtract, |d| c, the exponential's
# reduction, polynomial and scaling, its range selects, (1 + s), the product
# with alpha and the accumulation)
PREDICT_VALU_PER_EVAL = 109 / 4


def bench_predict(args, torch, H, wl, dev):
    """Prediction through the factor (§2.1) at the benchmark configuration:
    the n = 2^20 Matern-3/2 series, factor built once (untimed); one step =
    posterior means at --m new inputs ~ U(0, 1000) (hodlr_predict without
    variances: C^{-1} y through the factor, then the exact products
    k(xt, x) alpha over all n training points).  The product kernel is bound
    by FP64 vector arithmetic; its roofline peak is the VALU issue rate (256
    CUs x 4 SIMDs x 16 lanes x 2.4 GHz) over the instructions one evaluation
    takes.  Once, untimed in the rate: variances at 8 inputs (one solve
    each)."""
    import oracle
    p = wl.matern1d(args.n)
    m = args.m
    f = H.hodlr_build(p.x, p.kernel, p.theta, p.sigma2, p.leaf, p.tol, H.Opts(max_rank=64))
    xt = np.random.default_rng(2024).uniform(0.0, 1000.0, (m, 1))
    for _ in range(args.warmup):
        f.predict(p.y, xt, var=False)
    H.profile_select(["predict"])
    H.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mean, _ = f.predict(p.y, xt, var=False)
    el = time.perf_counter() - t0
    prof = H.profile_read()
    H.profile_enable(False)
    H.profile_select(None)
    k_ms, k_launches = prof["predict"]
    per_launch_s = k_ms / 1e3 / k_launches
    evals = float(p.n) * m
    peak = 256 * 4 * 16 * 2.4e9 / PREDICT_VALU_PER_EVAL / 1e9
    ach = evals / per_launch_s / 1e9
    roofline = {"bound": "alu", "achieved": ach, "peak": peak, "unit": "Geval/s",
                "frac": ach / peak, "traffic": None, "kernel": "predict_part_kernel<matern32,1>",
                "avg_launch_ms": per_launch_s * 1e3,
                "algorithmic_per_launch": {"kernel_evaluations": evals,
                                           "valu_per_evaluation": PREDICT_VALU_PER_EVAL},
                "note": "peak = 256 CUs x 64 FP64 lanes x 2.4 GHz / VALU instructions per "
                        "evaluation; the inputs (16 MB) are read once per slice from L2/LDS"}
    t1 = time.perf_counter()
    _, var8 = f.predict(p.y, xt[:8])
    t_var = time.perf_counter() - t1
    f.free()
    res = {"metric": "posterior means/s through the n=2^20 factor (exact k(xt, x) alpha)",
           "value": m * args.steps / el, "unit": "means/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "predict_matern32_n%d_m%d" % (p.n, m), "n": p.n, "m": m,
                      "kernel": "matern32", "theta": list(p.theta), "sigma2": p.sigma2,
                      "leaf": p.leaf, "tol": p.tol},
           "roofline": roofline,
           "variance": {"inputs": 8, "seconds": t_var, "values": var8.tolist()}}
    if not args.no_cpu_baseline:
        # the oracle: exact alpha from the O(n) Kalman solves, then entry-by-entry
        # kernel rows (OpenMP over rows) times alpha, for every new input
        oracle.build(force=False)
        t2 = time.perf_counter()
        alpha = oracle.kalman_matern32(p.x[:, 0], p.y, p.theta, p.sigma2)["alpha"]
        ref = np.empty(m)
        for j0 in range(0, m, 64):
            ref[j0:j0 + 64] = oracle.cross_matrix(xt[j0:j0 + 64], p.x, p.kernel, p.theta) @ alpha
        dt = time.perf_counter() - t2
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        res["cpu_baseline"] = {"value": m / dt, "unit": "means/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "all %d means of one step: Kalman alpha at n=%d plus "
                                         "%d x %d kernel entries times alpha, %.1f s on %d "
                                         "threads" % (m, p.n, m, p.n, dt, threads)}
        res["oracle_check"] = {"mean_max_rel_err": float(np.max(np.abs(mean - ref))
                                                         / max(1.0, np.max(np.abs(ref))))}
    print(json.dumps(res), flush=True)


# The paper's single-core timings at n = 10^6 (§5, one-dimensional rows of the
# Gaussian table tab_gauss_all, the exponential table tab_exp and the inverse
# multiquadric table tab_inv): assembly + factor + solve + determinant, seconds.
def profile_run(args, torch, H, p, dev):
    """The benchmark's likelihood, warmup + steps calls on one plan with the
    default tiles (512 rows per level chunk), nothing else: the command the
    counter profiles run, so that every dispatch of a kernel belongs to one of
    these calls."""
    perm = H.hodlr_order(p.x, p.leaf)
    xs, ys = p.x[perm], p.y[perm]
    spec = 0 if args.no_speculate else 1
    plan = H.Plan(p.n, p.dim, p.leaf, H.Opts(max_rank=64, presorted=1, speculate=spec,
                                             level_form=1 if args.level_by_level else 0))
    d_x = torch.from_numpy(np.ascontiguousarray(xs.T)).to(dev)
    d_y = torch.from_numpy(np.ascontiguousarray(ys)).to(dev)
    work = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    out = torch.zeros(8, dtype=torch.float64, device=dev)
    z = torch.empty(p.n, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                        plan.workspace_bytes, None, out, z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        H.gp_loglik_dev(plan, d_x, p.kernel, p.theta, p.sigma2, d_y, p.tol, work,
                        plan.workspace_bytes, None, out, z)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(json.dumps({"profile_run": "matern32_1d_n%d_leaf%d" % (p.n, p.leaf),
                      "calls": args.warmup + args.steps, "ms_per_call": el / args.steps * 1e3,
                      "logdet": float(out[1].item()), "speculated": plan.info()["speculated"]}),
          flush=True)


def bench_copy(args, torch, dev):
    """Calibration for the HBM byte counters: a plain elementwise copy of
    2^28 doubles (2 GiB read, 2 GiB written per launch), one launch per step."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gbs = 2 * 8 * n * args.steps / el / 1e9
    print(json.dumps({"metric": "copy bandwidth (counter calibration)", "value": gbs,
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                      "data": "synthetic",
                      "config": {"workload": "copy_2p28_f64", "bytes_read_per_launch": 8 * n,
                                 "bytes_written_per_launch": 8 * n}}), flush=True)


if __name__ == "__main__":
    main()
