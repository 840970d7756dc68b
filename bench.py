"""FKT MVM throughput on one MI355X.

One step = one fkt_mvm over the whole hot path (gather into tree order,
source-to-multipole moments, multipole-to-target far field, near field and
scatter) for one right-hand side, with the points' plan and x resident in
HBM. Workload: one million points uniform in [0,1]^3, leaf 256, order p = 6,
one RHS x ~ N(0,1) (seeds 1002 / 2002); the kernel (Laplace 1/r or
Matern-3/2 l = 0.05) and precision are flags. theta defaults to the largest
value on a 0.05 grid whose relative error against the dense FP64 sum stays
at or below 1e-5 for that kernel.

Prints one JSON line (rank 0). See the design doc for the roofline model.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import fkt_workloads as W  # noqa: E402

# largest theta on a 0.05 grid with rel err <= 1e-5 vs dense FP64 at the
# default workload (measured by the error sweep)
DEFAULT_THETA = {("laplace", "f64"): 0.32, ("laplace", "f32"): 0.32,
                 ("matern32", "f64"): 0.26, ("matern32", "f32"): 0.26}
KERNEL_KW = {"laplace": {}, "matern32": {"lengthscale": 0.05}}
ORACLE_KIND = {"laplace": ("power", {"shape": 1.0}), "matern32": ("matern32", {"lengthscale": 0.05})}

# MI355X peaks (published): FP64 vector 78.6 TFLOP/s = 256 CUs x 4 SIMDs x 16
# lanes x 2 (FMA) x 2.4 GHz, i.e. 39.3e12 FP64 lane-instructions/s; FP32
# without packed math issues at the same lane rate.
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

# VALU instructions per near-field pair of the near kernel's inner loop
# (counted in the gfx950 ISA of this build)
NEAR_OPS_PER_PAIR = {("laplace", "f64"): 17, ("laplace", "f32"): 9,
                     ("matern32", "f64"): 38, ("matern32", "f32"): 13}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel", default="laplace", choices=sorted(KERNEL_KW))
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"])
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--leaf", type=int, default=256)
    ap.add_argument("--order", type=int, default=6)
    ap.add_argument("--err-targets", type=int, default=2000,
                    help="targets sampled (seed 3002) for the error against the dense FP64 sum; 0 skips")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="time budget of the CPU-oracle baseline sample; 0 skips")
    a = ap.parse_args()

    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU path is a design, "
              "not a build (DESIGN.md, 'Sharding')", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2106_04487_amd as F

    theta = a.theta if a.theta is not None else DEFAULT_THETA[(a.kernel, a.prec)]
    X = W.uniform_cube(a.n, 3, 1002)
    x64 = W.normal_rhs(a.n, 1, 2002)[:, 0]
    dt = torch.float32 if a.prec == "f32" else torch.float64
    print(f"bench: n={a.n} kernel={a.kernel} prec={a.prec} theta={theta} leaf={a.leaf} p={a.order}", file=sys.stderr,
          flush=True)
    plan = F.fkt_plan(X, a.kernel, a.leaf, a.order, theta=theta, prec=a.prec, profile=True, **KERNEL_KW[a.kernel])
    info = plan.info()
    x = torch.as_tensor(x64, dtype=dt, device="cuda")
    y = torch.empty_like(x)

    for _ in range(a.warmup):
        F.fkt_mvm(plan, x, y)
    torch.cuda.synchronize()
    plan.stage_times(reset=True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(a.steps):
        F.fkt_mvm(plan, x, y)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(stop)
    stages, calls = plan.stage_times()
    ms_per_step = wall * 1e3 / a.steps
    value = a.n / (ms_per_step * 1e-3) / 1e6
    print(f"bench: {ms_per_step:.3f} ms/step (events {ev_ms / a.steps:.3f}); stages ms/step "
          + ", ".join(f"{k} {v / calls:.3f}" for k, v in stages.items()), file=sys.stderr, flush=True)

    # error against the dense FP64 sum on sampled targets (CPU oracle)
    rel_err = None
    z = y.double().cpu().numpy()
    import oracle
    okind, okw = ORACLE_KIND[a.kernel]
    if a.err_targets > 0:
        tg = W.subsample(a.n, a.err_targets, 3002)
        zd = oracle.dense_mvm(X, x64, okind, targets=tg, **okw)[:, 0]
        rel_err = float(np.linalg.norm(z[tg] - zd) / np.linalg.norm(zd))
        print(f"bench: rel err vs dense FP64 on {len(tg)} targets: {rel_err:.3e}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (near field): VALU-bound
    near_ms = stages["near"] / calls
    ops = info["near_pairs"] * NEAR_OPS_PER_PAIR[(a.kernel, a.prec)]
    achieved = ops / (near_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": "k_near", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "T lane-ops/s", "frac": achieved / PEAK_LANE_OPS, "traffic": None,
                "units_per_launch": info["near_pairs"], "ops_per_unit": NEAR_OPS_PER_PAIR[(a.kernel, a.prec)],
                "avg_launch_ms": near_ms}

    cpu = None
    if a.cpu_seconds > 0:
        # the oracle's rows (Algorithm 1 per target, pairwise expansion) on a
        # bounded sample of targets, on all host cores
        T = oracle.Tree(X, a.leaf)
        tg = W.subsample(a.n, 4096, 3003)
        done, t0 = 0, time.perf_counter()
        while done < len(tg) and time.perf_counter() - t0 < a.cpu_seconds:
            oracle.fkt_rows(T, x64, okind, theta, a.order, tg[done:done + 32], **okw)
            done += 32
        el = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        cpu = {"value": done / el / 1e6, "unit": "Mpoints/s", "cores": threads, "kind": "oracle",
               "sample": f"{done} of {a.n} target rows of the oracle's Algorithm 1 (pairwise far field), "
                         f"{el:.1f} s"}

    out = {
        "metric": "FKT MVM Mpoints/s at rel err <=1e-5",
        "value": value, "unit": "Mpoints/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": a.prec, "data": "synthetic",
        "config": {"workload": f"cube3_n{a.n}_{a.kernel}", "n": a.n, "d": 3, "kernel": a.kernel,
                   **KERNEL_KW[a.kernel], "leaf": a.leaf, "p": a.order, "theta": theta, "nrhs": 1},
        "rel_err_vs_dense": rel_err,
        "stages_ms": {k: v / calls for k, v in stages.items()},
        "plan": {k: info[k] for k in ("nnodes", "nleaves", "nblocks", "near_pairs", "near_lane_pairs",
                                      "far_pairs", "far_lane_pairs", "plan_seconds")},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
