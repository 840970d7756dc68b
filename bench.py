"""FKT MVM throughput on one MI355X.

One step = one fkt_mvm over the whole hot path -- gather of x into tree
order, source-to-multipole moments, multipole-to-target far field, near
field, scatter to the caller's order -- for one right-hand side, with the
plan and x resident in HBM.

Workload (headline): one million points uniform in [0,1]^3 (seed 1002),
x ~ N(0,1) (seed 2002), leaf 256, order p = 6, Matern-3/2 kernel with length
scale 0.05, FP64, theta = 0.26: the largest theta on a 0.01 grid whose
relative error against the dense FP64 sum (3000 sampled targets) stays at or
below 1e-5. Variants on the same points: Laplace 1/r (theta 0.32) in FP64,
and both kernels in FP32. Every line reports its measured error against the
dense FP64 sum on sampled targets.

Prints one JSON line. Roofline: algorithmic FP64 (or FP32) flops of the
dominant kernel (near field: 40 per pair; far field: 418 per pair at d = 3,
p = 6) over its launch time measured with HIP events, against the vector
peak.
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

# largest theta on a 0.01 grid with rel err <= 1e-5 against the dense FP64
# sum on the one-million-point workload (error sweep on 3,000 targets)
DEFAULT_THETA = {"laplace": 0.32, "matern32": 0.26}
KERNEL_KW = {"laplace": {}, "matern32": {"lengthscale": 0.05}}
ORACLE_KIND = {"laplace": ("power", {"shape": 1.0}), "matern32": ("matern32", {"lengthscale": 0.05})}

# Published MI355X vector peaks (TFLOP/s): FP64 78.6, FP32 157.3.
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
# Algorithmic work per unit, as the method's cost model prices it: one
# near-field pair evaluation (distance, kernel value, multiply-accumulate)
# at 40 vector flops, and one far (target, node) expansion at d = 3, p = 6
# at 418 flops (84 moment multiply-adds, 168, plus about 250 for the
# harmonics, the radial derivatives and the Tbar combinations).
NEAR_FLOPS_PER_PAIR = 40
M2T_FLOPS_PER_PAIR = {(3, 6): 418}
# HBM bytes per near-field launch from FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0
# (scale factors of a plain copy) of the current near kernel, from the
# counter profile under profiles/; empty until re-measured after a change.
NEAR_TRAFFIC_BYTES = {("matern32", "f64"): 2.368e9}
# the same for the node-major far-field launch (target coordinates re-read
# per pair, one atomic add per pair)
M2T_TRAFFIC_BYTES = {("matern32", "f64"): 1.825e10}


def run_variant(F, torch, X, x64, kernel, prec, theta, leaf, order, steps, warmup, err_targets, overlap=True,
                compress=False):
    dt = torch.float32 if prec == "f32" else torch.float64
    n = X.shape[0]
    print(f"bench: n={n} kernel={kernel} prec={prec} theta={theta} leaf={leaf} p={order} overlap={overlap} "
          f"compress={compress}", file=sys.stderr, flush=True)
    plan = F.fkt_plan(X, kernel, leaf, order, theta=theta, prec=prec, profile=True, overlap=overlap,
                      compress=compress, **KERNEL_KW[kernel])
    info = plan.info()
    x = torch.as_tensor(x64, dtype=dt, device="cuda")
    y = torch.empty_like(x)
    for _ in range(warmup):
        F.fkt_mvm(plan, x, y)
    torch.cuda.synchronize()
    plan.stage_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        F.fkt_mvm(plan, x, y)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages, calls = plan.stage_times()
    stages = {k: v / calls for k, v in stages.items()}
    ms = wall * 1e3 / steps
    print(f"bench: {ms:.3f} ms/step; stages ms/step " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()),
          file=sys.stderr, flush=True)
    rel_err = None
    if err_targets > 0:
        import oracle
        okind, okw = ORACLE_KIND[kernel]
        z = y.double().cpu().numpy()
        tg = W.subsample(n, err_targets, 3002)
        zd = oracle.dense_mvm(X, x64, okind, targets=tg, **okw)[:, 0]
        rel_err = float(np.linalg.norm(z[tg] - zd) / np.linalg.norm(zd))
        print(f"bench: rel err vs dense FP64 on {len(tg)} targets: {rel_err:.3e}", file=sys.stderr, flush=True)
    plan.close()
    return {"kernel": kernel, "prec": prec, "theta": theta, "radial_compression": compress,
            "radial_rank": info["radial_rank"], "ms_per_step": ms, "mpoints_per_s": n / ms / 1e3,
            "rel_err_vs_dense": rel_err, "stages_ms": stages, "plan": info}


def nsweep_leg(F, torch, steps, err_targets, kernel="matern32", prec="f64"):
    """The headline settings (uniform cube, leaf 256, p = 6, the kernel's
    theta) at N from 1e4 to 1e6: time per MVM against N shows the
    O(N log N) growth of the method."""
    out = []
    for n in (10_000, 31_623, 100_000, 316_228, 1_000_000):
        X = W.uniform_cube(n, 3, 1002)
        x64 = W.normal_rhs(n, 1, 2002)[:, 0]
        r = run_variant(F, torch, X, x64, kernel, prec, DEFAULT_THETA[kernel], 256, 6, steps, 3, min(err_targets, n))
        info = r.pop("plan")
        r.update({"n": n, "near_pairs": info["near_pairs"], "far_pairs": info["far_pairs"]})
        out.append(r)
    return out


def gp_solve(F, torch, n, theta, order, rank, rtol, maxit, train_steps, fp64_none=False):
    """Gaussian-process solve (K~ + sigma2 I) x = y by CG through the FKT MVM
    at the GP workload's settings (d = 4 mixture, Matern-5/2 length scale 0.3,
    sigma2 = 1e-2). Every solve stops at relative residual rtol under the
    FP64 operator:
      * none: plain CG, FP32 MVMs with the residual replaced by the FP64 one
        (fkt_cg_solve_refined; and plain FP64 CG with fp64_none);
      * block_jacobi: two-level (Nystrom coarse space of `rank` landmarks,
        block-Jacobi of the residual leaf blocks), FP64 MVMs and refined;
      * learned: the same two-level form with the learned per-leaf filter
        after train_steps Adam steps on the condition-number objective
        (30 Lanczos steps per draw), judged by block-Jacobi on 200 CG
        iterations (reverted to block-Jacobi exactly if worse)."""
    spec = W.WORKLOADS["gmm4_n200k_gp"]
    X = W.gaussian_mixture(n, spec["d"], spec["ncomp"], spec["std"], spec["pts_seed"])
    y = W.gp_targets(X, spec["lengthscale"], spec["sigma2"], spec["nfeat"], spec["rhs_seed"])
    ell, sig2, kern = spec["lengthscale"], spec["sigma2"], spec["kernel"]
    t0 = time.perf_counter()
    p64 = F.fkt_plan(X, kern, spec["leaf"], order, theta=theta, lengthscale=ell)
    p32 = F.fkt_plan(X, kern, spec["leaf"], order, theta=theta, prec="f32", lengthscale=ell)
    plan_s = time.perf_counter() - t0
    b = torch.as_tensor(y, device="cuda")
    out = {"workload": f"gmm{spec['d']}_n{n}_matern52_l{ell}_gp", "n": n, "d": spec["d"], "lengthscale": ell,
           "theta": theta, "p": order, "leaf": spec["leaf"], "sigma2": sig2, "rtol": rtol, "maxit": maxit,
           "coarse_rank": rank, "plan_seconds_f64_and_f32": plan_s}

    def timed(name, fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            res = fn()
            ok = True
        except F.FktError as e:
            if e.status != 5:
                raise
            res = (None, e.iters, getattr(e, "outer", None), e.relres) if hasattr(e, "outer") else (None, e.iters, e.relres)
            ok = False
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        if len(res) == 4:
            rec = {"iterations_f32": res[1], "fp64_replacements": res[2], "relres_fp64": res[3]}
        else:
            rec = {"iterations": res[1], "relres_fp64": res[2]}
        rec.update({"converged": ok, "seconds": sec})
        out[name] = rec
        print(f"bench: gp {name}: {rec}", file=sys.stderr, flush=True)

    refined = lambda pc: (lambda: F.fkt_cg_solve_refined(p64, p32, sig2, b, rtol=rtol, maxit=maxit, precond=pc))
    plain = lambda pc: (lambda: F.fkt_cg_solve(p64, sig2, b, rtol=rtol, maxit=maxit, precond=pc))
    timed("none_refined", refined("none"))
    if fp64_none:
        timed("none", plain("none"))
    # two-level preconditioning: the same landmarks on both plans
    lm = W.subsample(n, rank, 4242)
    t0 = time.perf_counter()
    F.fkt_precond_coarse(p64, sig2, lm)
    F.fkt_precond_coarse(p32, sig2, lm)
    out["coarse_setup_seconds_both_plans"] = time.perf_counter() - t0
    timed("block_jacobi", plain("block_jacobi"))
    timed("block_jacobi_refined", refined("block_jacobi"))
    t0 = time.perf_counter()
    k0, k1, accepted = F.fkt_learn_train_cond(p64, sig2, train_steps, lanczos=30, lr=1e-2, seed=1, judge_iters=200)
    torch.cuda.synchronize()
    out["learned_training"] = {"objective": "log condition number (Lanczos)", "steps": train_steps,
                               "seconds": time.perf_counter() - t0, "kappa_first": k0, "kappa_last": k1,
                               "kept_after_block_jacobi_judge": accepted}
    timed("learned", plain("learned"))
    out["learned"]["fallback_to_block_jacobi_at"] = p64.info()["cg_fallback_iter"]
    F.fkt_learn_params(p32, sig2, F.fkt_learn_params(p64, sig2))
    timed("learned_refined", refined("learned"))
    p32.close()
    p64.close()
    return out


def gp_mvm_leg(F, torch, steps, theta=0.3, order=8):
    """MVM time of the GP workload's operator (FP64 and FP32 plans), with
    stage times; the solves of gp_solve spend their time here."""
    spec = W.WORKLOADS["gmm4_n200k_gp"]
    X = W.gaussian_mixture(spec["n"], spec["d"], spec["ncomp"], spec["std"], spec["pts_seed"])
    out = {"workload": f"gmm{spec['d']}_n{spec['n']}_matern52_l{spec['lengthscale']}", "theta": theta, "p": order}
    for prec in ("f64", "f32"):
        plan = F.fkt_plan(X, spec["kernel"], spec["leaf"], order, theta=theta, prec=prec, profile=True,
                          lengthscale=spec["lengthscale"])
        x = torch.as_tensor(W.normal_rhs(spec["n"], 1, 7)[:, 0], dtype=torch.float32 if prec == "f32" else
                            torch.float64, device="cuda")
        y = torch.empty_like(x)
        F.fkt_mvm(plan, x, y)
        ms = _sync_time(torch, lambda: F.fkt_mvm(plan, x, y), steps)
        plan.stage_times(reset=True)
        F.fkt_mvm(plan, x, y)
        st, c = plan.stage_times()
        out[prec] = {"ms_per_mvm": ms, "stages_ms": {k: v / c for k, v in st.items()}, "far_pairs":
                     plan.info()["far_pairs"], "near_pairs": plan.info()["near_pairs"]}
        print(f"bench: gp mvm {prec}: {ms:.2f} ms", file=sys.stderr, flush=True)
        plan.close()
    return out


def _sync_time(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def batch_leg(F, torch, reps, theta, err_per_inst, leaf=0, per_instance=True):
    """Batched uneven instances: 256 sets in d = 3 with log-uniform sizes in
    [1e3, 1e5], rational quadratic kernel, 4 RHS, FP32: one forest plan
    (eager launches and one HIP graph) against per-instance plans and
    launches; leaf size from the library's autotuner."""
    import oracle
    spec = W.WORKLOADS["batch256_rq"]
    sizes = W.instance_sizes(spec["ninst"], spec["nmin"], spec["nmax"], spec["size_seed"])
    X, off = W.batched_instances(sizes, spec["d"], spec["pts_seed"])
    n = X.shape[0]
    x64 = W.normal_rhs(n, spec["nrhs"], spec["rhs_seed"])
    kw = dict(lengthscale=spec["lengthscale"], alpha=spec["alpha"])
    p = spec["order"]
    tune = None
    far_mode = "auto"
    if leaf <= 0:
        # leaf size and far-field schedule from the library's autotuner
        t0 = time.perf_counter()
        (leaf, far_mode), table = F.fkt_autotune((X, off), spec["kernel"], p, [256, 512, 1024], ("block", "node"),
                                                 nrhs=spec["nrhs"], reps=2, theta=theta, prec="f32", batch=True, **kw)
        tune = {f"{lf}/{m}": v for (lf, m), v in table.items()}
        tune_s = time.perf_counter() - t0
        print(f"bench: batch autotune {tune} -> leaf {leaf}, {far_mode} ({tune_s:.1f} s)", file=sys.stderr,
              flush=True)
    x = torch.as_tensor(x64, dtype=torch.float32, device="cuda").contiguous()
    y = torch.empty_like(x)
    t0 = time.perf_counter()
    plan = F.fkt_plan_batch((X, off), spec["kernel"], leaf, p, theta=theta, prec="f32", far_mode=far_mode, **kw)
    plan_s = time.perf_counter() - t0
    F.fkt_mvm(plan, x, y)
    eager_ms = _sync_time(torch, lambda: F.fkt_mvm(plan, x, y), reps)
    g = F.Graph(plan, x, y)
    g.launch()
    graph_ms = _sync_time(torch, g.launch, reps)
    yb = y.double().cpu().numpy()
    g.close()
    plan.close()
    # per-instance plans, one fkt_mvm each
    per_ms = plans_s = None
    if per_instance:
        t0 = time.perf_counter()
        plans = [F.fkt_plan(X[off[i]:off[i + 1]], spec["kernel"], leaf, p, theta=theta, prec="f32",
                            far_mode=far_mode, **kw) for i in range(len(sizes))]
        plans_s = time.perf_counter() - t0
        xs = [x[off[i]:off[i + 1]] for i in range(len(sizes))]
        ys = [y[off[i]:off[i + 1]] for i in range(len(sizes))]

        def per_instance_mvms():
            for q, xi, yi in zip(plans, xs, ys):
                F.fkt_mvm(q, xi, yi)
        per_instance_mvms()
        per_ms = _sync_time(torch, per_instance_mvms, reps)
        for q in plans:
            q.close()
    # error against the dense FP64 sum on sampled targets of a few instances
    errs = []
    for i in W.subsample(len(sizes), 8, 3005):
        a, b = off[i], off[i + 1]
        tg = W.subsample(b - a, err_per_inst, 3006 + int(i))
        zd = oracle.dense_mvm(X[a:b], x64[a:b], "ratquad", targets=tg, lengthscale=spec["lengthscale"],
                              shape=spec["alpha"])
        errs.append(float(np.linalg.norm(yb[a:b][tg] - zd) / np.linalg.norm(zd)))
    out = {"workload": f"batch{len(sizes)}_rq_d3_n{n}", "instances": len(sizes), "n_total": int(n),
           "size_min": int(sizes.min()), "size_max": int(sizes.max()), "nrhs": spec["nrhs"], "dtype": "f32",
           "theta": theta, "p": p, "leaf": leaf, "far_mode": far_mode, "autotune_ms": tune,
           "batched_graph_ms": graph_ms,
           "batched_eager_ms": eager_ms, "per_instance_ms": per_ms,
           "batched_graph_mpoints_per_s": n / graph_ms / 1e3,
           "speedup_graph_vs_per_instance": per_ms / graph_ms if per_ms else None,
           "plan_seconds_batched": plan_s, "plan_seconds_per_instance_total": plans_s,
           "rel_err_vs_dense_max_of_8_instances": max(errs)}
    print(f"bench: batch {len(sizes)} instances n={n}: graph {graph_ms:.2f} ms, eager {eager_ms:.2f} ms, "
          f"per-instance {per_ms} ms; err {max(errs):.2e}", file=sys.stderr, flush=True)
    return out


# column by column (FP32), and the matrix-core path: near field FP32 or bf16
# MFMA, far field bf16 high/low split MFMA (three products per tile) in both
MRHS_MODES = {"columns_f32": None, "mfma_near_f32_far_bf16x3": "f32", "mfma_near_bf16_far_bf16x3": "bf16"}


def batch_solve_leg(F, torch, ninst, theta, rtol=1e-6, maxit=1500, sig2=1.0, pcs=("none", "block_jacobi")):
    """Solves (K~ + sigma2 I) x = b on the first ninst instances of the
    batched workload (rational quadratic, d = 3): one CG call on the forest
    plan (every instance its own CG system, all advanced by one MVM per
    iteration) with the MVM in FP64 and in FP32, against plain FP64 CG on one
    plan per instance, one instance after another. Reports the worst
    per-instance relative residual of each batched solve (against the FP64
    operator) and its speedup over the per-instance solves."""
    spec = W.WORKLOADS["batch256_rq"]
    sizes = W.instance_sizes(spec["ninst"], spec["nmin"], spec["nmax"], spec["size_seed"])[:ninst]
    X, off = W.batched_instances(sizes, spec["d"], spec["pts_seed"])
    n = X.shape[0]
    b64 = W.normal_rhs(n, 1, spec["rhs_seed"])[:, 0]
    kw = dict(lengthscale=spec["lengthscale"], alpha=spec["alpha"])
    leaf, p = 128, spec["order"]
    out = {"workload": f"batch{ninst}_rq_d3_n{n}", "instances": ninst, "n_total": n, "sigma2": sig2, "rtol": rtol,
           "maxit": maxit, "theta": theta, "p": p, "leaf": leaf}

    def cg(plan, b, pc, solve=F.fkt_cg_solve):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            x, it, rr = solve(plan, sig2, b, rtol=rtol, maxit=maxit, precond=pc)
        except F.FktError as e:
            if e.status != 5:
                raise
            x, it, rr = e.x, e.iters, e.relres
        torch.cuda.synchronize()
        return x, it, rr, time.perf_counter() - t0

    its, secs = [], 0.0
    for i in range(ninst):
        plan = F.fkt_plan(X[off[i]:off[i + 1]], spec["kernel"], leaf, p, theta=theta, **kw)
        bi = torch.as_tensor(b64[off[i]:off[i + 1]], device="cuda")
        _, it, _, sec = cg(plan, bi, "none")
        its.append(it)
        secs += sec
        plan.close()
    out["per_instance_f64_none"] = {"seconds": secs, "iterations_max": max(its), "iterations_sum": int(sum(its))}
    print(f"bench: batched solve, per-instance FP64 plain CG: {secs:.2f} s, iterations max {max(its)}",
          file=sys.stderr, flush=True)
    # true residuals of every solution against the FP64 operator
    plan64 = F.fkt_plan_batch((X, off), spec["kernel"], leaf, p, theta=theta, prec="f64", **kw)
    b = torch.as_tensor(b64, device="cuda")
    bh = b64
    for prec in ("f64", "f32"):
        plan = plan64 if prec == "f64" else F.fkt_plan_batch((X, off), spec["kernel"], leaf, p, theta=theta,
                                                               prec=prec, **kw)
        # FP32 plans: FP32 MVMs, FP64 b, CG vectors and solution (fkt_cg_solve64)
        for pc in pcs:
            x, it, rr, sec = cg(plan, b, pc, solve=F.fkt_cg_solve64)
            x = x.double()
            r = (b - F.fkt_mvm(plan64, x) - sig2 * x).cpu().numpy()
            worst = max(float(np.linalg.norm(r[off[i]:off[i + 1]]) / np.linalg.norm(bh[off[i]:off[i + 1]]))
                        for i in range(ninst))
            out[f"batched_{prec}_{pc}"] = {"seconds": sec, "iterations": it, "relres": rr,
                                           "relres_worst_instance": worst, "speedup_vs_per_instance_f64": secs / sec}
            print(f"bench: batched solve {prec} {pc}: {sec:.2f} s, {it} iterations, relres {rr:.2e}, "
                  f"worst instance {worst:.2e}", file=sys.stderr, flush=True)
        if plan is not plan64:
            plan32 = plan
    # FP32 CG with the residual replaced by the FP64 one: every instance to
    # rtol under the FP64 operator
    for pc in ("none", "block_jacobi"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, outer, rr = F.fkt_cg_solve_refined(plan64, plan32, sig2, b, rtol=rtol, maxit=maxit, precond=pc)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[f"batched_refined_{pc}"] = {"seconds": sec, "iterations_f32": it, "fp64_replacements": outer, "relres": rr,
                                        "speedup_vs_per_instance_f64": secs / sec}
        print(f"bench: batched solve refined {pc}: {sec:.2f} s, {it} FP32 iterations, {outer} FP64 replacements, "
              f"relres {rr:.2e}", file=sys.stderr, flush=True)
    plan32.close()
    plan64.close()
    return out


def mrhs_leg(F, torch, reps, theta, err_targets, modes=tuple(MRHS_MODES)):
    """Mixed precision, many RHS: 500k points of a 10-component mixture in
    d = 5, Gaussian length scale 0.2, p = 8, 32 RHS, FP32 plan: column by
    column against the matrix-core near field in FP32 and in bf16."""
    import oracle
    spec = W.WORKLOADS["gmm5_n500k_gauss32"]
    n = spec["n"]
    X = W.gaussian_mixture(n, spec["d"], spec["ncomp"], spec["std"], spec["pts_seed"])
    x64 = W.normal_rhs(n, spec["nrhs"], spec["rhs_seed"])
    x = torch.as_tensor(x64, dtype=torch.float32, device="cuda").contiguous()
    tg = W.subsample(n, err_targets, 3007) if err_targets > 0 else None
    zd = oracle.dense_mvm(X, x64, spec["kernel"], targets=tg, lengthscale=spec["lengthscale"]) if tg is not None \
        else None
    out = {"workload": f"gmm5_n{n}_gauss_32rhs", "n": n, "d": 5, "p": spec["order"], "theta": theta, "nrhs": 32}
    for name in modes:
        mr = MRHS_MODES[name]
        plan = F.fkt_plan(X, spec["kernel"], 256, spec["order"], theta=theta, prec="f32", mrhs=mr,
                          lengthscale=spec["lengthscale"])
        y = F.fkt_mvm(plan, x)
        ms = _sync_time(torch, lambda: F.fkt_mvm(plan, x, y), reps)
        err = None
        if zd is not None:
            z = y.double().cpu().numpy()[tg]
            err = float(np.linalg.norm(z - zd) / np.linalg.norm(zd))
        out[name] = {"ms_per_mvm_32rhs": ms, "mpoints_rhs_per_s": n * 32 / ms / 1e3, "rel_err_vs_dense_fp64": err}
        print(f"bench: mrhs {name}: {ms:.1f} ms per 32-column MVM, err {err}", file=sys.stderr, flush=True)
        plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel", default="matern32", choices=sorted(KERNEL_KW))
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"])
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--leaf", type=int, default=256)
    ap.add_argument("--order", type=int, default=6)
    ap.add_argument("--err-targets", type=int, default=10000,
                    help="targets sampled (seed 3002) for the error against the dense FP64 sum (the headline "
                         "line; the secondary legs use at most 1000); 0 skips")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="time budget of the CPU-oracle baseline sample; 0 skips")
    ap.add_argument("--no-variants", action="store_true", help="headline workload only")
    ap.add_argument("--serial", action="store_true",
                    help="run near and far fields one after the other on one stream (default: concurrently)")
    ap.add_argument("--gp-n", type=int, default=200_000, help="points of the GP solves; 0 skips them")
    ap.add_argument("--gp-theta", type=float, default=0.3)
    ap.add_argument("--gp-order", type=int, default=8)
    ap.add_argument("--gp-rank", type=int, default=2048, help="landmarks of the two-level preconditioner")
    ap.add_argument("--gp-maxit", type=int, default=10000)
    ap.add_argument("--gp-train-steps", type=int, default=10)
    ap.add_argument("--gp-fp64-none", action="store_true", help="also plain FP64 CG without a preconditioner")
    ap.add_argument("--batch-theta", type=float, default=0.3)
    ap.add_argument("--batch-leaf", type=int, default=0, help="0: the library's autotuner picks it")
    ap.add_argument("--batch-no-per-instance", action="store_true")
    ap.add_argument("--mrhs-theta", type=float, default=0.4)
    ap.add_argument("--mrhs-modes", default=",".join(MRHS_MODES))
    ap.add_argument("--leg", default="all", choices=["all", "many_rhs", "batched", "gp", "gp_mvm", "nsweep",
                                                     "batched_solve"],
                    help="run one secondary leg alone and print its JSON (the default runs the headline line)")
    a = ap.parse_args()

    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}): the library has no multi-GPU path "
              "(the MVM would shard by target blocks).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2106_04487_amd as F

    if a.leg != "all":
        if a.leg == "many_rhs":
            out = mrhs_leg(F, torch, a.steps, a.mrhs_theta, min(a.err_targets, 1000), tuple(a.mrhs_modes.split(",")))
        elif a.leg == "batched":
            out = batch_leg(F, torch, a.steps, a.batch_theta, max(a.err_targets // 10, 20), a.batch_leaf,
                            not a.batch_no_per_instance)
        elif a.leg == "batched_solve":
            out = batch_solve_leg(F, torch, 32, a.batch_theta)
        elif a.leg == "nsweep":
            out = nsweep_leg(F, torch, a.steps, a.err_targets, a.kernel, a.prec)
        elif a.leg == "gp_mvm":
            out = gp_mvm_leg(F, torch, a.steps, a.gp_theta, a.gp_order)
        else:
            out = gp_solve(F, torch, a.gp_n, a.gp_theta, a.gp_order, a.gp_rank, 1e-6, a.gp_maxit, a.gp_train_steps,
                           a.gp_fp64_none)
        print(json.dumps(out))
        return

    X = W.uniform_cube(a.n, 3, 1002)
    x64 = W.normal_rhs(a.n, 1, 2002)[:, 0]
    theta = a.theta if a.theta is not None else DEFAULT_THETA[a.kernel]
    head = run_variant(F, torch, X, x64, a.kernel, a.prec, theta, a.leaf, a.order, a.steps, a.warmup,
                       a.err_targets, overlap=not a.serial)

    # roofline of the dominant kernel, the near field (vector-ALU bound), and
    # of the far-field evaluation beside it; launch times from the HIP events
    # bench records around each stage on the stream it runs on
    near_ms = head["stages_ms"]["near"]
    pairs = head["plan"]["near_pairs"]
    achieved = pairs * NEAR_FLOPS_PER_PAIR / (near_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_near", "achieved": achieved, "peak": PEAK_TFLOPS[a.prec],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[a.prec],
                "traffic": NEAR_TRAFFIC_BYTES.get((a.kernel, a.prec)) if a.n == 1_000_000 else None,
                "units": "near-field pair evaluations", "units_per_launch": pairs,
                "flops_per_unit": NEAR_FLOPS_PER_PAIR, "avg_launch_ms": near_ms}
    m2t = None
    if (3, a.order) in M2T_FLOPS_PER_PAIR:
        m2t_ms = head["stages_ms"]["m2t"]
        fpairs = head["plan"]["far_pairs"]
        ach = fpairs * M2T_FLOPS_PER_PAIR[(3, a.order)] / (m2t_ms * 1e-3) / 1e12
        m2t = {"bound": "alu", "kernel": "k_m2t_nodes", "achieved": ach, "peak": PEAK_TFLOPS[a.prec],
               "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS[a.prec],
               "traffic": M2T_TRAFFIC_BYTES.get((a.kernel, a.prec)) if a.n == 1_000_000 else None,
               "units": "far (target, node) expansions",
               "units_per_launch": fpairs, "flops_per_unit": M2T_FLOPS_PER_PAIR[(3, a.order)],
               "avg_launch_ms": m2t_ms}

    variants = []
    if not a.no_variants:
        # the Laplace kernel with and without radial compression (Appendix A.4)
        for kern, prec, comp in (("laplace", "f64", False), ("laplace", "f64", True), ("matern32", "f32", False),
                                 ("laplace", "f32", False), ("laplace", "f32", True)):
            if (kern, prec, comp) == (a.kernel, a.prec, False):
                continue
            v = run_variant(F, torch, X, x64, kern, prec, DEFAULT_THETA[kern], a.leaf, a.order, max(5, a.steps // 2),
                            1, min(a.err_targets, 1000), overlap=not a.serial, compress=comp)
            v.pop("plan")
            variants.append(v)

    gp = None
    if a.gp_n > 0 and not a.no_variants:
        gp = gp_solve(F, torch, a.gp_n, a.gp_theta, a.gp_order, a.gp_rank, 1e-6, a.gp_maxit, a.gp_train_steps,
                      a.gp_fp64_none)

    batch = mrhs = bsolve = None
    if not a.no_variants:
        batch = batch_leg(F, torch, 3, a.batch_theta, min(200, max(a.err_targets // 10, 50)), a.batch_leaf,
                          not a.batch_no_per_instance)
        bsolve = batch_solve_leg(F, torch, 32, a.batch_theta, pcs=("none",))
        mrhs = mrhs_leg(F, torch, 2, a.mrhs_theta, min(a.err_targets, 500), tuple(a.mrhs_modes.split(",")))

    cpu = None
    if a.cpu_seconds > 0:
        # the factorised CPU oracle (Cartesian moments of every node, then the
        # far and near field of each sampled target) at the full N, on all
        # host cores: rows in chunks until the time budget is spent
        import oracle
        okind, okw = ORACLE_KIND[a.kernel]
        T = oracle.Tree(X, a.leaf)
        tg = W.subsample(a.n, a.n, 3003)
        t0 = time.perf_counter()
        oracle.fkt_cart(T, x64, okind, theta, a.order, targets=tg[:0], **okw)  # moments only
        mom_s = time.perf_counter() - t0
        done, chunk = 0, 4096
        while done < len(tg) and time.perf_counter() - t0 < a.cpu_seconds:
            oracle.fkt_cart(T, x64, okind, theta, a.order, targets=tg[done:done + chunk], **okw)
            done += chunk
        el = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        # whole-MVM rate: every chunk recomputes the moments, so the rows
        # take el - (chunks + 1) mom_s; scale them to all N rows, add one
        row_s = max(el - (done // chunk + 1) * mom_s, 1e-9) / done
        mvm_s = mom_s + row_s * a.n
        cpu = {"value": a.n / mvm_s / 1e6, "unit": "Mpoints/s", "cores": threads, "kind": "oracle",
               "sample": f"factorised CPU FKT (Cartesian moments) at N = {a.n}: moments {mom_s:.2f} s, "
                         f"{done} sampled output rows in {el - (done // chunk + 1) * mom_s:.1f} s on {threads} "
                         f"threads; whole MVM {mvm_s:.1f} s by extrapolation"}

    info = head["plan"]
    out = {
        "metric": "FKT MVM Mpoints/s at rel err <=1e-5",
        "value": head["mpoints_per_s"], "unit": "Mpoints/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": a.prec, "data": "synthetic",
        "config": {"workload": f"uniform_cube3_n{a.n}_{a.kernel}", "n": a.n, "d": 3, "kernel": a.kernel,
                   **KERNEL_KW[a.kernel], "leaf": a.leaf, "p": a.order, "theta": theta, "nrhs": 1},
        "rel_err_vs_dense": head["rel_err_vs_dense"],
        "stages_ms": head["stages_ms"],
        "plan": {k: info[k] for k in ("nnodes", "nleaves", "nblocks", "near_pairs", "near_lane_pairs",
                                      "far_pairs", "far_lane_pairs", "plan_seconds")},
        "roofline": roofline,
        "roofline_m2t": m2t,
        "cpu_baseline": cpu,
        "variants": variants,
        "gp_solve": gp,
        "batched_instances": batch,
        "batched_solve": bsolve,
        "many_rhs": mrhs,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
