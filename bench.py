"""Benchmark: time to a 1e-8 relative residual of flexibly enlarged CG on one MI355X.

One step = one whole FP64 solve (every step of the hot path: split, SpMM, CGS2 Gram and
update, Pre-CholQR t x t factors, fused block update, flexible halving of t) of the 3D
anisotropic workload aniso3d128: 7-point finite differences on 128^3 cells
(n = 2097152), coefficients (1, 50, 0.01) along x/y/z, Dirichlet walls, t = 32 from
2 x 2 x 8 boxes, t halved once when |rho_k - rho_{k-1}| / rho_0 < 1e-5, x0 = 0,
b ~ U(-1, 1).  Inputs are resident in HBM before the timed region starts.

The 2D jumping-coefficient workload jump2d512 is not the timed step: without a
preconditioner its stored basis outgrows HBM long before 1e-8 (4000 iterations,
235 GB of stored blocks, residual still 0.45).  It is reported beside the step with the
block-Jacobi preconditioners of Section 5.3 of the paper: IC(0) on its 32 subdomains, and
the exact Cholesky of 64 blocks of 64 x 64 cells (the paper's best) with flexibly
SRE-CG2 and flexibly MSDO-CG.

Reported:
  value          seconds per FP64 solve of aniso3d128 (higher_is_better false)
  fp32_refined   the same solve with FP32 SpMM / Gram / block updates, FP64 t x t steps,
                 FP64 true residual and outer refinement to the same true residual
  roofline       the kernel class with the most time in the FP64 step: algorithmic bytes
                 per launch / HIP-event launch time, against 8 TB/s HBM
  jump2d512_bj   jump2d512 with block-Jacobi IC(0), FP64 and FP32-refined
  jump2d512_chol64  jump2d512 with block-Jacobi Cholesky on 64 blocks, FP64, flexibly
                 SRE-CG2 and flexibly MSDO-CG, and the restarted variants of SRE-CG2 (one
                 restart at restartTol 1e-5; restart at the halving): iterations, stored
                 vectors and the largest restart cycle
  learn2d256_learned  ECG with the trained G G^T vs its Jacobi start, block-Jacobi IC(0) and
                 no preconditioner on held-out 256x256 jumping-coefficient operators
  cpu_baseline   the FP64 oracle on the host (bounded sample, extrapolated; see 'sample')

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--t T]
                       [--precond none|bj_ic0|chol64] [--forms fp64,fp32] [--no-cpu] [--no-side]
                       [--kmax N] [--copy-calibration]
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

METRIC = "ECG time-to-1e-8 residual + SpMM HBM GB/s; FP32/learned vs FP64 plain"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def solve_once(ecg, op, P, b, x, opts, ws):
    x.zero_()
    rep, _ = ecg.solve(op, P, b, x, opts, workspace=ws)
    return rep


def run_form(args, torch, ecg, prob, op, P, b, form, M=None, steps=None, warmup=None, tag="", **extra):
    dev = b.device
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    common = dict(tol=prob.tol, kmax=args.kmax, reduce=prob.reduce, switch_tol=prob.switch_tol,
                  t_min=prob.t_min, M=M)
    common.update(extra)
    if form == "fp64":
        kw = dict(common, precision=ecg.FP64)
        w = 8
    else:
        kw = dict(common, precision=ecg.FP32_REFINED, inner_tol=args.inner_tol, replace_every=25,
                  max_outer=30)
        w = 4
    # stored blocks: as many columns as fit next to everything else
    free, _ = torch.cuda.mem_get_info()
    col = prob.n * w
    budget = max(prob.t * col, int(free * 0.93) - 4 * prob.t * col - (3 << 30))
    if args.q_cols:
        budget = args.q_cols * col
    opts = ecg.options(q_budget_bytes=budget, **kw)
    need = ecg.workspace_size(op, P, opts)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    x = torch.zeros_like(b)
    # priming (not a step): a 3-iteration solve loads every kernel of this path once
    prime = ecg.options(q_budget_bytes=budget, **dict(kw, kmax=4))
    solve_once(ecg, op, P, b, x, prime, ws)
    ecg.progress(args.progress)
    for i in range(warmup):
        rep = solve_once(ecg, op, P, b, x, opts, ws)
        log(f"[{tag}{form}] warmup {i}: iters={rep['iters']} {rep['seconds']:.3f}s relres_true={rep['relres_true']:.2e}")
    ecg.stats_read(reset=True)
    ecg.stats_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(steps):
        reps.append(solve_once(ecg, op, P, b, x, opts, ws))
        log(f"[{tag}{form}] step {i}: iters={reps[-1]['iters']} {reps[-1]['seconds']:.3f}s")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ecg.stats_enable(False)
    ecg.progress(0)
    stats = ecg.stats_read(reset=True)
    rep = reps[-1]
    log(f"[{tag}{form}] timed: {dt:.3f}s/solve iters={rep['iters']} switch={rep['switch_iters']} "
        f"mem={rep['vectors_stored']} dropped={rep['blocks_dropped']} relres_true={rep['relres_true']:.2e} "
        f"status={rep['status']}")
    xs = x.clone()
    del ws
    torch.cuda.empty_cache()
    return {"seconds": dt, "report": rep, "stats": stats, "x": xs, "q_cols": budget // col}


def roofline_from_stats(stats, steps):
    """The kernel class with the largest event time among the streaming classes."""
    streaming = ["cgs2_gram", "cgs2_update", "spmm", "final_update", "small_gram", "times_small"]
    best = max(streaming, key=lambda k: stats[k]["ms"])
    s = stats[best]
    if s["count"] == 0 or s["ms"] <= 0:
        return None, best
    per_launch_bytes = s["bytes"] / s["count"]
    per_launch_ms = s["ms"] / s["count"]
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    return {"kernel": best, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_us": round(per_launch_ms * 1e3, 2), "launches_per_step": s["count"] / steps,
            "algorithmic_bytes_per_launch": per_launch_bytes}, best


def profiled_traffic(workload, t, kernel):
    """Calibrated HBM bytes per launch from the committed rocprofv3 summary of this
    workload, or None when the kernels changed after the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"cgs2_{workload}_t{t}_fp64.md")
    if not os.path.exists(path):
        return None
    src = os.path.join(ROOT, "paper_2305_19013_amd", "csrc", "ecg_kernels.hip")
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    sha, val = None, None
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and parts[0] == "kernels_sha256_16":
            sha = parts[1]
        if len(parts) == 3 and parts[0] == "traffic_bytes_per_launch" and parts[1] == kernel:
            val = float(parts[2])
    return val if (sha == cur and val is not None) else None


def kernel_table(stats, steps):
    out = {}
    for k, s in stats.items():
        if s["count"] == 0:
            continue
        gbs = s["bytes"] / (s["ms"] * 1e-3) / 1e9 if s["ms"] > 0 else 0.0
        out[k] = {"launches_per_step": s["count"] / steps, "ms_per_step": round(s["ms"] / steps, 3),
                  "GB/s": round(gbs, 1), "TFLOP/s": round(s["flops"] / (s["ms"] * 1e-3) / 1e12, 3) if s["ms"] > 0 else 0}
    return out


class _StampedA:
    """A @ X for the oracle, with a wall-clock stamp taken before every product: the
    products fall at fixed points of each iteration, so the stamps split a run into
    per-iteration times without touching the oracle."""

    def __init__(self, A):
        self.A, self.shape, self.stamps = A, A.shape, []

    def __matmul__(self, X):
        self.stamps.append(time.perf_counter())
        return self.A @ X


def cpu_baseline(prob, widths_gpu, it_gpu, switch_gpu, kmax=8):
    """Bounded sample of the FP64 oracle on the same workload, extrapolated.

    The oracle runs the first kmax iterations of the same solve.  Iteration 1 makes two
    products with A, every later one four (two CGS2 passes, the A-step Gram, the fresh
    A W); the stamps of those products split each iteration into segments.  The cost per
    stored column b comes from the segments that carry it: the first CGS2 pass (product,
    Q^T Y, Q G; the second pass is the same work) and the stretch from the fresh product
    to the next iteration (which stacks Q), each fitted by least squares against m_k; it is
    b = 2 b_pass + b_stack.  The rest of an iteration is the constant a, the mean of
    T_k - b m_k.  T = a + b m_k is then summed over the GPU run's iteration history (same
    widths and switch) to estimate a whole solve.
    """
    import threadpoolctl

    from oracle import ecg as ora

    A = _StampedA(prob.A.to_scipy())
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] or [1])
    t0 = time.perf_counter()
    r = ora.flexible_sre_cg2(A, prob.b, prob.part, prob.t, tol=prob.tol, kmax=kmax + 1, reduce=prob.reduce,
                             switch_tol=prob.switch_tol, t_min=prob.t_min)
    t_end = time.perf_counter()
    log(f"[cpu] oracle first {r.it} iterations: {t_end - t0:.2f}s")
    st = A.stamps
    first = [1] + [3 + 4 * (k - 2) for k in range(2, r.it + 1)]  # stamp index opening iteration k
    assert len(st) == 1 + 2 + 4 * (r.it - 1), (len(st), r.it)
    opens = [st[i] for i in first] + [t_end]
    T = np.diff(opens)  # T[k-1] = time of iteration k
    cs = np.concatenate([[0], np.cumsum(r.widths)])
    ks = np.arange(2, r.it)  # complete iterations with a non-empty basis
    mk = cs[ks - 1].astype(float)
    stn = np.array(st + [t_end])
    i1 = np.array([first[k - 1] for k in ks])
    seg_pass = stn[i1 + 1] - stn[i1]  # CGS2 pass 1
    seg_stack = stn[i1 + 4] - stn[i1 + 3]  # fresh product .. next iteration (stacks Q)
    b_pass = max(np.polyfit(mk, seg_pass, 1)[0], 0.0)
    b_stack = max(np.polyfit(mk, seg_stack, 1)[0], 0.0)
    bcoef = 2.0 * b_pass + b_stack
    a = max(float(np.mean(T[ks - 1] - bcoef * mk)), 0.0)
    csg = np.concatenate([[0], np.cumsum(widths_gpu)])
    est = float(T[0] + sum(a + bcoef * csg[k - 1] for k in range(2, it_gpu + 1)))
    return {"value": round(est, 2), "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": (f"FP64 oracle (NumPy/SciPy, OpenBLAS {threads} threads) timed on the first {r.it} iterations "
                       f"of the same solve ({t_end - t0:.1f}s), per iteration from stamps taken at its products with "
                       f"A; T_k = a + b*m_k with b = 2*(slope of a CGS2 pass) + (slope of the Q stacking) fitted "
                       f"over iterations 2..{r.it - 1} (a={a:.3f}s, b={bcoef:.2e}s per stored column, m_k up to "
                       f"{int(mk.max())}), summed over the GPU run's {it_gpu} iterations and widths"),
            "measured_sample_s": round(t_end - t0, 2)}


def learned_section(args, torch, dev):
    """learn2d256 (256x256, log10 k ~ U(-3,3) on 16x16-cell blocks, t = 16): ECG with the
    trained G G^T against its untrained Jacobi start, block-Jacobi IC(0) and no
    preconditioner, on held-out operator seeds 2000.. (FP64, tol 1e-8).  The parameters were
    trained on the GPU by `python -m paper_2305_19013_amd.learned` and are read from
    paper_2305_19013_amd/trained/learn2d256.json."""
    import workloads as W
    from paper_2305_19013_amd import learned as LN

    path = os.path.join(ROOT, "paper_2305_19013_amd", "trained", "learn2d256.json")
    if not os.path.exists(path):
        return None
    meta = json.load(open(path))
    p0, _ = LN.family(0)
    nx, ny = p0.grid
    model = LN.LearnedFactor(nx, ny, np.asarray(meta["params"]), dev)
    seeds = list(range(2000, 2000 + args.learned_ops))
    kinds = ("learned", "jacobi", "bj_ic0")
    LN.evaluate(model, seeds[:1], dev, 1, kinds, params_jacobi=W.init_params(meta["init_seed"]))  # priming
    res = LN.evaluate(model, seeds, dev, 1, kinds, params_jacobi=W.init_params(meta["init_seed"]))
    res.update(LN.evaluate(model, seeds[:1], dev, 1, ("plain",), kmax=6000))
    out = {"train_ops": meta["train_ops"], "epochs": meta["epochs"], "best_epoch": meta.get("best_epoch"),
           "heldout_ops": len(seeds)}
    for k, v in res.items():
        out[k] = {"mean_iters": float(np.mean([r["iters"] for r in v])),
                  "mean_seconds": round(float(np.mean([r["seconds"] for r in v])), 4),
                  "mean_setup_seconds": round(float(np.mean([r["setup_s"] for r in v])), 4),
                  "max_relres_true": float(np.max([r["relres_true"] for r in v])),
                  "all_converged": all(r["status"] == "ok" for r in v), "ops": len(v)}
        log(f"[learn2d256 {k}] {out[k]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="aniso3d128")
    ap.add_argument("--t", type=int, default=32)
    ap.add_argument("--forms", default="fp64,fp32")
    ap.add_argument("--kmax", type=int, default=20000)
    ap.add_argument("--inner-tol", type=float, default=1e-4)
    ap.add_argument("--q-cols", type=int, default=0)
    ap.add_argument("--progress", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-ops", type=int, default=8)
    ap.add_argument("--precond", default="none", choices=("none", "bj_ic0", "chol64"),
                    help="preconditioner of the main solve (block-Jacobi IC(0) on the subdomains, or "
                         "exact Cholesky of 64 blocks of a 2D grid)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device-to-device before the solves (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2305_19013_amd import ecg

    ecg.lib()
    dev = torch.device("cuda:0")
    prob = W.config(args.workload, t=args.t) if args.workload == "aniso3d128" else W.config(args.workload)
    log(f"workload {args.workload}: n={prob.n} nnz={prob.A.nnz} t={prob.t}")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    op = ecg.Operator.from_csr(prob.A)
    P = ecg.Partition(prob.part, prob.t)
    b = torch.from_numpy(prob.b).to(dev)
    forms = [f for f in args.forms.split(",") if f]
    M = None
    if args.precond == "bj_ic0":
        M = ecg.Precond.bj_ic0(op, P)
    elif args.precond == "chol64":
        M = ecg.Precond.bj(op, W.box_partition(prob.grid, (8, 8)), ecg.BJ_CHOL)
    results = {}
    for f in forms:
        results[f] = run_form(args, torch, ecg, prob, op, P, b, f, M=M)
    main_form = "fp64" if "fp64" in results else forms[0]
    R = results[main_form]
    rep = R["report"]
    roof, best = roofline_from_stats(R["stats"], args.steps)
    if roof is not None and main_form == "fp64":
        roof["traffic"] = profiled_traffic(args.workload, prob.t, best)
    out = {
        "metric": METRIC,
        "value": round(R["seconds"], 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(R["seconds"] * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "precond": args.precond, "n": prob.n, "nnz": prob.A.nnz, "t": prob.t,
                   "reduce": {0: "none", 1: "halve once", 2: "halve repeatedly"}[prob.reduce],
                   "switch_tol": prob.switch_tol, "tol": prob.tol, "q_cols": R["q_cols"]},
        "solve": {"iters": rep["iters"], "switch_iters": rep["switch_iters"], "t_final": rep["t_final"],
                  "vectors_stored": rep["vectors_stored"], "blocks_dropped": rep["blocks_dropped"],
                  "relres_true": rep["relres_true"], "status": rep["status"]},
        "spmm_GBs": kernel_table(R["stats"], args.steps).get("spmm", {}).get("GB/s"),
        "roofline": roof,
        "kernels": kernel_table(R["stats"], args.steps),
    }
    for f, Rf in results.items():
        if f == main_form:
            continue
        rf = Rf["report"]
        err = None
        if "fp64" in results:
            xa = results["fp64"]["x"]
            err = float(torch.linalg.norm(Rf["x"] - xa) / torch.linalg.norm(xa))
        out[f + "_refined" if f == "fp32" else f] = {
            "seconds": round(Rf["seconds"], 4), "iters": rf["iters"], "outer_iters": rf["outer_iters"],
            "relres_true": rf["relres_true"], "status": rf["status"], "rel_err_vs_fp64": err,
            "speedup_vs_fp64": round(R["seconds"] / Rf["seconds"], 3) if main_form == "fp64" else None,
            "roofline": roofline_from_stats(Rf["stats"], args.steps)[0],
        }
    if not args.no_side and args.workload != "jump2d512":
        # side measurement: jump2d512 with block-Jacobi IC(0) on its 32 subdomains
        pj = W.config("jump2d512")
        opj = ecg.Operator.from_csr(pj.A)
        Pj = ecg.Partition(pj.part, pj.t)
        Mj = ecg.Precond.bj_ic0(opj, Pj)
        bj = torch.from_numpy(pj.b).to(dev)
        side = {"workload": "jump2d512", "precond": "block-Jacobi IC(0), 32 subdomains", "n": pj.n, "t": pj.t}
        for f in forms:
            Rj = run_form(args, torch, ecg, pj, opj, Pj, bj, f, M=Mj, steps=3, warmup=1, tag="jump2d512-bj ")
            rj = Rj["report"]
            side[f] = {"seconds": round(Rj["seconds"], 4), "iters": rj["iters"], "switch_iters": rj["switch_iters"],
                       "outer_iters": rj["outer_iters"], "relres_true": rj["relres_true"], "status": rj["status"]}
        out["jump2d512_bj"] = side
        # the paper's best preconditioner (Section 5.3): exact Cholesky of 64 blocks of
        # 64 x 64 cells, the same for every t; flexibly SRE-CG2 and flexibly MSDO-CG, FP64
        blocks = W.box_partition(pj.grid, (8, 8))
        t0 = time.perf_counter()
        Mc = ecg.Precond.bj(opj, blocks, ecg.BJ_CHOL)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        chol = {"workload": "jump2d512", "precond": "block-Jacobi Cholesky, 64 blocks", "n": pj.n, "t": pj.t,
                "setup_seconds": round(setup, 4)}
        # the memory-bounded alternatives of Section 3 beside the switch rule: one restart at
        # restartTol = 1e-5 with the same t, and the flexible run that also restarts at its halving
        runs = (("sre_cg2", dict(variant=ecg.SRE_CG2)), ("msdo_cg", dict(variant=ecg.MSDO_CG)),
                ("sre_cg2_restarted", dict(reduce=ecg.REDUCE_NONE, restart=ecg.RESTART_TOL, restart_tol=1e-5,
                                           max_restarts=1)),
                ("sre_cg2_restarted_flexible", dict(restart_at_switch=1)))
        for name, extra in runs:
            Rj = run_form(args, torch, ecg, pj, opj, Pj, bj, "fp64", M=Mc, steps=3, warmup=1,
                          tag=f"jump2d512-chol64-{name} ", **extra)
            rj = Rj["report"]
            chol[name] = {"seconds": round(Rj["seconds"], 4), "iters": rj["iters"],
                          "switch_iters": rj["switch_iters"], "restart_iters": rj["restart_iters"],
                          "vectors_stored": rj["vectors_stored"], "vectors_peak": rj["vectors_peak"],
                          "relres_true": rj["relres_true"], "status": rj["status"]}
        out["jump2d512_chol64"] = chol
    if not args.no_side and not args.no_learned:
        out["learn2d256_learned"] = learned_section(args, torch, dev)
    if not args.no_cpu:
        # widths history of the GPU run is reconstructed from its report
        it = rep["iters"]
        sw = rep["switch_iters"]
        widths = [prob.t if (not sw or k < sw[0]) else prob.t // 2 for k in range(1, it + 1)]
        out["cpu_baseline"] = cpu_baseline(prob, widths, it, sw)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
