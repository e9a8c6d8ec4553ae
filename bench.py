"""Benchmark: time to a 1e-8 relative residual of flexibly enlarged CG on one MI355X.

One step = one whole FP64 solve (every step of the hot path: split, SpMM, CGS2 Gram and
update, Pre-CholQR t x t factors, fused block update, flexible halving of t) of the 3D
anisotropic workload aniso3d128: 7-point finite differences on 128^3 cells
(n = 2097152), coefficients (1, 50, 0.01) along x/y/z, Dirichlet walls, t = 32 from
2 x 2 x 8 boxes, t halved once when |rho_k - rho_{k-1}| / rho_0 < 1e-5, x0 = 0,
b ~ U(-1, 1).  Inputs are resident in HBM before the timed region starts.

Wall-clock budget.  A step is a ~1 minute solve, so --steps and --warmup are maxima: the
run keeps to one budget (--budget-s, default 450 s from process start).  After a priming
solve of 3 iterations (loads every kernel) the first full FP64 solve is the warm-up; it
runs with per-launch HIP-event timing on (ecg_stats_enable) and gives the kernel table and
the roofline.  The timed steps run with that timing off; as many of them as the budget
leaves room for after reserving the other sections, at least one.  The JSON line carries
the steps and warm-up solves actually run and is printed even if a later section fails.

Sections, in order (a section that no longer fits the budget is recorded as skipped):
  value          seconds per FP64 solve of aniso3d128 (higher_is_better false)
  fp32_refined   the same solve with FP32 SpMM / Gram / block updates, FP64 t x t steps,
                 FP64 true residual and outer refinement to the same true residual
  roofline       the kernel class with the most time in the instrumented FP64 solve:
                 algorithmic bytes per launch / HIP-event launch time, against 8 TB/s HBM
  cpu_baseline   the FP64 oracle on the host: the first iterations of the same solve plus
                 its CGS2 step timed directly against a stored basis of up to thousands of
                 columns, summed over the GPU run's iteration history (see 'sample')
  poisson64      64x64 Poisson, t = 8: GPU FP64 and FP32-refined solves against the whole
                 oracle solve timed on the host; error of both against the oracle's x
  learn2d256_learned  ECG with the trained G G^T vs its Jacobi start, block-Jacobi IC(0) and
                 no preconditioner on held-out 256x256 jumping-coefficient operators
  jump2d512_bj   jump2d512 with block-Jacobi IC(0), FP64 and FP32-refined
  jump2d512_chol64  jump2d512 with block-Jacobi Cholesky on 64 blocks: flexibly SRE-CG2,
                 flexibly MSDO-CG, and two restarted variants of SRE-CG2

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget-s S] [--workload NAME]
                       [--t T] [--precond none|bj_ic0|chol64] [--forms fp64,fp32] [--no-cpu]
                       [--no-side] [--kmax N] [--copy-calibration] [--oracle-full]
       python bench.py --explore --workload NAME [--t T] [--precond ...] [--forms ...] [--kmax N]
                       (one solve per form, no timed series: the long configurations)
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
import traceback

T_START = time.time()

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ECG time-to-1e-8 residual + SpMM HBM GB/s; FP32/learned vs FP64 plain"
HBM_PEAK_GBS = 8000.0
# host-side estimates (seconds) of the sections after the headline, used to size the number
# of timed steps; refined by what the run measures
EST = {"fp32": 30.0, "cpu": 35.0, "poisson64": 12.0, "learned": 50.0, "jump2d512": 30.0}


def log(msg):
    print(f"[{time.time() - T_START:7.1f}s] {msg}", file=sys.stderr, flush=True)


class Budget:
    def __init__(self, total):
        self.total = total

    def left(self):
        return self.total - (time.time() - T_START)


def solve_once(ecg, op, P, b, x, opts, ws):
    x.zero_()
    rep, _ = ecg.solve(op, P, b, x, opts, workspace=ws)
    return rep


def form_options(args, ecg, prob, form, M=None, **extra):
    common = dict(tol=prob.tol, kmax=args.kmax, reduce=prob.reduce, switch_tol=prob.switch_tol,
                  t_min=prob.t_min, M=M)
    common.update(extra)
    if form == "fp64":
        return dict(common, precision=ecg.FP64), 8
    itol = args.inner_tol if args.inner_tol is not None else prob.fp32_inner_tol
    return dict(common, precision=ecg.FP32_REFINED, inner_tol=itol, replace_every=25, max_outer=30), 4


def run_form(args, torch, ecg, prob, op, P, b, form, M=None, steps=1, warmup=0, tag="", instrument=False,
             fit=None, **extra):
    """Priming solve, `warmup` untimed solves (the first instrumented when `instrument`), then
    timed solves.  fit(est_seconds) -> number of timed solves that fit (None: `steps`)."""
    dev = b.device
    kw, w = form_options(args, ecg, prob, form, M, **extra)
    free, _ = torch.cuda.mem_get_info()
    col = prob.n * w
    qbytes = max(prob.t * col, int(free * 0.93) - 4 * prob.t * col - (3 << 30))
    if args.q_cols:
        qbytes = args.q_cols * col
    opts = ecg.options(q_budget_bytes=qbytes, **kw)
    need = ecg.workspace_size(op, P, opts)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    x = torch.zeros_like(b)
    # priming (not a step): a 3-iteration solve loads every kernel of this path once
    solve_once(ecg, op, P, b, x, ecg.options(q_budget_bytes=qbytes, **dict(kw, kmax=4)), ws)
    ecg.progress(args.progress)
    stats, est, warm_times, inst_s = None, None, [], None
    for i in range(warmup):
        if instrument and i == 0:
            ecg.stats_read(reset=True)
            ecg.stats_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = solve_once(ecg, op, P, b, x, opts, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if instrument and i == 0:
            ecg.stats_enable(False)
            stats = ecg.stats_read(reset=True)
            inst_s = dt
        warm_times.append(dt)
        est = dt
        log(f"[{tag}{form}] warmup {i}{' (instrumented)' if instrument and i == 0 else ''}: iters={rep['iters']} "
            f"{dt:.3f}s relres_true={rep['relres_true']:.2e}")
        if fit is not None and i + 1 < warmup and fit(est) < 2:
            break  # another warm-up would leave no room for the timed steps
    k = steps if (fit is None or est is None) else max(1, min(steps, fit(est)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(k):
        reps.append(solve_once(ecg, op, P, b, x, opts, ws))
        log(f"[{tag}{form}] step {i}: iters={reps[-1]['iters']} {reps[-1]['seconds']:.3f}s")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / k
    ecg.progress(0)
    rep = reps[-1]
    log(f"[{tag}{form}] timed: {dt:.3f}s/solve over {k} iters={rep['iters']} switch={rep['switch_iters']} "
        f"mem={rep['vectors_stored']} dropped={rep['blocks_dropped']} relres_true={rep['relres_true']:.2e} "
        f"status={rep['status']}")
    xs = x.clone()
    del ws
    torch.cuda.empty_cache()
    return {"seconds": dt, "steps": k, "warmup": len(warm_times), "warmup_seconds": warm_times,
            "instrumented_seconds": inst_s, "report": rep, "stats": stats, "x": xs, "q_cols": qbytes // col,
            "step_seconds": [r["seconds"] for r in reps]}


def roofline_from_stats(stats):
    """The kernel class with the largest event time among the streaming classes."""
    if not stats:
        return None, None
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
            "avg_launch_us": round(per_launch_ms * 1e3, 2), "launches_per_solve": s["count"],
            "algorithmic_bytes_per_launch": per_launch_bytes,
            "timing": "HIP events on the solve's stream, instrumented warm-up solve of the same workload"}, best


def profiled_traffic(workload, t, kernel):
    """Calibrated HBM bytes per launch from the committed rocprofv3 summary of this
    workload, or None when the kernel source changed after the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"cgs2_{workload}_t{t}_fp64.md")
    if not os.path.exists(path):
        return None
    sha, val, src_name = None, None, "ecg_kernels.hip"
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and parts[0] == "kernel_source":
            src_name = parts[1]
        if len(parts) == 2 and parts[0] == "kernels_sha256_16":
            sha = parts[1]
        if len(parts) == 3 and parts[0] == "traffic_bytes_per_launch" and parts[1] == kernel:
            val = float(parts[2])
    src = os.path.join(ROOT, "paper_2305_19013_amd", "csrc", src_name)
    if not os.path.exists(src):
        return None
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return val if (sha == cur and val is not None) else None


def kernel_table(stats):
    out = {}
    for k, s in (stats or {}).items():
        if s["count"] == 0:
            continue
        gbs = s["bytes"] / (s["ms"] * 1e-3) / 1e9 if s["ms"] > 0 else 0.0
        out[k] = {"launches": s["count"], "ms": round(s["ms"], 3), "GB/s": round(gbs, 1),
                  "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                  "TFLOP/s": round(s["flops"] / (s["ms"] * 1e-3) / 1e12, 3) if s["ms"] > 0 else 0}
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


def _blas_threads():
    import threadpoolctl

    info = threadpoolctl.threadpool_info()
    return max([i.get("num_threads", 1) for i in info] or [1]), ",".join(
        sorted({f"{i.get('internal_api')}" for i in info}))


def cpu_baseline(prob, widths_gpu, kmax=6, m_probe=None, mem_fraction=0.3):
    """The FP64 oracle on the host for the same workload, from two bounded measurements.

    (1) The oracle's own solve, first kmax-1 iterations, split into iterations by stamps at
    its products with A (two products in iteration 1, four in every later one).
    (2) The oracle's CGS2 step (two passes W -= Q (Q^T A W), its function
    a_orthonormalize_against) timed on the workload's operator against a stored basis of m
    columns, for two values of m up to what `mem_fraction` of the available host memory
    holds: its cost per stored column b is the slope between them.
    An iteration of the oracle costs a + b m_k (m_k stored columns at iteration k; the rest
    of the iteration does not depend on m): a = mean over the sampled iterations of
    T_k - b m_k.  The estimate of the whole solve is T_1 + sum_k (a + b m_k) over the GPU
    run's iteration widths, plus the copies by which the oracle grows its stored-basis
    buffer (capacity doubling), at the copy rate measured while filling the probe basis.
    """
    import psutil

    from oracle import ecg as ora

    n, t = prob.n, prob.t
    A0 = prob.A.to_scipy()
    threads, api = _blas_threads()
    # (1) first iterations of the oracle's solve
    A = _StampedA(A0)
    t0 = time.perf_counter()
    r = ora.flexible_sre_cg2(A, prob.b, prob.part, t, tol=prob.tol, kmax=kmax, reduce=prob.reduce,
                             switch_tol=prob.switch_tol, t_min=prob.t_min)
    t_end = time.perf_counter()
    sample1 = t_end - t0
    st = A.stamps
    first = [1] + [3 + 4 * (k - 2) for k in range(2, r.it + 1)]  # stamp index opening iteration k
    assert len(st) == 1 + 2 + 4 * (r.it - 1), (len(st), r.it)
    opens = [st[i] for i in first] + [t_end]
    T = np.diff(opens)  # T[k-1] = time of iteration k
    cs = np.concatenate([[0], np.cumsum(r.widths)])
    log(f"[cpu] oracle first {r.it} iterations: {sample1:.2f}s  per iteration {np.round(T, 2).tolist()}")
    # (2) the CGS2 step against a synthetic stored basis of m columns
    avail = psutil.virtual_memory().available
    mmax = int(mem_fraction * avail // (8 * n))
    if m_probe is None:
        m2 = 1 << max(6, min(12, int(np.floor(np.log2(max(mmax, 64))))))
        m_probe = (max(32, m2 // 8), m2)
    m1, m2 = m_probe
    rng = np.random.default_rng(11)
    t0 = time.perf_counter()
    Q = np.empty((n, m2), order="F")
    Q[:, :t] = rng.standard_normal((n, t)) / np.sqrt(n)
    filled = t
    while filled < m2:  # fill by doubling copies (values do not change the BLAS cost)
        c = min(filled, m2 - filled)
        Q[:, filled:filled + c] = Q[:, :c]
        filled += c
    fill_s = time.perf_counter() - t0
    copy_rate = (m2 - t) * 8.0 * n / max(fill_s, 1e-9)  # bytes per second (first touch included)
    cand = rng.standard_normal((n, t))
    times = {}
    t0 = time.perf_counter()
    for m in (m1, m2, m1, m2):  # two calls each, the faster one kept
        s0 = time.perf_counter()
        ora.a_orthonormalize_against(cand, Q[:, :m], A0)
        times[m] = min(times.get(m, np.inf), time.perf_counter() - s0)
    sample2 = time.perf_counter() - t0
    del Q
    b_col = max((times[m2] - times[m1]) / (m2 - m1), 0.0)
    ks = np.arange(2, r.it + 1)
    a = max(float(np.mean(T[ks - 1] - b_col * cs[ks - 1])), 0.0)
    csg = np.concatenate([[0], np.cumsum(widths_gpu)])
    it_gpu = len(widths_gpu)
    m_final = int(csg[-1])
    cap, grow_cols = 4 * t, 0
    while cap < m_final:  # the oracle's buffer doubles, copying its columns each time
        grow_cols += cap
        cap *= 2
    grow_s = grow_cols * 8.0 * n / copy_rate
    est = float(T[0] + sum(a + b_col * csg[k - 1] for k in range(2, it_gpu + 1)) + grow_s)
    log(f"[cpu] CGS2 step m={m1}: {times[m1]:.2f}s, m={m2}: {times[m2]:.2f}s -> b={b_col:.3e}s/column, "
        f"a={a:.2f}s, estimate {est:.0f}s")
    return {"value": round(est, 1), "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": (f"FP64 oracle (NumPy/SciPy, BLAS {api} with {threads} threads; SciPy sparse products single "
                       f"threaded) on the host: (1) its solve of the same workload for the first {r.it} iterations "
                       f"({sample1:.1f}s); (2) its CGS2 step against a stored basis of m={m1} and m={m2} columns "
                       f"({sample2:.1f}s; basis filled in {fill_s:.1f}s). Per iteration a + b*m_k with "
                       f"b={b_col:.3e}s per stored column from (2) and a={a:.3f}s from (1), summed over the GPU "
                       f"run's {it_gpu} iterations (m up to {m_final} columns), plus {grow_s:.0f}s of buffer growth "
                       f"copies; the oracle's full stored basis ({m_final * 8.0 * n / 1e9:.0f} GB) is not held "
                       f"on the host"),
            "measured_sample_s": round(sample1 + sample2 + fill_s, 1),
            "cgs2_step_seconds": {str(m1): round(times[m1], 3), str(m2): round(times[m2], 3)},
            "per_iteration_const_s": round(a, 4), "per_column_s": b_col}


def poisson_section(args, torch, ecg, dev):
    """64x64 Poisson (t = 8): GPU FP64 and FP32-refined against the whole oracle solve."""
    import workloads as W
    from oracle import ecg as ora

    p = W.config("poisson64")
    op = ecg.Operator.from_csr(p.A)
    P = ecg.Partition(p.part, p.t)
    b = torch.from_numpy(p.b).to(dev)
    out = {"workload": "poisson64", "n": p.n, "t": p.t}
    threads, _ = _blas_threads()
    t0 = time.perf_counter()
    ref = ora.flexible_sre_cg2(p.A.to_scipy(), p.b, p.part, p.t, tol=p.tol)
    out["oracle"] = {"seconds": round(time.perf_counter() - t0, 3), "iters": ref.it, "cores": threads}
    xo = ref.x
    for form in ("fp64", "fp32"):
        R = run_form(args, torch, ecg, p, op, P, b, form, steps=5, warmup=1, tag="poisson64 ")
        xg = R["x"].cpu().numpy()
        rep = R["report"]
        out[form] = {"seconds": round(R["seconds"], 5), "iters": rep["iters"], "outer_iters": rep["outer_iters"],
                     "relres_true": rep["relres_true"], "status": rep["status"],
                     "rel_err_vs_oracle": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))}
    out["oracle_over_gpu_fp64"] = round(out["oracle"]["seconds"] / out["fp64"]["seconds"], 1)
    return out


def learned_section(args, torch, dev):
    """learn2d256 (256x256, log10 k ~ U(-3,3) on 16x16-cell blocks, t = 16): ECG with the
    trained G G^T against its untrained Jacobi start, the classical factor on the same
    pattern (FSAI), block-Jacobi IC(0) and no preconditioner, on held-out operator seeds
    2000.. (FP64, tol 1e-8).  The parameters were
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
    kinds = ("learned", "jacobi", "fsai", "bj_ic0")
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


def jump2d512_sections(args, torch, ecg, dev, forms):
    """jump2d512 with the block-Jacobi preconditioners of Section 5.3 (FP64, FP32-refined)."""
    import workloads as W

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
    # the paper's best preconditioner (Section 5.3): exact Cholesky of 64 blocks of
    # 64 x 64 cells, the same for every t
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
    Rj = run_form(args, torch, ecg, pj, opj, Pj, bj, "fp32", M=Mc, steps=3, warmup=1, tag="jump2d512-chol64 ")
    rj = Rj["report"]
    chol["sre_cg2_fp32_refined"] = {"seconds": round(Rj["seconds"], 4), "iters": rj["iters"],
                                    "outer_iters": rj["outer_iters"], "relres_true": rj["relres_true"],
                                    "status": rj["status"]}
    return side, chol


def oracle_full_section(args, torch, ecg, dev):
    """Whole oracle solve of jump2d512 with block-Jacobi Cholesky on 64 blocks, beside the
    GPU's FP64 and FP32-refined solves and their error against the oracle's x (minutes of
    host time: run with --oracle-full only)."""
    import workloads as W
    from oracle import ecg as ora
    from oracle import precond as opc

    pj = W.config("jump2d512")
    blocks = W.box_partition(pj.grid, (8, 8))
    threads, _ = _blas_threads()
    t0 = time.perf_counter()
    pre, _ = opc.bj_chol_preconditioner(pj.A.to_scipy(), blocks)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref = ora.flexible_sre_cg2(pj.A.to_scipy(), pj.b, pj.part, pj.t, tol=pj.tol, reduce=pj.reduce,
                               switch_tol=pj.switch_tol, t_min=pj.t_min, precond=pre)
    t_solve = time.perf_counter() - t0
    out = {"workload": "jump2d512", "precond": "block-Jacobi Cholesky, 64 blocks",
           "oracle": {"setup_seconds": round(t_setup, 1), "seconds": round(t_solve, 1), "iters": ref.it,
                      "switch_iters": ref.switch_iters, "cores": threads}}
    opj = ecg.Operator.from_csr(pj.A)
    Pj = ecg.Partition(pj.part, pj.t)
    bj = torch.from_numpy(pj.b).to(dev)
    Mc = ecg.Precond.bj(opj, blocks, ecg.BJ_CHOL)
    for f in ("fp64", "fp32"):
        R = run_form(args, torch, ecg, pj, opj, Pj, bj, f, M=Mc, steps=3, warmup=1, tag="oracle-full ")
        xg = R["x"].cpu().numpy()
        out[f] = {"seconds": round(R["seconds"], 4), "iters": R["report"]["iters"],
                  "relres_true": R["report"]["relres_true"],
                  "rel_err_vs_oracle": float(np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x))}
    return out


def explore(args):
    """One solve per requested form of one workload (no timed series): iterations, switch
    iterations, stored vectors, dropped blocks, true relative residual and seconds, with
    progress lines every --progress iterations.  For configurations too long for the timed
    series (jump3d160, aniso3d128 at t = 16 / 64)."""
    import torch

    import workloads as W
    from paper_2305_19013_amd import ecg

    ecg.lib()
    dev = torch.device("cuda:0")
    prob = W.config(args.workload, t=args.t) if args.workload == "aniso3d128" else W.config(args.workload)
    op = ecg.Operator.from_csr(prob.A)
    P = ecg.Partition(prob.part, prob.t)
    b = torch.from_numpy(prob.b).to(dev)
    M = None
    if args.precond == "bj_ic0":
        M = ecg.Precond.bj_ic0(op, P)
    elif args.precond == "chol64":
        M = ecg.Precond.bj(op, W.box_partition(prob.grid, (8, 8)), ecg.BJ_CHOL)
    out = {"mode": "explore", "workload": args.workload, "n": prob.n, "t": prob.t, "precond": args.precond,
           "kmax": args.kmax}
    for form in [f for f in args.forms.split(",") if f]:
        kw, w = form_options(args, ecg, prob, form, M)
        free, _ = torch.cuda.mem_get_info()
        col = prob.n * w
        qbytes = max(prob.t * col, int(free * 0.93) - 4 * prob.t * col - (3 << 30))
        opts = ecg.options(q_budget_bytes=qbytes, **kw)
        ws = torch.empty(ecg.workspace_size(op, P, opts), dtype=torch.uint8, device=dev)
        x = torch.zeros_like(b)
        ecg.progress(args.progress)
        log(f"[explore {args.workload} {form}] q budget {qbytes / 1e9:.1f} GB = {qbytes // col} columns")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = solve_once(ecg, op, P, b, x, opts, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ecg.progress(0)
        out[form] = {"seconds": round(dt, 3), "iters": rep["iters"], "switch_iters": rep["switch_iters"],
                     "t_final": rep["t_final"], "outer_iters": rep["outer_iters"],
                     "vectors_stored": rep["vectors_stored"], "blocks_dropped": rep["blocks_dropped"],
                     "q_cols": qbytes // col, "relres_recursive": rep["relres_recursive"],
                     "relres_true": rep["relres_true"], "status": rep["status"]}
        log(f"[explore {args.workload} {form}] {out[form]}")
        del ws
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall-clock budget of the whole run from process start; --steps and --warmup are maxima")
    ap.add_argument("--workload", default="aniso3d128")
    ap.add_argument("--t", type=int, default=32)
    ap.add_argument("--forms", default="fp64,fp32")
    ap.add_argument("--kmax", type=int, default=20000)
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="inner tolerance of the FP32 form (default: the workload's)")
    ap.add_argument("--q-cols", type=int, default=0)
    ap.add_argument("--progress", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-ops", type=int, default=8)
    ap.add_argument("--oracle-full", action="store_true",
                    help="also time the whole oracle solve of jump2d512 with 64-block Cholesky (minutes)")
    ap.add_argument("--precond", default="none", choices=("none", "bj_ic0", "chol64"),
                    help="preconditioner of the main solve (block-Jacobi IC(0) on the subdomains, or "
                         "exact Cholesky of 64 blocks of a 2D grid)")
    ap.add_argument("--explore", action="store_true",
                    help="one solve per form of --workload (no timed series; see explore())")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device-to-device before the solves (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    if args.explore:
        explore(args)
        return
    budget = Budget(args.budget_s)
    forms = [f for f in args.forms.split(",") if f]
    main_form = "fp64" if "fp64" in forms else forms[0]
    out = {"metric": METRIC, "value": None, "unit": "s", "n_gpus": 1, "steps": 0, "warmup": 0,
           "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if main_form == "fp64" else "f32+f64", "data": "synthetic",
           "config": {"workload": args.workload}, "steps_requested": args.steps, "warmup_requested": args.warmup,
           "budget_s": args.budget_s, "skipped": [], "roofline": None, "cpu_baseline": None}
    rc = 0
    try:
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
        M = None
        if args.precond == "bj_ic0":
            M = ecg.Precond.bj_ic0(op, P)
        elif args.precond == "chol64":
            M = ecg.Precond.bj(op, W.box_partition(prob.grid, (8, 8)), ecg.BJ_CHOL)
        out["config"].update({"precond": args.precond, "n": prob.n, "nnz": prob.A.nnz, "t": prob.t,
                              "reduce": {0: "none", 1: "halve once", 2: "halve repeatedly"}[prob.reduce],
                              "switch_tol": prob.switch_tol, "tol": prob.tol})
        # time needed after the headline series, for the sections that follow it
        later = 0.0
        if "fp32" in forms and main_form == "fp64":
            later += EST["fp32"] * 2
        if not args.no_cpu:
            later += EST["cpu"]
        if not args.no_side:
            later += EST["poisson64"] + EST["jump2d512"] + (0 if args.no_learned else EST["learned"])

        def fit_main(est):
            return int((budget.left() - later - 10.0) // est)

        # --warmup 0 (profiler runs): the priming solve and the timed steps only, no roofline
        R = run_form(args, torch, ecg, prob, op, P, b, main_form, M=M, steps=args.steps,
                     warmup=args.warmup, tag="", instrument=args.warmup > 0, fit=fit_main)
        rep = R["report"]
        out.update({"value": round(R["seconds"], 4), "steps": R["steps"], "warmup": R["warmup"],
                    "ms_per_step": round(R["seconds"] * 1e3, 2)})
        out["config"]["q_cols"] = R["q_cols"]
        out["step_seconds"] = [round(s, 4) for s in R["step_seconds"]]
        out["instrumented_warmup_s"] = round(R["instrumented_seconds"], 4) if R["instrumented_seconds"] else None
        out["solve"] = {"iters": rep["iters"], "switch_iters": rep["switch_iters"], "t_final": rep["t_final"],
                        "vectors_stored": rep["vectors_stored"], "blocks_dropped": rep["blocks_dropped"],
                        "relres_true": rep["relres_true"], "status": rep["status"]}
        roof, best = roofline_from_stats(R["stats"])
        if roof is not None and main_form == "fp64":
            roof["traffic"] = profiled_traffic(args.workload, prob.t, best)
        out["roofline"] = roof
        out["kernels"] = kernel_table(R["stats"])
        out["spmm_GBs"] = out["kernels"].get("spmm", {}).get("GB/s")
        xa = R["x"]
        for f in forms:
            if f == main_form:
                continue
            if budget.left() < EST["fp32"] + 10:
                out["skipped"].append(f)
                continue
            Rf = run_form(args, torch, ecg, prob, op, P, b, f, M=M, steps=args.steps, warmup=min(args.warmup, 1),
                          tag="", fit=lambda est: int((budget.left() - later + 2 * EST["fp32"] - 10.0) // est))
            rf = Rf["report"]
            out["fp32_refined" if f == "fp32" else f] = {
                "seconds": round(Rf["seconds"], 4), "steps": Rf["steps"], "warmup": Rf["warmup"],
                "iters": rf["iters"], "outer_iters": rf["outer_iters"], "relres_true": rf["relres_true"],
                "status": rf["status"],
                "rel_err_vs_fp64_gpu": float(torch.linalg.norm(Rf["x"] - xa) / torch.linalg.norm(xa)),
                "speedup_vs_fp64": round(R["seconds"] / Rf["seconds"], 3) if main_form == "fp64" else None,
            }
        if not args.no_cpu:
            later -= EST["cpu"]
            widths = []
            sw = rep["switch_iters"]
            for k in range(1, rep["iters"] + 1):
                widths.append(prob.t >> sum(1 for s in sw if s <= k))
            out["cpu_baseline"] = cpu_baseline(prob, widths)
        if not args.no_side:
            sections = [("poisson64", lambda: poisson_section(args, torch, ecg, dev))]
            if not args.no_learned:
                sections.append(("learn2d256_learned", lambda: learned_section(args, torch, dev)))
            sections.append(("jump2d512", lambda: jump2d512_sections(args, torch, ecg, dev, forms)))
            est_of = {"poisson64": EST["poisson64"], "learn2d256_learned": EST["learned"],
                      "jump2d512": EST["jump2d512"]}
            for name, fn in sections:
                if budget.left() < est_of[name] + 5:
                    out["skipped"].append(name)
                    log(f"skipped {name}: {budget.left():.0f}s left of the budget")
                    continue
                try:
                    res = fn()
                except Exception as e:  # a side section must not lose the headline line
                    out[name] = {"error": f"{type(e).__name__}: {e}"}
                    traceback.print_exc()
                    continue
                if name == "jump2d512":
                    out["jump2d512_bj"], out["jump2d512_chol64"] = res
                else:
                    out[name] = res
        if args.oracle_full:
            out["oracle_full_jump2d512_chol64"] = oracle_full_section(args, torch, ecg, dev)
    except Exception as e:
        out["error"] = f"{type(e).__name__}: {e}"
        traceback.print_exc()
        rc = 1
    finally:
        out["wall_s"] = round(time.time() - T_START, 1)
        print(json.dumps(out), flush=True)
    sys.exit(rc)


if __name__ == "__main__":
    main()
