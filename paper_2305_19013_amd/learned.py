"""Learned preconditioner M^{-1} = G G^T: binding of include/ecg_nn.h and its training loop.

Everything numerical runs in libecg.so: the network forward/backward, the loss and its
gradient, Adam, the CSR of G, and the ECG solves that produce the training solutions.
This module only moves arguments, picks minibatches and loops.

Usage (trains on operators 0..N-1 of the learn2d256 family, keeps the epoch with the fewest
ECG iterations on validation seeds 1900.., evaluates on held-out seeds 2000..):
    python -m paper_2305_19013_amd.learned --train 2000 --heldout 200 --epochs 40
"""

from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

from . import ecg as E

NPARAM = 1411
_sig_done = False


def _lib():
    global _sig_done
    L = E.lib()
    if not _sig_done:
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "ecg_nn_forward": [i32, i32, i32, vp, vp, vp, vp],
            "ecg_nn_workspace_size": [i32, i32, i32, C.POINTER(C.c_size_t)],
            "ecg_nn_loss_grad": [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp],
            "ecg_nn_backward": [i32, i32, i32, vp, vp, vp, C.c_double, vp, vp, C.c_size_t, vp],
            "ecg_nn_adam": [i32, vp, vp, vp, vp, i32, C.c_double, C.c_double, C.c_double, C.c_double, vp],
            "ecg_nn_factor_csr": [i32, i32, vp, vp, vp, vp, vp],
            "ecg_nn_fsai": [i32, i32, i32, vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = C.c_int32
            fn.argtypes = args
        _sig_done = True
    return L


def _p(t):
    return C.c_void_p(t.data_ptr())


class LearnedFactor:
    """Network parameters (FP32) and Adam state (FP64) on the device, for an nx x ny grid."""

    def __init__(self, nx: int, ny: int, params0, device):
        import torch

        self.torch = torch
        self.nx, self.ny, self.n = int(nx), int(ny), int(nx) * int(ny)
        self.device = device
        self.params = torch.tensor(np.asarray(params0), dtype=torch.float32, device=device)
        self.m = torch.zeros(NPARAM, dtype=torch.float64, device=device)
        self.v = torch.zeros(NPARAM, dtype=torch.float64, device=device)
        self.grad = torch.zeros(NPARAM, dtype=torch.float64, device=device)
        self.step = 0
        self._ws = {}

    def _workspace(self, nb):
        if nb not in self._ws:
            sz = C.c_size_t()
            E.check(_lib().ecg_nn_workspace_size(self.nx, self.ny, nb, C.byref(sz)))
            self._ws[nb] = self.torch.empty(sz.value, dtype=self.torch.uint8, device=self.device)
        return self._ws[nb]

    def forward(self, a5):
        nb = a5.shape[0]
        g3 = self.torch.empty((nb, 3, self.n), dtype=self.torch.float64, device=self.device)
        E.check(_lib().ecg_nn_forward(self.nx, self.ny, nb, _p(a5), _p(self.params), _p(g3), E._stream()))
        return g3

    def loss_grad(self, a5, g3, b, x):
        nb = a5.shape[0]
        ws = self._workspace(nb)
        loss = self.torch.empty(nb, dtype=self.torch.float64, device=self.device)
        dg3 = self.torch.empty_like(g3)
        E.check(_lib().ecg_nn_loss_grad(self.nx, self.ny, nb, _p(a5), _p(g3), _p(b), _p(x), _p(loss), _p(dg3),
                                        _p(ws), ws.numel(), E._stream()))
        return loss, dg3

    def backward(self, a5, dg3, scale):
        nb = a5.shape[0]
        ws = self._workspace(nb)
        E.check(_lib().ecg_nn_backward(self.nx, self.ny, nb, _p(a5), _p(self.params), _p(dg3), float(scale),
                                       _p(self.grad), _p(ws), ws.numel(), E._stream()))
        return self.grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        E.check(_lib().ecg_nn_adam(NPARAM, _p(self.params), _p(self.grad), _p(self.m), _p(self.v), self.step,
                                   lr, beta1, beta2, eps, E._stream()))

    def train_step(self, a5, b, x, lr):
        """One minibatch: forward, loss and dL/dG, backward (batch mean), Adam."""
        g3 = self.forward(a5)
        loss, dg3 = self.loss_grad(a5, g3, b, x)
        self.backward(a5, dg3, 1.0 / a5.shape[0])
        self.adam(lr)
        return loss

    def preconditioner(self, a5_one):
        """E.Precond for one operator (a5_one: [1, 5, n]) built from the network's G."""
        return factor_precond(self.nx, self.ny, self.forward(a5_one), self.device)


def fsai_g3(nx: int, ny: int, a5):
    """G of the classical factorised sparse approximate inverse on the same pattern
    (ecg_nn_fsai), for a5 [nb, 5, n] on the device; returns g3 [nb, 3, n]."""
    import torch

    g3 = torch.empty((a5.shape[0], 3, nx * ny), dtype=torch.float64, device=a5.device)
    E.check(_lib().ecg_nn_fsai(nx, ny, a5.shape[0], _p(a5), _p(g3), E._stream()))
    return g3


def factor_precond(nx: int, ny: int, g3, device):
    """E.Precond with M^{-1} = G G^T from g3 [1, 3, n] (CSR built on the device)."""
    import torch

    n = nx * ny
    nnz = 3 * n - nx - ny
    rowptr = torch.empty(n + 1, dtype=torch.int64, device=device)
    col = torch.empty(nnz, dtype=torch.int32, device=device)
    val = torch.empty(nnz, dtype=torch.float64, device=device)
    E.check(_lib().ecg_nn_factor_csr(nx, ny, _p(g3), _p(rowptr), _p(col), _p(val), E._stream()))
    return E.Precond.factor_device(n, nnz, rowptr, col, val)


# ----------------------------------------------------------------------------- data
def family(seed: int, scale: int = 1):
    """Operator `seed` of the learn2d256 family (problem, 5-point stencil)."""
    import workloads as W

    p = W.config("learn2d256", seed=seed, scale=scale)
    return p, W.stencil5(p.A, p.grid[0])


def solve_dataset(seeds, device, scale=1, tol=1e-10, log=print):
    """Solutions x_s = A_s^{-1} b_s produced by the ECG solver itself (FP64, block-Jacobi
    IC(0) on the t = 16 subdomains).  Returns device tensors a5 [N,5,n], b [N,n], x [N,n]."""
    import torch

    A5, B, X = [], [], []
    t0 = time.time()
    for j, s in enumerate(seeds):
        p, a5 = family(s, scale)
        op = E.Operator.from_csr(p.A)
        P = E.Partition(p.part, p.t)
        M = E.Precond.bj_ic0(op, P)
        b = torch.from_numpy(p.b).to(device)
        x = torch.zeros_like(b)
        rep, _ = E.solve(op, P, b, x, E.options(tol=tol, M=M, q_budget_bytes=4000 * p.n * 8))
        if rep["status"] != "ok":
            raise RuntimeError(f"training solve {s} did not converge: {rep}")
        A5.append(torch.from_numpy(a5).to(device))
        B.append(b)
        X.append(x)
        if log and (j + 1) % 64 == 0:
            log(f"[data] {j + 1}/{len(seeds)} solves, last {rep['iters']} iterations, {time.time() - t0:.1f}s")
    return torch.stack(A5), torch.stack(B), torch.stack(X)


def train(model: LearnedFactor, a5, b, x, epochs=4, batch=16, lr=3e-3, seed=0, log=print, val_seeds=(),
          val_scale=1, val_every=5):
    """Adam over shuffled minibatches; returns the mean loss of every epoch.

    With val_seeds, every val_every epochs the mean ECG iteration count on those validation
    operators is measured and the parameters with the fewest iterations are kept (the
    loss follows iteration counts only loosely, so training stops early on them)."""
    N = a5.shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    best = (float("inf"), model.params.clone(), 0)
    if val_seeds:
        best = (_val_iters(model, val_seeds, a5.device, val_scale), model.params.clone(), 0)
    for ep in range(epochs):
        order = rng.permutation(N)
        tot, cnt = 0.0, 0
        for i in range(0, N - batch + 1, batch):
            idx = model.torch.from_numpy(order[i:i + batch]).to(a5.device)
            loss = model.train_step(a5.index_select(0, idx), b.index_select(0, idx), x.index_select(0, idx), lr)
            tot += float(loss.sum())
            cnt += batch
        hist.append(tot / max(cnt, 1))
        msg = f"[train] epoch {ep + 1}/{epochs} mean loss {hist[-1]:.5f}"
        if val_seeds and ((ep + 1) % val_every == 0 or ep + 1 == epochs):
            it = _val_iters(model, val_seeds, a5.device, val_scale)
            msg += f" validation iterations {it:.1f}"
            if it < best[0]:
                best = (it, model.params.clone(), ep + 1)
        if log:
            log(msg)
    if val_seeds:
        model.params.copy_(best[1])
        model.best_epoch, model.best_val_iters = best[2], best[0]
        if log:
            log(f"[train] kept the parameters of epoch {best[2]} ({best[0]:.1f} validation iterations)")
    return hist


def _val_iters(model, seeds, device, scale):
    res = evaluate(model, seeds, device, scale, kinds=("learned",))
    return float(np.mean([r["iters"] for r in res["learned"]]))


def evaluate(model: LearnedFactor, seeds, device, scale=1, kinds=("learned", "jacobi", "bj_ic0", "plain"),
             kmax=4000, params_jacobi=None, log=None):
    """Iterations and seconds of ECG (t = 16, FP64, tol 1e-8) per preconditioner kind: learned
    (the network's G G^T), jacobi (the network at params_jacobi, its untrained start), fsai (the
    classical factor on the same pattern), bj_ic0 (block-Jacobi IC(0) on the subdomains) or
    plain (none)."""
    import torch

    out = {k: [] for k in kinds}
    jac = None
    if "jacobi" in kinds:
        jac = LearnedFactor(model.nx, model.ny, params_jacobi, device)
    for s in seeds:
        p, a5 = family(s, scale)
        op = E.Operator.from_csr(p.A)
        P = E.Partition(p.part, p.t)
        bt = torch.from_numpy(p.b).to(device)
        a5t = torch.from_numpy(a5).to(device)[None]
        for k in kinds:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if k == "learned":
                M = model.preconditioner(a5t)
            elif k == "jacobi":
                M = jac.preconditioner(a5t)
            elif k == "bj_ic0":
                M = E.Precond.bj_ic0(op, P)
            elif k == "fsai":
                M = factor_precond(model.nx, model.ny, fsai_g3(model.nx, model.ny, a5t), device)
            else:
                M = None
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            x = torch.zeros_like(bt)
            opts = E.options(tol=p.tol, kmax=kmax, M=M, q_budget_bytes=min(kmax, 4000) * p.t * p.n * 8)
            rep, _ = E.solve(op, P, bt, x, opts)
            out[k].append({"seed": s, "iters": rep["iters"], "seconds": rep["seconds"], "setup_s": setup,
                           "relres_true": rep["relres_true"], "status": rep["status"]})
        if log:
            log(f"[eval] seed {s}: " + ", ".join(f"{k} {out[k][-1]['iters']} it {out[k][-1]['seconds']:.3f}s"
                                                 for k in kinds))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=256, help="training operators (seeds 0..N-1)")
    ap.add_argument("--heldout", type=int, default=16, help="held-out operators (seeds 2000..)")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--scale", type=int, default=1)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--plain", type=int, default=0, help="unpreconditioned ECG on this many held-out operators")
    ap.add_argument("--val", type=int, default=4, help="validation operators (seeds 1900..)")
    ap.add_argument("--val-every", type=int, default=5)
    ap.add_argument("--out", default="")
    args = ap.parse_args()

    import torch

    import workloads as W

    dev = torch.device("cuda:0")
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    p0, _ = family(0, args.scale)
    nx, ny = p0.grid
    theta0 = W.init_params(args.init_seed)
    model = LearnedFactor(nx, ny, theta0, dev)
    t0 = time.time()
    a5, b, x = solve_dataset(range(args.train), dev, args.scale, log=log)
    t_data = time.time() - t0
    torch.cuda.synchronize()
    t0 = time.time()
    hist = train(model, a5, b, x, args.epochs, args.batch, args.lr, log=log,
                 val_seeds=tuple(range(1900, 1900 + args.val)), val_scale=args.scale, val_every=args.val_every)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    meta = {"train_ops": args.train, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
            "best_epoch": getattr(model, "best_epoch", None), "val_ops": args.val, "init_seed": args.init_seed,
            "val_iters": getattr(model, "best_val_iters", None),
            "params": model.params.cpu().numpy().astype(float).tolist()}
    if args.out:  # saved before the (long) evaluation
        with open(args.out, "w") as f:
            json.dump(meta, f)
    kinds = ("learned", "jacobi", "bj_ic0")
    res = evaluate(model, range(2000, 2000 + args.heldout), dev, args.scale, kinds, params_jacobi=theta0, log=log)
    if args.plain:  # unpreconditioned ECG is slow on this family: a few held-out operators only
        ecg_progress = E.progress
        ecg_progress(500)
        res.update(evaluate(model, range(2000, 2000 + args.plain), dev, args.scale, ("plain",), kmax=6000, log=log))
        ecg_progress(0)
    summary = {k: {"mean_iters": float(np.mean([r["iters"] for r in v])),
                   "mean_seconds": float(np.mean([r["seconds"] for r in v])),
                   "mean_setup_s": float(np.mean([r["setup_s"] for r in v])),
                   "max_relres_true": float(np.max([r["relres_true"] for r in v])),
                   "all_ok": all(r["status"] == "ok" for r in v)} for k, v in res.items()}
    meta.update({"heldout_ops": args.heldout, "data_seconds": t_data, "train_seconds": t_train,
                 "loss_per_epoch": hist, "summary": summary})
    if args.out:
        with open(args.out, "w") as f:
            json.dump(meta, f)
    meta.pop("params")
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
