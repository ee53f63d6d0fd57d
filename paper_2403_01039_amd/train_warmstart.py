"""Train the warm-start network on converged solves the library itself
produces, then measure what it gains.

Data: seeded 200-atom solutes in water (128^3 grid at 0.5 A, KH closure,
MDIIS depth 5, rms 1e-6), solved from tau0 = 0 on the GPU; the network input
is symlog(beta u) of each site (rism3d_net_input) and the target the
converged c_sr = g - 1 - tau (rism3d_csr), scaled by 1 / c_scale.  All of it
stays in device memory.  Training: one solute per step, the library's own
forward / backward kernels (rism3d_unet_gradient) and Adam with global-norm
clipping (rism3d_unet_adam); linear warm-up, then cosine decay over the
steps that fit in the time budget; a loss blow-up rolls back to the best
checkpoint at half the learning rate.  Evaluation: held-out seeds solved from
tau0 = 0 and from the warm start; iterations, time per solve, and the
difference of the two converged g and SFE.

    python -m paper_2403_01039_amd.train_warmstart --n-train 2000 --n-test 100 \\
        --out weights.npz --report report.json --budget 600
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2403_01039_amd import inputs
from paper_2403_01039_amd import rism3d as R

TRAIN_SEED0 = 10000
TEST_SEED0 = 20000


class Problems:
    """Device problems sharing one solver workspace (same grid and solvent)."""

    def __init__(self, device):
        self.device = device
        self.chi, self.dk = inputs.solvent_table("water")
        proto = inputs.warmstart_problem(TRAIN_SEED0)
        self.opts = R.make_opts(proto.options)
        self.shape = (3, proto.grid.nz, proto.grid.ny, proto.grid.nx)
        # the largest workspace any 200-atom solute needs
        self.ws = R.alloc_workspace(R.rism3d_workspace_bytes(self.dp(proto), self.opts), device)

    def dp(self, prob):
        return R.DeviceProblem(prob, self.chi, self.dk, device=self.device)

    def solve(self, dp, tau0=None, g=None):
        R.rism3d_potential(dp, self.opts, self.ws)
        return R.rism3d_solve(dp, self.opts, self.ws, tau0, g)


def generate(P: Problems, seeds, c_scale: float, log):
    n = len(seeds)
    X = torch.empty((n,) + P.shape, dtype=torch.float32, device=P.device)
    Y = torch.empty_like(X)
    its = []
    t0 = time.perf_counter()
    for i, seed in enumerate(seeds):
        dp = P.dp(inputs.warmstart_problem(seed))
        info = P.solve(dp)
        its.append(info.iterations)
        R.rism3d_net_input(dp, P.opts, P.ws, X[i])
        R.rism3d_csr(dp, P.opts, P.ws, Y[i])
        if (i + 1) % 100 == 0 or i + 1 == n:
            torch.cuda.synchronize()
            log(f"data {i + 1}/{n}: {time.perf_counter() - t0:.1f} s, mean iterations "
                f"{np.mean(its):.1f}")
    Y.mul_(1.0 / c_scale)
    return X, Y, its


def train(cfg, X, Y, epochs_max: int, budget_s: float, lr: float, seed: int, clip: float,
          warmup: int, log, init=None):
    """Adam on one solute per step: linear warm-up over `warmup` steps, then
    cosine decay; global-norm clipping; every CHECK steps the mean loss of the
    last CHECK steps is compared with the best so far and a blow-up (not
    finite, or 5x the best) rolls back to the best checkpoint at half the
    learning rate."""
    CHECK = 500
    n = X.shape[0]
    if init is None:
        init = inputs.unet_init_params(R.unet_layers(cfg), seed, slope=cfg.slope)
    theta = torch.tensor(np.asarray(init, dtype=np.float32), device=X.device)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    scratch = R.unet_adam_scratch(X.device)
    ws = R.alloc_workspace(R.unet_workspace_bytes(cfg, X.shape[2:], True), X.device)
    step_loss = torch.zeros(CHECK, dtype=torch.float64, device=X.device)
    norms = torch.zeros(CHECK, dtype=torch.float64, device=X.device)
    rng = np.random.default_rng(seed)
    R.unet_gradient(cfg, theta, X[0], Y[0], grad, ws, step_loss[:1])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        R.unet_gradient(cfg, theta, X[0], Y[0], grad, ws, step_loss[:1])
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t) / 3
    total = int(min(epochs_max * n, budget_s / (step_s * 1.05)))
    log(f"train: {step_s * 1e3:.1f} ms per step, {total} steps ({total / n:.2f} epochs), "
        f"peak lr {lr:g}, clip {clip:g}")
    best = (float("inf"), theta.clone(), m.clone(), v.clone(), 0)
    scale = 1.0
    history = []
    t0 = time.perf_counter()
    order = rng.permutation(n)
    pos = 0
    step = 0
    adam_t = 0
    while step < total:
        if pos == n:
            order, pos = rng.permutation(n), 0
        i = int(order[pos])
        pos += 1
        step += 1
        adam_t += 1
        frac = (step - 1) / total
        lr_t = scale * lr * min(1.0, step / warmup) * 0.5 * (1.0 + math.cos(math.pi * frac))
        k = (step - 1) % CHECK
        R.unet_gradient(cfg, theta, X[i], Y[i], grad, ws, step_loss[k:k + 1])
        R.unet_adam(theta, m, v, grad, adam_t, lr_t, clip_norm=clip, scratch=scratch)
        norms[k:k + 1].copy_(scratch[-2:-1])
        if step % CHECK == 0 or step == total:
            cnt = k + 1
            mean_loss = float(step_loss[:cnt].mean().item())
            mean_norm = float(norms[:cnt].mean().item())
            history.append({"step": step, "mean_loss": mean_loss, "mean_grad_norm": mean_norm,
                            "lr": lr_t, "seconds": time.perf_counter() - t0})
            log(f"  step {step}: loss {mean_loss:.4e}, |g| {mean_norm:.3e}, lr {lr_t:.2e} "
                f"({time.perf_counter() - t0:.0f} s)")
            if not math.isfinite(mean_loss) or mean_loss > 5.0 * best[0]:
                log(f"  blow-up: back to the checkpoint of step {best[4]}, learning rate halved")
                theta.copy_(best[1])
                m.copy_(best[2])
                v.copy_(best[3])
                scale *= 0.5
                history[-1]["rollback"] = best[4]
            elif mean_loss < best[0]:
                best = (mean_loss, theta.clone(), m.clone(), v.clone(), step)
    # the final parameters unless the last window is worse than the best
    if history and history[-1]["mean_loss"] > 1.5 * best[0]:
        theta.copy_(best[1])
    return theta, history, step_s


def evaluate(P: Problems, cfg, theta, c_scale: float, seeds, log):
    net_ws = R.alloc_workspace(R.unet_workspace_bytes(cfg, P.shape[1:], False), P.device)
    tau0 = torch.empty(P.shape, dtype=torch.float32, device=P.device)
    g_plain = torch.empty_like(tau0)
    g_warm = torch.empty_like(tau0)
    rows = []
    for seed in seeds:
        dp = P.dp(inputs.warmstart_problem(seed))
        torch.cuda.synchronize()
        t = time.perf_counter()
        R.rism3d_potential(dp, P.opts, P.ws)
        ip = R.rism3d_solve(dp, P.opts, P.ws, None, g_plain)
        sfe_p, _ = R.rism3d_thermo(dp, P.opts, P.ws)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        t = time.perf_counter()
        R.rism3d_potential(dp, P.opts, P.ws)
        R.rism3d_warmstart(dp, P.opts, cfg, theta, P.ws, net_ws, tau0, c_scale)
        iw = R.rism3d_solve(dp, P.opts, P.ws, tau0, g_warm)
        sfe_w, _ = R.rism3d_thermo(dp, P.opts, P.ws)
        torch.cuda.synchronize()
        tw = time.perf_counter() - t
        rows.append({"seed": seed, "it_plain": ip.iterations, "it_warm": iw.iterations,
                     "warm_used": iw.warm_start_used, "s_plain": tp, "s_warm": tw,
                     "max_dg": float((g_warm - g_plain).abs().max().item()),
                     "sfe_plain": sfe_p, "sfe_warm": sfe_w})
    it_p = np.mean([r["it_plain"] for r in rows])
    it_w = np.mean([r["it_warm"] for r in rows])
    sp = len(rows) / sum(r["s_plain"] for r in rows)
    sw = len(rows) / sum(r["s_warm"] for r in rows)
    summary = {"n": len(rows), "iterations_plain": it_p, "iterations_warm": it_w,
               "solves_per_s_plain": sp, "solves_per_s_warm": sw, "speedup": sw / sp,
               "max_dg": max(r["max_dg"] for r in rows),
               "max_sfe_rel": max(abs(r["sfe_warm"] - r["sfe_plain"]) / abs(r["sfe_plain"])
                                  for r in rows),
               "fallbacks": sum(1 for r in rows if not r["warm_used"])}
    log(f"eval: plain {it_p:.1f} it, {sp:.2f} solves/s; warm {it_w:.1f} it, {sw:.2f} solves/s; "
        f"speedup {sw / sp:.2f}; max|dg| {summary['max_dg']:.2e}")
    return summary, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-test", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--budget", type=float, default=600.0, help="training seconds")
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--clip", type=float, default=1.0, help="global gradient-norm clip")
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--c-scale", type=float, default=4.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--init", default=None,
                    help="continue from the parameters of a weights file (same configuration)")
    ap.add_argument("--out", default="warmstart_unet.npz")
    ap.add_argument("--report", default="warmstart_report.json")
    args = ap.parse_args()
    log = lambda s: print(s, flush=True)
    dev = torch.device("cuda:0")
    P = Problems(dev)
    cfg = R.unet_config(3, 3)
    X, Y, its = generate(P, range(TRAIN_SEED0, TRAIN_SEED0 + args.n_train), args.c_scale, log)
    log(f"targets / c_scale: mean {Y.mean().item():.3e} std {Y.std().item():.3e} "
        f"min {Y.min().item():.3e} max {Y.max().item():.3e}")
    init = None
    if args.init:
        with np.load(args.init, allow_pickle=False) as z:
            init = np.asarray(z["params"], dtype=np.float32)
            if float(z["c_scale"]) != args.c_scale:
                raise ValueError("--init weights were trained with another c_scale")
        log(f"continuing from {args.init}")
    theta, history, step_s = train(cfg, X, Y, args.epochs, args.budget, args.lr, args.seed,
                                   args.clip, args.warmup, log, init)
    np.savez(args.out, params=theta.cpu().numpy(), levels=cfg.levels, base=cfg.base,
             in_channels=cfg.in_channels, out_channels=cfg.out_channels, slope=cfg.slope,
             c_scale=args.c_scale)
    log(f"wrote {args.out}")
    del X, Y
    torch.cuda.empty_cache()
    summary, rows = evaluate(P, cfg, theta, args.c_scale,
                             range(TEST_SEED0, TEST_SEED0 + args.n_test), log)
    report = {"n_train": args.n_train, "train_seeds": [TRAIN_SEED0, TRAIN_SEED0 + args.n_train],
              "test_seeds": [TEST_SEED0, TEST_SEED0 + args.n_test], "c_scale": args.c_scale,
              "init": args.init, "lr": args.lr, "clip": args.clip, "warmup": args.warmup, "step_ms": step_s * 1e3, "data_iterations_mean": float(np.mean(its)),
              "history": history, "eval": summary, "eval_rows": rows}
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps(summary))


if __name__ == "__main__":
    main()
