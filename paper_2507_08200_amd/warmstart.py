"""Data, training and evaluation of the learned Poisson initial guess.

Snapshots come from the solver itself: streamer runs (the 15-species Ar-H2
state with seeded voltage and seed position) are stepped with vd_step, and
every few steps the charge density (as the network input of
vd_nn_features) and the converged potential / V (the target) are kept on
the GPU.  Training is plain Adam on the mean squared error through
vd_nn_train_step; evaluation times the multigrid solve to 1e-10 from zero,
from the previous step's potential and from the network's guess.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import inputs as I
from . import mechanisms as M
from . import vd as V

QE = 1.602176634e-19
EPS0 = 8.8541878128e-12


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def snapshots(ctx, runs, n, steps, every, dev="cuda:0"):
    """[(features bf16 [n,n,n,2], target f32 [n,n,n], rho f64, phi f64, bc, grid)] from solver runs."""
    species = M.arh2_15()
    Z = torch.tensor([s["Z"] for s in species], dtype=torch.float64, device=dev)
    out = []
    for r in runs:
        cfg = I.cfg3(seed=r["seed"], n=n, voltage=r["voltage"], seed_centre=r["centre"])
        state = {k: torch.tensor(cfg[k], device=dev) for k in ("n", "phi", "Te")}
        lfa = dict(cfg["lfa"])
        lfa["te_K"] = torch.tensor(cfg["lfa"]["te_K"], device=dev)
        P = V.step_params(cfg, species, lfa=lfa, poisson=V.mg_opts(rtol=1e-10),
                          species_mg=V.mg_opts(rtol=1e-10, n_levels=1, nu_pre=1, nu_post=1))
        for k in range(steps):
            ctx.vd_step(P, state, want_info=False)
            if (k + 1) % every == 0:
                rho = (QE * torch.tensordot(Z, state["n"], dims=1)).contiguous()
                feats, vref = ctx.vd_nn_features(cfg["grid"], cfg["phi_bc"], rho, eps=EPS0)
                out.append({"x": feats, "t": (state["phi"] / vref).float().contiguous(), "rho": rho,
                            "phi": state["phi"].clone(), "bc": cfg["phi_bc"], "grid": cfg["grid"], "vref": vref})
    return out


def train(ctx, data, cfg, params, seconds, lr, seed=0, max_steps=None):
    """Adam on the mean squared error, samples in a seeded random order,
    until the time budget (or max_steps) is spent."""
    ctx.vd_nn_create(cfg, params)
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    losses = []
    it = 0
    while True:
        for i in rng.permutation(len(data)):
            d = data[i]
            loss = ctx.vd_nn_train_step(d["grid"], d["x"], d["t"], lr, update=True)
            losses.append(loss)
            it += 1
            if it % 20 == 0:
                _log("[warmstart] step %d loss %.4g" % (it, float(np.mean(losses[-20:]))))
            if time.perf_counter() - t0 > seconds or (max_steps and it >= max_steps):
                return {"steps": it, "seconds": round(time.perf_counter() - t0, 2), "loss_first": losses[0],
                        "loss_last20": float(np.mean(losses[-20:]))}


def time_to_tol(ctx, d, guess, precision, phi0=None, reps=3):
    """Median event time of the Poisson solve to 1e-10 (the guess
    computation included)."""
    ts, info = [], None
    for _ in range(reps):
        phi = (phi0.clone() if phi0 is not None else torch.zeros_like(d["phi"]))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        info = ctx.vd_poisson_solve(d["grid"], d["bc"], d["rho"], phi, beta_c=EPS0,
                                    opts=V.mg_opts(rtol=1e-10, precision=precision, guess=guess, ir_inner=2))
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return {"ms": round(float(np.median(ts)), 4), "cycles": info["cycles"], "outer": info["outer_iters"],
            "rel_res0": info["rel_res0"], "fallback": info["fallback"]}


def evaluate(ctx, test):
    rows = []
    for d in test:
        rows.append({
            "plain_fp64_zero_guess": time_to_tol(ctx, d, V.GUESS_ZERO, V.FP64),
            "fp32_ir_zero_guess": time_to_tol(ctx, d, V.GUESS_ZERO, V.FP32_IR),
            "learned_fp64": time_to_tol(ctx, d, V.GUESS_LEARNED, V.FP64),
            "learned_fp32_ir": time_to_tol(ctx, d, V.GUESS_LEARNED, V.FP32_IR),
        })
    keys = rows[0].keys()
    return {k: {"ms": round(float(np.mean([r[k]["ms"] for r in rows])), 4),
                "cycles": float(np.mean([r[k]["cycles"] for r in rows])),
                "rel_res0": float(np.mean([r[k]["rel_res0"] for r in rows])),
                "fallback": int(sum(r[k]["fallback"] for r in rows))} for k in keys}


def main():
    ap = argparse.ArgumentParser(description="train the learned Poisson warm start on solver snapshots")
    ap.add_argument("--n", type=int, default=160)
    ap.add_argument("--runs", type=int, default=8)
    ap.add_argument("--test-runs", type=int, default=2)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None, help="network file to write")
    a = ap.parse_args()
    V.load()
    ctx = V.Context()
    t = time.perf_counter()
    data = snapshots(ctx, I.warmstart_runs(5, a.runs), a.n, a.steps, a.every)
    test = snapshots(ctx, I.warmstart_runs(6, a.test_runs), a.n, a.steps, a.every)[-a.test_runs:]
    _log("[warmstart] %d training / %d test snapshots in %.1f s" % (len(data), len(test), time.perf_counter() - t))
    rep = train(ctx, data, I.NN_CFG, I.nn_init(1), a.seconds, a.lr)
    _log("[warmstart] trained: %s" % rep)
    if a.out:
        ctx.vd_nn_save(a.out)
    ev = evaluate(ctx, test)
    print(json.dumps({"train": rep, "eval": ev}), flush=True)


if __name__ == "__main__":
    main()
