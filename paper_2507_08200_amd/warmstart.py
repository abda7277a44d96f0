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


def snapshots(ctx, runs, n, steps, every, dev="cuda:0", keep_solver_inputs=False):
    """[{"x": features bf16 [n,n,n,2], "t": target f32 [n,n,n], ...}] from
    solver runs: each run is stepped `steps` times (FP32-refined solves to
    1e-10 from extrapolated guesses) and every `every`-th step kept.  With
    keep_solver_inputs the charge density, the potential, the previous
    step's potential, the boundary and the grid are kept too (held-out
    evaluation)."""
    species = M.arh2_15()
    Z = torch.tensor([s["Z"] for s in species], dtype=torch.float64, device=dev)
    out = []
    t0 = time.perf_counter()
    for ir, r in enumerate(runs):
        cfg = I.cfg3(seed=r["seed"], n=n, voltage=r["voltage"], seed_centre=r["centre"])
        state = {k: torch.tensor(cfg[k], device=dev) for k in ("n", "phi", "Te")}
        lfa = dict(cfg["lfa"])
        lfa["te_K"] = torch.tensor(cfg["lfa"]["te_K"], device=dev)
        P = V.step_params(cfg, species, lfa=lfa,
                          poisson=V.mg_opts(rtol=1e-10, precision=V.FP32_IR, guess=V.GUESS_EXTRAP, ir_inner=1),
                          species_mg=V.mg_opts(rtol=1e-10, n_levels=1, nu_pre=1, nu_post=0, precision=V.FP32_IR,
                                               guess=V.GUESS_EXTRAP))
        ctx.vd_step_reset()
        prev = None
        for k in range(steps):
            if keep_solver_inputs and (k + 2) % every == 0:
                prev = state["phi"].clone()
            ctx.vd_step(P, state, want_info=False)
            if (k + 1) % every == 0:
                rho = (QE * torch.tensordot(Z, state["n"], dims=1)).contiguous()
                feats, vref = ctx.vd_nn_features(cfg["grid"], cfg["phi_bc"], rho, eps=EPS0)
                d = {"x": feats, "t": (state["phi"] / vref).float().contiguous(), "grid": cfg["grid"], "vref": vref}
                if keep_solver_inputs:
                    d.update({"rho": rho, "phi": state["phi"].clone(), "phi_prev": prev, "bc": cfg["phi_bc"]})
                out.append(d)
        if (ir + 1) % 10 == 0 or ir + 1 == len(runs):
            _log("[warmstart] %d/%d runs, %d snapshots, %.0f s" % (ir + 1, len(runs), len(out), time.perf_counter() - t0))
    return out


def train(ctx, data, cfg, params, seconds, lr, seed=0, max_steps=None, lr_final=None):
    """Adam on the mean squared error, samples in a seeded random order
    (reshuffled every epoch), until the time budget (or max_steps) is
    spent; the learning rate falls linearly with elapsed time to lr_final
    (default lr / 10)."""
    ctx.vd_nn_create(cfg, params)
    rng = np.random.default_rng(seed)
    lr_final = lr / 10 if lr_final is None else lr_final
    t0 = time.perf_counter()
    tlog = t0
    losses = []
    it = epochs = 0
    while True:
        for i in rng.permutation(len(data)):
            d = data[i]
            el = time.perf_counter() - t0
            rate = lr + (lr_final - lr) * min(1.0, el / seconds)
            loss = ctx.vd_nn_train_step(d["grid"], d["x"], d["t"], rate, update=True)
            losses.append(loss)
            it += 1
            if time.perf_counter() - tlog > 30:
                tlog = time.perf_counter()
                _log("[warmstart] step %d epoch %d loss %.4g lr %.2g (%.0f s)" % (it, epochs, float(np.mean(losses[-50:])), rate,
                                                                                  tlog - t0))
            if time.perf_counter() - t0 > seconds or (max_steps and it >= max_steps):
                return {"steps": it, "epochs": round(it / len(data), 2), "seconds": round(time.perf_counter() - t0, 2),
                        "loss_first": losses[0], "loss_last50": float(np.mean(losses[-50:]))}
        epochs += 1


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
    """Poisson solve to 1e-10 on each held-out snapshot: plain FP64 and
    FP32-refined from zero, from the previous step's potential, and from
    the network's guess (inference in the timed region); means over the
    snapshots."""
    rows = []
    for d in test:
        rows.append({
            "plain_fp64_zero_guess": time_to_tol(ctx, d, V.GUESS_ZERO, V.FP64),
            "fp32_ir_zero_guess": time_to_tol(ctx, d, V.GUESS_ZERO, V.FP32_IR),
            "fp32_ir_previous_step_guess": time_to_tol(ctx, d, V.GUESS_GIVEN, V.FP32_IR, phi0=d["phi_prev"]),
            "learned_fp64": time_to_tol(ctx, d, V.GUESS_LEARNED, V.FP64),
            "learned_fp32_ir": time_to_tol(ctx, d, V.GUESS_LEARNED, V.FP32_IR),
        })
    keys = rows[0].keys()
    return {k: {"ms": round(float(np.mean([r[k]["ms"] for r in rows])), 4),
                "cycles": float(np.mean([r[k]["cycles"] for r in rows])),
                "rel_res0": float(np.mean([r[k]["rel_res0"] for r in rows])),
                "fallback": int(sum(r[k]["fallback"] for r in rows))} for k in keys}


NET_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_arh2_160.bin")


def kernel_run(ctx, forwards, train_steps, n=160):
    """The network's kernels on one held-out 160^3 snapshot (for kernel
    traces and counters): `forwards` inferences of the stored network, then
    `train_steps` gradient evaluations (no update)."""
    d = snapshots(ctx, I.warmstart_runs(7, 1), n, 20, 20)[-1]
    ctx.vd_nn_load(NET_FILE)
    for _ in range(forwards):
        ctx.vd_nn_forward(d["grid"], d["x"])
    for _ in range(train_steps):
        ctx.vd_nn_train_step(d["grid"], d["x"], d["t"], 0.0, update=False)
    torch.cuda.synchronize()
    _log("[warmstart] %d forwards, %d gradient evaluations done" % (forwards, train_steps))


def main():
    ap = argparse.ArgumentParser(description="train the learned Poisson warm start on solver snapshots")
    ap.add_argument("--kernels", type=int, nargs=2, metavar=("FORWARDS", "GRADIENTS"), default=None,
                    help="only run the stored network's kernels on one snapshot (for profiling)")
    ap.add_argument("--n", type=int, default=160)
    ap.add_argument("--runs", type=int, default=100)
    ap.add_argument("--test-runs", type=int, default=10)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--every", type=int, default=5)
    ap.add_argument("--seconds", type=float, default=600.0)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None, help="network file to write")
    a = ap.parse_args()
    V.load()
    ctx = V.Context()
    if a.kernels:
        kernel_run(ctx, a.kernels[0], a.kernels[1], a.n)
        return
    t = time.perf_counter()
    data = snapshots(ctx, I.warmstart_runs(5, a.runs), a.n, a.steps, a.every)
    # held-out runs: other voltages and seed positions; their last snapshot
    test = []
    for r in I.warmstart_runs(6, a.test_runs):
        test += snapshots(ctx, [r], a.n, a.steps, a.every, keep_solver_inputs=True)[-1:]
    _log("[warmstart] %d training / %d held-out snapshots in %.1f s" % (len(data), len(test), time.perf_counter() - t))
    rep = train(ctx, data, I.NN_CFG, I.nn_init(1), a.seconds, a.lr)
    _log("[warmstart] trained: %s" % rep)
    if a.out:
        ctx.vd_nn_save(a.out)
    del data
    torch.cuda.empty_cache()
    ev = evaluate(ctx, test)
    print(json.dumps({"config": I.NN_CFG, "runs": a.runs, "test_runs": a.test_runs, "steps": a.steps, "every": a.every,
                      "train": rep, "eval": ev}), flush=True)


if __name__ == "__main__":
    main()
