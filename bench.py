#!/usr/bin/env python3
"""Benchmark of the semi-implicit plasma-fluid step on one MI355X.

Workload: the 15-species Ar-H2 streamer-shaped state on a 160^3 grid
(4,096,000 cells, dt = 1e-12 s, Te from the reduced-field table, electrode
plates at 15 kV / 0 V; seeded synthetic inputs from
paper_2507_08200_amd.inputs).  One step = Poisson solve, transport, WENO5
drift divergence with wall fluxes, chemistry and the batched implicit
species solve, all in libvd's HIP kernels.

Prints one JSON line: cell-steps/s, the roofline of the dominant kernel
(algorithmic bytes / HIP-event-timed duration over the timed region), the
Poisson time-to-1e-10 comparison and the FP64 CPU oracle timed on a bounded
sample on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-steps/s at 160^3×15 species; Poisson time-to-1e-10 plain vs learned+FP32"
HBM_PEAK_GBS = 8000.0
FAMILIES = ["gsrb", "gsrb_fine", "gsrb_uniform", "sweep", "resid_restrict", "prolong", "copy", "coarse", "norm", "finalize", "prep", "ir_update", "weno",
            "react", "transport", "rho", "guess", "setup"]
QE = 1.602176634e-19


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=160, help="grid edge (the workload is n^3)")
    # the 160^3 workload runs its multigrid smoothing in FP32 inside FP64
    # iterative refinement; the all-FP64 step is timed beside it
    ap.add_argument("--poisson-precision", choices=["fp64", "fp32_ir"], default="fp32_ir")
    ap.add_argument("--species-precision", choices=["fp64", "fp32_ir"], default="fp32_ir")
    ap.add_argument("--no-fp64-variant", action="store_true", help="skip the all-FP64 comparison run")
    ap.add_argument("--poisson-guess", choices=["extrap", "previous"], default="extrap",
                    help="Poisson initial guess: extrapolated in time from the last three potentials, or the "
                         "previous potential")
    ap.add_argument("--species-guess", choices=["extrap", "previous"], default="extrap",
                    help="species initial guesses: extrapolated from the last three steps, or the current "
                         "densities")
    ap.add_argument("--no-guess-variant", action="store_true",
                    help="skip the comparison run with the previous step's values as the guesses")
    ap.add_argument("--species-levels", type=int, default=1)
    ap.add_argument("--species-nu", type=int, nargs=2, default=(1, 0))
    ap.add_argument("--poisson-nu", type=int, nargs=2, default=(2, 2))
    ap.add_argument("--ir-inner", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default smoother tiling")
    ap.add_argument("--poisson-reps", type=int, default=5)
    ap.add_argument("--cpu-n", type=int, default=0,
                    help="grid edge of the oracle's timed sample (0: the workload's own grid, which also gives the "
                         "per-field error of the GPU step against the oracle)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", default="auto", help="kernel family for the roofline (auto = dominant)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batched Helmholtz timing")
    ap.add_argument("--nn-file", default=os.path.join(ROOT, "paper_2507_08200_amd", "warmstart_arh2_160.bin"),
                    help="trained warm-start network (trained in the benchmark if absent)")
    ap.add_argument("--nn-train-seconds", type=float, default=30.0)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess Poisson timing")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration under rocprofv3)")
    ap.add_argument("--batch-reps", type=int, default=3)
    return ap.parse_args()


def measured_traffic(family, alg_bytes_per_launch):
    """HBM bytes per launch of the kernel family: the committed rocprofv3
    counter summary gives the ratio of measured traffic (FETCH_SIZE and
    WRITE_SIZE, each scaled by a plain copy's reading) to algorithmic bytes
    over the same dispatches; it applies while the kernel source it was taken
    from is unchanged (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_hbm_traffic_arh2_160.txt" % family)
    if not os.path.exists(path) or not alg_bytes_per_launch:
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2507_08200_amd", "csrc", "mg.hip")
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha1") != sha or "traffic_to_algorithmic_ratio" not in fields:
        return None
    return round(float(fields["traffic_to_algorithmic_ratio"]) * alg_bytes_per_launch)


def learned_guess(ctx, V, I, cfg, rho, args):
    """Poisson time-to-1e-10 from the network's guess (inference included),
    FP64 and FP32-refined, on the benchmark's own streamer state (a voltage
    and seed position outside the training runs)."""
    import torch
    from paper_2507_08200_amd import warmstart as WS
    n = cfg["grid"][0]
    if os.path.exists(args.nn_file) and n == 160:
        ctx.vd_nn_load(args.nn_file)
        how = "loaded %s" % os.path.basename(args.nn_file)
    else:
        t = time.perf_counter()
        data = WS.snapshots(ctx, I.warmstart_runs(5, 4), n, 20, 10)
        rep = WS.train(ctx, data, I.NN_CFG, I.nn_init(1), args.nn_train_seconds, 1e-3)
        how = "trained in the benchmark: %d snapshots, %d Adam steps, %.0f s" % (len(data), rep["steps"],
                                                                                 time.perf_counter() - t)
    log("[bench] warm-start network: %s" % how)
    d = {"grid": cfg["grid"], "bc": cfg["phi_bc"], "rho": rho, "phi": torch.zeros_like(rho)}
    out = {"learned_fp64": WS.time_to_tol(ctx, d, V.GUESS_LEARNED, V.FP64, reps=args.poisson_reps),
           "learned_fp32_ir": WS.time_to_tol(ctx, d, V.GUESS_LEARNED, V.FP32_IR, reps=args.poisson_reps)}
    out["learned_network"] = how
    return out


def batch_bench(ctx, V, I, dev, reps):
    """The 64-problem batch (edges 32..160 in steps of 16, unit cube, alpha 1,
    a 1e-3..1 sheath jump, random Dirichlet/Neumann faces, N(0,1) rhs) solved
    to 1e-10 from zero: one call per problem, one batched call, and the
    batched call with graph replay and tile autotuning."""
    import numpy as np
    import torch
    probs = I.cfg4()
    cells = sum(p["grid"][0] ** 3 for p in probs)
    log("[bench] batch: %d problems, %d cells" % (len(probs), cells))
    gs = []
    for p in probs:
        gs.append({"grid": p["grid"], "bc": p["bc"], "mask": None, "alpha": None, "alpha_c": p["alpha_c"],
                   "beta": torch.tensor(p["beta"], device=dev), "beta_c": 0.0,
                   "rhs": torch.tensor(p["rhs"], device=dev), "x": torch.zeros(p["grid"][:3], dtype=torch.float64, device=dev)})
        p["beta"] = p["rhs"] = None

    def timed_solve(fn):
        ts, out = [], None
        for r in range(reps + 1):       # the first call builds hierarchies / captures / tunes
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            out = fn()
            e1.record()
            torch.cuda.synchronize()
            if r > 0:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), out

    def seq():
        return [ctx.vd_helmholtz_solve_batched([g], V.mg_opts(rtol=1e-10, guess=V.GUESS_ZERO))[0][0] for g in gs]

    def bat(**kw):
        return lambda: ctx.vd_helmholtz_solve_batched(gs, V.mg_opts(rtol=1e-10, guess=V.GUESS_ZERO, **kw))[0]

    res = {"problems": len(probs), "cells": cells, "rtol": 1e-10}
    ms, infos = timed_solve(seq)
    res["sequential_ms"] = round(ms, 3)
    res["cycles_max"] = max(i["cycles"] for i in infos)
    x_seq = [g["x"].clone() for g in gs]
    for name, kw in (("batched_ms", {}), ("batched_graph_ms", {"graph": True}),
                     ("batched_graph_autotune_ms", {"graph": True, "autotune": True})):
        ms, infos = timed_solve(bat(**kw))
        res[name] = round(ms, 3)
        # batching changes no arithmetic: same iterate as the sequential solves
        dmax = max(float((g["x"] - x).abs().max() / x.abs().max()) for g, x in zip(gs, x_seq))
        res[name.replace("_ms", "_max_rel_diff_vs_sequential")] = dmax
    res["cell_cycles_per_s_batched_graph"] = round(sum(i["cycles"] * p["grid"][0] ** 3 for i, p in zip(infos, probs))
                                                   / (res["batched_graph_ms"] * 1e-3), 1)
    log("[bench] batch: %s" % res)
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (requested --gpus %d, WORLD_SIZE %d)"
              % (args.gpus, world), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_08200_amd import inputs as I
    from paper_2507_08200_amd import mechanisms as M
    from paper_2507_08200_amd import vd as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    V.load()
    dev = "cuda:0"
    n = args.n
    cfg = I.cfg3(n=n)
    ncell = n ** 3
    log("[bench] building %d^3 x 15 state" % n)
    state = {k: torch.tensor(cfg[k], device=dev) for k in ("n", "phi", "Te")}
    lfa = dict(cfg["lfa"])
    lfa["te_K"] = torch.tensor(cfg["lfa"]["te_K"], device=dev)
    prec = {"fp64": V.FP64, "fp32_ir": V.FP32_IR}
    tune = not args.no_autotune
    pguess = V.GUESS_EXTRAP if args.poisson_guess == "extrap" else V.GUESS_GIVEN
    popts = V.mg_opts(rtol=1e-10, precision=prec[args.poisson_precision], ir_inner=args.ir_inner, autotune=tune,
                      guess=pguess, nu_pre=args.poisson_nu[0], nu_post=args.poisson_nu[1])
    sguess = V.GUESS_EXTRAP if args.species_guess == "extrap" else V.GUESS_GIVEN
    sopts = V.mg_opts(rtol=1e-10, precision=prec[args.species_precision], n_levels=args.species_levels,
                      nu_pre=args.species_nu[0], nu_post=args.species_nu[1], ir_inner=1, autotune=tune, guess=sguess)
    species = M.arh2_15()
    P = V.step_params(cfg, species, lfa=lfa, poisson=popts, species_mg=sopts)
    P64 = V.step_params(cfg, species, lfa=lfa, poisson=V.mg_opts(rtol=1e-10, autotune=tune, guess=pguess,
                                                                 nu_pre=args.poisson_nu[0], nu_post=args.poisson_nu[1]),
                        species_mg=V.mg_opts(rtol=1e-10, n_levels=args.species_levels, nu_pre=args.species_nu[0],
                                             nu_post=args.species_nu[1], autotune=tune, guess=sguess))
    state0 = {k: v.clone() for k, v in state.items()}
    ctx = V.Context()
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib * 2 ** 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration: 3 copies of %d MiB" % args.calibrate_copy_mib)

    # ---- warmup, with every kernel family timed to find the dominant one
    ctx.vd_timing_select(",".join(FAMILIES))
    infos = []
    for w in range(args.warmup):
        infos.append(ctx.vd_step(P, state))
        log("[bench] warmup step %d: %s" % (w, {k: infos[-1][k] for k in ("poisson_cycles", "species_cycles", "ms_total")}))
    torch.cuda.synchronize()
    prof = {}
    for f in FAMILIES:
        cnt, ms, by = ctx.vd_timing_read(f)
        if cnt:
            prof[f] = {"launches_per_step": cnt / max(1, args.warmup), "ms_per_step": ms / max(1, args.warmup),
                       "gb_per_s": (by / (ms * 1e-3) / 1e9) if ms > 0 and by > 0 else None}
    kernel = args.kernel
    if kernel == "auto":
        kernel = max(prof, key=lambda f: prof[f]["ms_per_step"]) if prof else "gsrb"
    log("[bench] per-family ms/step (warmup): %s" % {f: round(v["ms_per_step"], 3) for f, v in prof.items()})

    # ---- timed region: K steps; the dominant family is event-timed live
    ctx.vd_timing_select(kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc_p = cyc_s = 0
    for k in range(args.steps):
        ctx.vd_step(P, state, want_info=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    launches, kms, kbytes = ctx.vd_timing_read(kernel)
    ctx.vd_timing_select(None)
    info = ctx.vd_step(P, state)        # one more (untimed) step for the cycle counts
    cyc_p, cyc_s = info["poisson_cycles"], info["species_cycles"]
    ms_per_step = elapsed * 1e3 / args.steps
    value = ncell * args.steps / elapsed
    log("[bench] %d steps in %.3f s: %.3f ms/step, %.4g cell-steps/s" % (args.steps, elapsed, ms_per_step, value))

    # the same steps with every solve in FP64, from the same initial state
    fp64_variant = None
    if not args.no_fp64_variant:
        st64 = {k: v.clone() for k, v in state0.items()}
        for w in range(args.warmup):
            ctx.vd_step(P64, st64, want_info=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(args.steps):
            ctx.vd_step(P64, st64, want_info=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        i64 = ctx.vd_step(P64, st64)
        fp64_variant = {"value": round(ncell * args.steps / el, 1), "ms_per_step": round(el * 1e3 / args.steps, 4),
                        "poisson_cycles_last_step": i64["poisson_cycles"],
                        "species_cycles_last_step": i64["species_cycles"]}
        del st64
        log("[bench] all-FP64 variant: %s" % fp64_variant)

    # the same steps with the previous step's values as the guesses
    guess_variant = None
    if "extrap" in (args.poisson_guess, args.species_guess) and not args.no_guess_variant:
        PG = V.step_params(cfg, species, lfa=lfa, poisson=V.mg_opts(
            rtol=1e-10, precision=prec[args.poisson_precision], ir_inner=args.ir_inner, autotune=tune,
            nu_pre=args.poisson_nu[0], nu_post=args.poisson_nu[1]),
            species_mg=V.mg_opts(rtol=1e-10, precision=prec[args.species_precision], n_levels=args.species_levels,
                                 nu_pre=args.species_nu[0], nu_post=args.species_nu[1], ir_inner=1, autotune=tune))
        stg = {k: v.clone() for k, v in state0.items()}
        for w in range(args.warmup):
            ctx.vd_step(PG, stg, want_info=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(args.steps):
            ctx.vd_step(PG, stg, want_info=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ig = ctx.vd_step(PG, stg)
        guess_variant = {"value": round(ncell * args.steps / el, 1), "ms_per_step": round(el * 1e3 / args.steps, 4),
                         "poisson_cycles_last_step": ig["poisson_cycles"],
                         "species_cycles_last_step": ig["species_cycles"]}
        del stg
        log("[bench] previous-values guess variant: %s" % guess_variant)

    avg_ms = kms / launches if launches else 0.0
    achieved = (kbytes / launches) / (avg_ms * 1e-3) / 1e9 if launches and avg_ms > 0 else 0.0
    roofline = {"kernel": kernel, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kernel, kbytes / launches if launches else 0.0),
                "launches": launches, "avg_launch_us": round(avg_ms * 1e3, 3),
                "alg_bytes_per_launch": round(kbytes / launches) if launches else 0}

    # ---- Poisson time-to-1e-10 on the current streamer charge density
    Z = torch.tensor([s["Z"] for s in species], dtype=torch.float64, device=dev)
    rho = (QE * torch.tensordot(Z, state["n"], dims=1)).contiguous()
    phi_prev = state["phi"].clone()

    def poisson_time(precision, guess, x0, reps):
        times, info = [], None
        for r in range(reps):
            phi = x0.clone()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            info = ctx.vd_poisson_solve(cfg["grid"], cfg["phi_bc"], rho, phi, beta_c=8.8541878128e-12,
                                        opts=V.mg_opts(rtol=1e-10, precision=precision, guess=guess,
                                                       ir_inner=args.ir_inner))
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return {"ms": round(float(np.median(times)), 4), "cycles": info["cycles"], "outer": info["outer_iters"],
                "rel_res": info["rel_res"]}

    zero = torch.zeros_like(phi_prev)
    poisson = None if args.poisson_reps <= 0 else {
        "plain_fp64_zero_guess": poisson_time(V.FP64, V.GUESS_ZERO, zero, args.poisson_reps),
        "fp32_ir_zero_guess": poisson_time(V.FP32_IR, V.GUESS_ZERO, zero, args.poisson_reps),
        "plain_fp64_previous_step": poisson_time(V.FP64, V.GUESS_GIVEN, phi_prev, args.poisson_reps),
        "fp32_ir_previous_step": poisson_time(V.FP32_IR, V.GUESS_GIVEN, phi_prev, args.poisson_reps),
    }
    if poisson is not None and not args.no_learned:
        poisson.update(learned_guess(ctx, V, I, cfg, rho, args))
    log("[bench] poisson time-to-1e-10: %s" % poisson)

    # ---- 64 uneven sheath-jump Helmholtz problems: sequential vs batched
    batch = None if args.no_batch else batch_bench(ctx, V, I, dev, args.batch_reps)

    # ---- CPU baseline: the FP64 oracle on a bounded sample (one step of the
    # workload from its initial state), and the per-field error of the GPU
    # step from the same state against it
    cpu = None
    errors = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        O.build()
        cn = args.cpu_n if args.cpu_n > 0 else n
        ccfg = cfg if cn == n else I.cfg3(n=cn)
        log("[bench] oracle: one step at %d^3 on one host core" % cn)
        t = time.perf_counter()
        r = O.step(ccfg, O.species_arh2_15(), poisson=O.mg_opts(rtol=1e-10), species_mg=O.mg_opts(rtol=1e-10))
        dt_cpu = time.perf_counter() - t
        assert r["status"] == 0
        cpu = {"value": round(cn ** 3 / dt_cpu, 1), "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
               "sample": "one FP64 oracle step of the same Ar-H2 streamer workload at %d^3 (%d cells) from its initial "
                         "state (cold Poisson start, %d Poisson cycles), single-threaded, %.1f s; scaled per cell" %
                         (cn, cn ** 3, r["info"]["poisson_cycles"], dt_cpu),
               "host_cpus_available": len(os.sched_getaffinity(0))}
        log("[bench] oracle %.2f s -> %.4g cell-steps/s" % (dt_cpu, cpu["value"]))
        if cn == n:
            errors = {}
            for tag, PP in (("fp32_ir_step", P), ("fp64_step", P64)):
                st = {k: v.clone() for k, v in state0.items()}
                inf = ctx.vd_step(PP, st)
                assert inf["status"] == 0

                def rel(a, b):
                    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
                e = {"phi": rel(st["phi"].cpu().numpy(), r["phi"]), "Te": rel(st["Te"].cpu().numpy(), r["Te"])}
                nn = st["n"].cpu().numpy()
                for k2, sp in enumerate(M.ARH2_NAMES):
                    e["n_" + sp] = rel(nn[k2], r["n"][k2])
                errors[tag] = {f: float("%.3g" % v) for f, v in e.items()}
                errors[tag]["max"] = max(errors[tag].values())
                del st, nn
            log("[bench] error vs the FP64 oracle (max |gpu - oracle| / max |oracle| per field): %s" % errors)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32" if "fp32" in args.poisson_precision + args.species_precision else "f64",
        "data": "synthetic",
        "config": {"workload": "Ar-H2 15-species streamer step, %d^3 cells, dt 1e-12 s, LFA Te, 15 kV plates" % n,
                   "grid": [n, n, n], "species": 15, "dt": 1e-12,
                   "poisson": "%s%s V(%d,%d) rtol 1e-10, guess %s%s" % (
                       args.poisson_precision, " inner %d" % args.ir_inner if args.poisson_precision == "fp32_ir" else "",
                       args.poisson_nu[0], args.poisson_nu[1],
                       "extrapolated from the last three potentials" if args.poisson_guess == "extrap"
                       else "the previous potential", ", autotuned tiles" if tune else ""),
                   "species_solve": "%s levels %d nu %s rtol 1e-10, guess %s" % (
                       args.species_precision, args.species_levels, list(args.species_nu),
                       "extrapolated from the last three steps" if args.species_guess == "extrap"
                       else "the current densities"),
                   "mg_inner_dtype": "f32" if "fp32" in args.poisson_precision + args.species_precision else "f64",
                   "poisson_cycles_last_step": cyc_p, "species_cycles_last_step": cyc_s},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_variant": fp64_variant,
        "previous_values_guess_variant": guess_variant,
        "error_vs_fp64_oracle": errors,
        "poisson_time_to_1e-10": poisson,
        "batched_helmholtz_64": batch,
        "kernel_profile_warmup": prof,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
