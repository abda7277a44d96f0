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
Poisson time-to-1e-10 comparison, the 64-problem batched Helmholtz solve
with its roofline, the per-field error of GPU trajectories against FP64
oracle trajectories, and the FP64 CPU oracle timed on a warm step on all
host cores and on one.
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
    ap.add_argument("--no-widened", action="store_true",
                    help="skip the timings of the step with photoionization, surface charge / emission / adaptive "
                         "step, and an interior masked electrode")
    ap.add_argument("--no-guess-variant", action="store_true",
                    help="skip the comparison run with the previous step's values as the guesses")
    ap.add_argument("--species-levels", type=int, default=1)
    ap.add_argument("--species-nu", type=int, nargs=2, default=(1, 0))
    ap.add_argument("--poisson-nu", type=int, nargs=2, default=(2, 2))
    ap.add_argument("--ir-inner", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default smoother tiling")
    ap.add_argument("--poisson-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip every oracle leg")
    ap.add_argument("--traj-n", type=int, default=64, help="grid edge of the long accuracy trajectory")
    ap.add_argument("--traj-steps", type=int, default=100)
    ap.add_argument("--traj160-steps", type=int, default=5,
                    help="steps of the accuracy trajectory on the workload's own grid (its last oracle step is the "
                         "CPU baseline)")
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


def widened_variants(ctx, V, I, cfg, species, lfa, popts, sopts, state0, args, dev):
    """The same workload and solver options with each widened row switched
    on, from the same initial state: warmup steps, then timed steps
    (ms/step, cell-steps/s, cycles of the last step).  Photoionization:
    three Helmholtz terms with synthetic coefficients (A_j, lambda_j of the
    three-exponential form, p_O2 = 150 Torr, p = p_g = 760 Torr, p_q = 30
    Torr, xi = 0.06) into the electrons and Ar+, solved in FP64.  Surface charge: the y- face
    dielectric (sigma from 0), secondary emission gamma = 0.1, Eq. (20)
    limits with c_adv 0.3, c_diff 10, c_diel 0.5 and dt as their cap.
    Masked: a grounded post (covered box of n/8 x n/8 x n/8 cells at 0 V)
    three quarters of the way to the x+ plate."""
    import torch
    from paper_2507_08200_amd import mechanisms as M
    n = cfg["grid"][0]
    ncell = n ** 3
    steps = min(args.steps, 20)
    out = {}

    def run(tag, P, note, fam=None, init=None):
        st = {k: v.clone() for k, v in (init or state0).items()}
        ctx.vd_step_reset()
        for w in range(args.warmup):
            ctx.vd_step(P, st, want_info=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(steps):
            ctx.vd_step(P, st, want_info=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        if fam:
            ctx.vd_timing_select(fam)
        inf = ctx.vd_step(P, st)
        r = {"ms_per_step": round(el * 1e3 / steps, 4), "value": round(ncell * steps / el, 1), "steps": steps,
             "poisson_cycles_last_step": inf["poisson_cycles"], "species_cycles_last_step": inf["species_cycles"],
             "dt_used": inf["dt_used"], "note": note}
        if fam:
            r["family_ms_last_step"] = {}
            for f in fam.split(","):
                c, ms, by = ctx.vd_timing_read(f)
                if c:
                    r["family_ms_last_step"][f] = round(ms, 4)
            ctx.vd_timing_select(None)
        out[tag] = r
        log("[bench] widened %s: %s" % (tag, r))
        del st

    ph = {"A": [1.4e3, 2.6e4, 3.3e5], "lam": [21.0, 70.0, 330.0], "pO2": 150.0, "pg": 760.0, "xi": 0.06,
          "pq": 30.0, "p": 760.0, "e": 0, "ion": 1, "bc": I.bc([I.BC_DIRICHLET] * 6),
          "mg": V.mg_opts(rtol=1e-10, precision=V.FP32_IR)}
    run("photoionization", V.step_params(cfg, species, lfa=lfa, poisson=popts, species_mg=sopts, photo=ph),
        "NEXT-1: three photoionization Helmholtz terms (synthetic coefficients), FP32-in-FP64 refinement to 1e-10 "
        "from the previous step's terms, each term solved in units of a power of two near its largest right-hand "
        "side (~1e38 m^-3 s^-1 here)")
    sig = torch.zeros(n * n, dtype=torch.float64, device=dev)
    run("surface_charge_emission_adaptive_dt",
        V.step_params(cfg, species, lfa=lfa, poisson=popts, species_mg=sopts, diel=[0, 0, 1, 0, 0, 0], sigma=sig,
                      see_gamma=0.1, adaptive_dt={"c_adv": 0.3, "c_diff": 10.0, "c_diel": 0.5}, electron=0),
        "NEXT-3 and a12: y- face dielectric, gamma 0.1, Eq. (20) step capped at dt")
    mask = torch.ones((n, n, n), dtype=torch.uint8, device=dev)
    a, b = n * 3 // 4, n * 3 // 4 + n // 8
    c0, c1 = n * 7 // 16, n * 7 // 16 + n // 8
    mask[c0:c1, c0:c1, a:b] = 0
    init = {k: v.clone() for k, v in state0.items()}
    init["phi"][mask == 0] = 0.0
    run("masked_electrode", V.step_params(cfg, species, lfa=lfa, poisson=popts, species_mg=sopts, mask=mask),
        "NEXT-2: %d covered cells (a grounded post); drift: the tiled kernel, then the masked per-cell function on "
        "the cells within three of a covered cell" % int((mask == 0).sum().item()),
        fam=",".join(FAMILIES), init=init)
    del init
    return out


MG_FAMILIES = ["gsrb", "gsrb_fine", "gsrb_uniform", "sweep", "resid_restrict", "prolong", "copy", "coarse", "norm",
               "finalize", "prep", "ir_update", "setup"]


def batch_bench(ctx, V, I, dev, reps, oracle_sample=True):
    """The 64-problem batch (edges 32..160 in steps of 16, unit cube, alpha 1,
    a 1e-3..1 sheath jump, random Dirichlet/Neumann faces, N(0,1) rhs) solved
    to 1e-10 from zero: one call per problem, one batched call, and the
    batched call with graph replay and tile autotuning, with the tuned
    smoothing schedule and with FP32 refinement; then the small problems
    alone, plain, with graph replay and with persistent colour passes."""
    import numpy as np
    import torch
    probs = I.cfg4()
    cells = sum(p["grid"][0] ** 3 for p in probs)
    log("[bench] batch: %d problems, %d cells" % (len(probs), cells))
    # the oracle's sample: the two smallest problems, kept on the host
    order = sorted(range(len(probs)), key=lambda q: probs[q]["grid"][0] ** 3)
    sample = [dict(probs[q], beta=probs[q]["beta"].copy(), rhs=probs[q]["rhs"].copy()) for q in order[:2]]
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
                     ("batched_graph_autotune_ms", {"graph": True, "autotune": True}),
                     ("batched_tuned_schedule_ms", {"tune_nu": True})):
        ms, infos = timed_solve(bat(**kw))
        if name == "batched_graph_ms":
            infos_graph = infos
        res[name] = round(ms, 3)
        # batching changes no arithmetic: same iterate as the sequential solves
        dmax = max(float((g["x"] - x).abs().max() / x.abs().max()) for g, x in zip(gs, x_seq))
        if name == "batched_tuned_schedule_ms":
            # another smoothing schedule changes the iterates: report it and
            # its residuals instead of a comparison with the sequential solves
            res["tuned_schedule"] = [infos[0]["nu_pre"], infos[0]["nu_post"]]
            res["tuned_schedule_cycles_max"] = max(i["cycles"] for i in infos)
            res["tuned_schedule_max_rel_res"] = max(i["rel_res"] for i in infos)
        else:
            res[name.replace("_ms", "_max_rel_diff_vs_sequential")] = dmax
    # FP32 multigrid inside FP64 refinement on the same batch (same 1e-10)
    ms, infos = timed_solve(bat(precision=V.FP32_IR))
    res["batched_fp32_ir_ms"] = round(ms, 3)
    res["batched_fp32_ir_max_rel_res"] = max(i["rel_res"] for i in infos)
    # the batch's small problems (edges 32 and 48) alone: short launches,
    # where the host's launch rate rather than HBM bounds a cycle
    small = [g for g in gs if g["grid"][0] <= 48]
    x_small = None
    sm = {"problems": len(small), "cells": sum(g["grid"][0] ** 3 for g in small)}
    for name, kw in (("batched_ms", {}), ("batched_graph_ms", {"graph": True}),
                     ("batched_persistent_graph_ms", {"graph": True, "persistent": True})):
        ms, _ = timed_solve(lambda: ctx.vd_helmholtz_solve_batched(
            small, V.mg_opts(rtol=1e-10, guess=V.GUESS_ZERO, **kw))[0])
        sm[name] = round(ms, 3)
        xs = [g["x"].clone() for g in small]
        if x_small is None:
            x_small = xs
        else:
            sm[name.replace("_ms", "_max_rel_diff_vs_batched")] = max(
                float((a - b).abs().max() / b.abs().max()) for a, b in zip(xs, x_small))
    res["small_problems"] = sm
    infos = infos_graph
    cell_cycles = sum(i["cycles"] * p["grid"][0] ** 3 for i, p in zip(infos, probs))
    res["cell_cycles_per_s_batched_graph"] = round(cell_cycles / (res["batched_graph_ms"] * 1e-3), 1)
    # roofline of the batched solve: the algorithmic bytes of all its
    # multigrid launches (read from the library's per-family accounting in
    # one event-timed call) over the untimed batched call's duration
    ctx.vd_timing_select(",".join(MG_FAMILIES))
    bat()()
    torch.cuda.synchronize()
    alg = kms = 0.0
    for f in MG_FAMILIES:
        cnt, ms_f, by = ctx.vd_timing_read(f)
        alg += by
        kms += ms_f
    ctx.vd_timing_select(None)
    ach = alg / (res["batched_ms"] * 1e-3) / 1e9
    res["roofline"] = {"bound": "hbm", "alg_bytes_per_solve": round(alg), "achieved": round(ach, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                       "event_timed_kernel_ms": round(kms, 3),
                       "note": "algorithmic bytes of every multigrid launch of one batched solve / batched_ms"}
    if oracle_sample:
        res["oracle"] = batch_oracle(sample, infos, probs, order, cell_cycles)
    log("[bench] batch: %s" % res)
    return res


def batch_oracle(sample, infos, probs, order, cell_cycles):
    """The FP64 oracle solving the batch's two smallest problems one after
    the other from zero to 1e-10, single-threaded and on all host cores; the
    whole 64-problem sequential time is extrapolated from the measured cell
    cycles per second and the cycle counts of the GPU's solves."""
    import numpy as np
    from oracle import oracle as O
    out = {"sample": "problems %s (edges %s), solved one after the other" % (
        [int(q) for q in order[:len(sample)]], [p["grid"][0] for p in sample])}
    for tag, par in (("single_core", False), ("all_cores", True)):
        t = time.perf_counter()
        cc = 0
        for p in sample:
            x, info, st = O.mg_solve(p, p["rhs"], np.zeros(p["rhs"].shape), parallel=par, rtol=1e-10)
            assert st == 0
            cc += info["cycles"] * p["grid"][0] ** 3
        el = time.perf_counter() - t
        rate = cc / el
        out[tag] = {"ms": round(el * 1e3, 1), "cell_cycles_per_s": round(rate, 1),
                    "cores": 1 if not par else int(os.environ.get("OMP_NUM_THREADS", "1")),
                    "batch_ms_extrapolated": round(cell_cycles / rate * 1e3, 1)}
    return out


def field_errors(names, got, want):
    """Per field: max |gpu - oracle| / max |oracle| and the pointwise
    max |gpu - oracle| / max(|oracle|, 1e-6 max |oracle|)."""
    import numpy as np
    out = {}
    for name, g, w in zip(names, got, want):
        sc = np.abs(w).max()
        if sc == 0:
            out[name] = [float("%.3g" % np.abs(g).max())] * 2
            continue
        d = np.abs(g - w)
        out[name] = [float("%.3g" % (d.max() / sc)), float("%.3g" % (d / np.maximum(np.abs(w), 1e-6 * sc)).max())]
    out["max"] = [max(v[0] for v in out.values()), max(v[1] for v in out.values())]
    return out


def oracle_legs(args, ctx, V, I, M, P, P64, state0, cfg, n, dev):
    """GPU trajectories of the timed configuration (FP32-refined and all
    FP64) against FP64 oracle trajectories with the same solver schedule,
    tolerance and extrapolated guesses (formed from the oracle's own
    results): args.traj_steps steps at args.traj_n^3 and args.traj160_steps
    steps at the workload's grid.  The oracle's last step of the latter,
    a warm step like the timed ones, is the CPU baseline on all host cores;
    one more step from that state on one core is the single-core figure."""
    import numpy as np
    import torch
    from oracle import oracle as O
    O.build()
    O.build(parallel=True)
    threads = int(os.environ["OMP_NUM_THREADS"])
    names = ["phi", "Te"] + ["n_" + sp for sp in M.ARH2_NAMES]
    po, so = P.poisson, P.species_mg
    oP = O.mg_opts(rtol=po.rtol, nu_pre=po.nu_pre, nu_post=po.nu_post, n_levels=po.n_levels)
    oS = O.mg_opts(rtol=so.rtol, nu_pre=so.nu_pre, nu_post=so.nu_post, n_levels=so.n_levels)
    sp = O.species_arh2_15()

    def gpu_traj(PP, c, steps):
        st = {k: torch.tensor(c[k], device=dev) for k in ("n", "phi", "Te")}
        ctx.vd_step_reset()
        for t in range(steps):
            inf = ctx.vd_step(PP, st)
            assert inf["status"] == 0
        out = [st["phi"].cpu().numpy(), st["Te"].cpu().numpy()] + list(st["n"].cpu().numpy())
        del st
        return out

    errors = {"oracle": "FP64 oracle trajectory, Poisson V(%d,%d) and species %d-level V(%d,%d) to %.0e, "
                        "starting iterates extrapolated from its own results; [max-scaled, pointwise with a 1e-6 "
                        "floor] per field" % (po.nu_pre, po.nu_post, so.n_levels, so.nu_pre, so.nu_post, po.rtol)}
    legs = [(args.traj_n, args.traj_steps)]
    if args.traj160_steps > 0:
        legs.append((n, args.traj160_steps))
    warm = None
    for gn, steps in legs:
        c = cfg if gn == n else I.cfg3(n=gn)
        log("[bench] oracle trajectory: %d steps at %d^3 on %d threads" % (steps, gn, threads))
        t = time.perf_counter()
        ref = O.trajectory(c, sp, steps, poisson=oP, species_mg=oS, parallel=True)
        log("[bench]   %.1f s (last step %.2f s)" % (time.perf_counter() - t, ref["times"][-1]))
        want = [ref["phi"], ref["Te"]] + list(ref["n"])
        tight = None
        if gn != n:
            # the oracle's own tolerance error: the same trajectory with
            # every solve taken to 1e-13
            oPt = O.mg_opts(rtol=1e-13, nu_pre=po.nu_pre, nu_post=po.nu_post, n_levels=po.n_levels, max_cycles=200)
            oSt = O.mg_opts(rtol=1e-13, nu_pre=so.nu_pre, nu_post=so.nu_post, n_levels=so.n_levels, max_cycles=200)
            rt = O.trajectory(c, sp, steps, poisson=oPt, species_mg=oSt, parallel=True)
            tight = field_errors(names, want, [rt["phi"], rt["Te"]] + list(rt["n"]))
            del rt
        PPc = V.step_params(c, M.arh2_15(), lfa=lfa_dev(c, dev), poisson=P.poisson, species_mg=P.species_mg)
        PP64 = V.step_params(c, M.arh2_15(), lfa=lfa_dev(c, dev), poisson=P64.poisson, species_mg=P64.species_mg)
        key = "trajectory_%d^3_%d_steps" % (gn, steps)
        errors[key] = {"fp32_ir": field_errors(names, gpu_traj(PPc, c, steps), want),
                       "fp64": field_errors(names, gpu_traj(PP64, c, steps), want),
                       "oracle_cycles_last_step": {k: ref["infos"][-1][k] for k in ("poisson_cycles", "species_cycles")}}
        if tight is not None:
            errors[key]["oracle_1e-10_vs_oracle_1e-13"] = tight
        log("[bench]   error %s: fp32_ir max %s, fp64 max %s" % (key, errors[key]["fp32_ir"]["max"],
                                                                 errors[key]["fp64"]["max"]))
        if gn == n:
            warm = ref
    cpu = None
    if warm is not None:
        t_all = warm["times"][-1]
        # the trajectory's last step again, from the same inputs and guesses,
        # on a single core
        t = time.perf_counter()
        r1 = O.step(cfg, sp, poisson=oP, species_mg=oS, **warm["last_step_inputs"])
        t_one = time.perf_counter() - t
        assert r1["status"] == 0 and r1["info"] == warm["infos"][-1]
        cpu = {"value": round(n ** 3 / t_all, 1), "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
               "sample": "step %d of the FP64 oracle trajectory of the same %d^3 workload (warm: starting iterates "
                         "extrapolated from its earlier steps, %d Poisson cycles), OpenMP on %d threads, %.2f s" %
                         (len(warm["times"]), n, warm["infos"][-1]["poisson_cycles"], threads, t_all),
               "single_core": {"value": round(n ** 3 / t_one, 1), "cores": 1,
                               "sample": "the same step from the same inputs and guesses, single-threaded, %.2f s" %
                                         t_one},
               "host_cpus_available": len(os.sched_getaffinity(0))}
        log("[bench] oracle warm step: %.4g cell-steps/s on %d threads, %.4g on one core" %
            (cpu["value"], threads, cpu["single_core"]["value"]))
    return errors, cpu


def lfa_dev(c, dev):
    import torch
    lfa = dict(c["lfa"])
    lfa["te_K"] = torch.tensor(c["lfa"]["te_K"], device=dev)
    return lfa


def main():
    args = parse()
    os.environ.setdefault("OMP_NUM_THREADS", str(len(os.sched_getaffinity(0))))
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the step has no multi-GPU path (requested --gpus %d, WORLD_SIZE %d)"
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
            torch.add(src, 1.0, out=dst)       # one elementwise kernel: reads and writes the size once
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration: 3 copies of %d MiB" % args.calibrate_copy_mib)

    # ---- warmup; every kernel family is timed over the later warmup steps
    # (the first steps start the extrapolation histories and take more
    # cycles than the steady state) to find the dominant one
    infos = []
    n_prof = max(1, args.warmup // 2)
    for w in range(args.warmup):
        if w == args.warmup - n_prof:
            torch.cuda.synchronize()
            ctx.vd_timing_select(",".join(FAMILIES))
        infos.append(ctx.vd_step(P, state))
        log("[bench] warmup step %d: %s" % (w, {k: infos[-1][k] for k in ("poisson_cycles", "species_cycles", "ms_total")}))
    torch.cuda.synchronize()
    prof = {}
    for f in FAMILIES:
        cnt, ms, by = ctx.vd_timing_read(f)
        if cnt:
            prof[f] = {"launches_per_step": cnt / n_prof, "ms_per_step": ms / n_prof,
                       "gb_per_s": (by / (ms * 1e-3) / 1e9) if ms > 0 and by > 0 else None}
    kernel = args.kernel
    if kernel == "auto":
        kernel = max(prof, key=lambda f: prof[f]["ms_per_step"]) if prof else "gsrb"
    log("[bench] per-family ms/step (last %d warmup steps): %s" % (n_prof, {f: round(v["ms_per_step"], 3) for f, v in prof.items()}))

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

    widened = None if args.no_widened else widened_variants(ctx, V, I, cfg, species, lfa, popts, sopts, state0, args, dev)

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
    batch = None if args.no_batch else batch_bench(ctx, V, I, dev, args.batch_reps,
                                                    oracle_sample=not args.no_cpu_baseline)

    # ---- accuracy against the FP64 oracle over trajectories of the timed
    # configuration, and the oracle timed on the same kind of warm step
    cpu = None
    errors = None
    if not args.no_cpu_baseline:
        errors, cpu = oracle_legs(args, ctx, V, I, M, P, P64, state0, cfg, n, dev)

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
                   "background_gas": "Ar and H2 transported like the other 13 species (the paper holds the "
                                     "background constant)",
                   "mg_inner_dtype": "f32" if "fp32" in args.poisson_precision + args.species_precision else "f64",
                   "poisson_cycles_last_step": cyc_p, "species_cycles_last_step": cyc_s},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_variant": fp64_variant,
        "previous_values_guess_variant": guess_variant,
        "widened_rows": widened,
        "error_vs_fp64_oracle": errors,
        "poisson_time_to_1e-10": poisson,
        "batched_helmholtz_64": batch,
        "kernel_profile_warmup": prof,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
