"""More of the step on the GPU against the FP64 oracle.

* The electron-energy step at a size that runs the tiled WENO5 kernel
  (64 x 32 x 32), at pinned cycle counts (1e-12), and in tolerance mode with
  every solve FP32-refined, judged by the oracle's own residuals.
* The step's optional inputs: extra species and energy sources and a
  permittivity field, at pinned cycle counts.
* The path the benchmark times (FP32-refined Poisson V(2,2), single-level
  FP32-refined species V(1,0), both from guesses extrapolated in time) over
  several steps at 64^3: the oracle recomputes, from each step's starting
  state, the Poisson and species residuals of the GPU's results and checks
  them against the tolerance; the trajectory is compared with an oracle
  trajectory of plain solves from the previous values.

Errors are reported max-scaled (max |gpu - oracle| / max |oracle|) and
pointwise (|gpu - oracle| / max(|oracle|, 1e-6 max |oracle|))."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import dev, host, rel_err, rel_err_pointwise, say  # noqa: E402
from paper_2507_08200_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12
# pointwise bar of the pinned-cycle comparisons: |gpu - oracle| <= 1e-10 |oracle|
# in every cell whose value is at least 1e-6 of the field's largest (below
# that, 1e-16 of the largest in absolute terms)
PW_TOL = 1e-10
M_AR = 39.948 * 1.66053906660e-27
KB = 1.380649e-23


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_08200_amd import vd
    vd.load()
    return vd


@pytest.fixture(scope="module")
def ctx(V):
    return V.Context()


def _lfa(cfg):
    if "lfa" not in cfg:
        return None
    lfa = dict(cfg["lfa"])
    lfa["te_K"] = dev(cfg["lfa"]["te_K"])
    return lfa


def _errors(state, ref, names=("n", "phi", "Te", "Ee")):
    out = {}
    for k in names:
        if k not in state or ref.get(k) is None:
            continue
        g = host(state[k])
        if k == "n":
            for s in range(g.shape[0]):
                if np.abs(ref["n"][s]).max() > 0:
                    out["n%d" % s] = (rel_err(g[s], ref["n"][s]), rel_err_pointwise(g[s], ref["n"][s]))
        else:
            out[k] = (rel_err(g, ref[k]), rel_err_pointwise(g, ref[k]))
    return out


def _show(tag, errs):
    say(tag, {k: "%.1e/%.1e" % v for k, v in errs.items()})


def _energy_cfg(nx, ny, nz):
    cfg = I.cfg3(n=nx, ny=ny, nz=nz)
    cfg["te_mode"] = I.TE_ENERGY
    ne = cfg["n"][0]
    Ee = 1.5 * ne * KB * 23209.0
    return cfg, Ee


def test_step_energy_tiled_pinned(ctx, V, oracle):
    """64 x 32 x 32: the WENO5 divergence of the species and of the electron
    energy (with its wall flux 2 kB Te Gamma_e) runs in the LDS-tiled kernel;
    pinned cycle counts, 1e-12 of every field."""
    from paper_2507_08200_amd import mechanisms as M
    cfg, Ee = _energy_cfg(64, 32, 32)
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    state["Ee"] = dev(Ee)
    fx = dict(fixed_cycles=10)
    P = V.step_params(cfg, M.arh2_15(), lfa=_lfa(cfg), poisson=V.mg_opts(**fx), species_mg=V.mg_opts(fixed_cycles=2),
                      energy_mg=V.mg_opts(fixed_cycles=2), electron=0, m_bg=M_AR)
    say("energy step 64x32x32 pinned")
    info = ctx.vd_step(P, state)
    ref = oracle.step(cfg, oracle.species_arh2_15(), Ee=Ee, poisson=oracle.mg_opts(**fx),
                      species_mg=oracle.mg_opts(fixed_cycles=2), energy_mg=oracle.mg_opts(fixed_cycles=2),
                      electron=0, m_bg=M_AR)
    assert ref["status"] == 0
    errs = _errors(state, ref)
    _show("   errors max-scaled/pointwise", errs)
    say("   ", info)
    assert max(e[0] for e in errs.values()) <= TOL
    assert max(e[1] for e in errs.values()) <= PW_TOL


def test_step_energy_fp32_ir_checked_by_oracle(ctx, V, oracle):
    """The same energy step in tolerance mode with every solve FP32-refined
    (the species solves on the parity-split FP32 passes): the oracle takes
    the GPU's potential, electron energy and densities and recomputes the
    relative residual of each in its own discretisation; each must be within
    the tolerance (1e-10, up to the rounding of a residual that small)."""
    from paper_2507_08200_amd import mechanisms as M
    cfg, Ee = _energy_cfg(64, 32, 32)
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    state["Ee"] = dev(Ee)
    o = dict(rtol=1e-10, precision=V.FP32_IR, ir_inner=1)
    P = V.step_params(cfg, M.arh2_15(), lfa=_lfa(cfg), poisson=V.mg_opts(**o), species_mg=V.mg_opts(**o),
                      energy_mg=V.mg_opts(**o), electron=0, m_bg=M_AR)
    say("energy step 64x32x32 fp32-ir tolerance")
    info = ctx.vd_step(P, state)
    assert info["status"] == 0
    chk = oracle.step(cfg, oracle.species_arh2_15(), Ee=Ee, phi=host(state["phi"]), phi_fixed=True,
                      check_n=host(state["n"]), check_Ee=host(state["Ee"]), electron=0, m_bg=M_AR)
    assert chk["status"] == 0
    res = chk["check_res"]
    say("   oracle residuals: poisson %.2e species max %.2e energy %.2e" %
        (chk["info"]["poisson_rel"], res[:15].max(), res[15]), info)
    assert chk["info"]["poisson_rel"] <= 1.05e-10
    assert res[:15].max() <= 1.05e-10 and res[15] <= 1.05e-10
    assert rel_err(host(state["Te"]), chk["Te"]) <= TOL


def test_step_extra_source_and_permittivity(ctx, V, oracle):
    """Argon step with an extra species source and a permittivity field
    (variable-coefficient Poisson), pinned cycle counts."""
    from paper_2507_08200_amd import mechanisms as M
    cfg = I.cfg1()
    rng = np.random.default_rng(1101)
    extra = rng.uniform(-1e27, 1e27, cfg["n"].shape)
    eps = 8.8541878128e-12 * (1.0 + 4.0 * (rng.uniform(0, 1, cfg["phi"].shape) > 0.7))
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    P = V.step_params(cfg, M.ar3(), poisson=V.mg_opts(fixed_cycles=12), species_mg=V.mg_opts(fixed_cycles=2),
                      extra_source=dev(extra), eps_cell=dev(eps))
    say("step cfg1 + extra source + permittivity")
    ctx.vd_step(P, state)
    ref = oracle.step(cfg, oracle.species_ar3(), poisson=oracle.mg_opts(fixed_cycles=12),
                      species_mg=oracle.mg_opts(fixed_cycles=2), extra_source=extra, eps_cell=eps)
    assert ref["status"] == 0
    errs = _errors(state, ref)
    _show("   errors", errs)
    assert max(e[0] for e in errs.values()) <= TOL
    assert max(e[1] for e in errs.values()) <= PW_TOL
    # the source really entered: without it the densities differ
    plain = oracle.step(cfg, oracle.species_ar3(), poisson=oracle.mg_opts(fixed_cycles=12),
                        species_mg=oracle.mg_opts(fixed_cycles=2), eps_cell=eps)
    assert rel_err(plain["n"][2], ref["n"][2]) > 1e-6


def test_step_extra_energy(ctx, V, oracle):
    """Energy step with extra electron-energy and species sources."""
    from paper_2507_08200_amd import mechanisms as M
    cfg, Ee = _energy_cfg(32, 32, 32)
    rng = np.random.default_rng(1102)
    extra_e = rng.uniform(-1e9, 1e9, cfg["phi"].shape)
    extra_n = rng.uniform(-1e28, 1e28, cfg["n"].shape)
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    state["Ee"] = dev(Ee)
    P = V.step_params(cfg, M.arh2_15(), lfa=_lfa(cfg), poisson=V.mg_opts(fixed_cycles=10),
                      species_mg=V.mg_opts(fixed_cycles=2), energy_mg=V.mg_opts(fixed_cycles=2),
                      extra_source=dev(extra_n), extra_energy=dev(extra_e), electron=0, m_bg=M_AR)
    say("energy step 32^3 + extra energy + extra source")
    ctx.vd_step(P, state)
    ref = oracle.step(cfg, oracle.species_arh2_15(), Ee=Ee, poisson=oracle.mg_opts(fixed_cycles=10),
                      species_mg=oracle.mg_opts(fixed_cycles=2), energy_mg=oracle.mg_opts(fixed_cycles=2),
                      extra_source=extra_n, extra_energy=extra_e, electron=0, m_bg=M_AR)
    assert ref["status"] == 0
    errs = _errors(state, ref)
    _show("   errors", errs)
    assert max(e[0] for e in errs.values()) <= TOL
    assert max(e[1] for e in errs.values()) <= PW_TOL


def _bench_opts(V):
    p = V.mg_opts(rtol=1e-10, precision=V.FP32_IR, ir_inner=1, guess=V.GUESS_EXTRAP, nu_pre=2, nu_post=2,
                  autotune=True)
    s = V.mg_opts(rtol=1e-10, precision=V.FP32_IR, n_levels=1, nu_pre=1, nu_post=0, ir_inner=1,
                  guess=V.GUESS_EXTRAP, autotune=True)
    return p, s


def test_headline_path_checked_by_oracle(V, oracle):
    """Six steps of the benchmark's path at 64^3 (extrapolated guesses from
    the third step on).  For each of the last three the oracle starts from
    the GPU's state before the step, takes the GPU's potential and checks its
    Poisson residual, recomputes Te, and checks the relative residual of every
    species solve in its own discretisation (the GPU decided convergence on
    its own FP64 residual).  The final state is compared with six oracle
    steps of plain multigrid from the previous values."""
    from paper_2507_08200_amd import mechanisms as M
    cfg = I.cfg3(n=64)
    lfa = _lfa(cfg)
    popt, sopt = _bench_opts(V)
    P = V.step_params(cfg, M.arh2_15(transport_background=False), lfa=lfa, poisson=popt, species_mg=sopt)
    ctx = V.Context()
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    worst = {"poisson": 0.0, "species": 0.0, "Te": 0.0}
    sp_or = oracle.species_arh2_15()
    for s_ in sp_or[13:]:
        s_["transported"] = 0
    for step in range(6):
        before = {k: host(v) for k, v in state.items()}
        info = ctx.vd_step(P, state)
        assert info["status"] == 0
        say("   step %d cycles poisson %d species %d" % (step, info["poisson_cycles"], info["species_cycles"]))
        if step < 3:
            continue
        c = dict(cfg)
        c["n"], c["Te"] = before["n"], before["Te"]
        chk = oracle.step(c, sp_or, phi=host(state["phi"]), phi_fixed=True, check_n=host(state["n"]))
        assert chk["status"] == 0
        res = chk["check_res"][:13]
        worst["poisson"] = max(worst["poisson"], chk["info"]["poisson_rel"])
        worst["species"] = max(worst["species"], float(res.max()))
        worst["Te"] = max(worst["Te"], rel_err(host(state["Te"]), chk["Te"]))
    say("   oracle-recomputed residuals (worst of the last three steps):", worst)
    assert worst["poisson"] <= 1.05e-10 and worst["species"] <= 1.05e-10
    assert worst["Te"] <= TOL
    # the trajectory against plain oracle solves from the previous values
    ref = {"n": cfg["n"], "phi": cfg["phi"], "Te": cfg["Te"]}
    for step in range(6):
        c = dict(cfg)
        c["n"], c["phi"], c["Te"] = ref["n"], ref["phi"], ref["Te"]
        ref = oracle.step(c, sp_or, poisson=oracle.mg_opts(rtol=1e-10), species_mg=oracle.mg_opts(rtol=1e-10))
        assert ref["status"] == 0
    errs = _errors(state, ref)
    _show("   6-step trajectory vs oracle, max-scaled/pointwise (floor 1e-6 of max)", errs)
    assert max(e[0] for e in errs.values()) <= 1e-6


def test_step_energy_masked_electrode(ctx, V, oracle):
    """Electron energy with an interior covered box (an electrode at 5 kV):
    the masked drift of the energy and of the electrons in the Joule term,
    the homogeneous Dirichlet diffusive flux at the covered-valid faces and
    the masked energy solve against the oracle, pinned cycle counts, 32^3
    Ar-H2 streamer."""
    from paper_2507_08200_amd import mechanisms as M
    cfg, Ee = _energy_cfg(32, 32, 32)
    for sb in cfg["species_bc"] + [cfg["energy_bc"], cfg["phi_bc"]]:
        assert I.BC_PERIODIC not in list(sb["kind"])
    mask = np.ones((32, 32, 32), np.uint8)
    mask[12:20, 12:20, 18:24] = 0
    phi = cfg["phi"].copy()
    phi[mask == 0] = 5000.0
    cfg["phi"] = phi
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    state["Ee"] = dev(Ee)
    fx = dict(fixed_cycles=10)
    P = V.step_params(cfg, M.arh2_15(), lfa=_lfa(cfg), poisson=V.mg_opts(**fx), species_mg=V.mg_opts(fixed_cycles=2),
                      energy_mg=V.mg_opts(fixed_cycles=2), electron=0, m_bg=M_AR, mask=torch.tensor(mask, device="cuda"))
    say("energy step 32^3 masked electrode")
    ctx.vd_step(P, state)
    ref = oracle.step(cfg, oracle.species_arh2_15(), Ee=Ee, poisson=oracle.mg_opts(**fx),
                      species_mg=oracle.mg_opts(fixed_cycles=2), energy_mg=oracle.mg_opts(fixed_cycles=2),
                      electron=0, m_bg=M_AR, mask=mask.ravel())
    assert ref["status"] == 0
    assert np.all(host(state["phi"])[mask == 0] == 5000.0)
    errs = _errors(state, ref)
    _show("   errors max-scaled/pointwise", errs)
    assert max(e[0] for e in errs.values()) <= TOL
    assert max(e[1] for e in errs.values()) <= PW_TOL


def test_masked_production_path_matches_oracle_trajectory(ctx, V, oracle):
    """The production solver path with an interior electrode: FP32-refined
    Poisson and single-level species solves to 1e-10 from the guesses
    extrapolated in time, four steps of the 32^3 Ar-H2 streamer, against
    the oracle's trajectory with the same schedule and its own extrapolated
    guesses.  Both stop on residual tests, so the fields agree to the
    tolerance spread (well inside 1e-6 of each field's largest value); the
    covered cells keep their potential and hold no plasma."""
    from paper_2507_08200_amd import mechanisms as M
    cfg = I.cfg3(n=32)
    mask = np.ones((32, 32, 32), np.uint8)
    mask[12:20, 12:20, 20:26] = 0
    phi = cfg["phi"].copy()
    phi[mask == 0] = 2000.0
    cfg["phi"] = phi
    steps = 4
    P = V.step_params(cfg, M.arh2_15(), lfa=_lfa(cfg),
                      poisson=V.mg_opts(rtol=1e-10, precision=V.FP32_IR, guess=V.GUESS_EXTRAP, ir_inner=1),
                      species_mg=V.mg_opts(rtol=1e-10, precision=V.FP32_IR, n_levels=1, nu_pre=1, nu_post=0,
                                           guess=V.GUESS_EXTRAP), mask=torch.tensor(mask, device="cuda"))
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    ctx.vd_step_reset()
    for k in range(steps):
        ctx.vd_step(P, state)
    ref = oracle.trajectory(cfg, oracle.species_arh2_15(), steps, poisson=oracle.mg_opts(rtol=1e-10),
                            species_mg=oracle.mg_opts(rtol=1e-10, n_levels=1, nu_pre=1, nu_post=0), mask=mask.ravel())
    g = host(state["n"])
    errs = {"phi": rel_err(host(state["phi"]), ref["phi"]), "Te": rel_err(host(state["Te"]), ref["Te"])}
    for k in range(15):
        if np.abs(ref["n"][k]).max() > 0:
            errs["n%d" % k] = rel_err(g[k], ref["n"][k])
    _show("   masked trajectory max-scaled", {k: (v, v) for k, v in errs.items()})
    assert max(errs.values()) <= 1e-6
    assert np.all(host(state["phi"])[mask == 0] == 2000.0)
    assert np.all(g[:, mask == 0] == 0.0)
