"""GPU (HIP, through the C ABI) against the FP64 oracle on identical seeded
inputs.  Bars: bit-exact for colouring and masks; 1e-12 of each field's
maximum for FP64 results (solves compared at the same cycle count, the GPU
choosing the count in tolerance mode and the oracle replaying it)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import rel_err_pointwise, dev, gpu_problem, host, rel_err, say  # noqa: E402
from paper_2507_08200_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


# ------------------------------------------------------------ colouring, masks
@pytest.mark.parametrize("seed,shape,kinds,holes", [
    (101, (16, 16, 16), [0, 1, 3, 3, 1, 0], 3),
    (102, (24, 20, 12), [3, 3, 0, 0, 1, 1], 2),
    (103, (12, 12, 12), [0] * 6, 0),
])
def test_cell_flags_bit_exact(ctx, oracle, seed, shape, kinds, holes):
    prob = I.random_helmholtz(seed, shape, kinds=kinds, mask_holes=holes)
    g = gpu_problem(prob)
    L = 1
    nx, ny, nz = shape
    while nx % 2 == 0 and ny % 2 == 0 and nz % 2 == 0 and min(nx, ny, nz) > 4:
        nx, ny, nz, L = nx // 2, ny // 2, nz // 2, L + 1
    for level in range(L):
        say("flags", seed, shape, level)
        got = host(ctx.vd_cell_flags(g, level))
        want = oracle.cell_flags(prob, level)
        assert np.array_equal(got, want), (level, np.argwhere(got != want)[:5])


@pytest.mark.parametrize("ncolour", [1, 2, 5])
def test_half_sweeps(ctx, oracle, ncolour):
    prob = I.random_helmholtz(111, (20, 18, 16), mask_holes=2, kinds=[0, 1, 3, 3, 0, 1])
    g = gpu_problem(prob)
    say("half sweeps", ncolour)
    ctx.vd_smooth(g, ncolour)
    got = host(g["x"])
    want = oracle.smooth(prob, prob["rhs"], prob["x0"], ncolour)
    assert rel_err(got, want) <= TOL
    if ncolour == 1:
        # exactly the valid red cells changed, on both sides
        assert np.array_equal(got != prob["x0"], want != prob["x0"])
        k, j, i = np.meshgrid(*[np.arange(s) for s in (16, 18, 20)], indexing="ij")
        red = ((i + j + k) & 1) == 0
        assert np.array_equal(want != prob["x0"], red & (prob["mask"] != 0))


# ------------------------------------------------------------- pinned solves
SOLVE_CASES = [
    # seed, shape, alpha, beta, kinds, holes, n_levels, h
    (201, (16, 16, 16), "array", "array", None, 0, 0, None),
    (202, (48, 40, 24), "const", "array", None, 0, 0, None),
    (203, (32, 32, 32), "zero", "const", [0, 0, 1, 1, 1, 1], 0, 0, None),
    (204, (24, 24, 24), "array", "array", [0, 1, 3, 3, 1, 0], 3, 0, None),
    (205, (33, 20, 18), "array", "array", [1, 0, 1, 1, 0, 1], 0, 0, (1.0, 1.0, 1.0)),
    (206, (64, 32, 32), "array", "array", [0, 0, 1, 1, 3, 3], 0, 3, None),
    (207, (96, 96, 96), "zero", "const", [0, 0, 1, 1, 1, 1], 0, 0, None),
    (208, (40, 40, 40), "const", "array", None, 0, 0, None),
    (209, (40, 24, 20), "array", "array", [3, 3, 1, 0, 3, 3], 0, 0, None),
    (210, (40, 24, 20), "array", "const", [3, 3, 3, 3, 0, 1], 2, 0, None),
]


def _pinned_compare(oracle, prob, x_gpu, info, rtol, n_levels=0):
    k = info["cycles"]
    x_ref, i_ref, st = oracle.mg_solve(prob, prob["rhs"], prob["x0"], fixed_cycles=max(k, 0), n_levels=n_levels) \
        if k > 0 else (None, None, None)
    if k == 0:
        return
    assert st == 0
    err = rel_err(x_gpu, x_ref)
    say("   cycles", k, "rel", info["rel_res"], "oracle rel", i_ref["rel_res"], "err", err)
    assert err <= TOL, err
    assert i_ref["rel_res"] <= rtol * (1 + 1e-6)
    if k > 1:
        _, i_prev, _ = oracle.mg_solve(prob, prob["rhs"], prob["x0"], fixed_cycles=k - 1, n_levels=n_levels)
        assert i_prev["rel_res"] > rtol * (1 - 1e-6)


@pytest.mark.parametrize("case", SOLVE_CASES, ids=[str(c[0]) for c in SOLVE_CASES])
def test_solve_pinned_cycles(ctx, V, oracle, case):
    seed, shape, ak, bk, kinds, holes, nl, h = case
    prob = I.random_helmholtz(seed, shape, alpha_kind=ak, beta_kind=bk, kinds=kinds, mask_holes=holes, h=h,
                              beta_jump=(seed % 2 == 0))
    g = gpu_problem(prob)
    say("solve", seed, shape)
    infos, st = ctx.vd_helmholtz_solve_batched([g], V.mg_opts(rtol=1e-10, n_levels=nl))
    assert st == 0 and infos[0]["status"] == 0
    _pinned_compare(oracle, prob, host(g["x"]), infos[0], 1e-10, n_levels=nl)


def test_poisson_entry_point(ctx, V, oracle):
    """vd_poisson_solve: -div(beta grad phi) = rho with electrode plates."""
    n = 32
    h = 0.01 / n
    rng = np.random.default_rng(211)
    rho = rng.standard_normal((n, n, n)) * 1e-3
    eps = 8.8541878128e-12 * rng.uniform(1, 4, (n, n, n))
    pbc = I.bc([0, 0, 1, 1, 1, 1], (1000.0, 0, 0, 0, 0, 0))
    prob = {"grid": (n, n, n, h, h, h), "bc": pbc, "alpha": None, "alpha_c": 0.0, "beta": eps, "beta_c": 0.0,
            "mask": None, "rhs": rho, "x0": np.zeros((n, n, n))}
    phi = dev(np.zeros((n, n, n)))
    info = ctx.vd_poisson_solve(prob["grid"], pbc, dev(rho), phi, beta=dev(eps), opts=V.mg_opts(rtol=1e-10))
    assert info["status"] == 0
    _pinned_compare(oracle, prob, host(phi), info, 1e-10)


def test_batched_uneven(ctx, V, oracle):
    """Problems of different sizes, kinds and coefficients in one call give
    the same results as the oracle solving each alone at its cycle count."""
    shapes = [(16, 16, 16), (32, 24, 16), (40, 40, 40), (20, 20, 20), (48, 48, 48)]
    probs = [I.random_helmholtz(300 + p, s, beta_jump=True) for p, s in enumerate(shapes)]
    probs[1]["alpha"], probs[1]["alpha_c"] = None, 0.7
    probs[3]["beta"], probs[3]["beta_c"] = None, 0.3
    gs = [gpu_problem(p) for p in probs]
    say("batched", shapes)
    infos, st = ctx.vd_helmholtz_solve_batched(gs, V.mg_opts(rtol=1e-10))
    assert st == 0
    for p in range(len(probs)):
        assert infos[p]["status"] == 0
        _pinned_compare(oracle, probs[p], host(gs[p]["x"]), infos[p], 1e-10)


def test_fp32_refinement_reaches_tolerance(ctx, V, oracle):
    """FP32 cycles inside FP64 refinement: the FP64 residual (recomputed by
    the oracle's operator) meets the tolerance, and the solution agrees with
    the FP64 solution to the accuracy the tolerance implies."""
    for seed, shape in ((401, (48, 48, 48)), (402, (40, 24, 32))):
        prob = I.random_helmholtz(seed, shape, beta_jump=True)
        g = gpu_problem(prob)
        say("fp32-ir", seed, shape)
        infos, st = ctx.vd_helmholtz_solve_batched([g], V.mg_opts(rtol=1e-10, precision=V.FP32_IR, ir_inner=4))
        assert st == 0 and infos[0]["status"] == 0
        x = host(g["x"])
        r = oracle.residual(prob, prob["rhs"], x)
        b = oracle.residual(prob, prob["rhs"], np.zeros_like(x))
        rel = np.linalg.norm(r) / np.linalg.norm(b)
        say("   outer", infos[0]["outer_iters"], "cycles", infos[0]["cycles"], "rel", rel)
        assert rel <= 1e-10 * (1 + 1e-6)
        x64, _, _ = oracle.mg_solve(prob, prob["rhs"], prob["x0"], rtol=1e-12)
        assert rel_err(x, x64) <= 1e-6


def test_errors(ctx, V):
    prob = I.random_helmholtz(501, (8, 8, 8), alpha_kind="zero", kinds=[1] * 6)
    with pytest.raises(V.VDError) as e:
        ctx.vd_helmholtz_solve_batched([gpu_problem(prob)], V.mg_opts())
    assert e.value.status == V.VD_ESINGULAR
    prob = I.random_helmholtz(502, (8, 8, 8), kinds=[3, 1, 1, 1, 0, 0])
    with pytest.raises(V.VDError) as e:
        ctx.vd_helmholtz_solve_batched([gpu_problem(prob)], V.mg_opts())
    assert e.value.status == V.VD_EINVAL
    # odd periodic direction: red-black colouring would couple same-colour cells
    prob = I.random_helmholtz(505, (15, 8, 8), kinds=[3, 3, 0, 0, 1, 1])
    with pytest.raises(V.VDError) as e:
        ctx.vd_helmholtz_solve_batched([gpu_problem(prob)], V.mg_opts())
    assert e.value.status == V.VD_EINVAL
    prob = I.random_helmholtz(503, (16, 16, 16))
    infos, st = ctx.vd_helmholtz_solve_batched([gpu_problem(prob)], V.mg_opts(rtol=1e-30, max_cycles=3),
                                               allow_fail=True)
    assert st == V.VD_ENOCONV and infos[0]["cycles"] == 3
    prob = I.random_helmholtz(504, (16, 16, 16))
    prob["rhs"] = prob["rhs"] * np.nan
    infos, st = ctx.vd_helmholtz_solve_batched([gpu_problem(prob)], V.mg_opts(), allow_fail=True)
    assert st == V.VD_ENOCONV


# ------------------------------------------------------------ explicit terms
PHYS = {"qe": 1.602176634e-19, "eps0": 8.8541878128e-12, "kB": 1.380649e-23, "me": 9.1093837015e-31}


@pytest.mark.parametrize("shape", [(20, 18, 16), (64, 16, 16), (32, 24, 32), (128, 32, 16)])
@pytest.mark.parametrize("kinds", [[2, 2, 3, 3, 1, 1], [0, 0, 1, 1, 3, 3], [3, 3, 2, 2, 0, 1]])
def test_species_flux(ctx, oracle, kinds, shape):
    """Per-cell kernel (ragged shapes) and tiled kernel (32 x 8 tiles; at
    128 x 32 the tiles away from the x and y domain faces take the
    kernel's interior face loop)."""
    rng = np.random.default_rng(601)
    nx, ny, nz = shape
    h = 1e-4
    g = (nx, ny, nz, h, h, h)
    S = 4
    n = np.exp(rng.uniform(np.log(1e14), np.log(1e18), (S, nz, ny, nx)))
    phi = rng.uniform(-50, 50, (nz, ny, nx))
    Te = rng.uniform(1e4, 5e4, (nz, ny, nx))
    species = [
        {"Z": -1, "mass": PHYS["me"], "mob_kind": 0, "wall_kind": 1},
        {"Z": 1, "mass": 6.6e-26, "mob_kind": 0, "wall_kind": 2},
        {"Z": 0, "mass": 6.6e-26, "mob_kind": 0, "wall_kind": 3},
        {"Z": 1, "mass": 3.3e-27, "mob_kind": 0, "wall_kind": 2},
    ]
    mu = np.stack([-0.03 * (1 + 0.3 * rng.uniform(-1, 1, (nz, ny, nx))),
                   2e-4 * (1 + 0.3 * rng.uniform(-1, 1, (nz, ny, nx))),
                   np.zeros((nz, ny, nx)),
                   3e-3 * np.ones((nz, ny, nx))])
    pbc = I.bc([0, 0, 1, 1, 3, 3], (30.0, -10.0, 0, 0, 0, 0))
    sbc = [I.bc(kinds, rng.uniform(1e14, 1e16, 6)) for _ in range(S)]
    D = np.stack([0.05 * (1 + 0.5 * rng.uniform(-1, 1, (nz, ny, nx))) for _ in range(S)])
    say("species flux", kinds, shape)
    got = host(ctx.vd_species_flux(g, pbc, sbc, species, dev(n), dev(phi), dev(mu), dev(Te), 300.0, PHYS))
    want = oracle.species_flux(g, pbc, sbc, species, n, phi, mu, Te, 300.0, PHYS)
    for s in range(S):
        assert rel_err(got[s], want[s]) <= TOL, (s, rel_err(got[s], want[s]))
    # total face flux (drift + central diffusion) of the electrons and an ion
    for fs in (0, 1):
        div, faces = ctx.vd_species_flux(g, pbc, sbc, species, dev(n), dev(phi), dev(mu), dev(Te), 300.0, PHYS,
                                         D=dev(D), flux_species=fs)
        assert np.array_equal(host(div), got)
        ref = oracle.face_flux(g, pbc, sbc[fs], species[fs], n[fs], phi, mu[fs], D[fs], Te, 300.0, PHYS)
        for d in range(3):
            e, ep = rel_err(host(faces[d]), ref[d]), rel_err_pointwise(host(faces[d]), ref[d], 1e-6)
            say("   faces", fs, d, "%.2e %.2e" % (e, ep))
            assert e <= TOL, (fs, d, e)
            assert ep <= 1e-10, (fs, d, ep)      # pointwise, floor 1e-6 of the largest face flux


def test_reaction_source(ctx, oracle):
    rng = np.random.default_rng(701)
    nc = 4096
    n = np.exp(rng.uniform(np.log(1e12), np.log(1e20), (15, nc)))
    n[13], n[14] = 2.3e25, 1.2e24
    Te = np.exp(rng.uniform(np.log(3000), np.log(1.2e5), nc))
    say("reactions arh2")
    G, Sin = ctx.vd_reaction_source(I.MECH_ARH2_15, dev(n), dev(Te))
    Gr, Sr = oracle.reaction_source(I.MECH_ARH2_15, n, Te)
    for s in range(15):
        assert rel_err(host(G)[s], Gr[s]) <= TOL, s
    assert rel_err(host(Sin), Sr) <= TOL
    n3 = n[[0, 1, 7]].copy()
    G, Sin = ctx.vd_reaction_source(I.MECH_AR3, dev(n3), dev(Te), bg=(2.4e25,))
    Gr, Sr = oracle.reaction_source(I.MECH_AR3, n3, Te, bg=(2.4e25,))
    for s in range(3):
        assert rel_err(host(G)[s], Gr[s]) <= TOL, s
    assert rel_err(host(Sin), Sr) <= TOL
    G, _ = ctx.vd_reaction_source(I.MECH_DECAY, dev(n3), dev(Te), bg=(5.0,))
    assert np.array_equal(host(G), -5.0 * n3)


# ------------------------------------------------------------------- step
def _step_compare(V, oracle, ctx, cfg, sp_prod, sp_orc, pc, sc, ec=2, **kw):
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    Ee = kw.pop("Ee", None)
    if Ee is not None:
        state["Ee"] = dev(Ee)
    lfa = None
    if "lfa" in cfg:
        lfa = dict(cfg["lfa"])
        lfa["te_K"] = dev(cfg["lfa"]["te_K"])
    extra = kw.pop("extra_source", None)
    P = V.step_params(cfg, sp_prod, lfa=lfa, poisson=V.mg_opts(fixed_cycles=pc), species_mg=V.mg_opts(fixed_cycles=sc),
                      energy_mg=V.mg_opts(fixed_cycles=ec), extra_source=dev(extra), **kw)
    info = ctx.vd_step(P, state)
    ref = oracle.step(cfg, sp_orc, Ee=Ee, poisson=oracle.mg_opts(fixed_cycles=pc),
                      species_mg=oracle.mg_opts(fixed_cycles=sc), energy_mg=oracle.mg_opts(fixed_cycles=ec),
                      extra_source=extra, **kw)
    assert ref["status"] == 0
    n = host(state["n"])
    errs = {"phi": rel_err(host(state["phi"]), ref["phi"]), "Te": rel_err(host(state["Te"]), ref["Te"])}
    for s in range(n.shape[0]):
        errs["n%d" % s] = rel_err(n[s], ref["n"][s])
    if Ee is not None:
        errs["Ee"] = rel_err(host(state["Ee"]), ref["Ee"])
    say("   step errors", {k: "%.2e" % v for k, v in errs.items()}, info)
    return errs


def test_step_argon_cfg1(ctx, V, oracle):
    from paper_2507_08200_amd import mechanisms as M
    cfg = I.cfg1()
    say("step cfg1 32^3")
    errs = _step_compare(V, oracle, ctx, cfg, M.ar3(), oracle.species_ar3(), 12, 2)
    assert max(errs.values()) <= TOL


def test_step_arh2_small(ctx, V, oracle):
    from paper_2507_08200_amd import mechanisms as M
    cfg = I.cfg3(n=32)
    say("step cfg3-shaped 32^3")
    errs = _step_compare(V, oracle, ctx, cfg, M.arh2_15(), oracle.species_arh2_15(), 10, 2)
    assert max(errs.values()) <= TOL


@pytest.mark.parametrize("n", [16, 32])
def test_step_corrector_two(ctx, V, oracle, n):
    """Two correctors: at 16^3 the per-cell drift kernel (wall fluxes inside
    each cell's divergence); at 32^3 the tiled one, where the neutral
    field's right-hand side is formed with the reaction source and its wall
    flux added by the wall pass, from u^n while the rates are taken at the
    mid-point."""
    from paper_2507_08200_amd import mechanisms as M
    cfg = I.cfg1(n=n)
    cfg["n_t"] = 2
    say("step cfg1 %d^3 n_t=2" % n)
    errs = _step_compare(V, oracle, ctx, cfg, M.ar3(), oracle.species_ar3(), 10, 2)
    assert max(errs.values()) <= TOL


def test_step_energy_equation(ctx, V, oracle):
    """Electron energy solved (Eqs. (5)-(8)) with the fitted electron
    mobility, wall fluxes and the Ar-H2 chemistry."""
    from paper_2507_08200_amd import mechanisms as M
    cfg = I.cfg3(n=16)
    cfg["te_mode"] = I.TE_ENERGY
    ne = cfg["n"][0]
    Ee = 1.5 * ne * 1.380649e-23 * 23209.0
    say("step energy 16^3")
    errs = _step_compare(V, oracle, ctx, cfg, M.arh2_15(), oracle.species_arh2_15(), 10, 2, 2, Ee=Ee,
                         electron=0, m_bg=39.948 * 1.66053906660e-27)
    assert max(errs.values()) <= TOL


def test_cached_hierarchy_different_spacing(ctx, V, oracle):
    """Regression: two problems of the same shape but different mesh spacing
    solved one after the other on one context (the cached hierarchy must take
    the spacing of the current call)."""
    for seed, h in ((801, (1.0 / 32,) * 3), (802, (0.37 / 32, 0.5 / 32, 0.9 / 32))):
        prob = I.random_helmholtz(seed, (32, 32, 32), alpha_kind="zero", beta_kind="const",
                                  kinds=[0, 0, 1, 1, 1, 1], h=h)
        g = gpu_problem(prob)
        say("spacing", seed, h)
        infos, st = ctx.vd_helmholtz_solve_batched([g], V.mg_opts(rtol=1e-10))
        assert st == 0
        _pinned_compare(oracle, prob, host(g["x"]), infos[0], 1e-10)


# ------------------------------------------------ batch pins, graphs, autotune
def _cfg4_small(count, sizes):
    """The 64-problem sheath-jump recipe, at test sizes."""
    return I.cfg4(seed=4, count=count, sizes=sizes)


def test_batch_equals_alone(ctx, V):
    """Batching does not change the arithmetic: every problem of a batch of
    uneven sheath-jump problems equals the same problem solved alone at the
    same cycle count."""
    probs = _cfg4_small(8, (16, 32, 48))
    gs = [gpu_problem(p) for p in probs]
    say("batch vs alone", [p["grid"][0] for p in probs])
    infos, st = ctx.vd_helmholtz_solve_batched(gs, V.mg_opts(rtol=1e-10))
    assert st == 0
    for p, prob in enumerate(probs):
        g = gpu_problem(prob)
        i1, s1 = ctx.vd_helmholtz_solve_batched([g], V.mg_opts(rtol=1e-10, fixed_cycles=infos[p]["cycles"]))
        assert s1 == 0
        assert rel_err(host(gs[p]["x"]), host(g["x"])) <= TOL


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_graph_replay_and_autotune(ctx, V, oracle, precision):
    """Graph replay, smoother autotuning and the fused out-of-place sweep
    reproduce the kernel-by-kernel solve: same cycle counts, the same
    iterate to 1e-13; and the result is pinned against the oracle like every
    other solve (FP64)."""
    prec = V.FP64 if precision == "fp64" else V.FP32_IR
    shapes = [(32, 32, 32), (48, 40, 32), (24, 24, 24)]
    probs = [I.random_helmholtz(700 + p, s, beta_jump=True) for p, s in enumerate(shapes)]
    ref = [gpu_problem(p) for p in probs]
    say("graph/autotune", precision)
    i_ref, st = ctx.vd_helmholtz_solve_batched(ref, V.mg_opts(rtol=1e-10, precision=prec))
    assert st == 0
    for opts in (dict(graph=True), dict(autotune=True), dict(graph=True, autotune=True), dict(fused_sweep=True),
                 dict(fused_sweep=True, graph=True)):
        ctx2 = V.Context()
        for rep in range(3):   # capture, then replays (with eager work in between)
            gs = [gpu_problem(p) for p in probs]
            infos, st = ctx2.vd_helmholtz_solve_batched(gs, V.mg_opts(rtol=1e-10, precision=prec, **opts))
            assert st == 0
            torch.cuda.synchronize()
            for p in range(len(probs)):
                assert infos[p]["cycles"] == i_ref[p]["cycles"], (opts, rep, p)
                assert rel_err(host(gs[p]["x"]), host(ref[p]["x"])) <= 1e-13, (opts, rep, p)
    if prec == V.FP64:
        for p in range(len(probs)):
            _pinned_compare(oracle, probs[p], host(ref[p]["x"]), i_ref[p], 1e-10)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_persistent_colour_passes_bit_identical(V, precision):
    """Persistent colour passes (a fixed grid of workgroups walking the
    (problem, tile) items) compute every tile as the one-workgroup-per-tile
    launch does, and a colour pass reads only the other colour: the iterate
    is bit-identical, with the same cycle counts, for a batch that mixes
    uniform, variable-coefficient and masked problems, kernel by kernel and
    under graph replay."""
    prec = V.FP64 if precision == "fp64" else V.FP32_IR
    probs = [I.random_helmholtz(940, (64, 48, 32), alpha_kind="const", beta_kind="const"),
             I.random_helmholtz(941, (48, 40, 36), beta_jump=True),
             I.random_helmholtz(942, (32, 32, 32), mask_holes=2),
             I.random_helmholtz(943, (96, 64, 48), alpha_kind="zero", kinds=[I.BC_PERIODIC] * 4 + [I.BC_DIRICHLET] * 2)]
    ref = [gpu_problem(p) for p in probs]
    i_ref, st = V.Context().vd_helmholtz_solve_batched(ref, V.mg_opts(rtol=1e-10, precision=prec))
    assert st == 0
    for opts in (dict(persistent=True), dict(persistent=True, graph=True)):
        ctx2 = V.Context()
        for rep in range(3):
            gs = [gpu_problem(p) for p in probs]
            infos, st = ctx2.vd_helmholtz_solve_batched(gs, V.mg_opts(rtol=1e-10, precision=prec, **opts))
            assert st == 0
            torch.cuda.synchronize()
            say("   persistent", precision, opts, rep, [i["cycles"] for i in infos])
            for p in range(len(probs)):
                assert infos[p]["cycles"] == i_ref[p]["cycles"], (opts, rep, p)
                assert torch.equal(gs[p]["x"], ref[p]["x"]), (opts, rep, p)


def test_ir_fused_corrections_match_cleared(ctx, V, oracle):
    """FP32 corrections that start from zero without being cleared and add
    themselves to the FP64 unknown inside their last colour pass give the
    same solve as clearing them and adding them in a separate pass (forced
    here by the fused-sweep option, which smooths without colour passes):
    same cycle counts, same iterate to 1e-13, for a mixed batch (uniform,
    variable-coefficient and masked problems) in tolerance mode and as
    single-level smoothing (with and without post-smoothing, where the last
    pre-smoothing pass makes the update) at a fixed cycle count; the uniform
    problem's
    tolerance-mode residual is recomputed by the oracle."""
    probs = [I.random_helmholtz(910, (32, 32, 32), alpha_kind="const", beta_kind="const"),
             I.random_helmholtz(911, (48, 32, 40), beta_jump=True),
             I.random_helmholtz(912, (32, 32, 32), mask_holes=2)]
    for opts in (dict(), dict(n_levels=1, nu_pre=1, nu_post=1, fixed_cycles=6),
                 dict(n_levels=1, nu_pre=1, nu_post=0, fixed_cycles=6),
                 dict(n_levels=1, nu_pre=2, nu_post=0, fixed_cycles=4)):
        ref = [gpu_problem(p) for p in probs]
        i_ref, st = ctx.vd_helmholtz_solve_batched(ref, V.mg_opts(rtol=1e-10, precision=V.FP32_IR, **opts))
        assert st == 0
        gs = [gpu_problem(p) for p in probs]
        infos, st = V.Context().vd_helmholtz_solve_batched(
            gs, V.mg_opts(rtol=1e-10, precision=V.FP32_IR, fused_sweep=True, **opts))
        assert st == 0
        for p in range(len(probs)):
            say("   ir fused", opts, p, i_ref[p]["cycles"], infos[p]["cycles"], i_ref[p]["rel_res"])
            assert infos[p]["cycles"] == i_ref[p]["cycles"]
            assert rel_err(host(gs[p]["x"]), host(ref[p]["x"])) <= 1e-13
        if not opts:
            x = host(ref[0]["x"])
            r = oracle.residual(probs[0], probs[0]["rhs"], x)
            b = oracle.residual(probs[0], probs[0]["rhs"], np.zeros_like(x))
            assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10 * (1 + 1e-6)


@pytest.mark.parametrize("shapes,kinds", [
    ([(40, 24, 20), (64, 16, 12)], [I.BC_PERIODIC, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_DIRICHLET, I.BC_NEUMANN]),
    ([(36, 20, 16)], [I.BC_DIRICHLET, I.BC_NEUMANN, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_PERIODIC]),
    ([(40, 24, 20)], [I.BC_PERIODIC, I.BC_PERIODIC, I.BC_DIRICHLET, I.BC_NEUMANN, I.BC_PERIODIC, I.BC_PERIODIC]),
])
def test_ir_parity_split_rows(ctx, V, shapes, kinds):
    """Parity-split corrections on rows that end inside a workgroup's tile
    and across periodic faces give the same iterate as lexicographic ones,
    bit for bit up to 1e-13, at a fixed cycle count and in tolerance mode,
    and as single-level V(1,0) refinement (the species solves' schedule).
    The lexicographic run is the same batch plus a uniform problem whose nx
    is not a multiple of 4, which keeps the whole batch lexicographic
    (batching changes no arithmetic; its coarse levels, like the others',
    fit the LDS-resident coarse solve, so every problem keeps the same
    coarse solver)."""
    probs = [I.random_helmholtz(920 + q, s, alpha_kind="const", beta_kind="const", kinds=kinds) for q, s in enumerate(shapes)]
    extra = I.random_helmholtz(930, (38, 24, 24), alpha_kind="const", beta_kind="const",
                               kinds=[I.BC_DIRICHLET] * 6)
    for opts in (dict(fixed_cycles=3), dict(rtol=1e-10), dict(fixed_cycles=3, n_levels=1, nu_pre=1, nu_post=0)):
        split = [gpu_problem(p) for p in probs]
        i_s, st = ctx.vd_helmholtz_solve_batched(split, V.mg_opts(precision=V.FP32_IR, ir_inner=1, **opts))
        assert st == 0
        lex = [gpu_problem(p) for p in probs + [extra]]
        i_l, st = V.Context().vd_helmholtz_solve_batched(lex, V.mg_opts(precision=V.FP32_IR, ir_inner=1, **opts))
        assert st == 0
        for p in range(len(probs)):
            err = rel_err(host(split[p]["x"]), host(lex[p]["x"]))
            say("   parity-split", shapes[p], opts, i_s[p]["cycles"], i_l[p]["cycles"], err)
            assert i_s[p]["cycles"] == i_l[p]["cycles"]
            assert err <= 1e-13


def test_timing_credits_only_active_problems(V):
    """The smoother's algorithmic bytes count the problems that were still
    being cycled: a zero right-hand side added to a batch (inactive after
    the first check) adds launches but no smoother bytes."""
    prob = I.random_helmholtz(801, (32, 32, 32), beta_jump=True)
    zero = I.random_helmholtz(802, (32, 32, 32), beta_jump=True)
    zero["rhs"] = np.zeros_like(zero["rhs"])
    zero["bc"] = I.bc(list(zero["bc"]["kind"]), [0.0] * 6)     # no lifting either: b = 0
    res = []
    for batch in ([prob], [prob, zero]):
        c = V.Context()
        c.vd_timing_select("gsrb")
        infos, st = c.vd_helmholtz_solve_batched([gpu_problem(p) for p in batch], V.mg_opts(rtol=1e-10))
        assert st == 0
        res.append(c.vd_timing_read("gsrb"))
        say("   gsrb launches / ms / bytes", res[-1])
    assert res[0][0] == res[1][0] and res[0][2] > 0
    assert res[1][2] == res[0][2]
