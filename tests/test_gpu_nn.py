"""Warm-start network on the GPU (bfloat16 MFMA convolutions, backward,
Adam, learned Poisson guess) against the numpy oracle on the same seeded,
bfloat16-rounded inputs."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import dev, say  # noqa: E402
from oracle import nn_oracle as N  # noqa: E402
from paper_2507_08200_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


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


def bf16_dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").to(torch.bfloat16).contiguous()


def f32_dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def rel(got, want):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


@pytest.mark.parametrize("shape,ci,co,relu", [((12, 10, 8), 2, 8, True), ((16, 16, 16), 8, 16, False),
                                              ((9, 7, 5), 16, 1, False), ((10, 12, 6), 24, 48, True),
                                              ((8, 8, 8), 32, 32, True)])
def test_conv3d_forward(ctx, shape, ci, co, relu):
    nx, ny, nz = shape
    g = (nx, ny, nz, 1.0, 1.0, 1.0)
    rng = np.random.default_rng(ci * 100 + co)
    x = N.bf16(rng.standard_normal((nz, ny, nx, ci)))
    w = rng.standard_normal((co, 27, ci)).astype(np.float32)
    b = rng.standard_normal(co).astype(np.float32)
    say("conv", shape, ci, co)
    y = ctx.vd_nn_conv3d(g, bf16_dev(x.reshape(-1, ci)), f32_dev(w), f32_dev(b), relu=relu).cpu().numpy()
    ref = N.conv3d(x, N.bf16(w.reshape(co, 3, 3, 3, ci)), b)
    if relu:
        ref = N.relu(ref)
    assert rel(y.reshape(nz, ny, nx, co), ref) <= 1e-5


@pytest.mark.parametrize("shape,ci,co", [((12, 10, 8), 2, 8), ((16, 12, 10), 8, 16), ((6, 8, 10), 16, 8),
                                         ((8, 8, 8), 32, 32)])
def test_conv3d_backward(ctx, shape, ci, co):
    nx, ny, nz = shape
    g = (nx, ny, nz, 1.0, 1.0, 1.0)
    rng = np.random.default_rng(7 + ci + co)
    x = N.bf16(rng.standard_normal((nz, ny, nx, ci)))
    w = rng.standard_normal((co, 27, ci)).astype(np.float32)
    b = np.zeros(co, np.float32)
    dy = rng.standard_normal((nz * ny * nx, co)).astype(np.float32)
    say("conv bwd", shape, ci, co)
    _, dx, dw, db = ctx.vd_nn_conv3d(g, bf16_dev(x.reshape(-1, ci)), f32_dev(w), f32_dev(b), dy=f32_dev(dy))
    wq = N.bf16(w.reshape(co, 3, 3, 3, ci))
    # the input gradient runs on bfloat16 operands, the weight gradient in FP32
    dx_ref = N.conv3d_backward(x, wq, N.bf16(dy.reshape(nz, ny, nx, co)))[0]
    _, dw_ref, db_ref = N.conv3d_backward(x, wq, dy.reshape(nz, ny, nx, co))
    assert rel(dx.cpu().numpy().reshape(nz, ny, nx, ci), dx_ref) <= 1e-5
    assert rel(dw.cpu().numpy().reshape(co, 3, 3, 3, ci), dw_ref) <= 1e-5
    assert rel(db.cpu().numpy(), db_ref) <= 1e-5


CFG = {"levels": 3, "ch": [8, 16, 32], "cin": 2}


def _sample(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, n, n, 2))
    t = rng.standard_normal((n, n, n)) * 0.1
    return x, t


def test_network_forward(ctx):
    n = 16
    p = I.nn_init(21, CFG)
    x, _ = _sample(22, n)
    ctx.vd_nn_create(CFG, p)
    g = (n, n, n, 1.0, 1.0, 1.0)
    out = ctx.vd_nn_forward(g, bf16_dev(x)).cpu().numpy()
    ref, _ = N.forward(p.astype(np.float64), x, CFG, rounding=True)
    # identical up to FP32-vs-FP64 accumulation; a stored activation that sits
    # at a bfloat16 rounding boundary may round the other way (one bfloat16
    # step, 2^-8 of it), which moves the outputs downstream of it: most
    # outputs agree to the accumulation order (3e-8 of the scale at the 90th
    # percentile), a few percent carry a flip's footprint (below 1e-3)
    err = np.abs(out - ref[..., 0])
    scale = np.abs(ref).max()
    say("   forward max rel", err.max() / scale, "mean", err.mean() / scale,
        "quantiles 0.5/0.9/0.99/0.999", [float(np.quantile(err, q) / scale) for q in (0.5, 0.9, 0.99, 0.999)],
        "fraction above 1e-5", float(np.mean(err > 1e-5 * scale)))
    assert np.quantile(err, 0.9) <= 1e-6 * scale
    assert np.mean(err > 1e-5 * scale) <= 0.1
    assert err.max() <= 4e-3 * scale
    assert err.mean() <= 2e-5 * scale


def test_train_step_gradients_and_adam(ctx):
    n = 16
    p = I.nn_init(23, CFG)
    x, t = _sample(24, n)
    ctx.vd_nn_create(CFG, p)
    g = (n, n, n, 1.0, 1.0, 1.0)
    loss = ctx.vd_nn_train_step(g, bf16_dev(x), f32_dev(t), lr=1e-3, update=False)
    grads = ctx.vd_nn_get(1)
    out, cache = N.forward(p.astype(np.float64), x, CFG, rounding=True)
    l_ref, dout = N.mse(out[..., 0], t)
    g_ref = N.backward(p, cache, dout[..., None], CFG, grad_rounding=True)
    gl = np.linalg.norm(grads - g_ref) / np.linalg.norm(g_ref)
    gmax = np.abs(grads - g_ref).max() / np.abs(g_ref).max()
    say("   loss", loss, l_ref, "grad rel L2", gl, "grad max-scaled", gmax)
    # the device rounds dy to bfloat16 as the oracle's grad_rounding does;
    # what is left is FP32 accumulation (2.6e-7 relative L2 on this sample)
    assert abs(loss - l_ref) <= 1e-7 * l_ref
    assert gl <= 1e-5
    assert gmax <= 1e-5
    # the update: one Adam step from zero moments with the device gradients
    ctx.vd_nn_train_step(g, bf16_dev(x), f32_dev(t), lr=1e-3, update=True)
    g1 = ctx.vd_nn_get(1).astype(np.float64)
    p1 = ctx.vd_nn_get(0)
    p_ref, m_ref, v_ref = N.adam(p.astype(np.float64), g1, np.zeros(len(p)), np.zeros(len(p)), 1, 1e-3)
    assert np.abs(p1 - p_ref).max() <= 1e-6
    assert np.allclose(ctx.vd_nn_get(2), m_ref, rtol=1e-5, atol=1e-12)


def test_features(ctx):
    n = 16
    h = 0.0125 / n
    gr = (n, n, n, h, h, h)
    pbc = I.bc([0, 0, 1, 1, 1, 1], (15000.0, 0.0, 0, 0, 0, 0))
    rho = np.random.default_rng(25).standard_normal((n, n, n)) * 1e-2
    f, vref = ctx.vd_nn_features(gr, pbc, dev(rho), eps=8.8541878128e-12)
    ref, vr = N.features(rho, gr, pbc, 8.8541878128e-12)
    assert vref == vr
    got = f.float().cpu().numpy()
    want = N.bf16(ref)
    # one bfloat16 step at most (the two sides order the scaling differently)
    assert np.all(np.abs(got - want) <= np.abs(want) * 2.0 ** -7 + 1e-30)
    assert np.mean(got == want) > 0.999


def test_learned_guess_solve_and_fallback(ctx, V, oracle):
    """The multigrid solve from the network's guess reaches the tolerance
    (residual recomputed by the oracle); a guess worse than zero is replaced
    by zero, and the solve then equals the zero-guess solve exactly."""
    n = 32
    cfg3 = I.cfg3(n=n)
    gr = cfg3["grid"]
    Z = np.array([s["Z"] for s in oracle.species_arh2_15()])
    rho = 1.602176634e-19 * np.tensordot(Z, cfg3["n"], axes=1)
    pbc = cfg3["phi_bc"]
    prob = {"grid": gr, "bc": pbc, "alpha": None, "alpha_c": 0.0, "beta": None, "beta_c": 8.8541878128e-12,
            "mask": None, "rhs": rho, "x0": np.zeros_like(rho)}
    ctx.vd_nn_create(CFG, I.nn_init(26, CFG))
    phi = dev(np.zeros_like(rho))
    info = ctx.vd_poisson_solve(gr, pbc, dev(rho), phi, opts=V.mg_opts(rtol=1e-10, guess=V.GUESS_LEARNED))
    say("   learned: cycles", info["cycles"], "fallback", info["fallback"], "rel0", info["rel_res0"])
    x = phi.cpu().numpy()
    r = oracle.residual(prob, rho, x)
    b = oracle.residual(prob, rho, np.zeros_like(x))
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10 * (1 + 1e-6)
    # a hopeless guess: huge output bias
    p = I.nn_init(26, CFG)
    p[-1] = 1e6
    ctx.vd_nn_set(p)
    phi2 = dev(np.zeros_like(rho))
    info2 = ctx.vd_poisson_solve(gr, pbc, dev(rho), phi2, opts=V.mg_opts(rtol=1e-10, guess=V.GUESS_LEARNED))
    assert info2["fallback"] == 1
    phi3 = dev(np.full_like(rho, 3.0))
    info3 = ctx.vd_poisson_solve(gr, pbc, dev(rho), phi3, opts=V.mg_opts(rtol=1e-10, guess=V.GUESS_ZERO))
    assert info2["cycles"] == info3["cycles"]
    assert torch.equal(phi2, phi3)


def test_save_load_roundtrip(ctx, tmp_path):
    p = I.nn_init(27, CFG)
    ctx.vd_nn_create(CFG, p)
    path = tmp_path / "net.bin"
    ctx.vd_nn_save(path)
    ctx.vd_nn_create(CFG, None)
    assert ctx.vd_nn_load(path) == len(p)
    assert np.array_equal(ctx.vd_nn_get(0), p)


def test_trained_network_saves_cycles_on_held_out_state(V, oracle):
    """The stored network (4 levels, 16-64 channels, trained on solver
    snapshots of seeded streamer runs) on a held-out run (another noise
    seed, voltage and seed position, 20 steps in): the Poisson solve from
    its guess reaches 1e-10 (residual recomputed by the oracle) in fewer
    cycles than from zero, in FP64 and in FP32 refinement."""
    from paper_2507_08200_amd import warmstart as WS
    assert os.path.exists(WS.NET_FILE)
    ctx = V.Context()
    run = I.warmstart_runs(7, 1)[0]
    d = WS.snapshots(ctx, [run], 160, 20, 20, keep_solver_inputs=True)[-1]
    ctx.vd_nn_load(WS.NET_FILE)
    gr, pbc, rho = d["grid"], d["bc"], d["rho"]
    say("held-out run", run)
    for prec in (V.FP64, V.FP32_IR):
        phi0 = torch.zeros_like(rho)
        i0 = ctx.vd_poisson_solve(gr, pbc, rho, phi0, beta_c=8.8541878128e-12,
                                  opts=V.mg_opts(rtol=1e-10, precision=prec, guess=V.GUESS_ZERO))
        phi1 = torch.zeros_like(rho)
        i1 = ctx.vd_poisson_solve(gr, pbc, rho, phi1, beta_c=8.8541878128e-12,
                                  opts=V.mg_opts(rtol=1e-10, precision=prec, guess=V.GUESS_LEARNED))
        say("   precision", prec, "cycles zero", i0["cycles"], "learned", i1["cycles"], "rel0", i1["rel_res0"])
        assert i0["status"] == 0 and i1["status"] == 0 and i1["fallback"] == 0
        assert i1["cycles"] < i0["cycles"]
        rh = rho.cpu().numpy()
        prob = {"grid": gr, "bc": pbc, "alpha": None, "alpha_c": 0.0, "beta": None, "beta_c": 8.8541878128e-12,
                "mask": None, "rhs": rh, "x0": np.zeros_like(rh)}
        x = phi1.cpu().numpy()
        r = oracle.residual(prob, rh, x)
        b = oracle.residual(prob, rh, np.zeros_like(x))
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10 * (1 + 1e-6)
