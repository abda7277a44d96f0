"""The manufactured-solution workload (8 species, signed constant
mobilities, exact source passed as the step's extra source; the
verification method of Sec. 5.1 in 3D) on the GPU.

* One 128^3 step with four multigrid levels at pinned cycle counts equals
  the FP64 oracle's within 1e-12 of every field.
* Run to steady state on the GPU at 16^3 .. 128^3, the densities and the
  potential approach the analytic fields at second order (central
  diffusion, WENO5 on point values, second-order Poisson).
* The WENO5 drift divergence of exact cell averages of a smooth periodic
  profile in a uniform field converges at fifth order on the GPU (the
  tiled kernel at these shapes)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import dev, host, rel_err, rel_err_pointwise, say  # noqa: E402
from paper_2507_08200_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_08200_amd import vd
    vd.load()
    return vd


def test_cfg2_step_parity_128(V, oracle):
    cfg = I.cfg2(n=128)
    ctx = V.Context()
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    pc, sc = dict(fixed_cycles=4, n_levels=4), dict(fixed_cycles=2, n_levels=4)
    P = V.step_params(cfg, cfg["species"], consts=I.UNIT_CONSTS, poisson=V.mg_opts(**pc),
                      species_mg=V.mg_opts(**sc), extra_source=dev(cfg["extra_source"]))
    say("cfg2 128^3 step, pinned cycles")
    info = ctx.vd_step(P, state)
    ref = oracle.step(cfg, cfg["species"], consts=I.UNIT_CONSTS, extra_source=cfg["extra_source"],
                      poisson=oracle.mg_opts(**pc), species_mg=oracle.mg_opts(**sc))
    assert ref["status"] == 0
    errs = {"phi": (rel_err(host(state["phi"]), ref["phi"]), rel_err_pointwise(host(state["phi"]), ref["phi"]))}
    n = host(state["n"])
    for k in range(n.shape[0]):
        errs["n%d" % k] = (rel_err(n[k], ref["n"][k]), rel_err_pointwise(n[k], ref["n"][k]))
    say("   errors max-scaled/pointwise", {k: "%.1e/%.1e" % v for k, v in errs.items()}, info)
    assert max(e[0] for e in errs.values()) <= 1e-12
    assert max(e[1] for e in errs.values()) <= 1e-10     # pointwise, floor 1e-6 of the field's largest


def _steady(V, n, max_steps=600):
    cfg = I.cfg2(n=n, levels=min(4, int(np.log2(n)) - 2))
    ctx = V.Context()
    state = {k: dev(cfg[k]) for k in ("n", "phi", "Te")}
    o = dict(rtol=1e-12, n_levels=cfg["levels"], max_cycles=200)
    P = V.step_params(cfg, cfg["species"], consts=I.UNIT_CONSTS, poisson=V.mg_opts(**o), species_mg=V.mg_opts(**o),
                      extra_source=dev(cfg["extra_source"]))
    prev = state["n"].clone()
    for step in range(max_steps):
        info = ctx.vd_step(P, state, want_info=(step % 50 == 0))
        if step % 10 == 9:
            change = float((state["n"] - prev).abs().max())
            prev.copy_(state["n"])
            if change <= 1e-13:
                break
    ex = cfg["exact"]
    en = float(np.abs(host(state["n"]) - ex["n"]).max())
    ep = float(np.abs(host(state["phi"]) - ex["phi"]).max() / np.abs(ex["phi"]).max())
    return en, ep, step + 1


def test_cfg2_second_order_sweep(V):
    sizes = (16, 32, 64, 128)
    res = [_steady(V, n) for n in sizes]
    en = np.array([r[0] for r in res])
    ep = np.array([r[1] for r in res])
    rn = np.log2(en[:-1] / en[1:])
    rp = np.log2(ep[:-1] / ep[1:])
    say("cfg2 steady state: steps", [r[2] for r in res])
    say("   max |n - exact|", en, "slopes", rn)
    say("   max |phi - exact| / max |phi|", ep, "slopes", rp)
    assert np.all(rn > 1.8) and np.all(rp > 1.8), (rn, rp)


def _advection_error(V, ctx, n):
    """Exact cell averages of 1 + sin(2 pi x)/2 drifting at mu E along +x
    (periodic in x, plates give a uniform field): the divergence against the
    exact difference of the point values at the faces."""
    ny = nz = 8
    h = 1.0 / n
    xf = np.arange(n + 1) * h
    avg = 1.0 + 0.5 * (np.cos(2 * np.pi * xf[:-1]) - np.cos(2 * np.pi * xf[1:])) / (2 * np.pi * h)
    u = np.broadcast_to(avg, (nz, ny, n)).copy()[None]
    X, _, _ = I.cell_centres(n, ny, nz, h, h, h)
    Vp, mu = 2.0, 0.8
    phi = Vp * (1 - X)
    sp = [{"Z": 1, "mass": 1.0, "mob_kind": 0, "wall_kind": 0, "mu_const": mu}]
    div = host(ctx.vd_species_flux((n, ny, nz, h, h, h), I.bc([0, 0, 1, 1, 1, 1], (Vp, 0, 0, 0, 0, 0)),
                                   [I.bc([3, 3, 1, 1, 1, 1])], sp, dev(u), dev(phi),
                                   dev(np.full(u.shape, mu)), dev(np.full(phi.shape, 1.0)), 1.0, I.UNIT_CONSTS))
    f = lambda x: 1.0 + 0.5 * np.sin(2 * np.pi * x)
    exact = mu * Vp * (f(xf[1:]) - f(xf[:-1])) / h
    return float(np.abs(div[0] - exact[None, None, :]).max())


def test_weno5_fifth_order_gpu(V):
    ctx = V.Context()
    sizes = (32, 64, 128, 256)
    errs = np.array([_advection_error(V, ctx, n) for n in sizes])
    rates = np.log2(errs[:-1] / errs[1:])
    say("WENO5 periodic advection on the GPU: errors", errs, "slopes", rates)
    assert rates[-1] > 4.5 and rates[-2] > 4.5, rates
