"""vd_poisson_solve_noalloc (every work array in the library's static device
scratch) against vd_poisson_solve on the same inputs: identical results,
bit for bit, over consecutive calls of different sizes (the second call
finds the first call's data in the scratch), sizes beyond the scratch
rejected with the caller's arrays untouched, and no device memory taken."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import dev, say  # noqa: E402
from paper_2507_08200_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

EPS0 = 8.8541878128e-12


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


def _case(seed, shape, L=0.0125, var_eps=False):
    """Streamer-like charge density (a Gaussian space charge on noise)
    between a 15 kV plate at x = 0 and a grounded one at x = L."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    h = L / nx
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h, (np.arange(nx) + 0.5) * h,
                          indexing="ij")
    r2 = (x - 0.1 * L) ** 2 + (y - ny * h / 2) ** 2 + (z - nz * h / 2) ** 2
    rho = 1.602176634e-19 * (1e19 * np.exp(-r2 / (2 * (0.04 * L) ** 2)) + 1e13 * rng.uniform(-1, 1, shape))
    eps = EPS0 * rng.uniform(1, 4, shape) if var_eps else None
    g = (nx, ny, nz, h, h, h)
    pbc = I.bc([0, 0, 1, 1, 1, 1], (15000.0, 0, 0, 0, 0, 0))
    phi0 = 15000.0 * (1 - x / L) + rng.uniform(-1, 1, shape)
    return g, pbc, rho, eps, phi0


def _both(ctx, V, case, opts, want_info=True):
    """Solve with both entry points from the same starting potential."""
    g, pbc, rho, eps, phi0 = case
    r = dev(rho)
    e = dev(eps)
    a = dev(phi0)
    b = dev(phi0)
    ia = ctx.vd_poisson_solve(g, pbc, r, a, beta=e, beta_c=EPS0, opts=opts, want_info=want_info)
    ib = ctx.vd_poisson_solve_noalloc(g, pbc, r, b, beta=e, beta_c=EPS0, opts=opts, want_info=want_info)
    torch.cuda.synchronize()
    return a, b, ia, ib


def _same(a, b, ia, ib):
    d = (a - b).abs().max().item()
    assert torch.equal(a, b), "max |difference| %.3e" % d
    for k in ("cycles", "outer_iters", "status", "rel_res", "rel_res0", "bnorm", "levels"):
        if k in ia:
            assert ia[k] == ib[k], (k, ia[k], ib[k])


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_noalloc_matches_poisson_solve_two_calls(ctx, V, prec):
    """A 160^3 solve, then a smaller one of another shape that starts on the
    first call's leftovers in the scratch: both equal vd_poisson_solve."""
    p = V.FP64 if prec == "fp64" else V.FP32_IR
    for seed, shape in ((11, (160, 160, 160)), (12, (24, 40, 32))):
        say("noalloc", prec, shape)
        case = _case(seed, shape)
        a, b, ia, ib = _both(ctx, V, case, V.mg_opts(rtol=1e-10, precision=p))
        assert ia["status"] == 0 and ib["status"] == 0
        assert ib["rel_res"] <= 1e-10
        _same(a, b, ia, ib)


def test_noalloc_fixed_cycles_async_and_variable_permittivity(ctx, V):
    """Fixed cycles without an info struct (asynchronous), a variable
    permittivity with its face coefficients in the scratch, and a zero
    guess; each call follows a larger one."""
    runs = [((21, (64, 64, 64), True), V.mg_opts(fixed_cycles=3), False),
            ((22, (32, 32, 48), True), V.mg_opts(fixed_cycles=4, precision=V.FP32_IR, ir_inner=2), False),
            ((23, (16, 16, 16), False), V.mg_opts(rtol=1e-10, guess=V.GUESS_ZERO), True)]
    for (seed, shape, var), opts, want in runs:
        say("noalloc fixed", seed, shape, var)
        a, b, ia, ib = _both(ctx, V, _case(seed, shape, var_eps=var), opts, want_info=want)
        _same(a, b, ia, ib)


def test_noalloc_rejects_what_does_not_fit(ctx, V):
    """A 160^3 variable-permittivity hierarchy needs more than the scratch:
    VD_EINVAL and phi untouched; graph replay and autotuning are refused."""
    g, pbc, rho, eps, phi0 = _case(31, (160, 160, 160), var_eps=True)
    phi = dev(phi0)
    keep = phi.clone()
    with pytest.raises(V.VDError) as e:
        ctx.vd_poisson_solve_noalloc(g, pbc, dev(rho), phi, beta=dev(eps), opts=V.mg_opts())
    assert e.value.status == V.VD_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(phi, keep)
    g2, pbc2, rho2, _, phi2 = _case(32, (16, 16, 16))
    for opts in (V.mg_opts(graph=True), V.mg_opts(autotune=True), V.mg_opts(guess=V.GUESS_LEARNED)):
        with pytest.raises(V.VDError) as e:
            ctx.vd_poisson_solve_noalloc(g2, pbc2, dev(rho2), dev(phi2), opts=opts)
        assert e.value.status == V.VD_EINVAL
    # the context still works after the refusals
    a, b, ia, ib = _both(ctx, V, _case(33, (32, 32, 32)), V.mg_opts(rtol=1e-10))
    _same(a, b, ia, ib)


def test_noalloc_takes_no_device_memory(ctx, V):
    """Free device memory does not move across allocation-free solves of
    shapes this context has never solved (the same shapes through
    vd_poisson_solve build cached hierarchies that do take memory)."""
    cases = [_case(41, (96, 96, 96)), _case(42, (48, 80, 64))]
    opts = V.mg_opts(rtol=1e-10, precision=V.FP32_IR)
    dev_in = []
    for g, pbc, rho, eps, phi0 in cases:
        dev_in.append((g, pbc, dev(rho), dev(phi0), dev(phi0)))
    # one allocation-free call first, so that nothing measured below is a
    # first-call effect of the runtime
    g, pbc, r, p, _ = dev_in[1]
    ctx.vd_poisson_solve_noalloc(g, pbc, r, p, opts=opts)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for g, pbc, r, _, p in dev_in:
        info = ctx.vd_poisson_solve_noalloc(g, pbc, r, p, opts=opts)
        assert info["status"] == 0
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say("free device memory change (MiB):", (free0 - free1) / 2**20)
    assert free0 - free1 < 4 * 2**20
