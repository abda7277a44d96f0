"""Smoothing-schedule tuning (VD_MG_TUNE_NU) of batched Helmholtz solves.

The tuned solve stops on the same relative-residual test, reports the
schedule it took, and gives the same iterate as a plain solve with that
schedule from the same start; the persisted choice (VD_TUNE_CACHE) is
written once and read back by a fresh context, which then skips tuning."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_util import gpu_problem, say  # noqa: E402
from paper_2507_08200_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu
D, N, P = I.BC_DIRICHLET, I.BC_NEUMANN, I.BC_PERIODIC
CANDIDATES = {(1, 1), (2, 1), (1, 2), (2, 2), (3, 3)}


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_08200_amd import vd
    vd.load()
    return vd


def _batch():
    return [I.random_helmholtz(201, (64, 48, 32), kinds=[D, N, P, P, N, D], beta_jump=True),
            I.random_helmholtz(202, (32, 32, 32), alpha_kind="zero", kinds=[D, D, N, N, N, N]),
            I.random_helmholtz(203, (96, 64, 64), alpha_kind="const", kinds=[N, D, D, N, N, N])]


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_tuned_schedule_matches_plain_solve(V, tmp_path, precision):
    prec = V.FP64 if precision == "fp64" else V.FP32_IR
    path = str(tmp_path / "nu.txt")
    os.environ["VD_TUNE_CACHE"] = path
    try:
        probs = _batch()
        ctx = V.Context()
        g = [gpu_problem(p) for p in probs]
        infos, st = ctx.vd_helmholtz_solve_batched(g, V.mg_opts(rtol=1e-10, precision=prec, tune_nu=True))
        assert st == 0
        nu = (infos[0]["nu_pre"], infos[0]["nu_post"])
        say("tuned schedule", precision, nu, [i["cycles"] for i in infos])
        assert nu in CANDIDATES
        assert all((i["nu_pre"], i["nu_post"]) == nu for i in infos)
        assert all(i["status"] == 0 and i["rel_res"] <= 1e-10 * (1 + 1e-9) for i in infos)
        # the same solve with that schedule, untuned, in a fresh context
        ctx2 = V.Context()
        g2 = [gpu_problem(p) for p in probs]
        infos2, st2 = ctx2.vd_helmholtz_solve_batched(g2, V.mg_opts(rtol=1e-10, precision=prec, nu_pre=nu[0],
                                                                    nu_post=nu[1]))
        assert st2 == 0
        for a, b in zip(g, g2):
            assert torch.equal(a["x"], b["x"])
        # persisted once; a fresh context reads it (no second line)
        lines = [l for l in open(path) if l.startswith("vdnu")]
        assert len(lines) == 1
        ctx3 = V.Context()
        g3 = [gpu_problem(p) for p in probs]
        infos3, st3 = ctx3.vd_helmholtz_solve_batched(g3, V.mg_opts(rtol=1e-10, precision=prec, tune_nu=True))
        assert st3 == 0 and (infos3[0]["nu_pre"], infos3[0]["nu_post"]) == nu
        assert len([l for l in open(path) if l.startswith("vdnu")]) == 1
        for a, b in zip(g, g3):
            assert torch.equal(a["x"], b["x"])
    finally:
        del os.environ["VD_TUNE_CACHE"]
