"""The OpenMP timing build of the oracle (used only for the all-cores CPU
baseline) gives the same bits as the sequential build: it shares the
independent per-cell passes among threads and keeps every sum sequential."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_08200_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def threads():
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "4"
    O.build(parallel=True)
    yield
    if old is None:
        os.environ.pop("OMP_NUM_THREADS", None)
    else:
        os.environ["OMP_NUM_THREADS"] = old


def test_step_identical(tmp_path):
    cfg = I.cfg3(n=16)
    kw = dict(poisson=O.mg_opts(rtol=1e-10), species_mg=O.mg_opts(rtol=1e-10))
    a = O.step(cfg, O.species_arh2_15(), **kw)
    b = O.step(cfg, O.species_arh2_15(), parallel=True, **kw)
    assert a["status"] == 0 and b["status"] == 0
    assert a["info"] == b["info"]
    for k in ("n", "phi", "Te"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("shape,kinds", [((16, 12, 8), None), ((9, 8, 7), [3, 3, 1, 1, 3, 3])])
def test_solve_identical_including_odd_periodic(shape, kinds):
    prob = I.random_helmholtz(77, shape, kinds=kinds, beta_jump=True)
    xa, ia, sa = O.mg_solve(prob, prob["rhs"], prob["x0"], rtol=1e-10, n_levels=1 if shape[0] % 2 else 0)
    xb, ib, sb = O.mg_solve(prob, prob["rhs"], prob["x0"], parallel=True, rtol=1e-10,
                            n_levels=1 if shape[0] % 2 else 0)
    assert sa == sb and ia == ib
    assert np.array_equal(xa, xb)
