"""Host-side bounds check of the 2.5D tiled multigrid passes.

The lexicographic colour/residual pass (all modes, including the fused
first and last colour passes of the FP32 refinement corrections, and the
residual checks of uniform levels, which share its tile geometry), the
parity-split FP32 colour pass and the direct residual check of levels with
coefficient arrays (kernel 2) load from wrapped or clamped addresses with
no branches and store whole pairs, so an index mistake would fault the GPU
before it showed as a wrong value.  vd_check_tiles25 walks every access of
every thread of every tile with the kernels' own index functions, on the
CPU, for the shapes below: the finest and coarser levels of the 160^3
refinement workload at every tile depth the planner can pick, partial
x, y and z tiles, small and odd shapes, and periodic faces."""
import itertools

import pytest

from paper_2507_08200_amd import vd as V

LEVELS_160 = [(160, 160, 160), (80, 80, 80), (40, 40, 40), (20, 20, 20)]
RAGGED = [(36, 20, 9), (100, 34, 7), (4, 1, 1), (4, 3, 2), (68, 17, 33), (132, 50, 5), (8, 16, 16), (64, 15, 3)]


def _check(shape, periodic, kz, kernel):
    acc, bad = V.check_tiles25(*shape, periodic, kz, kernel)
    assert acc > 0
    assert bad == 0, (shape, periodic, kz, kernel, bad)


@pytest.mark.parametrize("kernel", [0, 1, 2])
@pytest.mark.parametrize("kz", [2, 4, 8, 16, 32])
def test_160_refinement_levels(kernel, kz):
    for shape in LEVELS_160:
        for periodic in (0, 7):
            _check(shape, periodic, kz, kernel)


@pytest.mark.parametrize("kernel", [0, 1, 2])
@pytest.mark.parametrize("shape", RAGGED, ids=[str(s) for s in RAGGED])
def test_partial_tiles(kernel, shape):
    for periodic, kz in itertools.product(range(8), (1, 2, 3, 8)):
        _check(shape, periodic, kz, kernel)


def test_rejects_unsupported_shapes():
    with pytest.raises(V.VDError):
        V.check_tiles25(6, 4, 4, 0, 8, 1)      # parity split needs nx % 4 == 0
    with pytest.raises(V.VDError):
        V.check_tiles25(5, 4, 4, 0, 8, 0)      # row pairs need an even nx
    with pytest.raises(V.VDError):
        V.check_tiles25(5, 4, 4, 0, 8, 2)
    with pytest.raises(V.VDError):
        V.check_tiles25(8, 4, 4, 0, 8, 3)      # no such kernel
