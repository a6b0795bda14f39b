"""Method AUTO on the GPU (Sec. 7: inverse iteration where Lanczos does not
converge): where Lanczos converges the result is Lanczos' own, where it is
capped below convergence every subgraph is solved again by inverse
iteration, with the same results as the inverse-iteration method run one
subgraph at a time, and within the oracle's tolerances.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb
from spectral_util import assert_fiedler_close, lambda23

pytestmark = pytest.mark.gpu

MESH = mg.uniform_holes(mg.box_hex(9, 7, 5), 0.1, 2)
HOLES = mg.uniform_holes(mg.box_hex(23, 17, 9), 0.07, 3)
CAPPED = dict(lanczos_m=6, max_restarts=0)


@pytest.mark.parametrize("keep", [0, 6])
def test_auto_equals_lanczos_when_converged(keep):
    kw = dict(tol=1e-8, lanczos_keep=keep, lanczos_m=30)
    st, lam, y, stats = rsb.fiedler(HOLES.ids, method="auto", **kw)
    st0, lam0, y0, _ = rsb.fiedler(HOLES.ids, method="lanczos", **kw)
    assert st == st0 == 0 and stats["fallbacks"] == 0
    assert lam == lam0 and np.array_equal(y, y0)


def test_auto_fiedler_falls_back(orc):
    kw = dict(tol=1e-8, **CAPPED)
    st, lam, y, stats = rsb.fiedler(HOLES.ids, method="auto", **kw)
    sti, lami, yi, _ = rsb.fiedler(HOLES.ids, method="inverse_cg", batched=0, **kw)
    ost, olam, oy, oinfo = orc.fiedler(HOLES.ids, method="auto", **kw)
    assert stats["fallbacks"] == 1 and oinfo["fallbacks"] == 1
    assert st == sti == ost
    assert lam == lami and np.array_equal(y, yi)
    assert abs(lam - olam) <= 1e-8 * olam
    l2, l3 = lambda23(orc, HOLES.ids)
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], l3 - l2)


@pytest.mark.parametrize("batched", [1, 0])
def test_auto_partition_falls_back_everywhere(orc, batched):
    kw = dict(tol=1e-8, **CAPPED)
    st, part, stats = rsb.partition(MESH.ids, 8, method="auto", batched=batched, **kw)
    sti, parti, _ = rsb.partition(MESH.ids, 8, method="inverse_cg", batched=0, **kw)
    ost, opart, oinfo = orc.partition(MESH.ids, 8, method="auto", **kw)
    assert stats["fallbacks"] == oinfo["fallbacks"] == 7
    assert st == sti and np.array_equal(part, parti)
    cut = orc.metrics(MESH.ids, part, 8)["weighted_cut"]
    ocut = orc.metrics(MESH.ids, opart, 8)["weighted_cut"]
    assert abs(cut - ocut) <= 0.01 * ocut


def test_auto_partition_equals_lanczos_when_converged():
    kw = dict(tol=1e-6, lanczos_keep=8, lanczos_m=30, warm_start=1)
    st, part, stats = rsb.partition(HOLES.ids, 16, method="auto", **kw)
    st0, part0, stats0 = rsb.partition(HOLES.ids, 16, method="lanczos", **kw)
    assert stats["fallbacks"] == 0 and st == st0
    assert np.array_equal(part, part0)


def test_auto_with_gather_scatter_operator():
    # the Lanczos part through the gather-scatter operator; every bisection
    # falls back, so the partition is inverse iteration's either way
    kw = dict(tol=1e-8, method="auto", **CAPPED)
    st, part, stats = rsb.partition(MESH.ids, 8, gather_scatter=1, **kw)
    st0, part0, stats0 = rsb.partition(MESH.ids, 8, **kw)
    assert stats["fallbacks"] == stats0["fallbacks"] == 7
    assert st == st0 and np.array_equal(part, part0)
