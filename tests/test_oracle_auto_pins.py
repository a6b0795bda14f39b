"""Pins of the oracle's method AUTO (Sec. 7: inverse iteration where Lanczos
does not converge).

AUTO is a composition, pinned to its two parts: where Lanczos converges its
result is Lanczos' own, bit for bit, with no fallback counted; where Lanczos
is capped so that it cannot converge, the result is inverse iteration's
from the random start, bit for bit, and one fallback is counted.
"""
import numpy as np
import pytest

import meshgen as mg

MESH = mg.uniform_holes(mg.box_hex(9, 7, 5), 0.1, 2)


@pytest.mark.parametrize("keep", [0, 6])
def test_auto_is_lanczos_when_it_converges(orc, keep):
    kw = dict(tol=1e-8, lanczos_keep=keep, lanczos_m=30)
    st, lam, y, info = orc.fiedler(MESH.ids, method="auto", **kw)
    st0, lam0, y0, info0 = orc.fiedler(MESH.ids, method="lanczos", **kw)
    assert st == st0 == 0 and info["fallbacks"] == 0
    assert lam == lam0 and np.array_equal(y, y0)


def test_auto_is_inverse_iteration_when_lanczos_is_capped(orc):
    kw = dict(tol=1e-8, lanczos_m=6, max_restarts=0)
    st_l, _, _, _ = orc.fiedler(MESH.ids, method="lanczos", **kw)
    assert st_l == 1  # not converged
    st, lam, y, info = orc.fiedler(MESH.ids, method="auto", **kw)
    st1, lam1, y1, info1 = orc.fiedler(MESH.ids, method="inverse_cg", **kw)
    assert st == st1 == 0 and info["fallbacks"] == 1
    assert lam == lam1 and np.array_equal(y, y1)


def test_auto_partition_counts_fallbacks(orc):
    # with Lanczos capped below convergence every one of the 7 bisections
    # falls back, so the partition is inverse iteration's, bisection by
    # bisection
    kw = dict(tol=1e-8, lanczos_m=6, max_restarts=0)
    st, part, info = orc.partition(MESH.ids, 8, method="auto", **kw)
    sti, parti, infoi = orc.partition(MESH.ids, 8, method="inverse_cg", **kw)
    assert info["fallbacks"] == 7 and infoi["fallbacks"] == 0
    assert st == sti and np.array_equal(part, parti)
    sizes = np.bincount(part, minlength=8)
    assert sizes.max() - sizes.min() <= 1
