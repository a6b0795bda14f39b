"""Pins of the oracle's warm start (a child subgraph's Lanczos solve starts
from its parent's second Ritz vector): at convergence the partition does not
depend on the start vector on boxes with a unique longest axis at every
level, and on a box whose parent's second eigenvector restricts to the
children's Fiedler vector (closed form) the children converge in fewer
steps.
"""
import numpy as np
import pytest

import meshgen as mg

KW = dict(lanczos_keep=8, lanczos_m=30, tol=1e-8)


@pytest.mark.parametrize("dims,graph,nparts", [((24, 20, 18), "face", 8),
                                              ((24, 20, 18), "weighted", 4),
                                              ((30, 14, 9), "face", 6)])
def test_warm_start_same_partition(orc, dims, graph, nparts):
    ids = mg.box_hex(*dims).ids
    st0, p0, i0 = orc.partition(ids, nparts, graph=graph, **KW)
    st1, p1, i1 = orc.partition(ids, nparts, graph=graph, warm_start=1, **KW)
    assert st0 == st1 == 0
    assert np.array_equal(p0, p1)


def test_warm_start_from_closed_form_second_eigenvector(orc):
    # 30 x 16 x 7 face box: the Fiedler vector runs along x; the second
    # eigenvector cos(pi (y + 1/2) / 16) (pi/16 < 2 pi/30) is, restricted to
    # either 15 x 16 x 7 half, that half's Fiedler vector
    ids = mg.box_hex(30, 16, 7).ids
    st0, p0, i0 = orc.partition(ids, 4, graph="face", **KW)
    st1, p1, i1 = orc.partition(ids, 4, graph="face", warm_start=1, **KW)
    assert st0 == st1 == 0 and np.array_equal(p0, p1)
    # the top solve is the same; the two child solves start next to their answer
    assert i1["matvecs"] < i0["matvecs"]
    top = orc.fiedler(ids, graph="face", **KW)[3]["matvecs"]
    assert i1["matvecs"] - top < 0.8 * (i0["matvecs"] - top)


def test_warm_start_fewer_steps_on_holey_box(orc):
    m = mg.clustered_holes(mg.box_hex(32, 32, 16), 0.1, 9)
    kw = dict(lanczos_keep=8, lanczos_m=40, tol=1e-2)
    st0, p0, i0 = orc.partition(m.ids, 16, **kw)
    st1, p1, i1 = orc.partition(m.ids, 16, warm_start=1, **kw)
    c0 = orc.metrics(m.ids, p0, 16)["weighted_cut"]
    c1 = orc.metrics(m.ids, p1, 16)["weighted_cut"]
    assert i1["matvecs"] < 0.85 * i0["matvecs"]
    assert abs(c1 - c0) <= 0.01 * c0
