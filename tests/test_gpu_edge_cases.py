"""Degenerate inputs through the whole path, against the oracle: the
smallest meshes, one part, one element per part, graphs without edges
(every element its own component), a complete graph (all elements share
their vertices), and a batch mixing such meshes with a normal one -- with the
one-vector Lanczos and with the block Lanczos (whose columns are dropped
where a graph has too few directions: a complete graph's single nonzero
eigenvalue ends its first block).
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb

pytestmark = pytest.mark.gpu

SOLVERS = {"lanczos": {}, "block": dict(method="block", lanczos_m=40, lanczos_keep=8)}


@pytest.fixture(params=list(SOLVERS))
def sk(request):
    return SOLVERS[request.param]


def check_balanced(part, n, p):
    sizes = np.bincount(part, minlength=p)
    assert part.min() >= 0 and part.max() < p
    assert sizes.min() == n // p and sizes.max() == -(-n // p)


def test_two_elements(orc, sk):
    ids = np.array([[0, 1, 2, 3], [2, 3, 4, 5]], dtype=np.int64)
    st, part, _ = rsb.partition(ids, 2, **sk)
    ost, opart, _ = orc.partition(ids, 2, **sk)
    assert st == ost == 0 and np.array_equal(part, opart)
    check_balanced(part, 2, 2)


def test_one_part_runs_no_solve(sk):
    ids = mg.box_hex(6, 5, 4).ids
    st, part, stats = rsb.partition(ids, 1, **sk)
    assert st == 0 and np.all(part == 0) and stats["level_steps"] == 0


@pytest.mark.parametrize("graph", ["weighted", "face"])
def test_one_element_per_part(orc, graph, sk):
    ids = mg.uniform_holes(mg.box_hex(5, 4, 3), 0.1, 1).ids
    n = len(ids)
    st, part, _ = rsb.partition(ids, n, graph=graph, tol=1e-10, **sk)
    ost, opart, _ = orc.partition(ids, n, graph=graph, tol=1e-10, **sk)
    assert st >= 0 and ost >= 0
    assert np.array_equal(np.sort(part), np.arange(n))
    cut = orc.metrics(ids, part, n)["weighted_cut"]
    assert cut == orc.metrics(ids, opart, n)["weighted_cut"]  # every edge is cut


def test_no_edges_follow_the_components_rule(orc, sk):
    # 23 elements with private vertex ids: every element is a component, so
    # the parts are consecutive runs of element ids
    ids = np.arange(23 * 8, dtype=np.int64).reshape(23, 8)
    for p in (2, 5, 23):
        st, part, _ = rsb.partition(ids, p, **sk)
        ost, opart, _ = orc.partition(ids, p, **sk)
        assert st == ost == 2 and np.array_equal(part, opart)
        assert np.all(np.diff(part) >= 0)
        check_balanced(part, 23, p)


def test_complete_graph(orc, sk):
    # every element has the same four ids: all pairs adjacent with weight 4,
    # every balanced split cuts the same weight
    ids = np.tile(np.arange(4, dtype=np.int64), (17, 1))
    st, part, stats = rsb.partition(ids, 4, **sk)
    assert st >= 0
    check_balanced(part, 17, 4)
    ost, opart, _ = orc.partition(ids, 4, **sk)
    assert stats["edge_cut"] == orc.metrics(ids, opart, 4)["weighted_cut"]


def test_batch_with_degenerate_meshes(orc, sk):
    # (one number of ids per element for the whole batch: hexes, 8 ids)
    two = mg.box_hex(2, 1, 1).ids
    meshes = [mg.box_hex(1, 1, 1).ids, two,
              np.arange(9 * 8, dtype=np.int64).reshape(9, 8),
              mg.uniform_holes(mg.box_hex(10, 8, 6), 0.05, 2).ids]
    nparts = [1, 2, 3, 6]
    st, parts, _ = rsb.partition_batch(meshes, nparts, **sk)
    for m, p, q in zip(meshes, nparts, parts):
        s1, p1, _ = rsb.partition(m, p, **sk)
        assert np.array_equal(np.asarray(q), p1)
        check_balanced(np.asarray(q), len(m), p)
    # the mesh without edges follows the components rule in the batch too
    ost, opart, _ = orc.partition(meshes[2], 3, **sk)
    assert np.array_equal(np.asarray(parts[2]), opart)
