"""GPU parity of the BFS start (opts bfs_start): the first solve of each mesh
starts from the graph distance to a pseudo-peripheral element, computed on
the GPU by breadth-first search.  Against the oracle's BFS start: Ritz
values after a fixed number of cycles (which depend on the start vector),
converged Fiedler pairs element by element, partitions identical on
unique-axis boxes and cuts within 1% on holed meshes (FP64 and mixed,
explicit and thick restart, one and two steps at a time); independent of the
locality order of the rows and of batching.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb
from spectral_util import assert_fiedler_close, lambda23

pytestmark = pytest.mark.gpu

MESHES = {
    "holes": lambda: mg.uniform_holes(mg.box_hex(23, 17, 9), 0.07, 3).ids,
    "clustered": lambda: mg.clustered_holes(mg.box_hex(30, 26, 22), 0.1, 9).ids,
    "quad": lambda: mg.uniform_holes(mg.box_quad(150, 97), 0.05, 4).ids,
    # two pieces: the search from element 0 reaches only the first one (holes
    # keep the sub-boxes of the recursion from exactly degenerate pairs)
    "two_boxes": lambda: np.concatenate([
        mg.uniform_holes(mg.box_hex(13, 9, 7), 0.05, 1).ids,
        mg.uniform_holes(mg.box_hex(11, 8, 5), 0.05, 2).ids + 100000]),
}


@pytest.mark.parametrize("restarts", [0, 2])
@pytest.mark.parametrize("keep,s", [(0, 1), (8, 1), (8, 2)])
@pytest.mark.parametrize("name", ["holes", "clustered", "quad"])
def test_cycles_match_oracle(orc, name, keep, s, restarts):
    ids = MESHES[name]()
    kw = dict(lanczos_m=30, lanczos_keep=keep, tol=1e-15, max_restarts=restarts, bfs_start=1)
    print(f"[bfs] cycles {name} keep {keep} s {s} restarts {restarts}", flush=True)
    st, lam, y, stats = rsb.fiedler(ids, lanczos_s=s, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, lanczos_s=s, **kw)
    assert stats["cycles"] == oinfo["cycles"] == restarts + 1
    assert abs(lam - olam) <= 1e-10 * olam
    # the random start gives a different value after the same cycles
    _, lam_r, _, _ = rsb.fiedler(ids, lanczos_s=s, **dict(kw, bfs_start=0))
    assert lam_r != lam


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["holes", "clustered", "quad"])
def test_fiedler_converged(orc, name, precision):
    ids = MESHES[name]()
    kw = dict(lanczos_m=40, lanczos_keep=8, max_restarts=400, bfs_start=1)
    st, lam, y, stats = rsb.fiedler(ids, precision=precision, tol=1e-8, lanczos_s=2, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, tol=1e-10, **kw)
    assert st == 0 and ost == 0
    assert abs(lam - olam) <= 1e-8 * olam
    l2, l3 = lambda23(orc, ids)
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], l3 - l2)


@pytest.mark.parametrize("dims,graph", [((24, 20, 18), "face"), ((48, 40, 36), "weighted")])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_partition_identical_on_boxes(orc, dims, graph, precision):
    mesh = mg.box_hex(*dims)
    kw = dict(graph=graph, lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1, bfs_start=1)
    st, part, _ = rsb.partition(mesh.ids, 8, precision=precision, lanczos_s=2, **kw)
    ost, opart, _ = orc.partition(mesh.ids, 8, **kw)
    assert st == ost == 0 and np.array_equal(part, opart)


@pytest.mark.parametrize("name,nparts", [("holes", 16), ("clustered", 32), ("two_boxes", 6)])
def test_partition_cut_within_one_percent(orc, name, nparts):
    ids = MESHES[name]()
    kw = dict(lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1, bfs_start=1)
    st, part, _ = rsb.partition(ids, nparts, precision="mixed", lanczos_s=2, **kw)
    ost, opart, _ = orc.partition(ids, nparts, **kw)
    assert st >= 0 and ost >= 0
    sizes = np.bincount(part, minlength=nparts)
    assert sizes.min() >= len(ids) // nparts and sizes.max() <= -(-len(ids) // nparts)
    cut = orc.metrics(ids, part, nparts)["weighted_cut"]
    ocut = orc.metrics(ids, opart, nparts)["weighted_cut"]
    assert abs(cut - ocut) <= 0.01 * ocut


def test_reorder_and_batch_do_not_change_it():
    meshes = [MESHES["holes"](), MESHES["clustered"](), MESHES["two_boxes"]()]
    kw = dict(precision="mixed", lanczos_m=40, lanczos_keep=8, tol=1e-6, warm_start=1,
              bfs_start=1, lanczos_s=2)
    st, parts, _ = rsb.partition_batch(meshes, [8, 12, 5], **kw)
    for b, ids in enumerate(meshes):
        s1, p1, _ = rsb.partition(ids, [8, 12, 5][b], **kw)
        s2, p2, _ = rsb.partition(ids, [8, 12, 5][b], reorder=1, **kw)
        assert np.array_equal(p1, parts[b]) and np.array_equal(p1, p2)
