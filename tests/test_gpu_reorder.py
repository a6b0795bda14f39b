"""The locality order of level-0 rows (option reorder) moves rows in memory
only: partitions, part numbering (sign rule), the components rule and the
batch path must match the oracle and the input-order runs exactly, also when
the elements arrive shuffled.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,graph,nparts", [((24, 20, 18), "face", 8),
                                              ((24, 20, 18), "weighted", 4),
                                              ((30, 14, 9), "face", 6)])
@pytest.mark.parametrize("shuffle", [False, True])
def test_reorder_partition_identical(orc, dims, graph, nparts, shuffle):
    mesh = mg.box_hex(*dims)
    if shuffle:
        mesh = mg.shuffle_elements(mesh, 31)
    kw = dict(graph=graph, lanczos_keep=8, lanczos_m=30, tol=1e-8)
    st, part, stats = rsb.partition(mesh.ids, nparts, reorder=1, **kw)
    st0, part0, _ = rsb.partition(mesh.ids, nparts, **kw)
    ost, opart, _ = orc.partition(mesh.ids, nparts, **kw)
    assert st == st0 == ost == 0
    assert np.array_equal(part, opart) and np.array_equal(part0, opart)


def test_reorder_components_rule(orc):
    # two boxes whose elements are interleaved: components must still be
    # taken in order of least global id
    a = mg.box_hex(10, 2, 2)
    b = mg.box_hex(2, 2, 2)
    ids = np.concatenate([a.ids, b.ids + 10_000])
    perm = np.random.default_rng(4).permutation(len(ids))
    ids = ids[perm]
    st, part, _ = rsb.partition(ids, 2, graph="face", reorder=1)
    ost, opart, _ = orc.partition(ids, 2, graph="face")
    assert st == ost == 2
    assert np.array_equal(part, opart)


def test_reorder_batch_equals_single_calls():
    meshes = [mg.shuffle_elements(mg.uniform_holes(mg.box_hex(12 + k, 10, 6), 0.05, k), k)
              for k in range(4)]
    kw = dict(lanczos_keep=8, lanczos_m=30, tol=1e-8, reorder=1)
    st, parts, stats = rsb.partition_batch([m.ids for m in meshes], [4] * len(meshes), **kw)
    for m, p in zip(meshes, parts):
        s1, p1, _ = rsb.partition(m.ids, 4, **kw)
        assert np.array_equal(p1, p)


def test_reorder_shuffled_holes_cut():
    m = mg.shuffle_elements(mg.clustered_holes(mg.box_hex(40, 40, 20), 0.1, 9), 17)
    kw = dict(lanczos_keep=8, lanczos_m=40, tol=1e-4)
    st0, p0, s0 = rsb.partition(m.ids, 32, **kw)
    st1, p1, s1 = rsb.partition(m.ids, 32, reorder=1, **kw)
    sizes = np.bincount(p1, minlength=32)
    assert sizes.max() - sizes.min() <= 1
    assert abs(s1["edge_cut"] - s0["edge_cut"]) <= 0.01 * s0["edge_cut"]


def _edges_csr(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = []
    for i in range(n):
        col += sorted(adj[i])
        rp[i + 1] = len(col)
    col = np.array(col, dtype=np.int32)
    return rp, col, np.ones(len(col), dtype=np.int32)


def _small_graphs():
    rng = np.random.default_rng(12)
    lab = rng.permutation(57)
    yield "path", _edges_csr(57, [(lab[t], lab[t + 1]) for t in range(56)])
    m, n = 13, 21
    e = [(i * n + j, (i + 1) * n + j) for i in range(m - 1) for j in range(n)]
    e += [(i * n + j, i * n + j + 1) for i in range(m) for j in range(n - 1)]
    yield "grid", _edges_csr(m * n, e)
    yield "pieces", _edges_csr(7, [(0, 3), (3, 5), (4, 1), (1, 2)])
    yield "no-edges", (np.zeros(6, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    yield "one-row", (np.zeros(2, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))


@pytest.mark.parametrize("name", ["path", "grid", "pieces", "no-edges", "one-row"])
def test_locality_order_small_graphs(orc, name):
    rp, col, w = dict(_small_graphs())[name]
    got = rsb.locality_order(rp, col, w)
    assert np.array_equal(got, orc.locality_order(rp, col, w))


@pytest.mark.parametrize("dims,graph,holes,seed", [
    ((24, 20, 18), "face", 0.0, 1),
    ((24, 20, 18), "weighted", 0.1, 2),
    ((30, 14, 9), "unit", 0.05, 3),
    ((64, 64, 24), "weighted", 0.1, 4),   # levels of several thousand rows
    ((64, 64, 24), "face", 0.3, 5),       # clustered holes: several pieces
])
def test_locality_order_dual_graphs(orc, dims, graph, holes, seed):
    m = mg.box_hex(*dims)
    if holes:
        m = mg.clustered_holes(m, holes, seed)
    m = mg.shuffle_elements(m, seed)
    rp, col, w = orc.dual_graph(m.ids, graph)
    got = rsb.locality_order(rp, col, w)
    want = orc.locality_order(rp, col, w)
    print(f"[order] {dims} {graph} holes={holes} n={len(rp) - 1}", flush=True)
    assert np.array_equal(got, want)
