"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Integer results (dual graph, split given a vector, partitions on boxes with a
unique longest axis) must be bit-exact; the Fiedler value within 1e-8
relative in FP64 and 1e-5 with FP32 vectors (mixed precision); edge cuts on
meshes with holes within 1%.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb
from spectral_util import assert_fiedler_close, lambda23

pytestmark = pytest.mark.gpu


def _meshes():
    out = {
        "paper": np.array([[1, 2, 3, 4], [2, 5, 4, 6], [3, 4, 7, 8]], dtype=np.int64),
        "box5x4x3": mg.box_hex(5, 4, 3).ids,
        "cube16": mg.cube16().ids,
        "holes": mg.uniform_holes(mg.box_hex(23, 17, 9), 0.07, 3).ids,
        "quad": mg.uniform_holes(mg.box_quad(40, 33), 0.1, 4).ids,
        "renum": mg.shuffle_elements(mg.renumber_vertices(
            mg.uniform_holes(mg.box_hex(19, 11, 13), 0.05, 6), 7), 8).ids,
        "collapsed": np.array([[1, 2, 3, 4], [4, 4, 5, 6], [3, 4, 7, 8]], dtype=np.int64),
        "clustered": mg.clustered_holes(mg.box_hex(30, 26, 22), 0.1, 9).ids,
    }
    return out


MESHES = _meshes()
_GAPS = {}


def gap(orc, name, graph="weighted"):
    """lambda_3 - lambda_2 of a test mesh (every one used here has a simple pair)."""
    if (name, graph) not in _GAPS:
        l2, l3 = lambda23(orc, MESHES[name], graph)
        _GAPS[(name, graph)] = l3 - l2
    return _GAPS[(name, graph)]


def graph_metrics(orc, ids, part, nparts, graph):
    """Cut weight, cut pairs and neighbour-part counts on the given graph kind."""
    rp, col, w = orc.dual_graph(ids, graph=graph)
    rows = np.repeat(np.arange(len(ids)), np.diff(rp))
    cross = part[rows] != part[col]
    upper = cross & (col > rows)
    nb = np.zeros((nparts, nparts), dtype=bool)
    nb[part[rows][cross], part[col][cross]] = True
    cnt = nb.sum(axis=1)
    return {"cut": float(w[upper].sum()), "pairs": int(upper.sum()), "max_nb": int(cnt.max()),
            "avg_nb": float(cnt.mean())}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("graph", ["weighted", "unit", "face"])
def test_dual_graph_bit_exact(orc, name, graph):
    ids = MESHES[name]
    print(f"dual graph {name} {graph} n={len(ids)}", flush=True)
    rp, col, w = rsb.dual_graph(ids, graph=graph)
    orp, ocol, ow = orc.dual_graph(ids, graph=graph)
    assert np.array_equal(rp, orp)
    assert np.array_equal(col, ocol)
    assert np.array_equal(w, ow)


def test_dual_graph_device_arrays(orc):
    import torch
    ids = MESHES["holes"]
    rp, col, w = rsb.dual_graph(torch.as_tensor(ids).cuda(), device=True)
    orp, ocol, ow = orc.dual_graph(ids)
    assert np.array_equal(rp.cpu().numpy(), orp)
    assert np.array_equal(col.cpu().numpy(), ocol)
    assert np.array_equal(w.cpu().numpy(), ow)


@pytest.mark.parametrize("name", ["holes", "quad", "renum", "cube16"])
def test_laplacian_apply(orc, name):
    ids = MESHES[name]
    rp, col, w = orc.dual_graph(ids)
    x = np.random.default_rng(1).standard_normal(len(ids))
    y = rsb.laplacian_apply(rp, col, w, x)
    oy = orc.laplacian_apply(rp, col, w, x)
    scale = np.abs(x).max() * max(1, w.max()) * 27
    assert np.max(np.abs(y - oy)) <= 1e-13 * scale


def test_split_bit_exact(orc):
    rng = np.random.default_rng(5)
    for trial in range(12):
        n = int(rng.integers(1, 5000)) if trial else 1
        vals = np.array([-1.5, -0.0, 0.0, 2.0, 1e-300, -1e-300, 7.0])
        y = rng.choice(vals, size=n) if trial % 2 else rng.standard_normal(n)
        gid = rng.permutation(3 * n)[:n].astype(np.int64)
        for n_low in sorted({0, n, n // 2, int(rng.integers(0, n + 1))}):
            side = rsb.split(y, gid, n_low)
            oside = orc.split(y, gid, n_low)
            assert np.array_equal(side, oside), (trial, n, n_low)


@pytest.mark.parametrize("name", ["paper", "box5x4x3", "holes", "quad", "renum"])
def test_fiedler_fp64(orc, name):
    ids = MESHES[name]
    print(f"fiedler fp64 {name}", flush=True)
    st, lam, y, stats = rsb.fiedler(ids, tol=1e-9)
    ost, olam, oy, oinfo = orc.fiedler(ids, tol=1e-9)
    assert st == ost
    assert abs(lam - olam) <= 1e-8 * olam
    assert abs(np.linalg.norm(y) - 1) < 1e-10
    assert abs(y.sum()) < 1e-9 * np.sqrt(len(y))
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], gap(orc, name))


def test_fiedler_face_cube_closed_form():
    ids = MESHES["cube16"]
    st, lam, y, stats = rsb.fiedler(ids, graph="face", tol=1e-10, lanczos_m=100)
    assert st == 0
    exact = 2 - 2 * np.cos(np.pi / 16)
    assert abs(lam - exact) <= 1e-10 * exact


@pytest.mark.parametrize("name", ["box5x4x3", "holes", "renum", "quad", "clustered"])
def test_fiedler_mixed(orc, name):
    ids = MESHES[name]
    st, lam, y, stats = rsb.fiedler(ids, precision="mixed", tol=1e-8)
    ost, olam, oy, oinfo = orc.fiedler(ids, tol=1e-10)
    assert st == ost
    assert abs(lam - olam) <= 1e-5 * olam
    # FP32 directions, FP64 restart vector: the pair still meets the FP64 tolerance
    assert stats["residual"] <= 1e-8 * lam
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], gap(orc, name))


@pytest.mark.parametrize("m,keep", [(12, 4), (30, 10)])
@pytest.mark.parametrize("name", ["box5x4x3", "holes", "renum", "clustered"])
def test_fiedler_thick_restart(orc, name, m, keep):
    ids = MESHES[name]
    print(f"thick restart {name} m={m} keep={keep}", flush=True)
    kw = dict(lanczos_m=m, lanczos_keep=keep, max_restarts=400)
    st, lam, y, stats = rsb.fiedler(ids, tol=1e-8, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, tol=1e-10, **kw)
    assert st == 0 and ost == 0
    assert abs(lam - olam) <= 1e-8 * olam
    assert stats["residual"] <= 1.01e-8 * lam
    assert abs(y.sum()) < 1e-9 * np.sqrt(len(y))
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], gap(orc, name))


@pytest.mark.parametrize("m,keep", [(30, 10), (40, 8)])
@pytest.mark.parametrize("tol", [1e-4, 1e-8, 1e-10])
@pytest.mark.parametrize("name", ["box5x4x3", "holes", "renum", "clustered"])
def test_fiedler_thick_restart_mixed(orc, name, tol, m, keep):
    # FP32 directions, FP64 kept Ritz vectors: FP32 rounding stalls the
    # residual near 0.6 u ||L|| (u = 2^-24: 7e-7 to 1e-4 lambda on these
    # meshes); a solve that stalls short of the tolerance continues from its
    # Ritz vector with FP64 directions until the FP64 residual meets it
    ids = MESHES[name]
    print(f"thick restart mixed {name} tol={tol} m={m} keep={keep}", flush=True)
    kw = dict(lanczos_m=m, lanczos_keep=keep, max_restarts=400)
    st, lam, y, stats = rsb.fiedler(ids, precision="mixed", tol=tol, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, tol=1e-10, **kw)
    assert st == 0 and ost == 0
    assert abs(lam - olam) <= 1e-8 * olam
    assert stats["residual"] <= 1.01 * tol * lam
    assert abs(y.sum()) < 1e-9 * np.sqrt(len(y))
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], gap(orc, name))
    # tolerances below the stall level take FP64 cycles (level launches with
    # FP64 vectors: steps 1 and 2 and the residual of every cycle, and every
    # step of the FP64 cycles)
    refined = stats["spmv_fp64"] > 3 * stats["cycles"]
    if tol <= 1e-8:
        assert refined, (stats["spmv_fp64"], stats["cycles"])


NEAR_DEGENERATE = mg.uniform_holes(mg.box_hex(16, 16, 8), 0.05, 3).ids


def test_thick_restart_keep_one_is_explicit_restart():
    kw = dict(lanczos_m=8, tol=1e-15, max_restarts=4)
    _, lam0, y0, _ = rsb.fiedler(NEAR_DEGENERATE, lanczos_keep=0, **kw)
    _, lam1, y1, _ = rsb.fiedler(NEAR_DEGENERATE, lanczos_keep=1, **kw)
    assert abs(lam0 - lam1) <= 1e-11 * lam0
    assert abs(abs(float(y0 @ y1)) - 1.0) < 1e-8


def test_thick_restart_cycles_match_oracle(orc):
    # a fixed number of cycles, so the intermediate iterates are compared
    kw = dict(lanczos_m=12, lanczos_keep=4, tol=1e-15, max_restarts=6)
    st, lam, y, stats = rsb.fiedler(NEAR_DEGENERATE, **kw)
    ost, olam, oy, oinfo = orc.fiedler(NEAR_DEGENERATE, **kw)
    assert st == ost == 1
    assert stats["cycles"] == oinfo["cycles"] == 7
    assert abs(lam - olam) <= 1e-10 * olam


def test_thick_restart_does_not_stagnate(orc):
    kw = dict(lanczos_m=12, tol=1e-8, max_restarts=100)
    st0, lam0, _, s0 = rsb.fiedler(NEAR_DEGENERATE, lanczos_keep=0, **kw)
    st4, lam4, _, s4 = rsb.fiedler(NEAR_DEGENERATE, lanczos_keep=4, **kw)
    ost, olam, _, _ = orc.fiedler(NEAR_DEGENERATE, lanczos_keep=4, **kw)
    assert st0 == 1 and s0["residual"] > 1e-6 * lam4
    assert st4 == 0 and ost == 0 and s4["cycles"] < 40
    assert abs(lam4 - olam) <= 1e-8 * olam


@pytest.mark.parametrize("name", ["box5x4x3", "holes", "quad"])
def test_fiedler_inverse_cg(orc, name):
    ids = MESHES[name]
    st, lam, y, stats = rsb.fiedler(ids, method="inverse_cg", tol=1e-9, inv_max_outer=400)
    ost, olam, oy, _ = orc.fiedler(ids, method="inverse_cg", tol=1e-9, inv_max_outer=400)
    lst, llam, ly, _ = orc.fiedler(ids, tol=1e-10)
    assert st == ost == 0
    assert abs(lam - llam) <= 1e-8 * llam
    assert abs(abs(float(y @ ly)) - 1) < 1e-6


@pytest.mark.parametrize("method,keep", [("lanczos", 0), ("lanczos", 6), ("inverse_cg", 0)])
def test_unbatched_equals_batched(method, keep):
    ids = MESHES["holes"]
    kw = dict(method=method, tol=1e-8, inv_max_outer=300, lanczos_m=40, lanczos_keep=keep)
    st1, p1, s1 = rsb.partition(ids, 12, **kw)
    st2, p2, s2 = rsb.partition(ids, 12, batched=0, **kw)
    assert st1 == st2
    assert np.array_equal(p1, p2)


def test_profile_counts():
    ids = MESHES["clustered"]
    st, part, stats = rsb.partition(ids, 16, precision="mixed", profile=1, tol=1e-6)
    assert stats["kernel_launches"] > 0 and stats["kernel_ms"] > 0 and stats["kernel_bytes"] > 0
    st2, part2, _ = rsb.partition(ids, 16, precision="mixed", tol=1e-6)
    assert np.array_equal(part, part2)


@pytest.mark.parametrize("dims,graph,nparts", [((24, 20, 18), "face", 8),
                                              ((48, 40, 36), "weighted", 8),
                                              ((24, 20, 18), "weighted", 4),
                                              ((30, 14, 9), "face", 6)])
@pytest.mark.parametrize("precision,keep", [("fp64", 0), ("mixed", 0), ("fp64", 10),
                                            ("mixed", 8)])
def test_partition_identical_on_boxes(orc, dims, graph, nparts, precision, keep):
    mesh = mg.box_hex(*dims)
    print(f"partition {dims} {graph} {nparts} {precision} keep={keep}", flush=True)
    # (mixed precision with thick restart: FP32 directions to 1e-4, then FP64)
    tol = 1e-8
    st, part, stats = rsb.partition(mesh.ids, nparts, graph=graph, precision=precision, tol=tol,
                                    lanczos_keep=keep)
    ost, opart, _ = orc.partition(mesh.ids, nparts, graph=graph, tol=1e-8, lanczos_keep=keep)
    assert st == ost == 0
    assert np.array_equal(part, opart)
    met = graph_metrics(orc, mesh.ids, part, nparts, graph)
    assert stats["edge_cut"] == met["cut"]
    assert stats["cut_pairs"] == met["pairs"]
    assert stats["max_neighbors"] == met["max_nb"]
    assert abs(stats["avg_neighbors"] - met["avg_nb"]) < 1e-12


@pytest.mark.parametrize("name,nparts", [("holes", 16), ("renum", 8), ("clustered", 32),
                                         ("quad", 10)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_partition_cut_within_one_percent(orc, name, nparts, precision):
    ids = MESHES[name]
    print(f"partition {name} {nparts} {precision}", flush=True)
    st, part, stats = rsb.partition(ids, nparts, precision=precision, tol=1e-8)
    ost, opart, _ = orc.partition(ids, nparts, tol=1e-8)
    assert st >= 0
    sizes = np.bincount(part, minlength=nparts)
    assert sizes.min() >= len(ids) // nparts and sizes.max() <= -(-len(ids) // nparts)
    assert np.array_equal(np.sort(sizes), np.sort(np.bincount(opart, minlength=nparts)))
    cut = orc.metrics(ids, part, nparts)["weighted_cut"]
    ocut = orc.metrics(ids, opart, nparts)["weighted_cut"]
    assert abs(cut - ocut) <= 0.01 * ocut


@pytest.mark.parametrize("rpt", [2, 4, 8])
def test_tile_sizes_identical_partition(orc, rpt):
    # 69,120 elements: many tiles and reduction groups and a ragged last
    # tile for every tile size; unique longest axis at every level
    mesh = mg.box_hex(48, 40, 36)
    print(f"tile rows_per_thread={rpt}", flush=True)
    st, part, stats = rsb.partition(mesh.ids, 8, precision="mixed", tol=1e-8,
                                    rows_per_thread=rpt)
    ost, opart, _ = orc.partition(mesh.ids, 8, tol=1e-8)
    assert st == ost == 0
    assert np.array_equal(part, opart)


@pytest.mark.parametrize("steps", [1, 2])
def test_autotune_cache(tmp_path, steps):
    # one- and two-step launch sequences are timed and cached as separate
    # classes (the last key field before the tile)
    ids = MESHES["clustered"]
    path = str(tmp_path / "tiles.txt")
    kw = dict(precision="mixed", lanczos_keep=8, lanczos_m=40, lanczos_s=steps,
              autotune_cache=path)
    st1, p1, _ = rsb.partition(ids, 16, autotune=2, **kw)
    lines = open(path).read().splitlines()
    assert lines
    for line in lines:
        f = line.split()
        assert f[:2] == ["rsb-tile", "2"] and f[2].startswith("gfx") and len(f) == 10
        assert int(f[-2]) == steps and int(f[-1]) in (2, 4, 8)
    keys = [" ".join(line.split()[2:9]) for line in lines]
    assert len(keys) == len(set(keys))  # each class timed once per call
    st2, p2, _ = rsb.partition(ids, 16, autotune=1, **kw)
    assert st1 == st2
    assert np.array_equal(p1, p2)
    assert open(path).read().splitlines() == lines  # served from the cache


def test_disconnected_rule(orc):
    # Two separate boxes.  Components are ordered by smallest element id, so
    # box A (ids 0..35) comes first.  Exact ties of a box's symmetric Fiedler
    # vector are broken by rounding, so only rule-fixed facts are compared.
    a = mg.box_hex(4, 3, 3)
    b = mg.box_hex(3, 3, 2)
    ids = np.concatenate([a.ids, b.ids + 10_000])
    for nparts in (2, 3, 5):
        st, part, _ = rsb.partition(ids, nparts)
        ost, opart, _ = orc.partition(ids, nparts)
        assert st == ost == 2
        assert np.array_equal(np.bincount(part), np.bincount(opart))
    # P = 2: 27 low elements cut out of box A, box B entirely high
    st, part, _ = rsb.partition(ids, 2)
    assert np.all(part[36:] == 1) and np.sum(part[:36] == 0) == 27
    # A = 10x2x2 (40), B = 2x2x2 (8): the cut of A falls between slabs, so
    # the whole partition is unique (face graph)
    a = mg.box_hex(10, 2, 2)
    b = mg.box_hex(2, 2, 2)
    ids = np.concatenate([a.ids, b.ids + 10_000])
    st, part, _ = rsb.partition(ids, 2, graph="face")
    ost, opart, _ = orc.partition(ids, 2, graph="face")
    assert st == ost == 2
    assert np.array_equal(part, opart)
    assert np.all(part[40:] == 1)
    ids2 = np.concatenate([b.ids, b.ids + 10_000])
    st, lam, y, _ = rsb.fiedler(ids2)
    ost, olam, oy, _ = orc.fiedler(ids2)
    assert st == ost == 2 and lam == 0.0 and np.all(y == 0)


def test_batch_equals_single_calls():
    meshes = mg.batch64(seed=77, count=6, smin=2e3, smax=2e4)
    nparts = [4, 7, 16, 1, 3, 8]
    st, parts, stats = rsb.partition_batch([m.ids for m in meshes], nparts)
    for m, p, q in zip(meshes, nparts, parts):
        s1, part1, _ = rsb.partition(m.ids, p)
        assert np.array_equal(part1, q)


def test_repeated_partitions_identical(orc):
    # Component labels must not depend on thread timing: every row's label
    # is its component's root.  Many repetitions, with other solves between
    # them, give the same converged partition as the oracle's each time.
    ids = mg.box_hex(24, 20, 18).ids
    kw = dict(graph="face", lanczos_keep=8, lanczos_m=30, tol=1e-8)
    ost, opart, _ = orc.partition(ids, 8, **kw)
    for it in range(60):
        st, part, stats = rsb.partition(ids, 8, **kw)
        assert st == 0 and stats["disconnected"] == 0, it
        assert np.array_equal(part, opart), it
        m = mg.uniform_holes(mg.box_hex(10 + it % 7, 10, 4), 0.06, it)
        rsb.fiedler(m.ids, lanczos_keep=8, lanczos_m=30, tol=1e-10)
