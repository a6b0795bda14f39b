"""GPU: the packed copy of the sliced-ELL slices and the LDS staging of the
tiles' gathers (opts pack_matrix: 0 words, 1 packed (the default), 2 packed
and staged).

A slice whose column offsets from the row fit in at most four windows of
1024 is read as 16-bit entries (weight, window, offset) instead of 32-bit
words; the other slices stay in words.  A tile whose packed slices reach at
most 4864 values of the vector (in up to six intervals) copies them into LDS
and gathers there.  The entries, their order and the values are the same, so
every result is bitwise the one of the 32-bit reading: Fiedler vectors,
eigenvalues, partitions, for every solver path that applies the level matrix
(one-step and two-step Lanczos, explicit restart, FP64 and mixed, inverse
iteration), every tile size.  Meshes in lexicographic order pack and stage
completely; shuffled elements leave most slices in words, and a partly
shuffled mesh mixes both forms within a level.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb

pytestmark = pytest.mark.gpu


def _partly_shuffled(mesh, frac, seed):
    # the last `frac` of the elements in random order, the rest in place
    n = mesh.ids.shape[0]
    k = int(n * (1 - frac))
    tail = k + mg.random_permutation(seed, n - k)
    order = np.concatenate([np.arange(k), tail])
    return mesh.ids[order]


MESHES = {
    "holes": lambda: mg.uniform_holes(mg.box_hex(23, 17, 9), 0.07, 3).ids,
    "clustered_renum": lambda: mg.renumber_vertices(
        mg.clustered_holes(mg.box_hex(30, 26, 22), 0.1, 9), 7).ids,
    "quad": lambda: mg.uniform_holes(mg.box_quad(150, 97), 0.05, 4).ids,
    # 16,302 elements in random order: a slice's offsets spread over the
    # whole mesh, far more than four windows
    "shuffled": lambda: mg.shuffle_elements(mg.uniform_holes(mg.box_hex(30, 26, 22), 0.05, 6),
                                            8).ids,
    "half_shuffled": lambda: _partly_shuffled(mg.uniform_holes(mg.box_hex(34, 30, 20), 0.05, 2),
                                              0.5, 5),
}

SOLVERS = {
    "thick_s2_mixed": dict(precision="mixed", lanczos_m=40, lanczos_keep=8, lanczos_s=2),
    "thick_s1_fp64": dict(precision="fp64", lanczos_m=40, lanczos_keep=8, lanczos_s=1),
    "explicit_mixed": dict(precision="mixed", lanczos_m=60, lanczos_keep=0),
    "inverse_cg": dict(method="inverse_cg"),
}


@pytest.mark.parametrize("solver", list(SOLVERS))
@pytest.mark.parametrize("name", list(MESHES))
def test_fiedler_bitwise_packed_vs_words(name, solver):
    ids = MESHES[name]()
    kw = dict(SOLVERS[solver], tol=1e-8, max_restarts=400)
    print(f"[pack] fiedler {name} {solver}", flush=True)
    st0, lam0, y0, s0 = rsb.fiedler(ids, pack_matrix=0, **kw)
    # (inverse iteration on the shuffled meshes stops at its CG cap in every
    # reading: status 1, the same vector)
    assert st0 == 0 or solver == "inverse_cg"
    for pack in (1, 2):
        st1, lam1, y1, s1 = rsb.fiedler(ids, pack_matrix=pack, **kw)
        assert st1 == st0
        assert lam1 == lam0
        assert np.array_equal(y1.view(np.uint64), y0.view(np.uint64))
        assert s1["cycles"] == s0["cycles"] and s1["level_steps"] == s0["level_steps"]


@pytest.mark.parametrize("solver", ["thick_s2_mixed", "thick_s1_fp64", "inverse_cg"])
@pytest.mark.parametrize("name", ["holes", "clustered_renum", "half_shuffled"])
def test_partition_bitwise_packed_vs_words(name, solver):
    ids = MESHES[name]()
    kw = dict(SOLVERS[solver], tol=1e-6, warm_start=0 if solver == "inverse_cg" else 1)
    print(f"[pack] partition {name} {solver}", flush=True)
    st0, p0, s0 = rsb.partition(ids, 24, pack_matrix=0, **kw)
    for pack in (1, 2):
        st1, p1, s1 = rsb.partition(ids, 24, pack_matrix=pack, **kw)
        assert st1 == st0
        assert np.array_equal(p1, p0)
        assert s1["lambda2"] == s0["lambda2"] and s1["level_steps"] == s0["level_steps"]


@pytest.mark.parametrize("rpt", [2, 4, 8])
@pytest.mark.parametrize("name", ["holes", "half_shuffled"])
def test_tile_sizes_bitwise(name, rpt):
    # 512-, 1024- and 2048-row tiles: the 2048-row ones reach more than the
    # LDS holds on a mesh with long planes and are not staged
    ids = MESHES[name]()
    kw = dict(precision="mixed", lanczos_m=40, lanczos_keep=8, lanczos_s=2, tol=1e-6,
              warm_start=1, rows_per_thread=rpt)
    st0, p0, s0 = rsb.partition(ids, 12, pack_matrix=0, **kw)
    st2, p2, s2 = rsb.partition(ids, 12, pack_matrix=2, **kw)
    assert st2 == st0 and np.array_equal(p2, p0) and s2["lambda2"] == s0["lambda2"]


def test_staged_fraction_large_planes():
    # 250 x 120 x 12 box: 1024-row tiles reach three intervals of about
    # 1,530 values (staged), 2048-row tiles two or three of about 2,550 (not
    # staged)
    ids = mg.uniform_holes(mg.box_hex(250, 120, 12), 0.03, 11).ids
    kw = dict(precision="mixed", lanczos_m=40, lanczos_keep=8, lanczos_s=2, tol=1e-4)
    st4, p4, s4 = rsb.partition(ids, 4, rows_per_thread=4, pack_matrix=2, **kw)
    st8, p8, s8 = rsb.partition(ids, 4, rows_per_thread=8, pack_matrix=2, **kw)
    assert s4["staged_fraction"] > 0.95
    assert s8["staged_fraction"] < 0.05
    for rpt, p, s in ((4, p4, s4), (8, p8, s8)):
        st0, p0, s0 = rsb.partition(ids, 4, rows_per_thread=rpt, pack_matrix=0, **kw)
        assert np.array_equal(p, p0) and s["lambda2"] == s0["lambda2"]


def _bytes_expected(stats, packed_nnz_frac_bounds):
    nnz = stats["nnz"]
    lo, hi = packed_nnz_frac_bounds
    assert lo <= stats["packed_fraction"] <= hi
    pn = stats["packed_fraction"] * nnz
    # 4 per nonzero in words, 2 per packed nonzero + 16 per packed slice
    mb = stats["matrix_bytes"]
    slices = mb - (4.0 * (nnz - pn) + 2.0 * pn)
    return slices / 16.0


@pytest.mark.parametrize("name,bounds,staged", [
    ("holes", (0.999, 1.0), (1.0, 1.0)), ("clustered_renum", (0.999, 1.0), (1.0, 1.0)),
    ("quad", (0.999, 1.0), (1.0, 1.0)), ("shuffled", (0.0, 0.0), (0.0, 0.0)),
    ("half_shuffled", (0.4, 0.5), (0.2, 0.8))])
def test_packed_fraction_and_bytes(name, bounds, staged):
    ids = MESHES[name]()
    st, part, s = rsb.partition(ids, 2, tol=1e-4, pack_matrix=2)
    assert st == 0
    assert staged[0] <= s["staged_fraction"] <= staged[1]
    nslices_packed = _bytes_expected(s, bounds)
    nslices = -(-len(ids) // 64)
    assert -1e-6 <= nslices_packed <= nslices + 1e-6
    assert abs(nslices_packed - round(nslices_packed)) < 1e-6
    st, part, s1 = rsb.partition(ids, 2, tol=1e-4, pack_matrix=1)
    assert s1["staged_fraction"] == 0.0 and s1["matrix_bytes"] == s["matrix_bytes"]
    st, part, s0 = rsb.partition(ids, 2, tol=1e-4, pack_matrix=0)
    assert s0["packed_fraction"] == 0.0 and s0["matrix_bytes"] == 4.0 * s0["nnz"]
    assert s0["staged_fraction"] == 0.0


def test_face_graph_packs_and_matches_oracle(orc):
    # the unique-axis box: identical octant partition with packed slices
    box = mg.box_hex(24, 20, 18)
    kw = dict(graph="face", lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1)
    st, part, s = rsb.partition(box.ids, 8, lanczos_s=2, **kw)
    ost, opart, _ = orc.partition(box.ids, 8, **kw)
    assert s["packed_fraction"] == 1.0
    assert st == ost == 0 and np.array_equal(part, opart)


@pytest.mark.parametrize("dims,bounds", [((3000, 3), (1.0, 1.0)), ((1500, 4, 4), (0.0, 0.3))])
def test_windows_limit(dims, bounds):
    # a quad strip: offsets -1..1 and +-(3000 + {-1, 0, 1}), three windows,
    # every slice packs.  A 1500 x 4 x 4 hex bar: offsets in up to nine groups
    # 1500 apart; only the four corner lines (four groups) pack, the other
    # slices stay in words
    ids = mg.box_quad(*dims).ids if len(dims) == 2 else mg.box_hex(*dims).ids
    kw = dict(tol=1e-6, lanczos_keep=8, lanczos_s=2, max_restarts=200)
    st1, p1, s1 = rsb.partition(ids, 4, pack_matrix=2, **kw)
    st0, p0, s0 = rsb.partition(ids, 4, pack_matrix=0, **kw)
    assert bounds[0] <= s1["packed_fraction"] <= bounds[1]
    assert st1 == st0 and np.array_equal(p1, p0) and s1["lambda2"] == s0["lambda2"]
