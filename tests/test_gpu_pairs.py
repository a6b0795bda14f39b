"""GPU parity of the two-step Lanczos (lanczos_s = 2; thick restart): from
step 3 on, steps j and j+1 come from one block [L q_j, L^2 q_j].  Against the
oracle's two-step recurrence (and the one-step one, equal in exact
arithmetic): Ritz values cycle by cycle, converged Fiedler pairs (FP64 and
mixed precision, element-wise vectors), partitions on unique-axis boxes,
cuts within 1%, batched = unbatched, every tile size, cycle lengths and
kept counts that give odd and even first steps and a one-column last pair.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb
from spectral_util import assert_fiedler_close, lambda23

pytestmark = pytest.mark.gpu

MESHES = {
    "box12x7x5": lambda: mg.box_hex(12, 7, 5).ids,
    "holes": lambda: mg.uniform_holes(mg.box_hex(23, 17, 9), 0.07, 3).ids,
    "renum": lambda: mg.shuffle_elements(mg.renumber_vertices(
        mg.uniform_holes(mg.box_hex(19, 11, 13), 0.05, 6), 7), 8).ids,
    "clustered": lambda: mg.clustered_holes(mg.box_hex(30, 26, 22), 0.1, 9).ids,
}
_GAP = {}


def gap(orc, name):
    if name not in _GAP:
        l2, l3 = lambda23(orc, MESHES[name]())
        _GAP[name] = l3 - l2
    return _GAP[name]


# (m, keep): even m with odd first steps; odd first step 8 (keep 7: a one-step
# launch at step 8, then pairs); odd m (a one-column pair ends every cycle)
SHAPES = [(40, 8), (30, 7), (13, 4)]


@pytest.mark.parametrize("m,keep", SHAPES)
@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fiedler_two_step(orc, name, m, keep, precision):
    ids = MESHES[name]()
    print(f"[pairs] {name} {precision} m={m} keep={keep}", flush=True)
    kw = dict(lanczos_m=m, lanczos_keep=keep, max_restarts=400)
    st, lam, y, stats = rsb.fiedler(ids, precision=precision, tol=1e-8, lanczos_s=2, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, tol=1e-10, lanczos_s=2, **kw)
    assert st == 0 and ost == 0
    assert abs(lam - olam) <= 1e-8 * olam
    assert stats["residual"] <= 1.01e-8 * lam
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], gap(orc, name))


@pytest.mark.parametrize("m,keep", SHAPES)
@pytest.mark.parametrize("restarts", [0, 3, 6])
def test_cycles_match_oracle(orc, m, keep, restarts):
    # a fixed number of cycles: the intermediate Ritz values of the GPU's
    # two-step recurrence against the oracle's, FP64
    ids = MESHES["holes"]()
    kw = dict(lanczos_m=m, lanczos_keep=keep, tol=1e-15, max_restarts=restarts)
    st, lam, y, stats = rsb.fiedler(ids, lanczos_s=2, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, lanczos_s=2, **kw)
    assert stats["cycles"] == oinfo["cycles"] == restarts + 1
    assert abs(lam - olam) <= 1e-10 * olam


@pytest.mark.parametrize("dims,graph,nparts", [((24, 20, 18), "face", 8),
                                              ((48, 40, 36), "weighted", 8),
                                              ((30, 14, 9), "face", 6)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_partition_identical_on_boxes(orc, dims, graph, nparts, precision):
    mesh = mg.box_hex(*dims)
    kw = dict(graph=graph, lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1)
    st, part, stats = rsb.partition(mesh.ids, nparts, precision=precision, lanczos_s=2, **kw)
    ost, opart, _ = orc.partition(mesh.ids, nparts, lanczos_s=2, **kw)
    assert st == ost == 0
    assert np.array_equal(part, opart)


@pytest.mark.parametrize("name,nparts", [("holes", 16), ("renum", 8), ("clustered", 32)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_partition_cut_within_one_percent(orc, name, nparts, precision):
    ids = MESHES[name]()
    kw = dict(lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1)
    st, part, stats = rsb.partition(ids, nparts, precision=precision, lanczos_s=2, **kw)
    ost, opart, _ = orc.partition(ids, nparts, lanczos_s=2, **kw)
    assert st >= 0
    sizes = np.bincount(part, minlength=nparts)
    assert sizes.min() >= len(ids) // nparts and sizes.max() <= -(-len(ids) // nparts)
    cut = orc.metrics(ids, part, nparts)["weighted_cut"]
    ocut = orc.metrics(ids, opart, nparts)["weighted_cut"]
    assert abs(cut - ocut) <= 0.01 * ocut


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_step_equals_one_step_partition(precision):
    # the same octant partition from both recurrences
    mesh = mg.box_hex(48, 40, 36)
    kw = dict(precision=precision, lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1)
    st1, p1, s1 = rsb.partition(mesh.ids, 8, lanczos_s=1, **kw)
    st2, p2, s2 = rsb.partition(mesh.ids, 8, lanczos_s=2, **kw)
    assert st1 == st2 == 0 and np.array_equal(p1, p2)


@pytest.mark.parametrize("rpt", [2, 4, 8])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tile_sizes(orc, rpt, precision):
    # 69,120 elements: many tiles, ragged last tiles, every tile size
    mesh = mg.box_hex(48, 40, 36)
    kw = dict(lanczos_m=40, lanczos_keep=8, tol=1e-8)
    st, part, _ = rsb.partition(mesh.ids, 8, precision=precision, lanczos_s=2,
                                rows_per_thread=rpt, **kw)
    ost, opart, _ = orc.partition(mesh.ids, 8, **kw)
    assert st == ost == 0 and np.array_equal(part, opart)


@pytest.mark.parametrize("keep", [8, 7])
def test_batched_equals_unbatched(keep):
    ids = MESHES["holes"]()
    kw = dict(tol=1e-8, lanczos_m=40, lanczos_keep=keep, lanczos_s=2, warm_start=1)
    st1, p1, s1 = rsb.partition(ids, 12, **kw)
    st0, p0, s0 = rsb.partition(ids, 12, batched=0, **kw)
    assert st1 == st0 and np.array_equal(p1, p0)


def test_mixed_refinement_two_step(orc):
    # FP32 directions to their stall, then FP64 directions, both two-step
    ids = MESHES["clustered"]()
    kw = dict(lanczos_m=40, lanczos_keep=8, max_restarts=400)
    st, lam, y, stats = rsb.fiedler(ids, precision="mixed", tol=1e-10, lanczos_s=2, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, tol=1e-11, **kw)
    assert st == 0 and stats["residual"] <= 1.01e-10 * lam
    assert abs(lam - olam) <= 1e-9 * olam
    assert stats["spmv_fp64"] > 3 * stats["cycles"]


def test_batch_call_two_step():
    meshes = [mg.uniform_holes(mg.box_hex(14 + 3 * b, 9 + b, 7), 0.05, b).ids for b in range(5)]
    kw = dict(precision="mixed", lanczos_m=40, lanczos_keep=8, tol=1e-6, warm_start=1,
              lanczos_s=2)
    st, parts, _ = rsb.partition_batch(meshes, [3, 4, 5, 6, 7], **kw)
    for b, ids in enumerate(meshes):
        s1, p1, _ = rsb.partition(ids, 3 + b, **kw)
        assert np.array_equal(p1, parts[b])
