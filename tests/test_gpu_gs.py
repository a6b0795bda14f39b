"""GPU parity of the gather-scatter operator (Sec. 5: L = diag(A_w 1) - A_w,
A_w = P^T Q Q^T P), used by the Lanczos SpMV when gather_scatter = 1.

The operator itself is compared with the oracle's gather-scatter apply and
its assembled weighted Laplacian (FP64, 1e-12 relative).  Solves and
partitions through it must meet the same bars as the assembled operator:
Fiedler values within 1e-8 (FP64) of the oracle, identical partitions on
boxes with a unique longest axis, cuts within 1% elsewhere, and the batched,
unbatched, batch-call and reordered paths identical to each other.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb
from spectral_util import assert_fiedler_close, lambda23

pytestmark = pytest.mark.gpu


def _meshes():
    return {
        "paper": np.array([[1, 2, 3, 4], [2, 5, 4, 6], [3, 4, 7, 8]], dtype=np.int64),
        "box5x4x3": mg.box_hex(5, 4, 3).ids,
        "holes": mg.uniform_holes(mg.box_hex(23, 17, 9), 0.07, 3).ids,
        "quad": mg.uniform_holes(mg.box_quad(40, 33), 0.1, 4).ids,
        "renum": mg.shuffle_elements(mg.renumber_vertices(
            mg.uniform_holes(mg.box_hex(19, 11, 13), 0.05, 6), 7), 8).ids,
        "collapsed": np.array([[1, 2, 3, 4], [4, 4, 5, 6], [3, 4, 7, 8]], dtype=np.int64),
        "clustered": mg.clustered_holes(mg.box_hex(30, 26, 22), 0.1, 9).ids,
    }


MESHES = _meshes()


@pytest.mark.parametrize("name", list(MESHES))
def test_gs_apply(orc, name):
    ids = MESHES[name]
    x = np.random.default_rng(5).standard_normal(len(ids))
    y = rsb.gs_apply(ids, x)
    want = orc.gs_apply(ids, x)
    scale = np.abs(want).max() + 1e-300
    assert np.abs(y - want).max() <= 1e-12 * scale
    rp, col, w = orc.dual_graph(ids, "weighted")
    assert np.abs(y - orc.laplacian_apply(rp, col, w, x)).max() <= 1e-12 * scale


def test_gs_apply_device_arrays_and_size(orc):
    import torch
    m = mg.shuffle_elements(mg.clustered_holes(mg.box_hex(64, 64, 32), 0.1, 2), 3)
    x = np.random.default_rng(6).standard_normal(m.nelem)
    print(f"[gs] apply n={m.nelem}", flush=True)
    y = rsb.gs_apply(torch.as_tensor(m.ids).cuda(), torch.as_tensor(x).cuda(), device=True)
    want = orc.gs_apply(m.ids, x)
    assert np.abs(y.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(rsb.gs_apply(m.ids, np.ones(m.nelem))).max() == 0.0


def test_gs_vertex_in_too_many_slots(orc):
    # vertex 0 in every element; consecutive elements also share a chain
    ids = np.array([[0, i + 1, i + 2, 1000 + i] for i in range(65)], dtype=np.int64)
    with pytest.raises(rsb.RsbError):
        rsb.gs_apply(ids, np.ones(65))
    with pytest.raises(rsb.RsbError):
        rsb.partition(ids, 2, gather_scatter=1)
    x = np.random.default_rng(7).standard_normal(64)
    y = rsb.gs_apply(ids[:64], x)
    assert np.abs(y - orc.gs_apply(ids[:64], x)).max() <= 1e-12 * np.abs(y).max()
    # 64 slots are accepted (the clustered spectrum near 64 need not
    # converge under the default caps; the split is still balanced)
    st, part, _ = rsb.partition(ids[:64], 2, gather_scatter=1)
    assert st >= 0 and np.bincount(part).tolist() == [32, 32]


@pytest.mark.parametrize("name", ["paper", "box5x4x3", "holes", "quad", "renum"])
@pytest.mark.parametrize("keep", [0, 8])
def test_fiedler_fp64(orc, name, keep):
    ids = MESHES[name]
    kw = dict(tol=1e-9, lanczos_keep=keep, lanczos_m=30 if keep else 100)
    st, lam, y, stats = rsb.fiedler(ids, gather_scatter=1, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, **kw)
    assert st == ost
    assert abs(lam - olam) <= 1e-8 * olam
    l2, l3 = lambda23(orc, ids)
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], l3 - l2)


@pytest.mark.parametrize("name", ["box5x4x3", "holes", "clustered"])
def test_fiedler_mixed_thick(orc, name):
    ids = MESHES[name]
    # FP32 directions to the switch point, then FP64 directions to 1e-8
    st, lam, y, stats = rsb.fiedler(ids, gather_scatter=1, precision="mixed", tol=1e-8,
                                    lanczos_keep=8, lanczos_m=30, max_restarts=400)
    ost, olam, oy, oinfo = orc.fiedler(ids, tol=1e-9, lanczos_keep=8, lanczos_m=30,
                                       max_restarts=400)
    assert st == ost == 0
    assert abs(lam - olam) <= 1e-8 * olam
    assert stats["residual"] <= 1.01e-8 * lam
    l2, l3 = lambda23(orc, ids)
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], l3 - l2)


@pytest.mark.parametrize("dims,nparts", [((48, 40, 36), 8), ((24, 20, 18), 4)])
@pytest.mark.parametrize("precision,keep", [("fp64", 0), ("mixed", 0), ("fp64", 10),
                                            ("mixed", 8)])
def test_partition_identical_on_boxes(orc, dims, nparts, precision, keep):
    mesh = mg.box_hex(*dims)
    print(f"[gs] partition {dims} {nparts} {precision} keep={keep}", flush=True)
    tol = 1e-8
    st, part, stats = rsb.partition(mesh.ids, nparts, precision=precision, tol=tol,
                                    lanczos_keep=keep, gather_scatter=1)
    ost, opart, _ = orc.partition(mesh.ids, nparts, tol=1e-8, lanczos_keep=keep)
    assert st == ost == 0
    assert np.array_equal(part, opart)


@pytest.mark.parametrize("name,nparts", [("holes", 16), ("renum", 8), ("clustered", 32),
                                         ("quad", 10)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_partition_cut_within_one_percent(orc, name, nparts, precision):
    ids = MESHES[name]
    st, part, stats = rsb.partition(ids, nparts, precision=precision, tol=1e-8, gather_scatter=1)
    ost, opart, _ = orc.partition(ids, nparts, tol=1e-8)
    assert st >= 0
    sizes = np.bincount(part, minlength=nparts)
    assert np.array_equal(np.sort(sizes), np.sort(np.bincount(opart, minlength=nparts)))
    cut = orc.metrics(ids, part, nparts)["weighted_cut"]
    ocut = orc.metrics(ids, opart, nparts)["weighted_cut"]
    assert abs(cut - ocut) <= 0.01 * ocut


@pytest.mark.parametrize("keep", [0, 6])
def test_unbatched_equals_batched(keep):
    ids = MESHES["holes"]
    kw = dict(tol=1e-8, lanczos_m=40, lanczos_keep=keep, gather_scatter=1)
    st1, p1, s1 = rsb.partition(ids, 12, **kw)
    st2, p2, s2 = rsb.partition(ids, 12, batched=0, **kw)
    assert st1 == st2
    assert np.array_equal(p1, p2)


def test_batch_equals_single_calls():
    meshes = mg.batch64(seed=78, count=5, smin=2e3, smax=2e4)
    nparts = [4, 7, 1, 3, 8]
    kw = dict(gather_scatter=1, lanczos_keep=8, lanczos_m=30, tol=1e-6)
    st, parts, stats = rsb.partition_batch([m.ids for m in meshes], nparts, **kw)
    for m, p, q in zip(meshes, nparts, parts):
        s1, part1, _ = rsb.partition(m.ids, p, **kw)
        assert np.array_equal(part1, q)


def test_benchmark_settings_match_assembled_operator(orc):
    # the benchmark's solver settings (FP32 directions, thick restart, warm
    # start), with the locality order too: same partition as the oracle
    mesh = mg.shuffle_elements(mg.box_hex(40, 24, 18), 5)
    kw = dict(precision="mixed", lanczos_keep=8, lanczos_m=40, tol=1e-4, warm_start=1)
    st0, p0, s0 = rsb.partition(mesh.ids, 16, **kw)
    st1, p1, s1 = rsb.partition(mesh.ids, 16, gather_scatter=1, **kw)
    st2, p2, s2 = rsb.partition(mesh.ids, 16, gather_scatter=1, reorder=1, **kw)
    ost, op, _ = orc.partition(mesh.ids, 16, lanczos_keep=8, lanczos_m=40, tol=1e-8, warm_start=1)
    assert st0 == st1 == st2 == ost == 0
    assert np.array_equal(p1, op) and np.array_equal(p2, op) and np.array_equal(p0, op)


def test_profile_counts_gs():
    ids = MESHES["clustered"]
    st, part, stats = rsb.partition(ids, 16, precision="mixed", profile=1, tol=1e-6,
                                    gather_scatter=1)
    assert stats["kernel_launches"] > 0 and stats["kernel_ms"] > 0 and stats["kernel_bytes"] > 0
    st2, part2, _ = rsb.partition(ids, 16, precision="mixed", tol=1e-6, gather_scatter=1)
    assert np.array_equal(part, part2)
