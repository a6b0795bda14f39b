"""Inverse iteration with CG "augmented with full projection" (Sec. 7): each
new direction L-orthogonalised against the last k directions of the solve.
GPU against the oracle with the same k: the Fiedler value within 1e-8, CG
step counts within a few steps, partitions identical on a box with a
unique longest axis, the batched and one-subgraph paths identical, and the
AMG-preconditioned variant within the same bars.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb
from spectral_util import assert_fiedler_close, lambda23

pytestmark = pytest.mark.gpu

MESHES = {
    "box5x4x3": mg.box_hex(5, 4, 3).ids,
    "holes": mg.uniform_holes(mg.box_hex(23, 17, 9), 0.07, 3).ids,
    "quad": mg.uniform_holes(mg.box_quad(40, 33), 0.1, 4).ids,
    "clustered": mg.clustered_holes(mg.box_hex(30, 26, 22), 0.1, 9).ids,
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("k", [4, 32])
@pytest.mark.parametrize("precond", ["none", "amg"])
def test_fiedler_full_projection(orc, name, k, precond):
    ids = MESHES[name]
    kw = dict(method="inverse_cg", tol=1e-9, inv_max_outer=400, cg_full_projection=k,
              inv_precond=precond)
    st, lam, y, stats = rsb.fiedler(ids, **kw)
    ost, olam, oy, oinfo = orc.fiedler(ids, **kw)
    print(f"[fp] {name} k={k} {precond}: gpu cg {stats['segment_steps']} "
          f"oracle cg {oinfo['cg_iters']}", flush=True)
    assert st == ost == 0
    assert abs(lam - olam) <= 1e-8 * olam
    l2, l3 = lambda23(orc, ids)
    assert_fiedler_close(y, oy, stats["residual"], oinfo["residual"], l3 - l2)
    assert abs(stats["segment_steps"] - oinfo["cg_iters"]) <= max(3, 0.05 * oinfo["cg_iters"])


def test_full_projection_takes_fewer_steps():
    ids = MESHES["clustered"]
    kw = dict(method="inverse_cg", tol=1e-8, inv_max_outer=400)
    _, _, _, s0 = rsb.fiedler(ids, **kw)
    _, _, _, s1 = rsb.fiedler(ids, cg_full_projection=32, **kw)
    print(f"[fp] cg steps plain {s0['segment_steps']} projected {s1['segment_steps']}", flush=True)
    assert s1["segment_steps"] <= s0["segment_steps"]


def test_partition_identical_on_box(orc):
    ids = mg.box_hex(24, 20, 18).ids
    kw = dict(method="inverse_cg", tol=1e-8, inv_max_outer=400, cg_full_projection=8,
              graph="face")
    st, part, _ = rsb.partition(ids, 8, **kw)
    st1, part1, _ = rsb.partition(ids, 8, batched=0, **kw)
    ost, opart, _ = orc.partition(ids, 8, **kw)
    assert st == st1 == ost == 0
    assert np.array_equal(part, opart) and np.array_equal(part1, part)
