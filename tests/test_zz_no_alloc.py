"""The entry point for callers that cannot allocate (rsb_partition_noalloc):
through the C ABI its partitions equal rsb_partition's on the same inputs,
on two calls in a row (the second with a smaller mesh, so the region holds
the first call's contents), with host and device arrays, default and
benchmark solver settings, the block Lanczos, and at the documented maximum size."""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb

pytestmark = pytest.mark.gpu

BENCH = dict(precision="mixed", lanczos_keep=8, lanczos_m=40, tol=1e-2, warm_start=1, lanczos_s=2)
BFS = dict(BENCH, bfs_start=1)
BLOCK = dict(method="block", lanczos_m=40, lanczos_keep=8, tol=1e-6, warm_start=1, fiedler_sweep=8)


def _pair(ids, nparts, device=False, **kw):
    st0, p0, s0 = rsb.partition(ids, nparts, device=device, **kw)
    st1, p1, s1 = rsb.partition_noalloc(ids, nparts, device=device, **kw)
    if device:
        p0, p1 = p0.cpu().numpy(), p1.cpu().numpy()
    assert st1 == st0
    assert np.array_equal(p1, p0)
    assert s1["edge_cut"] == s0["edge_cut"] and s1["level_steps"] == s0["level_steps"]
    return p1


@pytest.mark.parametrize("kw", [{}, BENCH, BFS, BLOCK], ids=["default", "bench", "bfs_start", "block"])
def test_two_calls_second_smaller(kw):
    big = mg.uniform_holes(mg.box_hex(40, 30, 24), 0.05, 31)
    small = mg.clustered_holes(mg.box_hex(23, 17, 11), 0.1, 32)
    print(f"[noalloc] {big.nelem} elements -> 16 parts, then {small.nelem} -> 5", flush=True)
    _pair(big.ids, 16, **kw)
    _pair(small.ids, 5, **kw)


def test_device_arrays():
    import torch
    mesh = mg.renumber_vertices(mg.uniform_holes(mg.box_hex(30, 22, 17), 0.04, 33), 34)
    ids = torch.as_tensor(mesh.ids).cuda()
    print(f"[noalloc] device arrays, {mesh.nelem} elements -> 12 parts", flush=True)
    _pair(ids, 12, device=True, **BENCH)
    _pair(ids[: mesh.nelem // 3].contiguous(), 3, device=True, **BENCH)


def test_maximum_size():
    # 65536 elements (the documented maximum) into 1024 parts (the maximum):
    # the default solver settings fit the region
    mesh = mg.box_hex(64, 32, 32)
    assert mesh.nelem == rsb.NOALLOC_MAX_ELEMS
    print("[noalloc] maximum size, 65536 elements -> 1024 parts", flush=True)
    _pair(mesh.ids, 1024)
    _pair(mesh.ids, 1024, **BENCH)
    _pair(mesh.ids, 1024, **BLOCK)
    # and a smaller call after it
    _pair(mg.box_hex(9, 7, 5).ids, 4)


def test_beyond_maximum_rejected():
    mesh = mg.box_hex(65, 32, 32)
    with pytest.raises(rsb.RsbError) as e:
        rsb.partition_noalloc(mesh.ids, 8)
    assert e.value.code == rsb.EINVAL and "at most 65536 elements" in str(e.value)
    with pytest.raises(rsb.RsbError) as e:
        rsb.partition_noalloc(mg.box_hex(20, 20, 10).ids, 1025)
    assert e.value.code == rsb.EINVAL
    # a call after the rejections still works
    _pair(mg.box_hex(12, 10, 8).ids, 6)
