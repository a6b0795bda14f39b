"""CPU-side checks of the GPU library: it loads, exports every function that
include/rsb.h declares, and its host-side argument checks reject bad input
(no kernel runs in any of these)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2606_14659_amd as rsb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rsb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsb_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("rsb_opts_init", "rsb_partition", "rsb_fiedler", "rsb_dual_graph",
                 "rsb_partition_batch", "rsb_strerror", "rsb_last_error", "rsb_split",
                 "rsb_laplacian_apply", "rsb_locality_order", "rsb_gs_apply"):
        assert need in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(rsb.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(rsb._SIGNATURES)


def test_struct_sizes_match():
    o = rsb.Opts()
    assert rsb.lib().rsb_opts_init(C.byref(o)) == 0
    assert o.struct_size == C.sizeof(rsb.Opts)
    assert o.lanczos_m == 100 and o.max_restarts == 50 and o.seed == 20261203
    assert o.inv_precond == 0 and o.amg_smooth == 1 and abs(o.amg_sigma - 2.0 / 3.0) < 1e-15
    assert rsb.lib().rsb_opts_init(None) == rsb.EINVAL


def test_strerror():
    for code in (0, 1, 2, -1, -2, -3, -4, -5):
        assert rsb.lib().rsb_strerror(code)
    assert rsb.lib().rsb_strerror(99) == b"unknown code"


def test_bad_options_rejected_before_any_device_call():
    ids = np.array([[0, 1, 2, 3], [2, 3, 4, 5]], dtype=np.int64)
    o = rsb.Opts()
    rsb.lib().rsb_opts_init(C.byref(o))
    bad = []
    for field, value in (("struct_size", 4), ("graph", 7), ("method", 4), ("method", -1),
                         ("lanczos_m", 0), ("lanczos_m", 251),
                         ("tol", 0.0), ("cg_full_projection", 33), ("cg_full_projection", -1),
                         ("precision", 5),
                         ("rows_per_thread", 3), ("rows_per_thread", 16), ("autotune", 3),
                         ("lanczos_keep", -1), ("lanczos_keep", 17), ("lanczos_keep", 100),
                         ("inv_precond", 2), ("inv_precond", -1), ("amg_smooth", -1),
                         ("amg_smooth", 17), ("amg_sigma", 0.0), ("amg_sigma", 2.0),
                         ("fiedler_sweep", -1), ("fiedler_sweep", 65), ("sweep_gap", -1.0),
                         ("warm_start", 2), ("warm_start", -1), ("reorder", 2),
                         ("gather_scatter", 2), ("gather_scatter", -1), ("lanczos_s", 3),
                         ("lanczos_s", 0), ("pack_matrix", 3), ("pack_matrix", -1),
                         ("bfs_start", 2), ("bfs_start", -1)):
        oo = rsb.Opts.from_buffer_copy(o)
        setattr(oo, field, value)
        part = np.zeros(2, dtype=np.int32)
        code = rsb.lib().rsb_partition(2, 4, ids.ctypes.data_as(C.c_void_p), 2, C.byref(oo),
                                       part.ctypes.data_as(C.c_void_p), None)
        bad.append(code)
        assert rsb.lib().rsb_last_error()
    assert all(c == rsb.EINVAL for c in bad), bad
    # the sweep needs thick-restart Lanczos
    for method, keep in ((0, 0), (0, 1), (1, 8)):
        oo = rsb.Opts.from_buffer_copy(o)
        oo.fiedler_sweep, oo.method, oo.lanczos_keep = 8, method, keep
        part = np.zeros(2, dtype=np.int32)
        assert rsb.lib().rsb_partition(2, 4, ids.ctypes.data_as(C.c_void_p), 2, C.byref(oo),
                                       part.ctypes.data_as(C.c_void_p), None) == rsb.EINVAL
        oo.fiedler_sweep, oo.warm_start = 0, 1
        part = np.zeros(2, dtype=np.int32)
        assert rsb.lib().rsb_partition(2, 4, ids.ctypes.data_as(C.c_void_p), 2, C.byref(oo),
                                       part.ctypes.data_as(C.c_void_p), None) == rsb.EINVAL
    # the block solver: an even basis of 4..48 vectors, an even kept count
    # leaving two blocks, no gather-scatter operator, no second solve
    for m, keep, gs, second in ((41, 8, 0, 0), (50, 8, 0, 0), (2, 0, 0, 0), (40, 7, 0, 0),
                                (40, 38, 0, 0), (40, 8, 1, 0), (40, 8, 0, 1)):
        oo = rsb.Opts.from_buffer_copy(o)
        oo.method, oo.lanczos_m, oo.lanczos_keep = 3, m, keep
        oo.gather_scatter, oo.second_solve, oo.fiedler_sweep = gs, second, 8 * second
        part = np.zeros(2, dtype=np.int32)
        assert rsb.lib().rsb_partition(2, 4, ids.ctypes.data_as(C.c_void_p), 2, C.byref(oo),
                                       part.ctypes.data_as(C.c_void_p), None) == rsb.EINVAL, \
            (m, keep, gs, second)
    # the gather-scatter operator is the weighted Laplacian, applied by Lanczos
    for graph, method in ((1, 0), (2, 0), (0, 1)):
        oo = rsb.Opts.from_buffer_copy(o)
        oo.gather_scatter, oo.graph, oo.method = 1, graph, method
        oo.warm_start = 0
        part = np.zeros(2, dtype=np.int32)
        assert rsb.lib().rsb_partition(2, 4, ids.ctypes.data_as(C.c_void_p), 2, C.byref(oo),
                                       part.ctypes.data_as(C.c_void_p), None) == rsb.EINVAL


def test_bad_arguments_rejected():
    ids = np.array([[0, 1, 2, 3], [2, 3, 4, 5]], dtype=np.int64)
    o = rsb.make_opts()
    part = np.zeros(2, dtype=np.int32)
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    L = rsb.lib()
    assert L.rsb_partition(2, 4, None, 2, C.byref(o), P(part), None) == rsb.EINVAL
    assert L.rsb_partition(0, 4, P(ids), 1, C.byref(o), P(part), None) == rsb.EINVAL
    assert L.rsb_partition(2, 0, P(ids), 1, C.byref(o), P(part), None) == rsb.EINVAL
    assert L.rsb_partition(2, 4, P(ids), 3, C.byref(o), P(part), None) == rsb.EINVAL
    assert L.rsb_partition(2, 4, P(ids), 0, C.byref(o), P(part), None) == rsb.EINVAL
    st = rsb.Stats()
    st.struct_size = 3
    assert L.rsb_partition(2, 4, P(ids), 2, C.byref(o), P(part), C.byref(st)) == rsb.EINVAL
    y = np.array([0.0, np.nan])
    g = np.array([0, 1], dtype=np.int64)
    side = np.zeros(2, dtype=np.uint8)
    assert L.rsb_split(2, P(y), P(g), 1, P(side), C.byref(o)) == rsb.EINVAL
    y = np.array([0.0, 1.0])
    assert L.rsb_split(2, P(y), P(g), 3, P(side), C.byref(o)) == rsb.EINVAL
    assert L.rsb_fiedler(1, 4, P(ids), C.byref(o), P(y), C.byref(C.c_double()), None) == rsb.EINVAL
    nnz = C.c_int64(0)
    assert L.rsb_dual_graph(2, 4, P(ids), C.byref(o), None, None, None, None) == rsb.EINVAL


def test_python_binding_raises_without_library(monkeypatch):
    monkeypatch.setattr(rsb, "_lib", None)
    monkeypatch.setattr(rsb, "LIB_PATH", "/nonexistent/librsb.so")
    with pytest.raises(RuntimeError):
        rsb.lib()


def test_batch_rejects_mixed_element_sizes():
    quads = np.array([[0, 1, 2, 3]], dtype=np.int64)
    hexes = np.arange(16, dtype=np.int64).reshape(2, 8)
    with pytest.raises(ValueError):
        rsb.partition_batch([quads, hexes], [1, 2])


def test_batch_bad_arguments_rejected_before_any_device_call():
    L = rsb.lib()
    o = rsb.make_opts()
    ids = np.array([[0, 1, 2, 3], [2, 3, 4, 5]], dtype=np.int64)
    part = np.zeros(2, dtype=np.int32)
    nelem = (C.c_int64 * 2)(2, 2)
    idp = (C.c_void_p * 2)(ids.ctypes.data, ids.ctypes.data)
    parts_ok = (C.c_int32 * 2)(2, 1)
    out_ok = (C.c_void_p * 2)(part.ctypes.data, part.ctypes.data)
    out_null = (C.c_void_p * 2)(part.ctypes.data, None)
    too_many = (C.c_int32 * 2)(2, 3)
    none = (C.c_int32 * 2)(0, 1)
    for nmesh, pa, out, why in ((0, parts_ok, out_ok, b"bad arguments"),
                                (2, parts_ok, out_null, b"part_out entry NULL"),
                                (2, too_many, out_ok, b"nparts out of range"),
                                (2, none, out_ok, b"nparts out of range")):
        code = L.rsb_partition_batch(nmesh, nelem, 4, idp, pa, C.byref(o), out, None)
        assert code == rsb.EINVAL and why in L.rsb_last_error()
    assert L.rsb_partition_batch(2, nelem, 4, idp, parts_ok, C.byref(o), None, None) == rsb.EINVAL
    assert L.rsb_partition_batch(2, None, 4, idp, parts_ok, C.byref(o), out_ok, None) == rsb.EINVAL


def test_noalloc_limits_rejected_before_any_device_call():
    # the entry point for callers that cannot allocate: sizes beyond its
    # documented maximum are refused on the host, with the limits named
    hdr = open(os.path.join(ROOT, "include", "rsb.h")).read()
    assert f"#define RSB_NOALLOC_MAX_ELEMS {rsb.NOALLOC_MAX_ELEMS}" in hdr
    assert f"#define RSB_NOALLOC_MAX_PARTS {rsb.NOALLOC_MAX_PARTS}" in hdr
    assert "#define RSB_NOALLOC_SCRATCH_BYTES (256ll << 20)" in hdr
    assert rsb.NOALLOC_SCRATCH_BYTES == 256 << 20
    L = rsb.lib()
    o = rsb.make_opts()
    n = rsb.NOALLOC_MAX_ELEMS + 1
    ids = np.arange(4 * n, dtype=np.int64).reshape(n, 4)
    part = np.zeros(n, dtype=np.int32)
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    assert L.rsb_partition_noalloc(n, 4, P(ids), 2, C.byref(o), P(part), None) == rsb.EINVAL
    assert b"at most 65536 elements and 1024 parts" in L.rsb_last_error()
    assert L.rsb_partition_noalloc(2000, 4, P(ids), 1025, C.byref(o), P(part), None) == rsb.EINVAL
    assert L.rsb_partition_noalloc(2, 4, None, 2, C.byref(o), P(part), None) == rsb.EINVAL
