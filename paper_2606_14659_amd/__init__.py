"""Python binding of librsb.so, the gfx950 recursive spectral bisection library.

Argument marshalling only: every step of the computation runs in the HIP
library behind the C ABI of ``include/rsb.h``.  Arrays may be numpy arrays
(host memory) or torch tensors on a ROCm device; in the latter case the
library reads and writes them in place (``device_pointers = 1``) and queues
its work on torch's current stream.  There is no CPU fallback: if the
library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsb.so")

GRAPH = {"weighted": 0, "unit": 1, "face": 2}
METHOD = {"lanczos": 0, "inverse_cg": 1, "auto": 2, "block": 3}
PRECISION = {"fp64": 0, "mixed": 1}
PRECOND = {"none": 0, "amg": 1}

OK, WARN_NOT_CONVERGED, WARN_DISCONNECTED = 0, 1, 2
EINVAL, ENOMEM, EDEVICE, EBUFFER, EINTERNAL = -1, -2, -3, -4, -5
# rsb_partition_noalloc limits (RSB_NOALLOC_* in rsb.h)
NOALLOC_SCRATCH_BYTES, NOALLOC_MAX_ELEMS, NOALLOC_MAX_PARTS = 256 << 20, 65536, 1024


class Opts(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32), ("graph", C.c_int32), ("method", C.c_int32),
        ("precision", C.c_int32), ("lanczos_m", C.c_int32), ("max_restarts", C.c_int32),
        ("tol", C.c_double), ("inv_max_outer", C.c_int32), ("cg_max_iter", C.c_int32),
        ("cg_tol", C.c_double), ("cg_full_projection", C.c_int32), ("batched", C.c_int32),
        ("seed", C.c_uint64), ("use_hipgraph", C.c_int32), ("autotune", C.c_int32),
        ("autotune_cache", C.c_char_p), ("device", C.c_int32), ("device_pointers", C.c_int32),
        ("stream", C.c_void_p), ("device_mem_limit", C.c_int64), ("verbose", C.c_int32),
        ("profile", C.c_int32), ("rows_per_thread", C.c_int32), ("lanczos_keep", C.c_int32),
        ("inv_precond", C.c_int32), ("amg_smooth", C.c_int32), ("amg_sigma", C.c_double),
        ("fiedler_sweep", C.c_int32), ("warm_start", C.c_int32), ("sweep_gap", C.c_double),
        ("reorder", C.c_int32), ("gather_scatter", C.c_int32), ("second_solve", C.c_int32),
        ("lanczos_s", C.c_int32),
        ("pack_matrix", C.c_int32), ("bfs_start", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32), ("levels", C.c_int32), ("level_steps", C.c_int64),
        ("segment_steps", C.c_int64), ("cycles", C.c_int64), ("spmv_fp64", C.c_int64),
        ("not_converged", C.c_int32), ("disconnected", C.c_int32), ("lambda2", C.c_double),
        ("residual", C.c_double), ("ms_graph", C.c_double), ("ms_solve", C.c_double),
        ("ms_split", C.c_double), ("ms_total", C.c_double), ("edge_cut", C.c_double),
        ("cut_pairs", C.c_int64), ("max_neighbors", C.c_int32), ("avg_neighbors", C.c_double),
        ("nnz", C.c_int64), ("kernel_bytes", C.c_double), ("kernel_ms", C.c_double),
        ("kernel_launches", C.c_int64), ("tile_rows", C.c_int32), ("amg_levels", C.c_int32),
        ("sweeps", C.c_int32), ("sweep_moved", C.c_int32), ("fallbacks", C.c_int32),
        ("reserved", C.c_int32), ("ms_reorder", C.c_double), ("spmv_alone_us", C.c_double),
        ("spmv_alone_bytes", C.c_double), ("packed_fraction", C.c_double),
        ("matrix_bytes", C.c_double), ("staged_fraction", C.c_double),
        ("spmv_words_us", C.c_double), ("spmv_words_bytes", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("reserved", "struct_size")}


class RsbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rsb error {code}: {msg}")
        self.code = code


_lib = None

# Every function of the C ABI, with its ctypes signature.
_SIGNATURES = {
    "rsb_opts_init": ([C.c_void_p], C.c_int),
    "rsb_dual_graph": ([C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                        C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "rsb_laplacian_apply": ([C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p], C.c_int),
    "rsb_gs_apply": ([C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
                     C.c_int),
    "rsb_locality_order": ([C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p], C.c_int),
    "rsb_fiedler": ([C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                     C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "rsb_split": ([C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "rsb_partition": ([C.c_int64, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                       C.c_void_p], C.c_int),
    "rsb_partition_noalloc": ([C.c_int64, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                               C.c_void_p, C.c_void_p], C.c_int),
    "rsb_partition_batch": ([C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rsb_amg_level": ([C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                       C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "rsb_amg_vcycle": ([C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                        C.c_void_p], C.c_int),
    "rsb_hbm_probe": ([C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.POINTER(C.c_double)],
                      C.c_int),
    "rsb_strerror": ([C.c_int], C.c_char_p),
    "rsb_last_error": ([], C.c_char_p),
}


def _share_torch_hip_runtime():
    """Load PyTorch's HIP runtime before librsb.so.

    PyTorch-ROCm ships its own libamdhip64; two HIP runtimes in one process
    cannot both open the GPU.  Loading torch's copy first makes the loader
    resolve librsb.so's libamdhip64 dependency to it, so torch tensors and the
    library share one runtime whichever is imported first.
    """
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if not (spec and spec.origin):
        return
    path = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
    if os.path.exists(path):
        C.CDLL(path, mode=C.RTLD_GLOBAL)


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2606_14659_amd.build`")
        _share_torch_hip_runtime()
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code: int, what: str) -> int:
    if code < 0:
        msg = lib().rsb_last_error().decode()
        raise RsbError(code, f"{what}: {msg or lib().rsb_strerror(code).decode()}")
    return code


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def make_opts(device_arrays: bool = False, **kw) -> Opts:
    o = Opts()
    _check(lib().rsb_opts_init(C.byref(o)), "rsb_opts_init")
    for k, v in kw.items():
        if k == "graph" and isinstance(v, str):
            v = GRAPH[v]
        elif k == "method" and isinstance(v, str):
            v = METHOD[v]
        elif k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        elif k == "inv_precond" and isinstance(v, str):
            v = PRECOND[v]
        elif k == "autotune_cache" and isinstance(v, str):
            v = v.encode()
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    if device_arrays:
        import torch
        o.device_pointers = 1
        o.device = torch.cuda.current_device()
        o.stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return o


class _Arr:
    """An argument array: numpy (host) or torch (device) with its pointer."""

    def __init__(self, a, dtype, device: bool):
        if device:
            import torch
            tdt = {np.int64: torch.int64, np.int32: torch.int32, np.float64: torch.float64,
                   np.uint8: torch.uint8}[dtype]
            if not _is_torch(a):
                a = torch.as_tensor(np.ascontiguousarray(a, dtype=dtype))
            self.a = a.to(device="cuda", dtype=tdt).contiguous()
            self.ptr = C.c_void_p(self.a.data_ptr())
        else:
            self.a = np.ascontiguousarray(a, dtype=dtype)
            self.ptr = self.a.ctypes.data_as(C.c_void_p)


def _out(shape, dtype, device: bool):
    if device:
        import torch
        tdt = {np.int64: torch.int64, np.int32: torch.int32, np.float64: torch.float64,
               np.uint8: torch.uint8}[dtype]
        t = torch.empty(shape, dtype=tdt, device="cuda")
        return t, C.c_void_p(t.data_ptr())
    a = np.zeros(shape, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _ids_shape(ids):
    if len(ids.shape) != 2:
        raise ValueError("ids must be a [nelem, nv] array")
    return int(ids.shape[0]), int(ids.shape[1])


def dual_graph(ids, device: bool = False, **kw):
    """Off-diagonal CSR of the dual-graph Laplacian: (row_ptr, col, weight)."""
    n, nv = _ids_shape(ids)
    o = make_opts(device, **kw)
    a = _Arr(ids, np.int64, device)
    nnz = C.c_int64(0)
    _check(lib().rsb_dual_graph(n, nv, a.ptr, C.byref(o), None, None, None, C.byref(nnz)),
           "rsb_dual_graph")
    rp, rpp = _out(n + 1, np.int64, device)
    col, colp = _out(max(nnz.value, 1), np.int32, device)
    w, wp = _out(max(nnz.value, 1), np.int32, device)
    _check(lib().rsb_dual_graph(n, nv, a.ptr, C.byref(o), rpp, colp, wp, C.byref(nnz)),
           "rsb_dual_graph")
    return rp, col[: nnz.value], w[: nnz.value]


def laplacian_apply(row_ptr, col, weight, x, device: bool = False, **kw):
    n = len(row_ptr) - 1
    o = make_opts(device, **kw)
    rp = _Arr(row_ptr, np.int64, device)
    c = _Arr(col if len(col) else np.zeros(1), np.int32, device)
    w = _Arr(weight if len(weight) else np.zeros(1), np.int32, device)
    xx = _Arr(x, np.float64, device)
    y, yp = _out(n, np.float64, device)
    _check(lib().rsb_laplacian_apply(n, rp.ptr, c.ptr, w.ptr, xx.ptr, yp, C.byref(o)),
           "rsb_laplacian_apply")
    return y


def gs_apply(ids, x, device: bool = False, **kw):
    """y = L x in the gather-scatter form (element -> vertex -> element)."""
    n, nv = _ids_shape(ids)
    ids_a = _Arr(ids, np.int64, device)
    o = make_opts(device, **kw)
    xx = _Arr(x, np.float64, device)
    y, yp = _out(n, np.float64, device)
    _check(lib().rsb_gs_apply(n, nv, ids_a.ptr, xx.ptr, yp, C.byref(o)), "rsb_gs_apply")
    return y


def locality_order(row_ptr, col, weight, device: bool = False, **kw):
    """Cuthill-McKee order of a CSR graph: order[k] = row placed at position k."""
    n = len(row_ptr) - 1
    o = make_opts(device, **kw)
    rp = _Arr(row_ptr, np.int64, device)
    c = _Arr(col if len(col) else np.zeros(1), np.int32, device)
    w = _Arr(weight if len(weight) else np.zeros(1), np.int32, device)
    out, op = _out(n, np.int32, device)
    _check(lib().rsb_locality_order(n, rp.ptr, c.ptr, w.ptr, op, C.byref(o)),
           "rsb_locality_order")
    return out


def amg_level(row_ptr, col, weight, level: int, **kw) -> dict:
    """Level `level` of the AMG hierarchy of a CSR graph (host arrays):
    nlevels, row_ptr, col, weight, gid, agg (-1 on the coarsest level)."""
    n = len(row_ptr) - 1
    o = make_opts(False, **kw)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col if len(col) else np.zeros(1), dtype=np.int32)
    w = np.ascontiguousarray(weight if len(weight) else np.zeros(1), dtype=np.int32)
    nl, nr, nz = C.c_int32(0), C.c_int64(0), C.c_int64(0)
    L = lib()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    _check(L.rsb_amg_level(n, ptr(rp), ptr(c), ptr(w), int(level), C.byref(o), C.byref(nl),
                           C.byref(nr), C.byref(nz), None, None, None, None, None),
           "rsb_amg_level")
    out = {"nlevels": nl.value, "row_ptr": np.zeros(nr.value + 1, dtype=np.int64),
           "col": np.zeros(max(nz.value, 1), dtype=np.int64),
           "weight": np.zeros(max(nz.value, 1), dtype=np.int64),
           "gid": np.zeros(max(nr.value, 1), dtype=np.int64),
           "agg": np.zeros(max(nr.value, 1), dtype=np.int64)}
    _check(L.rsb_amg_level(n, ptr(rp), ptr(c), ptr(w), int(level), C.byref(o), C.byref(nl),
                           C.byref(nr), C.byref(nz), ptr(out["row_ptr"]), ptr(out["col"]),
                           ptr(out["weight"]), ptr(out["gid"]), ptr(out["agg"])),
           "rsb_amg_level")
    out["col"] = out["col"][:nz.value]
    out["weight"] = out["weight"][:nz.value]
    out["gid"] = out["gid"][:nr.value]
    out["agg"] = out["agg"][:nr.value]
    return out


def amg_vcycle(row_ptr, col, weight, f, device: bool = False, **kw):
    """u = M f, one V-cycle of the AMG hierarchy of a CSR graph."""
    n = len(row_ptr) - 1
    o = make_opts(device, **kw)
    rp = _Arr(row_ptr, np.int64, device)
    c = _Arr(col if len(col) else np.zeros(1), np.int32, device)
    w = _Arr(weight if len(weight) else np.zeros(1), np.int32, device)
    ff = _Arr(f, np.float64, device)
    u, up = _out(n, np.float64, device)
    _check(lib().rsb_amg_vcycle(n, rp.ptr, c.ptr, w.ptr, ff.ptr, up, C.byref(o)), "rsb_amg_vcycle")
    return u


def split(y, gid, n_low, device: bool = False, **kw):
    n = len(y)
    o = make_opts(device, **kw)
    yy = _Arr(y, np.float64, device)
    g = _Arr(gid, np.int64, device)
    side, sp = _out(n, np.uint8, device)
    _check(lib().rsb_split(n, yy.ptr, g.ptr, int(n_low), sp, C.byref(o)), "rsb_split")
    return side


def fiedler(ids, device: bool = False, **kw):
    """(status, lambda2, y, stats) of the mesh's dual-graph Laplacian."""
    n, nv = _ids_shape(ids)
    o = make_opts(device, **kw)
    a = _Arr(ids, np.int64, device)
    y, yp = _out(n, np.float64, device)
    lam = C.c_double(0)
    st = Stats()
    st.struct_size = C.sizeof(Stats)
    code = _check(lib().rsb_fiedler(n, nv, a.ptr, C.byref(o), yp, C.byref(lam), C.byref(st)),
                  "rsb_fiedler")
    return code, lam.value, y, st.as_dict()


def partition(ids, nparts: int, device: bool = False, **kw):
    """(status, part, stats): recursive spectral bisection into nparts parts."""
    n, nv = _ids_shape(ids)
    o = make_opts(device, **kw)
    a = _Arr(ids, np.int64, device)
    part, pp = _out(n, np.int32, device)
    st = Stats()
    st.struct_size = C.sizeof(Stats)
    code = _check(lib().rsb_partition(n, nv, a.ptr, int(nparts), C.byref(o), pp, C.byref(st)),
                  "rsb_partition")
    return code, part, st.as_dict()


def partition_noalloc(ids, nparts: int, device: bool = False, **kw):
    """(status, part, stats): rsb_partition with its device scratch in the
    library's fixed region (no device allocation by the library)."""
    n, nv = _ids_shape(ids)
    o = make_opts(device, **kw)
    a = _Arr(ids, np.int64, device)
    part, pp = _out(n, np.int32, device)
    st = Stats()
    st.struct_size = C.sizeof(Stats)
    code = _check(lib().rsb_partition_noalloc(n, nv, a.ptr, int(nparts), C.byref(o), pp,
                                              C.byref(st)), "rsb_partition_noalloc")
    return code, part, st.as_dict()


def hbm_probe(kind: str, nbytes: int, reps: int = 10, **kw) -> float:
    """GB/s of a plain HBM stream: kind 'read', 'copy' (read + write bytes) or 'write'."""
    o = make_opts(False, **kw)
    gbs = C.c_double(0)
    _check(lib().rsb_hbm_probe({"read": 0, "copy": 1, "write": 2}[kind], int(nbytes), int(reps),
                               C.byref(o), C.byref(gbs)), "rsb_hbm_probe")
    return gbs.value


def partition_batch(ids_list, nparts_list, device: bool = False, **kw):
    """(status, [part], stats) for independent meshes in one call."""
    nmesh = len(ids_list)
    nv = _ids_shape(ids_list[0])[1]
    if any(_ids_shape(a)[1] != nv for a in ids_list):
        raise ValueError("every mesh of a batch must have the same number of ids per element")
    o = make_opts(device, **kw)
    arrs = [_Arr(a, np.int64, device) for a in ids_list]
    nelem = (C.c_int64 * nmesh)(*[int(a.shape[0]) for a in ids_list])
    nparts = (C.c_int32 * nmesh)(*[int(p) for p in nparts_list])
    idp = (C.c_void_p * nmesh)(*[a.ptr.value for a in arrs])
    outs = [_out(int(a.shape[0]), np.int32, device) for a in ids_list]
    pp = (C.c_void_p * nmesh)(*[p.value for _, p in outs])
    st = Stats()
    st.struct_size = C.sizeof(Stats)
    code = _check(lib().rsb_partition_batch(nmesh, nelem, nv, idp, nparts, C.byref(o), pp,
                                            C.byref(st)), "rsb_partition_batch")
    return code, [p for p, _ in outs], st.as_dict()
