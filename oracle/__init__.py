"""ctypes binding of the plain FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the partitioning library never does.
``build()`` compiles ``oracle.cpp`` with g++ into ``liboracle.so`` next to it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.cpp")

GRAPH = {"weighted": 0, "unit": 1, "face": 2}
METHOD = {"lanczos": 0, "inverse_cg": 1, "auto": 2, "block": 3}
PRECOND = {"none": 0, "amg": 1}


class Opts(C.Structure):
    _fields_ = [("graph", C.c_int32), ("method", C.c_int32), ("lanczos_m", C.c_int32),
                ("max_restarts", C.c_int32), ("tol", C.c_double), ("inv_max_outer", C.c_int32),
                ("cg_max_iter", C.c_int32), ("cg_tol", C.c_double),
                ("cg_full_projection", C.c_int32), ("seed", C.c_uint64),
                ("lanczos_keep", C.c_int32), ("inv_precond", C.c_int32),
                ("amg_smooth", C.c_int32), ("amg_sigma", C.c_double),
                ("fiedler_sweep", C.c_int32), ("sweep_gap", C.c_double),
                ("warm_start", C.c_int32), ("second_solve", C.c_int32),
                ("lanczos_s", C.c_int32), ("bfs_start", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("converged", C.c_int32), ("matvecs", C.c_int64),
                ("theta", C.c_double), ("residual", C.c_double), ("ncomp", C.c_int32),
                ("cg_iters", C.c_int32), ("amg_levels", C.c_int32), ("sweeps", C.c_int32),
                ("sweep_moved", C.c_int32), ("fallbacks", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# IEEE double without contraction into fused multiply-adds (the same bits
# with or without an FMA unit), element loops threaded by OpenMP.
CXXFLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off"]


def build(force: bool = True, out: str = LIB, native: bool = False) -> str:
    """Compile the oracle into `out`.  native=True adds -march=native (for
    timing on the machine that runs it; the committed tests use the portable
    build)."""
    if force or not os.path.exists(out):
        cmd = ["g++"] + CXXFLAGS + (["-march=native"] if native else []) + [
            "-o", out + ".tmp", SRC]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = load(LIB)
    return _lib


def use_library(path: str):
    """Load the oracle from another build of the same source (for example a
    -march=native build for timing) and use it from now on."""
    global _lib
    _lib = load(path)
    return _lib


def load(path: str):
    """Load an oracle library file and declare its functions."""
    L = C.CDLL(path)
    P = C.POINTER
    L.orc_opts_default.argtypes = [P(Opts)]
    L.orc_start_value.argtypes = [C.c_uint64, C.c_int64]
    L.orc_start_value.restype = C.c_double
    L.orc_dual_graph.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_void_p, P(C.c_int64)]
    L.orc_laplacian_apply.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]
    L.orc_tridiag_smallest.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                       P(C.c_double), C.c_void_p]
    L.orc_jacobi_eigen.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_fiedler.argtypes = [C.c_int64, C.c_int32, C.c_void_p, P(Opts), C.c_void_p,
                              P(C.c_double), P(Info)]
    L.orc_fiedler_csr.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  P(Opts), C.c_void_p, P(C.c_double), P(Info)]
    L.orc_split.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    L.orc_gs_apply.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_locality_order.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_bfs_start.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_partition.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_int32, P(Opts),
                                C.c_void_p, P(Info)]
    L.orc_metrics.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                              C.c_void_p]
    L.orc_amg_level.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int32, P(C.c_int32), P(C.c_int64), P(C.c_int64),
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_amg_vcycle.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_double, C.c_int32, C.c_void_p, C.c_void_p]
    L.orc_cg_solve.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               P(Opts), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                               P(C.c_int32)]
    L.orc_block_pair.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 P(Opts), C.c_void_p, C.c_void_p, C.c_void_p, P(Info)]
    L.orc_set_threads.argtypes = [C.c_int32]
    return L


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's element loops (0: unchanged); returns the count."""
    return lib().orc_set_threads(int(n))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def opts(**kw) -> Opts:
    o = Opts()
    lib().orc_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "graph" and isinstance(v, str):
            v = GRAPH[v]
        if k == "method" and isinstance(v, str):
            v = METHOD[v]
        if k == "inv_precond" and isinstance(v, str):
            v = PRECOND[v]
        setattr(o, k, v)
    return o


def jacobi_eigen(A):
    """(eigenvalues ascending, eigenvectors as columns) of a symmetric matrix."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    k = A.shape[0]
    ev = np.zeros(k)
    V = np.zeros((k, k))
    lib().orc_jacobi_eigen(k, _ptr(A), _ptr(ev), _ptr(V))
    return ev, V


def start_value(seed: int, gid: int) -> float:
    return lib().orc_start_value(seed, gid)


def _ids(ids) -> np.ndarray:
    a = np.ascontiguousarray(ids, dtype=np.int64)
    if a.ndim != 2:
        raise ValueError("ids must be [nelem, nv]")
    return a


def dual_graph(ids, graph="weighted"):
    """(row_ptr int64[n+1], col int32[nnz], weight int32[nnz])."""
    a = _ids(ids)
    n, nv = a.shape
    g = GRAPH[graph] if isinstance(graph, str) else graph
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    nnz = C.c_int64(0)
    rc = lib().orc_dual_graph(n, nv, _ptr(a), g, _ptr(row_ptr), None, None, C.byref(nnz))
    if rc != 0:
        raise RuntimeError(f"orc_dual_graph: {rc}")
    col = np.zeros(max(nnz.value, 1), dtype=np.int32)
    w = np.zeros(max(nnz.value, 1), dtype=np.int32)
    rc = lib().orc_dual_graph(n, nv, _ptr(a), g, _ptr(row_ptr), _ptr(col), _ptr(w), C.byref(nnz))
    if rc != 0:
        raise RuntimeError(f"orc_dual_graph: {rc}")
    return row_ptr, col[: nnz.value], w[: nnz.value]


def laplacian_apply(row_ptr, col, w, x) -> np.ndarray:
    n = len(row_ptr) - 1
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(n, dtype=np.float64)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    lib().orc_laplacian_apply(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(x), _ptr(y))
    return y


def gs_apply(ids, x) -> np.ndarray:
    """y = L x in the gather-scatter form (element -> vertex -> element)."""
    a = _ids(ids)
    n, nv = a.shape
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(n, dtype=np.float64)
    rc = lib().orc_gs_apply(n, nv, _ptr(a), _ptr(xx), _ptr(y))
    if rc != 0:
        raise RuntimeError(f"orc_gs_apply: {rc}")
    return y


def locality_order(row_ptr, col, w) -> np.ndarray:
    """Cuthill-McKee order: order[k] = row placed at position k."""
    n = len(row_ptr) - 1
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    out = np.zeros(n, dtype=np.int32)
    rc = lib().orc_locality_order(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"orc_locality_order: {rc}")
    return out


def bfs_start(row_ptr, col, w) -> np.ndarray:
    """Start values of bfs_start on a CSR graph (NaN where not reached)."""
    n = len(row_ptr) - 1
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    out = np.zeros(n, dtype=np.float64)
    rc = lib().orc_bfs_start(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"orc_bfs_start: {rc}")
    return out


def tridiag_smallest(a, b, thr=0.0):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    k = len(a)
    t = np.zeros(k, dtype=np.float64)
    th = C.c_double(0)
    rc = lib().orc_tridiag_smallest(k, _ptr(a), _ptr(b), thr, C.byref(th), _ptr(t))
    if rc != 0:
        raise RuntimeError(f"orc_tridiag_smallest: {rc}")
    return th.value, t


def fiedler(ids, **kw):
    """(status, lambda2, y, info) for the whole mesh."""
    a = _ids(ids)
    n, nv = a.shape
    o = opts(**kw)
    y = np.zeros(n, dtype=np.float64)
    lam = C.c_double(0)
    info = Info()
    rc = lib().orc_fiedler(n, nv, _ptr(a), C.byref(o), _ptr(y), C.byref(lam), C.byref(info))
    if rc < 0:
        raise RuntimeError(f"orc_fiedler: {rc}")
    return rc, lam.value, y, info.as_dict()


def fiedler_csr(row_ptr, col, w, gid=None, **kw):
    n = len(row_ptr) - 1
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    g = np.arange(n, dtype=np.int64) if gid is None else np.ascontiguousarray(gid, dtype=np.int64)
    o = opts(**kw)
    y = np.zeros(n, dtype=np.float64)
    lam = C.c_double(0)
    info = Info()
    rc = lib().orc_fiedler_csr(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(g), C.byref(o), _ptr(y),
                               C.byref(lam), C.byref(info))
    if rc < 0:
        raise RuntimeError(f"orc_fiedler_csr: {rc}")
    return rc, lam.value, y, info.as_dict()


def block_pair(row_ptr, col, w, gid=None, **kw):
    """Block Lanczos pair on a connected CSR graph: (status, y1, y2,
    (theta1, theta2), info); theta2 = inf when there is no second direction."""
    n, rp, c, ww, g = _csr_args(row_ptr, col, w, gid)
    o = opts(**dict(kw, method="block"))
    y1 = np.zeros(n, dtype=np.float64)
    y2 = np.zeros(n, dtype=np.float64)
    th = np.zeros(2, dtype=np.float64)
    info = Info()
    rc = lib().orc_block_pair(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(g), C.byref(o), _ptr(y1),
                              _ptr(y2), _ptr(th), C.byref(info))
    if rc < 0:
        raise RuntimeError(f"orc_block_pair: {rc}")
    return rc, y1, y2, (float(th[0]), float(th[1])), info.as_dict()


def _csr_args(row_ptr, col, w, gid):
    n = len(row_ptr) - 1
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    g = np.arange(n, dtype=np.int64) if gid is None else np.ascontiguousarray(gid, dtype=np.int64)
    return n, rp, c, ww, g


def amg_level(row_ptr, col, w, level, gid=None):
    """Level `level` of the AMG hierarchy: dict with nlevels, row_ptr, col,
    weight, gid (per row) and agg (row -> row of the next level, -1 on the
    coarsest level)."""
    n, rp, c, ww, g = _csr_args(row_ptr, col, w, gid)
    nl, nr, nz = C.c_int32(0), C.c_int64(0), C.c_int64(0)
    rc = lib().orc_amg_level(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(g), int(level), C.byref(nl),
                             C.byref(nr), C.byref(nz), None, None, None, None, None)
    if rc != 0:
        raise RuntimeError(f"orc_amg_level: {rc} (levels {nl.value})")
    out = {"nlevels": nl.value,
           "row_ptr": np.zeros(nr.value + 1, dtype=np.int64),
           "col": np.zeros(max(nz.value, 1), dtype=np.int64),
           "weight": np.zeros(max(nz.value, 1), dtype=np.int64),
           "gid": np.zeros(nr.value, dtype=np.int64),
           "agg": np.zeros(nr.value, dtype=np.int64)}
    rc = lib().orc_amg_level(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(g), int(level), C.byref(nl),
                             C.byref(nr), C.byref(nz), _ptr(out["row_ptr"]), _ptr(out["col"]),
                             _ptr(out["weight"]), _ptr(out["gid"]), _ptr(out["agg"]))
    if rc != 0:
        raise RuntimeError(f"orc_amg_level: {rc}")
    out["col"] = out["col"][:nz.value]
    out["weight"] = out["weight"][:nz.value]
    return out


def amg_vcycle(row_ptr, col, w, f, sigma=2.0 / 3.0, nsmooth=1, gid=None) -> np.ndarray:
    """u = M f, one V-cycle of the AMG hierarchy of the graph."""
    n, rp, c, ww, g = _csr_args(row_ptr, col, w, gid)
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.zeros(n, dtype=np.float64)
    rc = lib().orc_amg_vcycle(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(g), float(sigma), int(nsmooth),
                              _ptr(f), _ptr(u))
    if rc != 0:
        raise RuntimeError(f"orc_amg_vcycle: {rc}")
    return u


def cg_solve(row_ptr, col, w, b, gid=None, max_dirs=0, **kw):
    """One inner CG solve of inverse iteration: (steps, x, directions) with
    directions[k] = the k-th search direction (at most max_dirs of them)."""
    n, rp, c, ww, g = _csr_args(row_ptr, col, w, gid)
    o = opts(**kw)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n, dtype=np.float64)
    dirs = np.zeros((max(max_dirs, 1), n), dtype=np.float64)
    nd = C.c_int32(0)
    its = lib().orc_cg_solve(n, _ptr(rp), _ptr(c), _ptr(ww), _ptr(g), C.byref(o), _ptr(bb),
                             _ptr(x), int(max_dirs), _ptr(dirs) if max_dirs > 0 else None,
                             C.byref(nd))
    if its < 0:
        raise RuntimeError(f"orc_cg_solve: {its}")
    return its, x, dirs[:nd.value]


def split(y, gid, n_low) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.ascontiguousarray(gid, dtype=np.int64)
    side = np.zeros(len(y), dtype=np.uint8)
    rc = lib().orc_split(len(y), _ptr(y), _ptr(g), int(n_low), _ptr(side))
    if rc != 0:
        raise RuntimeError(f"orc_split: {rc}")
    return side


def partition(ids, nparts, **kw):
    """(status, part int32[n], info)."""
    a = _ids(ids)
    n, nv = a.shape
    o = opts(**kw)
    part = np.zeros(n, dtype=np.int32)
    info = Info()
    rc = lib().orc_partition(n, nv, _ptr(a), int(nparts), C.byref(o), _ptr(part), C.byref(info))
    if rc < 0:
        raise RuntimeError(f"orc_partition: {rc}")
    return rc, part, info.as_dict()


def metrics(ids, part, nparts) -> dict:
    a = _ids(ids)
    n, nv = a.shape
    p = np.ascontiguousarray(part, dtype=np.int32)
    out = np.zeros(6, dtype=np.float64)
    rc = lib().orc_metrics(n, nv, _ptr(a), int(nparts), _ptr(p), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"orc_metrics: {rc}")
    return {"weighted_cut": out[0], "cut_pairs": out[1], "max_neighbors": out[2],
            "avg_neighbors": out[3], "min_size": out[4], "max_size": out[5]}
