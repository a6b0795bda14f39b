"""Seeded synthetic mesh generators shared by the tests and the benchmark.

This module only produces inputs: per-element global vertex ids, the form in
which the paper's partitioner receives a mesh (each rank lists the global
vertex ids of its elements, Section 5, gather-scatter setup).  It holds none
of the partitioning arithmetic, so both the CPU oracle and the GPU library can
be fed from it without sharing any of the method.

Every random choice comes from a splitmix64 stream (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014), computed
here with numpy's wrapping uint64 arithmetic.

Meshes
------
* ``box_hex(nx, ny, nz)``: structured hexahedra.  Element (i, j, k) has index
  i + nx*(j + ny*k); its eight vertices are (i+a, j+b, k+c), a, b, c in {0, 1},
  numbered a' + (nx+1)*(b' + (ny+1)*c') and listed in the usual hex order
  (bottom face counter-clockwise, then top face).
* ``box_quad(nx, ny)``: the same in 2D (four vertices per element).
* ``uniform_holes``: removes exactly round(f*N) elements chosen uniformly at
  random; survivors keep their lexicographic order.
* ``clustered_holes``: removes elements whose centroids fall inside random
  spheres (radius uniform in [3, 12] element widths), sphere by sphere and in
  order of distance to each centre, until exactly round(f*N) are gone.
* ``renumber_vertices``: applies a random permutation pi to the vertex ids and
  spreads them over 64 bits as pi(v) * 2**31 + 7.
* ``shuffle_elements``: random element order (for invariance tests).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

BASE_SEED = 20261203


def splitmix64_stream(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset+1 .. offset+count of the splitmix64 stream started at ``seed``."""
    k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of the stream."""
    z = splitmix64_stream(seed, count, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def random_permutation(seed: int, count: int) -> np.ndarray:
    """A uniformly random permutation of range(count): ranks of stream values."""
    z = splitmix64_stream(seed, count)
    return np.argsort(z, kind="stable").astype(np.int64)


@dataclass
class Mesh:
    """A mesh as the partitioner receives it, plus how it was made."""

    ids: np.ndarray                      # int64 [nelem, nv] global vertex ids
    dims: tuple                          # box dimensions (nx, ny[, nz])
    lex: np.ndarray                      # lexicographic box index of every element
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nelem(self) -> int:
        return int(self.ids.shape[0])

    @property
    def nv(self) -> int:
        return int(self.ids.shape[1])


def box_hex(nx: int, ny: int, nz: int) -> Mesh:
    i = np.arange(nx, dtype=np.int64)
    j = np.arange(ny, dtype=np.int64)
    k = np.arange(nz, dtype=np.int64)
    kk, jj, ii = np.meshgrid(k, j, i, indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    corners = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
               (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    ids = np.stack([(ii + a) + sx * (jj + b) + sy * (kk + c) for a, b, c in corners], axis=1)
    return Mesh(ids=np.ascontiguousarray(ids, dtype=np.int64), dims=(nx, ny, nz),
                lex=np.arange(nx * ny * nz, dtype=np.int64), name=f"box{nx}x{ny}x{nz}")


def box_quad(nx: int, ny: int) -> Mesh:
    i = np.arange(nx, dtype=np.int64)
    j = np.arange(ny, dtype=np.int64)
    jj, ii = np.meshgrid(j, i, indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    sx = nx + 1
    corners = [(0, 0), (1, 0), (1, 1), (0, 1)]
    ids = np.stack([(ii + a) + sx * (jj + b) for a, b in corners], axis=1)
    return Mesh(ids=np.ascontiguousarray(ids, dtype=np.int64), dims=(nx, ny),
                lex=np.arange(nx * ny, dtype=np.int64), name=f"quad{nx}x{ny}")


def _keep(mesh: Mesh, keep_mask: np.ndarray, tag: str) -> Mesh:
    idx = np.nonzero(keep_mask)[0]
    return Mesh(ids=np.ascontiguousarray(mesh.ids[idx]), dims=mesh.dims, lex=mesh.lex[idx],
                name=mesh.name + tag, meta=dict(mesh.meta))


def uniform_holes(mesh: Mesh, frac: float, seed: int) -> Mesh:
    n = mesh.nelem
    r = int(round(frac * n))
    order = random_permutation(seed, n)
    keep = np.ones(n, dtype=bool)
    keep[order[:r]] = False
    out = _keep(mesh, keep, f"-u{frac:g}")
    out.meta["removed"] = r
    return out


def clustered_holes(mesh: Mesh, frac: float, seed: int,
                    rmin: float = 3.0, rmax: float = 12.0) -> Mesh:
    if len(mesh.dims) != 3:
        raise ValueError("clustered holes are defined for hex boxes")
    nx, ny, nz = mesh.dims
    n = mesh.nelem
    target = int(round(frac * n))
    removed = np.zeros(nx * ny * nz, dtype=bool)  # indexed by lexicographic index
    present = np.zeros(nx * ny * nz, dtype=bool)
    present[mesh.lex] = True
    count = 0
    sphere = 0
    while count < target:
        u = uniform01(seed, 4, offset=4 * sphere)
        sphere += 1
        c = np.array([u[0] * nx, u[1] * ny, u[2] * nz])
        rad = rmin + (rmax - rmin) * u[3]
        lo = np.maximum(np.floor(c - rad - 1).astype(np.int64), 0)
        hi = np.minimum(np.ceil(c + rad + 1).astype(np.int64), [nx, ny, nz])
        ks, js, is_ = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]),
                                  np.arange(lo[0], hi[0]), indexing="ij")
        is_, js, ks = is_.ravel(), js.ravel(), ks.ravel()
        d2 = (is_ + 0.5 - c[0]) ** 2 + (js + 0.5 - c[1]) ** 2 + (ks + 0.5 - c[2]) ** 2
        lexi = is_ + nx * (js + ny * ks)
        sel = (d2 <= rad * rad) & present[lexi] & ~removed[lexi]
        lexi, d2 = lexi[sel], d2[sel]
        order = np.lexsort((lexi, d2))
        take = lexi[order[: target - count]]
        removed[take] = True
        count += take.size
    keep = ~removed[mesh.lex]
    out = _keep(mesh, keep, f"-c{frac:g}")
    out.meta["removed"] = count
    out.meta["spheres"] = sphere
    return out


def renumber_vertices(mesh: Mesh, seed: int) -> Mesh:
    """Random vertex relabelling onto sparse 64-bit ids pi(v)*2**31 + 7."""
    nvert = int(mesh.ids.max()) + 1
    pi = random_permutation(seed, nvert)
    new_ids = pi[mesh.ids] * np.int64(2 ** 31) + np.int64(7)
    out = Mesh(ids=np.ascontiguousarray(new_ids), dims=mesh.dims, lex=mesh.lex.copy(),
               name=mesh.name + "-r", meta=dict(mesh.meta))
    return out


def shuffle_elements(mesh: Mesh, seed: int) -> Mesh:
    perm = random_permutation(seed, mesh.nelem)
    return Mesh(ids=np.ascontiguousarray(mesh.ids[perm]), dims=mesh.dims, lex=mesh.lex[perm],
                name=mesh.name + "-s", meta=dict(mesh.meta, perm=perm))


# --------------------------------------------------------------------------
# The benchmark workloads (sizes, graph kind and precision of each)
# --------------------------------------------------------------------------

def config_seed(index: int) -> int:
    return BASE_SEED + index


def cube16() -> Mesh:
    """16x16x16 hex box, no holes (used with the face-connected unit graph)."""
    return box_hex(16, 16, 16)


def box128_holes5() -> Mesh:
    """128x128x64 box with 5% of the elements removed uniformly at random."""
    return uniform_holes(box_hex(128, 128, 64), 0.05, config_seed(1))


def box256_holes3() -> Mesh:
    """256x256x64 box with 3% of the elements removed uniformly at random."""
    return uniform_holes(box_hex(256, 256, 64), 0.03, config_seed(2))


def box256x128_clustered10() -> Mesh:
    """256x256x128 box, 10% removed in spherical clusters, vertex ids renumbered."""
    seed = config_seed(4)
    m = clustered_holes(box_hex(256, 256, 128), 0.10, seed)
    return renumber_vertices(m, seed + 1)


def batch64(seed: int | None = None, count: int = 64, smin: float = 1e4, smax: float = 5e5,
            holes: float = 0.03) -> list:
    """64 boxes of log-uniform size in [1e4, 5e5] elements with 3% holes each."""
    seed = config_seed(4) + 100 if seed is None else seed
    u = uniform01(seed, 3 * count)
    meshes = []
    for b in range(count):
        s = math.exp(math.log(smin) + (math.log(smax) - math.log(smin)) * u[3 * b])
        a2 = 0.5 + 0.5 * u[3 * b + 1]
        a3 = 0.5 + 0.5 * u[3 * b + 2]
        nx = max(1, int(round((s / (a2 * a3)) ** (1.0 / 3.0))))
        ny = max(1, int(round(a2 * nx)))
        nz = max(1, int(round(a3 * nx)))
        m = uniform_holes(box_hex(nx, ny, nz), holes, seed + 1000 + b)
        meshes.append(m)
    return meshes


def box_counts(nx: int, ny: int, nz: int) -> dict:
    """Closed-form numbers of face, edge and corner neighbour pairs on a full box."""
    F = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    E = 2 * ((nx - 1) * (ny - 1) * nz + (nx - 1) * ny * (nz - 1) + nx * (ny - 1) * (nz - 1))
    K = 4 * (nx - 1) * (ny - 1) * (nz - 1)
    return {"face": F, "edge": E, "corner": K}
