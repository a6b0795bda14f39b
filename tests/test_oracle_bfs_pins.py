"""Pins of the oracle's BFS start (opts bfs_start; not in the paper, which
leaves the start vector open): the first solve of a mesh starts from the
number of edges between each element and a pseudo-peripheral element (the
element farthest from element 0, smallest index among the farthest),
centred and scaled to unit root-mean-square over the elements the search
reaches.

What fixes it independently of the code: on a box the graph distance has a
closed form -- with the vertex-shared graph two elements are adjacent when
their indices differ by at most 1 in every axis, so the distance is the
Chebyshev distance max|dx|, |dy|, |dz|; with the face graph it is the
Manhattan distance.  The farthest set from the corner element 0 is then the
plane x = nx - 1 (vertex graph: smallest index (nx - 1, 0, 0)) or the
opposite corner alone (face graph).  A search from the largest index of the
farthest set, or from element 0 itself, fails the affine check below.
Elements of another component get no value.  Started this way, the solve
still converges to the dense eigenpair, and the octant partition of the
unique-axis box is unchanged.
"""
import numpy as np
import pytest

import meshgen as mg
from spectral_util import assert_fiedler_close
from test_oracle_pins import dense_laplacian


def _coords(dims):
    idx = np.arange(int(np.prod(dims)))
    out = []
    for n in dims:
        out.append(idx % n)
        idx = idx // n
    return out


def _assert_affine_in(values, d):
    # values = a d + b with a > 0, to rounding; unit RMS and zero mean
    A = np.stack([d.astype(np.float64), np.ones(len(d))], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, values, rcond=None)
    assert a > 0
    assert np.abs(A @ np.array([a, b]) - values).max() <= 1e-12
    assert abs(values.mean()) <= 1e-12
    assert abs(np.sqrt(np.mean(values ** 2)) - 1.0) <= 1e-12


@pytest.mark.parametrize("dims", [(12, 7, 5), (9, 9, 4), (5, 11, 3)])
def test_vertex_graph_box_is_chebyshev_from_far_plane(orc, dims):
    mesh = mg.box_hex(*dims)
    rp, col, w = orc.dual_graph(mesh.ids)
    v = orc.bfs_start(rp, col, w)
    x, y, z = _coords(dims)
    # element 0 is a corner; the farthest elements (Chebyshev) are the ones
    # at the largest axis length - 1; the smallest index among them
    far_d = max(dims) - 1
    cheb0 = np.maximum(np.maximum(x, y), z)
    far = int(np.flatnonzero(cheb0 == far_d).min())
    fx, fy, fz = x[far], y[far], z[far]
    d = np.maximum(np.maximum(np.abs(x - fx), np.abs(y - fy)), np.abs(z - fz))
    _assert_affine_in(v, d)


@pytest.mark.parametrize("dims", [(12, 7, 5), (6, 6, 6)])
def test_face_graph_box_is_manhattan_from_opposite_corner(orc, dims):
    mesh = mg.box_hex(*dims)
    rp, col, w = orc.dual_graph(mesh.ids, graph="face")
    v = orc.bfs_start(rp, col, w)
    x, y, z = _coords(dims)
    d = (dims[0] - 1 - x) + (dims[1] - 1 - y) + (dims[2] - 1 - z)
    _assert_affine_in(v, d)


def test_quad_mesh_is_chebyshev(orc):
    mesh = mg.box_quad(9, 6)
    rp, col, w = orc.dual_graph(mesh.ids)
    v = orc.bfs_start(rp, col, w)
    x, y = _coords((9, 6))
    d = np.maximum(np.abs(x - 8), y)  # from (8, 0): the smallest index at distance 8
    _assert_affine_in(v, d)


def test_unreached_component_has_no_value(orc):
    a = mg.box_hex(6, 5, 4)
    b = mg.box_hex(3, 3, 3)
    ids = np.concatenate([a.ids, b.ids + a.ids.max() + 1])
    rp, col, w = orc.dual_graph(ids)
    v = orc.bfs_start(rp, col, w)
    na = a.ids.shape[0]
    assert np.all(np.isnan(v[na:])) and not np.any(np.isnan(v[:na]))
    x, y, z = _coords((6, 5, 4))
    d = np.maximum(np.maximum(np.abs(x - 5), y), z)
    _assert_affine_in(v[:na], d)


@pytest.mark.parametrize("name,make", [
    ("holes", lambda: mg.uniform_holes(mg.box_hex(14, 10, 7), 0.07, 3)),
    ("clustered", lambda: mg.clustered_holes(mg.box_hex(13, 11, 8), 0.1, 9)),
    ("quad", lambda: mg.uniform_holes(mg.box_quad(36, 25), 0.1, 4)),
])
@pytest.mark.parametrize("keep,m", [(0, 40), (8, 40)])
def test_solve_from_bfs_start_matches_dense_eigh(orc, name, make, keep, m):
    mesh = make()
    rp, col, w = orc.dual_graph(mesh.ids)
    ev, V = np.linalg.eigh(dense_laplacian(rp, col, w))
    st, lam, y, info = orc.fiedler(mesh.ids, lanczos_m=m, lanczos_keep=keep, bfs_start=1,
                                   tol=1e-10, max_restarts=2000)
    assert st == 0
    assert abs(lam - ev[1]) <= 1e-10 * ev[1]
    assert_fiedler_close(y, V[:, 1], info["residual"], 1e-14 * ev[-1], ev[2] - ev[1])


def test_bfs_start_changes_the_start(orc):
    # one cycle from each start gives different Ritz values (the option is
    # not a no-op), both above lambda_2
    mesh = mg.uniform_holes(mg.box_hex(30, 9, 7), 0.05, 2)
    kw = dict(lanczos_m=12, lanczos_keep=0, tol=1e-15, max_restarts=0)
    _, lam0, _, i0 = orc.fiedler(mesh.ids, **kw)
    _, lam1, _, i1 = orc.fiedler(mesh.ids, bfs_start=1, **kw)
    st, lam, _, _ = orc.fiedler(mesh.ids, tol=1e-12, lanczos_m=60, max_restarts=500)
    assert abs(lam0 - lam1) > 1e-9 * lam
    assert lam0 >= lam * (1 - 1e-12) and lam1 >= lam * (1 - 1e-12)


def test_partition_unique_axis_box_unchanged(orc):
    box = mg.box_hex(24, 20, 18)
    kw = dict(graph="face", lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1)
    st0, p0, _ = orc.partition(box.ids, 8, **kw)
    st1, p1, _ = orc.partition(box.ids, 8, bfs_start=1, **kw)
    assert st0 == st1 == 0 and np.array_equal(p0, p1)
