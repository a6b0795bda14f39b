"""Pins of the oracle's CG inner solve of inverse iteration (Sec. 7, Alg. 2)
and of its threading.

The CG "augmented with full projection" L-orthogonalises every new search
direction against the kept ones.  What fixes it independently of the code:

* the kept directions are pairwise L-orthogonal (conjugate): that is what
  the projection is for, and it fails at once if a projection coefficient
  has the wrong sign or the wrong denominator;
* in exact arithmetic CG directions are already conjugate, so projection
  changes nothing there: on a small mesh the projected solve takes the same
  number of steps as plain CG, and whole inverse iterations the same total;
* conjugate directions make CG terminate: with every direction kept, a solve
  takes at most as many steps as L has distinct nonzero eigenvalues;
* the solution is L^+ b (dense pseudo-inverse) for b orthogonal to the ones.

Threads: every sum over elements is taken in one fixed order, so one thread
and several threads give the same bits.
"""
import numpy as np
import pytest

import meshgen as mg

from test_oracle_pins import dense_laplacian


def _mesh_graph(orc, mesh, graph="weighted"):
    rp, col, w = orc.dual_graph(mesh.ids, graph=graph)
    return rp, col, w, len(rp) - 1


def _rhs(orc, n, seed=20261203):
    b = np.array([orc.start_value(seed, i) for i in range(n)])
    b -= b.mean()
    return b / np.linalg.norm(b)


def _conjugacy(orc, rp, col, w, dirs):
    """|p_i^T L p_j| / (||p_i||_L ||p_j||_L) for all pairs."""
    ld = np.array([orc.laplacian_apply(rp, col, w, d) for d in dirs])
    G = dirs @ ld.T
    nrm = np.sqrt(np.diag(G))
    return np.abs(G) / np.outer(nrm, nrm)


@pytest.mark.parametrize("k", [1, 3, 8, 32])
def test_projected_directions_are_conjugate(orc, k):
    # every direction is L-orthogonal to the k directions before it; the
    # solve runs long enough (tolerance 1e-12) that any error in the
    # projection compounds from step to step
    mesh = mg.uniform_holes(mg.box_hex(7, 6, 5), 0.05, 11)
    rp, col, w, n = _mesh_graph(orc, mesh)
    its, x, dirs = orc.cg_solve(rp, col, w, _rhs(orc, n), max_dirs=4000, cg_full_projection=k,
                                cg_tol=1e-12, cg_max_iter=4000)
    assert len(dirs) == its > 20
    C = _conjugacy(orc, rp, col, w, dirs)
    worst = max(C[i, j] for i in range(len(dirs)) for j in range(max(0, i - k), i))
    assert worst <= 1e-10, worst


def test_projection_changes_no_step_count_on_a_small_mesh(orc):
    # conjugacy holds in exact arithmetic, so the projection only removes
    # rounding: the same step counts as plain CG, per solve and over the
    # whole inverse iteration
    mesh = mg.uniform_holes(mg.box_hex(7, 6, 5), 0.05, 11)
    rp, col, w, n = _mesh_graph(orc, mesh)
    b = _rhs(orc, n)
    plain, _, _ = orc.cg_solve(rp, col, w, b, cg_tol=1e-10)
    for k in (3, 8):
        its, _, _ = orc.cg_solve(rp, col, w, b, cg_full_projection=k, cg_tol=1e-10)
        assert abs(its - plain) <= 2
    kw = dict(method="inverse_cg", tol=1e-10, inv_max_outer=400)
    _, _, _, i0 = orc.fiedler(mesh.ids, **kw)
    _, _, _, i8 = orc.fiedler(mesh.ids, cg_full_projection=8, **kw)
    assert abs(i8["cg_iters"] - i0["cg_iters"]) <= 2


@pytest.mark.parametrize("dims,graph", [((4, 4, 4), "face"), ((6, 5, 1), "face"),
                                        ((3, 3, 3), "weighted")])
def test_finite_termination_with_all_directions_kept(orc, dims, graph):
    # exact CG needs at most as many steps as there are distinct nonzero
    # eigenvalues (the face graph of a box has many repeated ones); keeping
    # every direction conjugate reproduces that in floating point
    mesh = mg.box_hex(*dims)
    rp, col, w, n = _mesh_graph(orc, mesh, graph)
    ev = np.linalg.eigvalsh(dense_laplacian(rp, col, w))
    nz = ev[ev > 1e-9 * ev.max()]
    distinct = 1 + int(np.sum(np.diff(nz) > 1e-8 * ev.max()))
    assert distinct < n - 1
    its, x, dirs = orc.cg_solve(rp, col, w, _rhs(orc, n), max_dirs=n, cg_full_projection=32,
                                cg_tol=1e-12)
    assert its <= distinct, (its, distinct)


@pytest.mark.parametrize("k", [0, 4])
def test_solution_is_the_pseudo_inverse(orc, k):
    mesh = mg.uniform_holes(mg.box_hex(6, 5, 4), 0.1, 3)
    rp, col, w, n = _mesh_graph(orc, mesh)
    b = _rhs(orc, n, seed=7)
    its, x, _ = orc.cg_solve(rp, col, w, b, cg_full_projection=k, cg_tol=1e-13)
    ref = np.linalg.pinv(dense_laplacian(rp, col, w)) @ b
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


def test_threads_give_identical_bits(orc):
    # 40k rows: threaded element loops and many summation chunks
    mesh = mg.uniform_holes(mg.box_hex(40, 32, 32), 0.05, 2)
    rp, col, w, n = _mesh_graph(orc, mesh)
    assert n > 8 * 4096
    runs = []
    prev = orc.set_threads(0)
    for t in (1, 4):
        assert orc.set_threads(t) == t
        lz = orc.fiedler_csr(rp, col, w, tol=1e-6, lanczos_m=30, lanczos_keep=6, max_restarts=4)
        cg = orc.cg_solve(rp, col, w, _rhs(orc, n), cg_full_projection=4, cg_tol=1e-6)
        runs.append((lz, cg))
    orc.set_threads(prev)
    (l1, c1), (l4, c4) = runs
    assert l1[0] == l4[0] and l1[1] == l4[1] and np.array_equal(l1[2], l4[2])
    assert c1[0] == c4[0] and np.array_equal(c1[1], c4[1])
