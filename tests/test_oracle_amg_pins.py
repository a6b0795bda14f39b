"""Pins of the oracle's aggregation multigrid preconditioner (paper Sec. 7,
Alg. 3) against facts fixed by the mathematics rather than by its own code:

* every coarse Laplacian equals the dense Galerkin product J^T L J with the
  Boolean prolongation J read from the aggregate map;
* aggregates are single rows or adjacent pairs, numbered by first member,
  carrying the smaller global id, and an edge of largest weight is always
  collapsed at the first level;
* the V-cycle, applied to unit vectors, equals the closed-form operator
  M = S^v [B + J M_c J^T (I - A B)] + B' of damped Jacobi (S = I - sigma D A,
  B = sum_{k<=v} S^k sigma D, B' = sum_{k<v} S^k sigma D), built level by
  level with dense matrices;
* AMG-preconditioned inverse iteration reaches the dense eigen-decomposition's
  Fiedler pair, and, with an exact eigenvector as right-hand side, still
  stops after one CG step (the first direction is not preconditioned, Sec. 7).
"""
import numpy as np
import pytest

import meshgen as mg


def dense(rp, col, w, n=None):
    n = len(rp) - 1 if n is None else n
    A = np.zeros((n, n))
    for i in range(len(rp) - 1):
        for p in range(rp[i], rp[i + 1]):
            A[i, col[p]] -= w[p]
            A[i, i] += w[p]
    return A


def meshes():
    return [
        ("box6x5x4-holes", mg.uniform_holes(mg.box_hex(6, 5, 4), 0.15, 7)),
        ("quad14x9-holes", mg.uniform_holes(mg.box_quad(14, 9), 0.1, 3)),
        ("box5x4x3-renum-shuffle", mg.shuffle_elements(mg.renumber_vertices(mg.box_hex(5, 4, 3), 5), 9)),
    ]


def hierarchy(orc, rp, col, w):
    first = orc.amg_level(rp, col, w, 0)
    return [orc.amg_level(rp, col, w, l) for l in range(first["nlevels"])]


@pytest.mark.parametrize("name,mesh", meshes())
def test_galerkin_product_is_the_coarse_laplacian(orc, name, mesh):
    rp, col, w = orc.dual_graph(mesh.ids)
    lv = hierarchy(orc, rp, col, w)
    assert len(lv) >= 3
    for a, b in zip(lv[:-1], lv[1:]):
        na, nb = len(a["gid"]), len(b["gid"])
        J = np.zeros((na, nb))
        J[np.arange(na), a["agg"]] = 1.0
        La = dense(a["row_ptr"], a["col"], a["weight"])
        Lb = dense(b["row_ptr"], b["col"], b["weight"])
        assert np.array_equal(J.T @ La @ J, Lb)
        assert np.all(b["weight"] > 0)
        for i in range(nb):  # columns ascending, no diagonal entry
            c = b["col"][b["row_ptr"][i]:b["row_ptr"][i + 1]]
            assert np.all(np.diff(c) > 0) and i not in c
    assert np.all(lv[-1]["agg"] == -1)


@pytest.mark.parametrize("name,mesh", meshes())
def test_aggregates_are_adjacent_pairs(orc, name, mesh):
    rp, col, w = orc.dual_graph(mesh.ids)
    gid = np.arange(len(rp) - 1, dtype=np.int64)[::-1].copy()  # ids need not follow rows
    lv = [orc.amg_level(rp, col, w, l, gid=gid) for l in range(orc.amg_level(rp, col, w, 0, gid=gid)["nlevels"])]
    assert np.array_equal(lv[0]["gid"], gid)
    for a, b in zip(lv[:-1], lv[1:]):
        na, nb = len(a["gid"]), len(b["gid"])
        assert 10 * nb <= 9 * na                     # the stop rule
        members = [[] for _ in range(nb)]
        for i in range(na):
            members[a["agg"][i]].append(i)
        firsts = [m[0] for m in members]
        assert firsts == sorted(firsts)              # numbered by first member
        A = dense(a["row_ptr"], a["col"], a["weight"])
        for I, m in enumerate(members):
            assert len(m) in (1, 2)
            if len(m) == 2:
                assert A[m[0], m[1]] < 0             # an edge of the finer level
            assert b["gid"][I] == min(a["gid"][k] for k in m)
    # an edge of the largest weight is collapsed at the first level
    A = dense(rp, col, w)
    off = -A + np.diag(np.diag(A))
    wmax = off.max()
    agg = lv[0]["agg"]
    heavy = np.argwhere(off == wmax)
    assert any(agg[i] == agg[j] for i, j in heavy)


def closed_form_vcycle(lv, sigma, nu):
    """M of every level from the coarsest up, dense."""
    M_next = None
    for l in range(len(lv) - 1, -1, -1):
        a = lv[l]
        A = dense(a["row_ptr"], a["col"], a["weight"])
        n = A.shape[0]
        d = np.diag(A)
        D = np.diag(np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0))
        S = np.eye(n) - sigma * D @ A
        B = sum(np.linalg.matrix_power(S, k) for k in range(nu + 1)) @ (sigma * D)
        if l == len(lv) - 1:
            M = B
        else:
            Bp = sum((np.linalg.matrix_power(S, k) for k in range(nu)), np.zeros((n, n))) @ (sigma * D)
            J = np.zeros((n, len(lv[l + 1]["gid"])))
            J[np.arange(n), a["agg"]] = 1.0
            M = np.linalg.matrix_power(S, nu) @ (B + J @ M_next @ J.T @ (np.eye(n) - A @ B)) + Bp
        M_next = M
    return M_next


@pytest.mark.parametrize("sigma,nu", [(2.0 / 3.0, 1), (0.9, 2), (0.5, 0)])
def test_vcycle_equals_closed_form(orc, sigma, nu):
    mesh = mg.uniform_holes(mg.box_hex(5, 4, 4), 0.1, 13)
    rp, col, w = orc.dual_graph(mesh.ids)
    n = len(rp) - 1
    lv = hierarchy(orc, rp, col, w)
    assert len(lv) >= 3
    M = np.column_stack([orc.amg_vcycle(rp, col, w, np.eye(n)[:, k], sigma=sigma, nsmooth=nu)
                         for k in range(n)])
    Mc = closed_form_vcycle(lv, sigma, nu)
    assert np.abs(M - Mc).max() <= 1e-12 * np.abs(Mc).max()


def test_vcycle_two_elements_is_jacobi(orc):
    # two adjacent elements collapse into one row whose Laplacian is 0, so
    # without smoothing steps the cycle is the first Jacobi step sigma D f
    ids = np.array([[0, 1, 2, 3], [2, 3, 4, 5]])
    rp, col, w = orc.dual_graph(ids)
    f = np.array([0.75, -0.25])
    u = orc.amg_vcycle(rp, col, w, f, sigma=0.6, nsmooth=0)
    assert np.allclose(u, 0.6 * f / 2.0, rtol=0, atol=1e-16)


def test_vcycle_is_a_convergent_iteration(orc):
    mesh = mg.uniform_holes(mg.box_hex(8, 6, 5), 0.05, 3)
    rp, col, w = orc.dual_graph(mesh.ids)
    n = len(rp) - 1
    A = dense(rp, col, w)
    M = np.column_stack([orc.amg_vcycle(rp, col, w, np.eye(n)[:, k]) for k in range(n)])
    # error propagation on the complement of the ones vector
    Q = np.linalg.qr(np.column_stack([np.ones(n), np.random.default_rng(1).standard_normal((n, n - 1))]))[0][:, 1:]
    E = Q.T @ (np.eye(n) - M @ A) @ Q
    rho = np.abs(np.linalg.eigvals(E)).max()
    assert rho < 0.9


def test_amg_inverse_iteration_matches_dense_eigh(orc):
    mesh = mg.uniform_holes(mg.box_hex(9, 6, 5), 0.05, 11)
    rp, col, w = orc.dual_graph(mesh.ids)
    ev, V = np.linalg.eigh(dense(rp, col, w))
    assert ev[2] - ev[1] > 1e-2 * ev[1]
    st, lam, y, info = orc.fiedler(mesh.ids, method="inverse_cg", inv_precond="amg", tol=1e-10,
                                   inv_max_outer=400)
    assert st == 0 and info["amg_levels"] >= 3
    assert abs(lam - ev[1]) <= 1e-9 * ev[1]
    assert abs(abs(y @ V[:, 1]) - 1.0) < 1e-7
    st0, lam0, _, info0 = orc.fiedler(mesh.ids, method="inverse_cg", tol=1e-10, inv_max_outer=400)
    assert info["cg_iters"] < 0.5 * info0["cg_iters"]


def test_amg_first_cg_direction_is_not_preconditioned(orc):
    # b an exact eigenvector: CG from x0 = 0 with the plain residual as first
    # direction returns b / lambda in one step, so inverse iteration stops
    # after one outer pass with one CG step, preconditioner or not (Sec. 7)
    ids = np.array([[0, 1, 2, 3], [2, 3, 4, 5]])
    st, lam, y, info = orc.fiedler(ids, method="inverse_cg", inv_precond="amg")
    assert st == 0 and info["cycles"] == 1 and info["cg_iters"] == 1
    assert abs(lam - 4.0) < 1e-14
