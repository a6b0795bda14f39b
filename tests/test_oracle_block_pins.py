"""Pins of the oracle's block Lanczos of two vectors (method "block", the
paper's Sec. 9 proposal for degenerate Fiedler pairs).

What fixes it independently of its code:
  * the first cycle is the Rayleigh-Ritz procedure on the block Krylov space
    span{X0, L X0, ..., L^(m/2-1) X0} of the two seeded start vectors, ones
    component removed: recomputed with numpy's QR and eigh on that space;
  * an explicit restart is the same procedure on the Krylov space of the
    first cycle's pair;
  * converged pairs are the dense eigen-decomposition's (lambda_2, lambda_3,
    the Fiedler vector element-wise and the pair's plane), also where
    lambda_2 = lambda_3 exactly -- which a one-vector solve cannot resolve;
  * on graphs whose whole space fits one cycle the result is exact after it
    (the deflation of exhausted columns), with no second vector on a
    two-element graph;
  * Ritz values never fall below the eigenvalues they approximate
    (Courant-Fischer) and a thick restart never raises them;
  * the swept cut of an exactly degenerate box equals the sweep over the
    dense eigenspace with y1 the projection of the random start on it.
A dropped coefficient, a wrong sign in the projection or a transposed block
fails the first two pins by orders of magnitude.
"""
import numpy as np
import pytest

import meshgen as mg
from spectral_util import assert_fiedler_close
from test_oracle_pins import dense_laplacian
from test_oracle_sweep_pins import canonical, half_cut

SEED = 20240611
SECOND = 0x9E3779B97F4A7C15


def _starts(orc, n, seed=SEED):
    x0 = np.array([orc.start_value(seed, i) for i in range(n)])
    x1 = np.array([orc.start_value(seed ^ SECOND, i) for i in range(n)])
    return x0, x1


def _rayleigh_ritz_block_krylov(Ld, X, nb):
    """Two smallest Ritz values of Ld on span{X, Ld X, ..., Ld^(nb-1) X},
    ones vector removed."""
    n = Ld.shape[0]
    u = np.ones(n) / np.sqrt(n)
    X = X - np.outer(u, u @ X)
    cols = [X]
    for _ in range(nb - 1):
        cols.append(Ld @ cols[-1])
    K = np.concatenate([u[:, None]] + cols, axis=1)
    Qf, _ = np.linalg.qr(K)
    Qk = Qf[:, 1:]
    return np.linalg.eigvalsh(Qk.T @ Ld @ Qk)[:2]


MESHES = {
    "holes": lambda: mg.uniform_holes(mg.box_hex(9, 7, 5), 0.06, 3).ids,
    "quad": lambda: mg.uniform_holes(mg.box_quad(21, 17), 0.05, 4).ids,
    "clustered": lambda: mg.clustered_holes(mg.box_hex(10, 9, 6), 0.1, 9).ids,
}


@pytest.mark.parametrize("name", list(MESHES))
def test_first_cycle_is_rayleigh_ritz_on_block_krylov(orc, name):
    ids = MESHES[name]()
    rp, col, w = orc.dual_graph(ids)
    Ld = dense_laplacian(rp, col, w)
    n = Ld.shape[0]
    x0, x1 = _starts(orc, n)
    ref = _rayleigh_ritz_block_krylov(Ld, np.stack([x0, x1], 1), 4)
    for keep in (0, 4):
        st, y1, y2, th, info = orc.block_pair(rp, col, w, lanczos_m=8, lanczos_keep=keep,
                                              tol=1e-15, max_restarts=0, seed=SEED)
        assert info["cycles"] == 1
        assert np.allclose(th, ref, rtol=1e-7, atol=0)
        # the returned vectors are the Ritz vectors: orthonormal, off the ones vector
        assert abs(y1 @ y2) < 1e-12 and abs(np.linalg.norm(y1) - 1) < 1e-12
        assert abs(y1.sum()) < 1e-10 and abs(y2.sum()) < 1e-10


@pytest.mark.parametrize("name", ["holes", "quad"])
def test_explicit_restart_is_rayleigh_ritz_from_the_pair(orc, name):
    ids = MESHES[name]()
    rp, col, w = orc.dual_graph(ids)
    Ld = dense_laplacian(rp, col, w)
    kw = dict(lanczos_m=8, lanczos_keep=0, tol=1e-15, seed=SEED)
    _, y1, y2, th0, _ = orc.block_pair(rp, col, w, max_restarts=0, **kw)
    _, _, _, th1, info = orc.block_pair(rp, col, w, max_restarts=1, **kw)
    assert info["cycles"] == 2
    ref = _rayleigh_ritz_block_krylov(Ld, np.stack([y1, y2], 1), 4)
    assert np.allclose(th1, ref, rtol=1e-7, atol=0)
    assert th1[0] < th0[0] and th1[1] < th0[1]


@pytest.mark.parametrize("keep,tol", [(0, 1e-8), (8, 1e-10)])
@pytest.mark.parametrize("name", list(MESHES))
def test_converged_pair_matches_dense_eigh(orc, name, keep, tol):
    ids = MESHES[name]()
    rp, col, w = orc.dual_graph(ids)
    ev, V = np.linalg.eigh(dense_laplacian(rp, col, w))
    st, y1, y2, th, info = orc.block_pair(rp, col, w, lanczos_m=20, lanczos_keep=keep, tol=tol,
                                          max_restarts=3000, seed=SEED)
    assert st == 0
    assert abs(th[0] - ev[1]) <= 1e-9 * ev[1] and abs(th[1] - ev[2]) <= 1e-9 * ev[2]
    assert_fiedler_close(y1, V[:, 1], info["residual"], 1e-14 * ev[-1], ev[2] - ev[1])
    # the pair's plane: projector error bounded by residual / distance to lambda_4
    P = np.outer(y1, y1) + np.outer(y2, y2)
    E = V[:, 1:3]
    bound = 4 * tol * ev[2] / (ev[3] - ev[2]) + 1e-12
    assert np.abs(P - E @ E.T).max() <= bound


@pytest.mark.parametrize("dims", [(8, 8, 3), (12, 12, 2), (16, 16, 4)])
def test_exactly_degenerate_pair_is_found(orc, dims):
    ids = mg.box_hex(*dims).ids
    rp, col, w = orc.dual_graph(ids, "face")
    ev, V = np.linalg.eigh(dense_laplacian(rp, col, w))
    assert abs(ev[2] - ev[1]) < 1e-12 * ev[1] and ev[3] - ev[2] > 0.1 * ev[1]
    st, y1, y2, th, info = orc.block_pair(rp, col, w, graph="face", lanczos_m=20,
                                          lanczos_keep=8, tol=1e-10, max_restarts=500, seed=SEED)
    assert st == 0
    assert abs(th[0] - ev[1]) <= 1e-9 * ev[1] and abs(th[1] - ev[1]) <= 1e-9 * ev[1]
    E = V[:, 1:3]
    P = np.outer(y1, y1) + np.outer(y2, y2)
    assert np.abs(P - E @ E.T).max() <= 1e-8
    # a one-vector solve finds one direction of that plane only: with the
    # sweep on, its second Ritz value is the next eigenvalue and no sweep runs
    _, _, _, i1 = orc.fiedler(ids, graph="face", lanczos_m=20, lanczos_keep=8, tol=1e-10,
                              fiedler_sweep=8, seed=SEED)
    _, _, _, ib = orc.fiedler(ids, graph="face", lanczos_m=20, lanczos_keep=8, tol=1e-10,
                              fiedler_sweep=8, seed=SEED, method="block")
    assert i1["sweeps"] == 0 and ib["sweeps"] == 1


@pytest.mark.parametrize("make", [lambda: mg.box_quad(3, 1), lambda: mg.box_quad(2, 2),
                                  lambda: mg.box_hex(2, 2, 2), lambda: mg.box_quad(4, 3),
                                  lambda: mg.box_hex(3, 2, 2)])
def test_small_graph_is_exact_after_one_cycle(orc, make):
    ids = make().ids
    rp, col, w = orc.dual_graph(ids)
    ev = np.linalg.eigvalsh(dense_laplacian(rp, col, w))
    st, y1, y2, th, info = orc.block_pair(rp, col, w, lanczos_m=20, lanczos_keep=0, tol=1e-10,
                                          max_restarts=0, seed=SEED)
    assert st == 0 and info["cycles"] == 1
    assert abs(th[0] - ev[1]) <= 1e-12 * ev[-1] and abs(th[1] - ev[2]) <= 1e-12 * ev[-1]
    assert abs(y1 @ y2) < 1e-12


def test_two_elements_have_no_second_vector(orc):
    ids = mg.box_quad(2, 1).ids
    rp, col, w = orc.dual_graph(ids)
    st, y1, y2, th, info = orc.block_pair(rp, col, w, lanczos_m=8, lanczos_keep=0, tol=1e-10,
                                          max_restarts=0, seed=SEED)
    lam = 2.0 * w[0]
    assert st == 0 and abs(th[0] - lam) <= 1e-13 * lam and np.isinf(th[1])
    assert np.all(y2 == 0.0)
    assert np.allclose(np.abs(y1), np.sqrt(0.5), atol=1e-14) and y1[0] == -y1[1]


def test_ritz_values_bound_and_decrease(orc):
    ids = MESHES["clustered"]()
    rp, col, w = orc.dual_graph(ids)
    ev = np.linalg.eigvalsh(dense_laplacian(rp, col, w))
    prev = (np.inf, np.inf)
    for r in range(6):
        _, _, _, th, info = orc.block_pair(rp, col, w, lanczos_m=12, lanczos_keep=6, tol=1e-15,
                                           max_restarts=r, seed=SEED)
        assert info["cycles"] == r + 1
        assert th[0] >= ev[1] * (1 - 1e-12) and th[1] >= ev[2] * (1 - 1e-12)
        assert th[0] <= prev[0] * (1 + 1e-12) and th[1] <= prev[1] * (1 + 1e-12)
        prev = th


def test_block_sweep_of_a_degenerate_box_equals_dense_eigenspace_sweep(orc):
    ids = mg.box_hex(16, 16, 4).ids
    rp, col, w = orc.dual_graph(ids, "face")
    n = len(rp) - 1
    ev, V = np.linalg.eigh(dense_laplacian(rp, col, w))
    S = 16
    kw = dict(graph="face", lanczos_m=20, lanczos_keep=8, tol=1e-10, seed=SEED)
    st, lam, y, info = orc.fiedler(ids, fiedler_sweep=S, method="block", **kw)
    st0, lam0, y0, _ = orc.fiedler(ids, **kw)
    assert st == st0 == 0 and info["sweeps"] == 1
    # y1: the random start projected on the eigenspace; y2 its rotation there
    E = V[:, 1:3]
    x0, _ = _starts(orc, n)
    p1 = E @ (E.T @ x0)
    p1 = canonical(p1 / np.linalg.norm(p1))
    rot = np.array([[0.0, -1.0], [1.0, 0.0]])
    p2 = canonical(E @ (rot @ (E.T @ p1)))
    cuts = [half_cut(orc, rp, col, w,
                     canonical(np.cos(np.pi * k / S) * p1 + np.sin(np.pi * k / S) * p2))
            for k in range(S)]
    assert half_cut(orc, rp, col, w, y) == min(cuts)
    assert half_cut(orc, rp, col, w, y) < half_cut(orc, rp, col, w, y0)


def test_block_partition_equals_lanczos_on_unique_axis_box(orc):
    ids = mg.box_hex(24, 20, 18).ids
    kw = dict(graph="face", lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1)
    st0, p0, _ = orc.partition(ids, 8, **kw)
    st1, p1, _ = orc.partition(ids, 8, method="block", **kw)
    assert st0 == st1 == 0 and np.array_equal(p0, p1)
