"""Pins of the oracle's sweep over the Fiedler pair (the paper's suggestion
for near-degenerate pairs: search the combinations of the two lowest
eigenvectors for the smallest cut).

The sweep's cut is pinned to the same sweep run on the dense
eigen-decomposition's eigenvectors (library routine), it never cuts more than
the Fiedler vector alone, one angle reproduces the plain method, and an
exactly degenerate pair (which a single-vector Krylov space cannot resolve)
leaves the method unchanged.
"""
import numpy as np
import pytest

import meshgen as mg


def dense(rp, col, w):
    n = len(rp) - 1
    A = np.zeros((n, n))
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            A[i, col[p]] -= w[p]
            A[i, i] += w[p]
    return A


def canonical(y):
    big = np.abs(y).max()
    k = np.flatnonzero(np.abs(y) >= 1e-3 * big)[0]
    return -y if y[k] > 0 else y


def half_cut(orc, rp, col, w, y):
    n = len(y)
    side = orc.split(y, np.arange(n), n // 2)
    rows = np.repeat(np.arange(n), np.diff(rp))
    c = (side[rows] != side[col]) & (col > rows)
    return int(w[c].sum())


KW = dict(lanczos_keep=8, lanczos_m=30, tol=1e-10)


@pytest.mark.parametrize("seed", range(6))
def test_sweep_equals_dense_eigenvector_sweep(orc, seed):
    mesh = mg.uniform_holes(mg.box_hex(10, 10, 4), 0.06, seed)
    rp, col, w = orc.dual_graph(mesh.ids)
    ev, V = np.linalg.eigh(dense(rp, col, w))
    assert (ev[2] - ev[1]) / ev[1] < 0.1            # a near-degenerate pair
    S = 16
    v1, v2 = canonical(V[:, 1]), canonical(V[:, 2])
    cuts = [half_cut(orc, rp, col, w, canonical(np.cos(np.pi * k / S) * v1 + np.sin(np.pi * k / S) * v2))
            for k in range(S)]
    st, lam, y, info = orc.fiedler(mesh.ids, fiedler_sweep=S, **KW)
    st0, lam0, y0, _ = orc.fiedler(mesh.ids, **KW)
    assert st == st0 == 0 and info["sweeps"] == 1
    assert half_cut(orc, rp, col, w, y) == min(cuts)
    assert half_cut(orc, rp, col, w, y) <= half_cut(orc, rp, col, w, y0)
    assert abs(np.linalg.norm(y) - 1) < 1e-12 and abs(y.sum()) < 1e-10
    assert lam == lam0


def test_one_angle_is_the_plain_method(orc):
    mesh = mg.uniform_holes(mg.box_hex(12, 12, 6), 0.05, 2)
    st0, p0, _ = orc.partition(mesh.ids, 8, **KW)
    st1, p1, info = orc.partition(mesh.ids, 8, fiedler_sweep=1, **KW)
    assert info["sweeps"] > 0 and info["sweep_moved"] == 0
    assert np.array_equal(p0, p1)


def test_exactly_degenerate_pair_is_not_swept(orc):
    # a 16 x 16 x 4 face-graph box: lambda_2 = lambda_3 exactly; the Krylov
    # space of one start vector holds a single vector of that eigenspace, so
    # the second Ritz value is the next distinct eigenvalue and no sweep runs
    ids = mg.box_hex(16, 16, 4).ids
    st, lam, y, info = orc.fiedler(ids, graph="face", fiedler_sweep=32, **KW)
    assert st == 0 and info["sweeps"] == 0


def test_second_solve_sweeps_an_exactly_degenerate_pair(orc):
    # the same box with the pair taken from two solves (second random start):
    # the swept cut equals the sweep over y1 projected on the dense
    # eigenspace and its orthogonal complement in that space, and is never
    # above the plain cut
    ids = mg.box_hex(16, 16, 4).ids
    rp, col, w = orc.dual_graph(ids, "face")
    ev, V = np.linalg.eigh(dense(rp, col, w))
    assert abs(ev[2] - ev[1]) < 1e-10 * ev[1] and ev[3] - ev[2] > 0.1 * ev[1]
    S = 16
    st, lam, y, info = orc.fiedler(ids, graph="face", fiedler_sweep=S, second_solve=1, **KW)
    st0, lam0, y0, _ = orc.fiedler(ids, graph="face", **KW)
    assert st == st0 == 0 and info["sweeps"] == 1
    E = V[:, 1:3]
    p1 = E @ (E.T @ y0)
    p1 = canonical(p1 / np.linalg.norm(p1))
    rot = np.array([[0.0, -1.0], [1.0, 0.0]])
    p2 = canonical(E @ (rot @ (E.T @ p1)))
    cuts = [half_cut(orc, rp, col, w, canonical(np.cos(np.pi * k / S) * p1 + np.sin(np.pi * k / S) * p2))
            for k in range(S)]
    assert half_cut(orc, rp, col, w, y) == min(cuts)
    assert half_cut(orc, rp, col, w, y) <= half_cut(orc, rp, col, w, y0)


def test_second_solve_leaves_a_simple_pair_alone(orc):
    # unique longest axis: the second solve returns the same vector, which
    # is not swept; the partition is the plain one
    ids = mg.box_hex(20, 12, 8).ids
    st0, p0, _ = orc.partition(ids, 8, fiedler_sweep=8, **KW)
    st1, p1, info = orc.partition(ids, 8, fiedler_sweep=8, second_solve=1, **KW)
    assert st0 == st1 == 0 and info["sweeps"] == 0
    assert np.array_equal(p0, p1)


@pytest.mark.parametrize("seed", range(6))
def test_second_solve_falls_back_to_the_thick_restart_pair(orc, seed):
    # a near-degenerate pair whose second solve comes back to y1 (not 0.1
    # off it): the thick restart's own pair is swept, exactly as without the
    # option
    mesh = mg.uniform_holes(mg.box_hex(10, 10, 4), 0.06, seed)
    st0, lam0, y0, i0 = orc.fiedler(mesh.ids, fiedler_sweep=16, **KW)
    st1, lam1, y1, i1 = orc.fiedler(mesh.ids, fiedler_sweep=16, second_solve=1, **KW)
    assert i0["sweeps"] == i1["sweeps"] == 1
    assert np.array_equal(y0, y1)
