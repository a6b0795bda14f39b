"""Pins of the oracle's gather-scatter Laplacian (Sec. 5: A_w = P^T Q Q^T P,
L = diag(A_w 1) - A_w).

It is pinned to the explicit product of the copy matrices P and Q (built
with numpy from the paper's definition), to the Laplacian of the assembled
weighted dual graph, to the printed worked example (z = A_w x with
x = (1, 0, 0) has z_2 = 2), and to the Laplacian's invariants: L 1 = 0 and
x^T L x = sum over element pairs of s_ij (x_i - x_j)^2.
"""
import json
import os

import numpy as np
import pytest

import meshgen as mg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def copy_matrix_product(ids):
    ids = np.asarray(ids)
    m, v = ids.shape
    uniq = np.unique(ids)
    P = np.zeros((m * v, m))
    for e in range(m):
        P[e * v:(e + 1) * v, e] = 1.0
    Q = np.zeros((m * v, len(uniq)))
    Q[np.arange(m * v), np.searchsorted(uniq, ids.ravel())] = 1.0
    return P.T @ Q @ Q.T @ P


def meshes():
    yield "box5x4x3", mg.box_hex(5, 4, 3)
    yield "box6x5x4-holes", mg.uniform_holes(mg.box_hex(6, 5, 4), 0.15, 7)
    yield "quad12x9-holes", mg.uniform_holes(mg.box_quad(12, 9), 0.1, 3)
    m = mg.uniform_holes(mg.box_hex(7, 6, 5), 0.1, 11)
    yield "box7x6x5-renum-shuffle", mg.shuffle_elements(mg.renumber_vertices(m, 5), 9)


@pytest.mark.parametrize("name,mesh", list(meshes()))
def test_equals_copy_matrix_product(orc, name, mesh):
    A = copy_matrix_product(mesh.ids)
    x = np.random.default_rng(1).standard_normal(mesh.nelem)
    want = A.sum(axis=1) * x - A @ x
    got = orc.gs_apply(mesh.ids, x)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("name,mesh", list(meshes()))
def test_equals_assembled_laplacian(orc, name, mesh):
    rp, col, w = orc.dual_graph(mesh.ids, "weighted")
    x = np.random.default_rng(2).standard_normal(mesh.nelem)
    want = orc.laplacian_apply(rp, col, w, x)
    got = orc.gs_apply(mesh.ids, x)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_invariants(orc):
    m = mg.clustered_holes(mg.box_hex(9, 8, 6), 0.1, 4)
    assert np.abs(orc.gs_apply(m.ids, np.ones(m.nelem))).max() == 0.0
    rp, col, w = orc.dual_graph(m.ids, "weighted")
    x = np.random.default_rng(3).standard_normal(m.nelem)
    quad = 0.0
    for i in range(m.nelem):
        for p in range(rp[i], rp[i + 1]):
            if col[p] > i:
                quad += w[p] * (x[i] - x[col[p]]) ** 2
    assert abs(x @ orc.gs_apply(m.ids, x) - quad) <= 1e-11 * quad


def test_paper_worked_example(orc):
    g = json.load(open(os.path.join(GOLD, "paper_gs_example.json")))
    ids = np.array(g["elements"])
    x = np.array(g["printed"]["x"], dtype=float)
    # A_w x = diag(A_w 1) x - L x; with x = e_1 the second entry is s_21
    A1 = copy_matrix_product(ids).sum(axis=1)
    z = A1 * x - orc.gs_apply(ids, x)
    assert z[1] == g["printed"]["z2"]


def test_repeated_id_counts_once(orc):
    # element 0 lists vertex 1 twice: the same Laplacian as the assembled
    # graph, which takes each element's ids as a set
    ids = np.array([[0, 1, 1, 2], [1, 2, 3, 4], [3, 4, 5, 6]], dtype=np.int64)
    rp, col, w = orc.dual_graph(ids, "weighted")
    x = np.array([1.0, -2.0, 0.5])
    assert np.allclose(orc.gs_apply(ids, x), orc.laplacian_apply(rp, col, w, x), rtol=0, atol=1e-14)
