"""Pins of the oracle's two-step Lanczos (lanczos_s = 2): from step 3 on,
steps j+1 and j+2 come from one block [L q_j, L^2 q_j], orthogonalised
against the basis and split by a Cholesky QR; the projected matrix entries
alpha_{j+1} = R01/R00 - alpha_j and beta_{j+2} = R11/R00 follow from the
Lanczos relation (only q_j of the old basis couples to q_{j+1}).

What fixes it independently of the code: in exact arithmetic the block
spans the same Krylov space and gives the same projected matrix as one step
at a time (the paper's Sec. 6 recurrence), so

* cycle by cycle -- a fixed number of cycles from the same start, explicit
  and thick restart, even and odd cycle lengths (a trailing single step) --
  the Ritz value agrees with the one-step recurrence to rounding;
* converged, the pair agrees with the dense eigendecomposition (eigenvalue
  to 1e-10, vector element by element within the gap bound).

A sign flipped in the derived alpha_{j+1} moves the Ritz values of the first
check by orders of magnitude more than rounding.
"""
import numpy as np
import pytest

import meshgen as mg
from spectral_util import assert_fiedler_close
from test_oracle_pins import dense_laplacian

MESHES = {
    "holes": lambda: mg.uniform_holes(mg.box_hex(14, 10, 7), 0.07, 3),
    "clustered": lambda: mg.clustered_holes(mg.box_hex(13, 11, 8), 0.1, 9),
    "box": lambda: mg.box_hex(12, 7, 5),
    "quad": lambda: mg.uniform_holes(mg.box_quad(36, 25), 0.1, 4),
}
_EIGH = {}


def _eigh(orc, name, ids):
    if name not in _EIGH:
        rp, col, w = orc.dual_graph(ids)
        _EIGH[name] = np.linalg.eigh(dense_laplacian(rp, col, w))
    return _EIGH[name]


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("keep,m", [(0, 30), (8, 40), (4, 13), (3, 8)])
@pytest.mark.parametrize("cycles", [1, 4])
def test_two_step_equals_one_step_cycle_by_cycle(orc, name, keep, m, cycles):
    ids = MESHES[name]().ids
    kw = dict(lanczos_m=m, lanczos_keep=keep, tol=1e-15, max_restarts=cycles - 1)
    st1, lam1, y1, i1 = orc.fiedler(ids, **kw)
    st2, lam2, y2, i2 = orc.fiedler(ids, lanczos_s=2, **kw)
    assert i1["cycles"] == i2["cycles"] == cycles
    assert i1["matvecs"] == i2["matvecs"]
    assert abs(i1["theta"] - i2["theta"]) <= 1e-11 * i1["theta"]
    assert abs(lam1 - lam2) <= 1e-11 * lam1


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("keep,m", [(0, 40), (8, 40), (5, 20)])
def test_two_step_matches_dense_eigh(orc, name, keep, m):
    mesh = MESHES[name]()
    ev, V = _eigh(orc, name, mesh.ids)
    assert int(np.sum(np.abs(ev) < 1e-9)) == 1 and ev[2] - ev[1] > 1e-6 * ev[1]
    st, lam, y, info = orc.fiedler(mesh.ids, lanczos_m=m, lanczos_keep=keep, lanczos_s=2,
                                   tol=1e-10, max_restarts=2000)
    assert st == 0
    assert abs(lam - ev[1]) <= 1e-10 * ev[1]
    assert_fiedler_close(y, V[:, 1], info["residual"], 1e-14 * ev[-1], ev[2] - ev[1])


def test_two_step_partition_equals_one_step(orc):
    # a unique longest axis at every level: the same octant partition
    box = mg.box_hex(24, 20, 18)
    kw = dict(graph="face", lanczos_m=40, lanczos_keep=8, tol=1e-8, warm_start=1)
    st1, p1, _ = orc.partition(box.ids, 8, **kw)
    st2, p2, _ = orc.partition(box.ids, 8, lanczos_s=2, **kw)
    assert st1 == st2 == 0 and np.array_equal(p1, p2)
