"""Pins of the oracle's Lanczos where the Krylov space is exhausted (Sec. 6):
on a graph of n elements a cycle of m >= n - 1 steps spans every direction
orthogonal to the ones vector that the start vector reaches (fewer where the
Laplacian has repeated eigenvalues), so the next step must end the cycle by
breakdown.  Deep in a recursion the subgraphs are this small.

What fixes it independently of the code: the dense eigen-decomposition of
the Laplacian.  Every setting (one step at a time with explicit and thick
restart, two steps at a time) must return lambda_2 and the Fiedler vector of
the dense solver.  The two-step form takes beta_{j+2} from the Cholesky QR
(R11^2 = g11 - R01^2), a difference that cancellation empties as the second
column falls into the span of the basis; without the rule that ends the
cycle there, the next basis vector is not of unit norm and the cycle returns
Ritz values far from the spectrum (a box of 4x2x2 elements gave 24.9 for
lambda_2 = 5.27).
"""
import numpy as np
import pytest

import meshgen as mg
from spectral_util import assert_fiedler_close
from test_oracle_pins import dense_laplacian


def tiny_meshes(count, seed=5):
    """Seeded small boxes (quad and hex, some with holes), connected ones only."""
    import oracle
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        if t % 2:
            base = mg.box_quad(int(rng.integers(2, 9)), int(rng.integers(2, 7)))
        else:
            base = mg.box_hex(*(int(v) for v in rng.integers(2, 5, size=3)))
        mesh = mg.uniform_holes(base, 0.1, t) if t % 3 else base
        rp, col, w = oracle.dual_graph(mesh.ids)
        if len(rp) - 1 < 3:
            continue
        ev = np.linalg.eigvalsh(dense_laplacian(rp, col, w))
        if ev[1] < 1e-9 * ev[-1]:
            continue  # disconnected: another rule applies
        out.append(mesh.ids)
    return out


SETTINGS = {
    "one-step explicit": dict(lanczos_keep=0, lanczos_s=1),
    "one-step thick": dict(lanczos_keep=8, lanczos_s=1),
    "two-step thick": dict(lanczos_keep=8, lanczos_s=2),
}


@pytest.mark.parametrize("setting", list(SETTINGS))
def test_exhausted_cycles_match_dense_eigh(orc, setting):
    for ids in tiny_meshes(120):
        rp, col, w = orc.dual_graph(ids)
        ev, V = np.linalg.eigh(dense_laplacian(rp, col, w))
        m = 40 if len(rp) - 1 <= 41 else 60
        st, lam, y, info = orc.fiedler(ids, lanczos_m=m, tol=1e-10, max_restarts=20,
                                       **SETTINGS[setting])
        assert st == 0, (setting, len(rp) - 1)
        assert abs(lam - ev[1]) <= 1e-10 * ev[-1], (setting, len(rp) - 1, lam, ev[1])
        if ev[2] - ev[1] > 1e-6 * ev[-1]:
            assert_fiedler_close(y, V[:, 1], info["residual"], 1e-14 * ev[-1], ev[2] - ev[1])


def test_one_step_explicit_is_exact_in_one_cycle(orc):
    # one cycle that runs into the exhaustion ends by breakdown with the
    # exact pair: no restart needed
    for ids in tiny_meshes(60):
        rp, col, w = orc.dual_graph(ids)
        ev = np.linalg.eigvalsh(dense_laplacian(rp, col, w))
        m = 40 if len(rp) - 1 <= 41 else 60
        st, lam, _, info = orc.fiedler(ids, lanczos_m=m, lanczos_keep=0, tol=1e-10,
                                       max_restarts=0)
        assert st == 0 and info["cycles"] == 1
        assert abs(lam - ev[1]) <= 1e-10 * ev[-1]


def test_two_step_box_with_repeated_eigenvalues(orc):
    # 4 x 2 x 2 hex box: four double eigenvalues, so the Krylov space of a
    # start vector has 11 dimensions; the Ritz value of the first cycle is
    # an upper bound of lambda_2 (Courant-Fischer) close to it, never a
    # value from the middle of the spectrum
    ids = mg.box_hex(4, 2, 2).ids
    rp, col, w = orc.dual_graph(ids)
    ev = np.linalg.eigvalsh(dense_laplacian(rp, col, w))
    _, lam, _, info = orc.fiedler(ids, lanczos_m=40, lanczos_keep=8, lanczos_s=2, tol=1e-10,
                                  max_restarts=0)
    assert info["theta"] >= ev[1] * (1 - 1e-12)
    assert abs(lam - ev[1]) <= 1e-6 * ev[1]
    st, lam, _, _ = orc.fiedler(ids, lanczos_m=40, lanczos_keep=8, lanczos_s=2, tol=1e-10,
                                max_restarts=5)
    assert st == 0 and abs(lam - ev[1]) <= 1e-12 * ev[-1]


def test_two_step_only_above_four_m_elements(orc):
    # at most 4 m elements: one step at a time (bit for bit the one-step
    # result, whose breakdown the pins above check); above: the two-step
    # recurrence (the same values to rounding, not bit for bit)
    kw = dict(lanczos_m=20, lanczos_keep=8, tol=1e-10, max_restarts=50)
    small = mg.uniform_holes(mg.box_hex(5, 4, 4), 0.05, 3).ids  # 76 elements <= 80
    big = mg.uniform_holes(mg.box_hex(9, 7, 5), 0.05, 3).ids    # 299 elements
    assert len(small) <= 80 < len(big)
    _, l1, y1, _ = orc.fiedler(small, lanczos_s=1, **kw)
    _, l2, y2, _ = orc.fiedler(small, lanczos_s=2, **kw)
    assert l1 == l2 and np.array_equal(y1, y2)
    _, l1, y1, _ = orc.fiedler(big, lanczos_s=1, **kw)
    _, l2, y2, _ = orc.fiedler(big, lanczos_s=2, **kw)
    assert abs(l1 - l2) <= 1e-9 * l1 and not np.array_equal(y1, y2)
