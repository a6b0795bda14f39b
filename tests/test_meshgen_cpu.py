"""The seeded input generators that both the library and the oracle are fed
from: shapes, exact removal counts, clustering, relabelling and shuffling
behave as their recipes state (no method arithmetic here)."""
import numpy as np

import meshgen as mg


def test_box_hex_elements_are_unit_cubes():
    nx, ny, nz = 5, 4, 3
    m = mg.box_hex(nx, ny, nz)
    assert m.ids.shape == (nx * ny * nz, 8) and m.ids.dtype == np.int64
    assert np.unique(m.ids).size == (nx + 1) * (ny + 1) * (nz + 1)
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    x, y, z = m.ids % sx, (m.ids // sx) % (ny + 1), m.ids // sy
    for c in (x, y, z):
        assert np.all(c.max(axis=1) - c.min(axis=1) == 1)
    # every element holds 8 distinct corners; interior vertices are shared by 8 elements
    assert all(len(set(r)) == 8 for r in m.ids.tolist())
    shared = np.bincount(m.ids.ravel())
    assert np.sum(shared == 8) == (nx - 1) * (ny - 1) * (nz - 1)


def test_uniform_holes_remove_exactly_the_fraction():
    m = mg.box_hex(20, 10, 10)
    h = mg.uniform_holes(m, 0.07, 3)
    assert h.nelem == m.nelem - round(0.07 * m.nelem) == m.nelem - h.meta["removed"]
    assert np.unique(h.lex).size == h.nelem
    assert np.array_equal(h.ids, m.ids[h.lex])


def _removed_neighbour_counts(dims, lex_kept):
    nx, ny, nz = dims
    present = np.zeros(nx * ny * nz, dtype=bool)
    present[lex_kept] = True
    gone = np.nonzero(~present)[0]
    i, j, k = gone % nx, (gone // nx) % ny, gone // (nx * ny)
    cnt = np.zeros(gone.size, dtype=np.int64)
    for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        a, b, c = i + di, j + dj, k + dk
        ok = (a >= 0) & (a < nx) & (b >= 0) & (b < ny) & (c >= 0) & (c < nz)
        li = np.where(ok, a + nx * (b + ny * c), 0)
        cnt += ok & ~present[li]
    return cnt


def test_clustered_holes_remove_exactly_the_fraction_in_clusters():
    m = mg.box_hex(40, 40, 20)
    c = mg.clustered_holes(m, 0.10, 9)
    u = mg.uniform_holes(m, 0.10, 9)
    assert c.nelem == u.nelem == m.nelem - round(0.10 * m.nelem)
    assert np.array_equal(c.ids, m.ids[c.lex])
    # removed elements sit inside spheres: most of their face neighbours are gone too
    cc = _removed_neighbour_counts(m.dims, c.lex)
    cu = _removed_neighbour_counts(m.dims, u.lex)
    assert np.mean(cc >= 3) > 0.7 and np.mean(cu >= 3) < 0.05


def test_renumbering_is_a_consistent_bijection():
    m = mg.uniform_holes(mg.box_hex(9, 8, 7), 0.1, 2)
    r = mg.renumber_vertices(m, 5)
    old, new = m.ids.ravel(), r.ids.ravel()
    pairs = np.unique(np.stack([old, new], axis=1), axis=0)
    assert np.unique(pairs[:, 0]).size == np.unique(pairs[:, 1]).size == pairs.shape[0]
    assert np.all(new % (2 ** 31) == 7) and new.max() > 2 ** 32


def test_shuffle_is_a_row_permutation():
    m = mg.box_hex(7, 6, 5)
    s = mg.shuffle_elements(m, 4)
    perm = s.meta["perm"]
    assert np.array_equal(np.sort(perm), np.arange(m.nelem))
    assert np.array_equal(s.ids, m.ids[perm]) and np.array_equal(s.lex, m.lex[perm])
    assert not np.array_equal(perm, np.arange(m.nelem))


def test_streams_are_reproducible_and_uniform():
    a = mg.uniform01(123, 100000)
    assert np.array_equal(a, mg.uniform01(123, 100000))
    assert np.array_equal(a[500:600], mg.uniform01(123, 100, offset=500))
    assert a.min() >= 0.0 and a.max() < 1.0
    hist = np.bincount((a * 10).astype(int), minlength=10)
    assert np.all(np.abs(hist - 10000) < 500)


def test_benchmark_mesh_size():
    m = mg.box256x128_clustered10()
    assert m.nelem == 7_549_747 and m.meta["removed"] == 838_861
