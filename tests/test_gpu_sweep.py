"""GPU parity of the sweep over the Fiedler pair against the CPU oracle.

The cut of every swept bisection must equal the oracle's (both pick the
smallest cut among the same combinations of the converged pair); one angle
reproduces the plain method exactly; an exactly degenerate pair is not swept.
"""
import numpy as np
import pytest

import meshgen as mg
import paper_2606_14659_amd as rsb

pytestmark = pytest.mark.gpu

KW = dict(lanczos_keep=8, lanczos_m=30, tol=1e-10)


def half_cut(orc, ids, y):
    rp, col, w = orc.dual_graph(ids)
    n = len(y)
    side = orc.split(y, np.arange(n), n // 2)
    rows = np.repeat(np.arange(n), np.diff(rp))
    c = (side[rows] != side[col]) & (col > rows)
    return int(w[c].sum())


@pytest.mark.parametrize("seed", range(6))
def test_sweep_fiedler_cut_matches_oracle(orc, seed):
    ids = mg.uniform_holes(mg.box_hex(10, 10, 4), 0.06, seed).ids
    st, lam, y, stats = rsb.fiedler(ids, fiedler_sweep=16, **KW)
    ost, olam, oy, oinfo = orc.fiedler(ids, fiedler_sweep=16, **KW)
    assert st == ost == 0
    assert stats["sweeps"] == oinfo["sweeps"] == 1
    assert abs(lam - olam) <= 1e-8 * olam
    assert half_cut(orc, ids, y) == half_cut(orc, ids, oy)
    assert abs(np.linalg.norm(y) - 1) < 1e-10


def test_sweep_one_angle_is_plain():
    ids = mg.uniform_holes(mg.box_hex(24, 24, 12), 0.05, 3).ids
    kw = dict(lanczos_keep=8, lanczos_m=40, tol=1e-6)
    st0, p0, s0 = rsb.partition(ids, 16, **kw)
    st1, p1, s1 = rsb.partition(ids, 16, fiedler_sweep=1, **kw)
    assert s1["sweeps"] > 0 and s1["sweep_moved"] == 0
    assert np.array_equal(p0, p1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep_partition_cut_vs_oracle(orc, precision):
    m = mg.uniform_holes(mg.box_hex(24, 24, 12), 0.05, 3)
    tol = 1e-4 if precision == "mixed" else 1e-6
    kw = dict(lanczos_keep=8, lanczos_m=40, tol=tol)
    st, part, stats = rsb.partition(m.ids, 16, precision=precision, fiedler_sweep=8, **kw)
    st0, part0, stats0 = rsb.partition(m.ids, 16, precision=precision, **kw)
    ost, opart, oinfo = orc.partition(m.ids, 16, fiedler_sweep=8, lanczos_keep=8, lanczos_m=40,
                                      tol=1e-6)
    ocut = orc.metrics(m.ids, opart, 16)["weighted_cut"]
    print(f"24x24x12 holes -> 16 ({precision}): cut plain {stats0['edge_cut']:.0f}, swept "
          f"{stats['edge_cut']:.0f} ({stats['sweeps']} swept, {stats['sweep_moved']} moved); "
          f"oracle swept {ocut:.0f} ({oinfo['sweeps']}, {oinfo['sweep_moved']})", flush=True)
    sizes = np.bincount(part, minlength=16)
    assert sizes.max() - sizes.min() <= 1
    assert stats["sweeps"] == oinfo["sweeps"]
    assert abs(stats["edge_cut"] - ocut) <= 0.01 * ocut
    assert stats["edge_cut"] < stats0["edge_cut"]


def test_exactly_degenerate_pair_is_not_swept():
    ids = mg.box_hex(16, 16, 4).ids
    st, lam, y, stats = rsb.fiedler(ids, graph="face", fiedler_sweep=32, **KW)
    assert st == 0 and stats["sweeps"] == 0


def test_sweep_unbatched_equals_batched():
    ids = mg.uniform_holes(mg.box_hex(20, 20, 10), 0.05, 5).ids
    kw = dict(lanczos_keep=8, lanczos_m=40, tol=1e-8, fiedler_sweep=8)
    st1, p1, s1 = rsb.partition(ids, 8, **kw)
    st2, p2, s2 = rsb.partition(ids, 8, batched=0, **kw)
    assert s1["sweeps"] == s2["sweeps"] > 0
    assert np.array_equal(p1, p2)


# --- warm start of the child solves from the parent's second Ritz vector ---

@pytest.mark.parametrize("dims,graph,nparts", [((24, 20, 18), "face", 8),
                                              ((30, 14, 9), "face", 6),
                                              ((30, 16, 7), "face", 4)])
def test_warm_start_partition_identical(orc, dims, graph, nparts):
    ids = mg.box_hex(*dims).ids
    kw = dict(graph=graph, lanczos_keep=8, lanczos_m=30, tol=1e-8)
    import os
    st, part, stats = rsb.partition(ids, nparts, warm_start=1,
                                    verbose=int(os.environ.get("RSB_TEST_VERBOSE", "0")), **kw)
    ost, opart, _ = orc.partition(ids, nparts, warm_start=1, **kw)
    st0, part0, stats0 = rsb.partition(ids, nparts, **kw)
    print(f"{dims} {graph} {nparts}: status warm {st} oracle {ost} plain {st0}; segment steps "
          f"{stats['segment_steps']} / {stats0['segment_steps']}", flush=True)
    assert st == ost == st0 == 0
    assert np.array_equal(part, opart) and np.array_equal(part, part0)
    assert stats["segment_steps"] <= stats0["segment_steps"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_warm_start_fewer_steps_same_cut(orc, precision):
    m = mg.clustered_holes(mg.box_hex(48, 48, 24), 0.1, 9)
    kw = dict(lanczos_keep=8, lanczos_m=40, tol=1e-2)
    st0, p0, s0 = rsb.partition(m.ids, 64, precision=precision, **kw)
    st1, p1, s1 = rsb.partition(m.ids, 64, precision=precision, warm_start=1, **kw)
    ost, op, oinfo = orc.partition(m.ids, 64, warm_start=1, **kw)
    ocut = orc.metrics(m.ids, op, 64)["weighted_cut"]
    print(f"48x48x24 clustered -> 64 ({precision}): level-steps {s0['level_steps']} -> "
          f"{s1['level_steps']}, segment-steps {s0['segment_steps']} -> {s1['segment_steps']}; "
          f"cut {s0['edge_cut']:.0f} -> {s1['edge_cut']:.0f} (oracle warm {ocut:.0f})", flush=True)
    assert s1["segment_steps"] < 0.85 * s0["segment_steps"]
    assert abs(s1["edge_cut"] - ocut) <= 0.01 * ocut
    sizes = np.bincount(p1, minlength=64)
    assert sizes.max() - sizes.min() <= 1


def test_warm_start_unbatched_equals_batched():
    ids = mg.uniform_holes(mg.box_hex(20, 20, 10), 0.05, 5).ids
    kw = dict(lanczos_keep=8, lanczos_m=40, tol=1e-8, warm_start=1)
    st1, p1, s1 = rsb.partition(ids, 8, **kw)
    st2, p2, s2 = rsb.partition(ids, 8, batched=0, **kw)
    assert np.array_equal(p1, p2)


def _cut(orc, ids, y, graph):
    rp, col, w = orc.dual_graph(ids, graph)
    n = len(y)
    side = orc.split(y, np.arange(n), n // 2)
    rows = np.repeat(np.arange(n), np.diff(rp))
    c = (side[rows] != side[col]) & (col > rows)
    return int(w[c].sum())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_second_solve_sweeps_exactly_degenerate_pair(orc, precision):
    # lambda_2 = lambda_3 on a 16 x 16 x 4 face box: the pair from two solves
    # (second random start) is swept; the swept cut equals the oracle's and
    # is never above the plain one
    ids = mg.box_hex(16, 16, 4).ids
    kw = dict(graph="face", fiedler_sweep=16, second_solve=1, **KW)
    tol = 1e-4 if precision == "mixed" else 1e-10
    st, lam, y, stats = rsb.fiedler(ids, precision=precision, **dict(kw, tol=tol))
    ost, olam, oy, oinfo = orc.fiedler(ids, **kw)
    st0, lam0, y0, _ = rsb.fiedler(ids, graph="face", **KW)
    assert st == ost == st0 == 0
    assert stats["sweeps"] == oinfo["sweeps"] == 1
    cut, ocut = _cut(orc, ids, y, "face"), _cut(orc, ids, oy, "face")
    print(f"[second solve] {precision}: cut {cut} oracle {ocut} plain {_cut(orc, ids, y0, 'face')}",
          flush=True)
    assert cut == ocut
    assert cut <= _cut(orc, ids, y0, "face")


def test_second_solve_leaves_simple_pair_alone(orc):
    ids = mg.box_hex(20, 12, 8).ids
    kw = dict(fiedler_sweep=8, **KW)
    st0, p0, s0 = rsb.partition(ids, 8, **kw)
    st1, p1, s1 = rsb.partition(ids, 8, second_solve=1, **kw)
    st2, p2, s2 = rsb.partition(ids, 8, second_solve=1, batched=0, **kw)
    ost, op, oinfo = orc.partition(ids, 8, second_solve=1, **kw)
    assert st0 == st1 == st2 == ost == 0
    assert s1["sweeps"] == s2["sweeps"] == oinfo["sweeps"] == 0
    assert np.array_equal(p1, p0) and np.array_equal(p2, p0) and np.array_equal(p0, op)


def test_second_solve_partition_degenerate_box(orc):
    ids = mg.box_hex(16, 16, 8).ids
    kw = dict(graph="face", fiedler_sweep=16, second_solve=1, **KW)
    st, part, stats = rsb.partition(ids, 4, **kw)
    st1, part1, _ = rsb.partition(ids, 4, batched=0, **kw)
    ost, opart, oinfo = orc.partition(ids, 4, **kw)
    assert st == st1 == ost == 0 and stats["sweeps"] == oinfo["sweeps"] >= 1
    assert np.array_equal(part, part1)
    cut = orc.metrics(ids, part, 4)["weighted_cut"]
    ocut = orc.metrics(ids, opart, 4)["weighted_cut"]
    assert abs(cut - ocut) <= 0.01 * ocut


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", range(3))
def test_second_solve_falls_back_to_thick_pair(orc, seed, precision):
    # the second solve comes back to y1 on these near-degenerate pairs: the
    # thick restart's own pair is swept, exactly as without the option
    ids = mg.uniform_holes(mg.box_hex(10, 10, 4), 0.06, seed).ids
    kw = dict(KW, precision=precision, fiedler_sweep=16)
    st0, lam0, y0, s0 = rsb.fiedler(ids, **kw)
    st1, lam1, y1, s1 = rsb.fiedler(ids, second_solve=1, **kw)
    assert s0["sweeps"] == s1["sweeps"] == 1 and np.array_equal(y0, y1)
    ost, olam, oy, oinfo = orc.fiedler(ids, second_solve=1, **dict(KW, fiedler_sweep=16))
    assert oinfo["sweeps"] == 1 and half_cut(orc, ids, y1) == half_cut(orc, ids, oy)
