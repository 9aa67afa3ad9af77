"""Host analysis (ordering, pattern, level schedule) against the oracle, bit for bit."""
import numpy as np
import pytest

import oracle as O
import paper_1706_02205_amd as K
from paper_1706_02205_amd import workloads as W


def assert_same(x, rho, rule):
    p = K.analyze(x, rho, rule)
    perm, l, colptr, rowidx = p.export()
    P = O.pattern(x, rho, O.RULE_MAX if rule == "max" else O.RULE_MIN)
    np.testing.assert_array_equal(perm, P.perm)
    np.testing.assert_array_equal(l, P.l)
    np.testing.assert_array_equal(colptr, P.colptr)
    np.testing.assert_array_equal(rowidx, P.rowidx)
    return p, P


@pytest.mark.parametrize("n,d,rho,rule,seed", [
    (2000, 2, 3.0, "max", 1001), (2000, 2, 3.0, "min", 1001), (3000, 3, 2.0, "max", 2), (800, 5, 1.5, "max", 3),
    (1500, 2, 0.5, "max", 4), (1500, 2, 0.5, "min", 4), (700, 2, 9.0, "max", 5), (64, 2, 1e9, "max", 6),
    (300, 1, 3.0, "max", 7), (1200, 3, 4.0, "min", 8)])
def test_matches_oracle(n, d, rho, rule, seed):
    assert_same(W.uniform_points(n, d, seed), rho, rule)


def test_jittered_grid_and_sphere_embedding():
    assert_same(W.jittered_grid(40, 9), 4.0, "max")
    assert_same(W.embedded_sincos(900, 10), 3.0, "max")


def test_ties_and_duplicates():
    lattice = np.array([(a, b) for a in range(9) for b in range(7)], dtype=np.float64)
    assert_same(lattice, 2.0, "max")
    assert_same(lattice, 2.0, "min")
    x = W.uniform_points(300, 2, 11)
    x = np.concatenate([x, x[:25], x[:5]])
    assert_same(x, 2.5, "max")
    assert_same(x, 2.5, "min")


@pytest.mark.parametrize("name", ["grid2d", "sincos20d", "lattice", "duplicates"])
def test_ordering_on_several_threads_matches_oracle(name):
    """From 16,384 points and 8 analysis threads on, the ordering runs in batches on several threads;
    it must still be the oracle's greedy maximin ordering bit for bit, ties and duplicates included."""
    if name == "grid2d":
        x = W.jittered_grid(140, 21)
    elif name == "sincos20d":
        x = W.embedded_sincos(17000, 22)
    elif name == "lattice":
        x = np.array([(a, b) for a in range(130) for b in range(130)], dtype=np.float64)
    else:
        base = W.uniform_points(9000, 2, 23)
        x = np.concatenate([base, base[:8000], base[:500]])
    assert len(x) >= 16384
    perm, l = O.maximin(x)
    for nthreads in (8, 16):
        pp, ll, _, _ = K.analyze(x, 3.0, "max", nthreads).export()
        np.testing.assert_array_equal(pp, perm)
        np.testing.assert_array_equal(ll, l)


def test_tiny_inputs():
    for n in (1, 2, 3):
        assert_same(W.uniform_points(n, 2, 12), 2.0, "max")
    assert_same(np.array([[0.0, 0.0], [1.0, 0.0], [0.4, 0.0]]), 1.0, "min")


def test_level_schedule_is_topological():
    x = W.uniform_points(2500, 2, 13)
    p = K.analyze(x, 3.0)
    perm, l, colptr, rowidx = p.export()
    lv = p.levels()
    n = p.n
    cols = np.repeat(np.arange(n), np.diff(colptr))
    off = rowidx != cols
    # an entry (k, j) below the diagonal makes column k wait for column j
    assert np.all(lv[rowidx[off]] > lv[cols[off]])
    # level = 1 + max level of the parents (tight schedule)
    best = np.full(n, -1)
    np.maximum.at(best, rowidx[off], lv[cols[off]])
    assert np.array_equal(lv, best + 1)
    assert p.info()["nlevels"] == lv.max() + 1


@pytest.mark.slow
def test_full_size_pattern_matches_paper(golden):
    """nnz(L)/N^2 at N = 10^6 uniform points in 2-D, rho = 3 (Section 4.4 vary-rho table)."""
    g = golden["vary_rho_1e6_2d"]
    p = K.analyze(W.uniform_points(g["N"], 2, 14), 3.0)
    assert p.nnz / g["N"] ** 2 == pytest.approx(g["nnz_over_N2"][1], rel=0.03)


def test_batched_plan_is_the_union_of_instances():
    xs = [W.uniform_points(n, 2, 30 + i) for i, n in enumerate([300, 1, 50, 700, 2])]
    pb = K.analyze_batched(xs, 3.0)
    assert pb.info()["ninst"] == len(xs)
    perm, l, cp, ri = pb.export()
    lv = pb.levels()
    off = eo = 0
    depth = 0
    for x in xs:
        P = O.pattern(x, 3.0)
        n = len(x)
        np.testing.assert_array_equal(perm[off:off + n] - off, P.perm)
        np.testing.assert_array_equal(l[off:off + n], P.l)
        np.testing.assert_array_equal(cp[off:off + n + 1] - eo, P.colptr)
        np.testing.assert_array_equal(ri[eo:eo + P.nnz] - off, P.rowidx)
        np.testing.assert_array_equal(lv[off:off + n], K.analyze(x, 3.0).levels())
        depth = max(depth, K.analyze(x, 3.0).info()["nlevels"])
        off += n
        eo += P.nnz
    assert pb.info()["nlevels"] == depth


@pytest.mark.parametrize("n,d,rho,seed", [(3000, 3, 3.0, 5), (2500, 2, 2.0, 6), (800, 5, 1.5, 7)])
def test_supernodal_plan_matches_oracle(n, d, rho, seed):
    x = W.uniform_points(n, d, seed)
    Pn, sptr = O.supernodal_pattern(x, rho)
    p = K.analyze_supernodal(x, rho)
    perm, l, cp, ri = p.export()
    np.testing.assert_array_equal(perm, Pn.perm)
    np.testing.assert_array_equal(l, Pn.l)
    np.testing.assert_array_equal(cp, Pn.colptr)
    np.testing.assert_array_equal(ri, Pn.rowidx)
    np.testing.assert_array_equal(p.supernodes(), sptr)


def test_supernodal_plan_of_a_worked_example():
    """The host's supernodal ordering on the hand-worked example (tests/golden/supernodes_line9.json)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "supernodes_line9.json")) as f:
        g = json.load(f)
    x = np.array(g["points"], dtype=np.float64).reshape(-1, 1)
    p = K.analyze_supernodal(x, g["rho"])
    np.testing.assert_array_equal(p.export()[0], g["supernodal_perm"])
    np.testing.assert_array_equal(p.supernodes(), g["supernode_ptr"])
