"""Pins for the oracle's supernodal construction (Section 5, supernodal ordering
and pattern) and for the equivalence of ICHOL(0) on it with the block algorithm."""
import numpy as np
import pytest
from scipy.spatial import distance_matrix

import oracle as O
from paper_1706_02205_amd import workloads as W


@pytest.mark.parametrize("n,d,rho", [(600, 2, 3.0), (500, 3, 2.0)])
def test_greedy_aggregation_and_block_closure(n, d, rho):
    x = W.uniform_points(n, d, 7)
    P = O.pattern(x, rho)
    Pn, sptr = O.supernodal_pattern(x, rho)
    ns = len(sptr) - 1
    # positions of the new order in the maximin order
    inv = np.empty(n, np.int64)
    inv[P.perm] = np.arange(n)
    old = inv[Pn.perm]
    node = np.repeat(np.arange(ns), np.diff(sptr))
    D = distance_matrix(P.xh, P.xh)
    leaders = np.array([old[sptr[s]] for s in range(ns)])
    assert np.all(np.diff(leaders) > 0)  # supernodes ordered by their first point
    for q in range(n):
        a = old[q]
        # the supernode of a is the first earlier leader that may claim it (or a itself)
        elig = [s for s in range(ns) if leaders[s] < a and P.l[a] >= 0.5 * P.l[leaders[s]]
                and D[a, leaders[s]] <= 0.5 * rho * P.l[leaders[s]] * (1 + 1e-12)]
        want = elig[0] if elig else np.nonzero(leaders == a)[0][0]
        assert node[q] == want
    # block closure containing S_rho: adjacency of supernodes, then all member pairs
    full = O.dense_from_csc(Pn, np.ones(Pn.nnz)) != 0
    S = O.dense_from_csc(P, np.ones(P.nnz)) != 0
    Snew = S[np.ix_(old, old)]
    Snew = Snew | Snew.T
    assert np.all(full[np.tril(Snew)])
    for s in range(ns):
        for t in range(s, ns):
            blk = full[sptr[t]:sptr[t + 1], sptr[s]:sptr[s + 1]]
            if t > s:
                assert blk.all() or not blk.any()
                assert blk.any() == Snew[sptr[t]:sptr[t + 1], sptr[s]:sptr[s + 1]].any()


def test_elementwise_equals_block_algorithm():
    x = W.uniform_points(400, 2, 6)
    Pn, sptr = O.supernodal_pattern(x, 2.0)
    th = O.theta_on_pattern(Pn, 0.5, 0.1)
    R = O.ichol(Pn, th)
    assert R.nonpositive == 0
    np.testing.assert_allclose(O.dense_from_csc(Pn, R.L), O.block_ichol(Pn, sptr, th), rtol=0, atol=1e-13)


def test_supernodal_pattern_is_at_least_as_accurate():
    x = W.uniform_points(2000, 2, 8)
    P = O.pattern(x, 2.0)
    e_plain = O.frob_error(P, O.ichol(P, O.theta_on_pattern(P, 0.5, 0.2)).L, 0.5, 0.2)
    Pn, _ = O.supernodal_pattern(x, 2.0)
    e_super = O.frob_error(Pn, O.ichol(Pn, O.theta_on_pattern(Pn, 0.5, 0.2)).L, 0.5, 0.2)
    assert e_super <= e_plain


def test_supernodes_of_a_worked_example():
    """Nine points on a line, rho = 2: the ordering and supernodes worked out by hand from the paper's
    construction (tests/golden/supernodes_line9.json holds the derivation)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "supernodes_line9.json")) as f:
        g = json.load(f)
    x = np.array(g["points"], dtype=np.float64).reshape(-1, 1)
    P = O.pattern(x, g["rho"])
    np.testing.assert_array_equal(P.perm, g["maximin_perm"])
    np.testing.assert_array_equal(P.l, [float(v) for v in g["maximin_l"]])
    Pn, sptr = O.supernodal_pattern(x, g["rho"])
    np.testing.assert_array_equal(Pn.perm, g["supernodal_perm"])
    np.testing.assert_array_equal(sptr, g["supernode_ptr"])
