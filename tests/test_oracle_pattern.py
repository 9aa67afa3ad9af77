"""Pins for the oracle's maximin ordering and sparsity pattern (Section 2.3).

The ordering is checked against invariants that characterise the greedy
maximin order (with ties to the lowest original index), the pattern against a
dense scipy distance matrix, and both against the nnz(L)/N^2 values printed
in the paper's Section 4.4 tables.
"""
import numpy as np
import pytest
from scipy.spatial import distance_matrix

import oracle as O
from paper_1706_02205_amd import workloads as W


def check_maximin(x, perm, l):
    n = len(x)
    assert sorted(perm.tolist()) == list(range(n))
    assert perm[0] == 0 and np.isinf(l[0])
    xh = x[perm]
    D = distance_matrix(xh, xh)
    # C[a, k] = min distance of point a to the first k+1 selected points
    C = np.minimum.accumulate(D, axis=1)
    for k in range(1, n):
        # l[k] is the distance to the earlier points ...
        assert l[k] == pytest.approx(C[k, k - 1], rel=1e-14, abs=0)
        # ... and no later point is farther from them (greedy argmax)
        later = C[k + 1:, k - 1]
        assert np.all(later <= l[k] * (1 + 1e-14))
        # ties go to the lowest original index
        tied = np.nonzero(np.abs(later - l[k]) <= 1e-14 * l[k])[0] + k + 1
        assert np.all(perm[tied] > perm[k])
    assert np.all(np.diff(l[1:]) <= 0)


def test_hand_example():
    # three collinear points: order 0, 1, 2 with l = inf, 1, 0.4
    x = np.array([[0.0, 0.0], [1.0, 0.0], [0.4, 0.0]])
    perm, l = O.maximin(x)
    assert perm.tolist() == [0, 1, 2]
    assert np.isinf(l[0]) and l[1] == 1.0 and l[2] == 0.4
    Pmax = O.pattern(x, 1.0, O.RULE_MAX)
    assert Pmax.nnz == 6  # full lower triangle: 0.6 <= 1*max(1, 0.4)
    Pmin = O.pattern(x, 1.0, O.RULE_MIN)
    # (2,0) sits exactly on the boundary 0.4 <= 0.4 (inclusive), (2,1): 0.6 > 0.4
    assert Pmin.nnz == 5
    assert Pmin.rowidx.tolist() == [0, 1, 2, 1, 2]


@pytest.mark.parametrize("n,d,seed", [(300, 2, 1), (250, 3, 2), (200, 5, 3)])
def test_maximin_invariants_random(n, d, seed):
    x = W.uniform_points(n, d, seed)
    check_maximin(x, *O.maximin(x))


def test_maximin_ties_on_lattice():
    # integer coordinates: squared distances are exact, so equal distances are exact ties
    x = np.array([(a, b) for a in range(7) for b in range(6)], dtype=np.float64)
    check_maximin(x, *O.maximin(x))


def test_maximin_duplicates():
    x = W.uniform_points(100, 2, 4)
    x = np.concatenate([x, x[:10]])
    perm, l = O.maximin(x)
    check_maximin(x, perm, l)
    assert np.sum(l == 0.0) == 10  # each duplicate is last in its pair, at distance 0


@pytest.mark.parametrize("rule", [O.RULE_MAX, O.RULE_MIN])
@pytest.mark.parametrize("rho", [0.7, 2.0, 3.5])
def test_pattern_against_distance_matrix(rule, rho):
    x = W.uniform_points(400, 2, 11)
    P = O.pattern(x, rho, rule)
    D = distance_matrix(P.xh, P.xh)
    n = P.n
    la, lb = np.meshgrid(P.l, P.l, indexing="ij")
    sc = np.maximum(la, lb) if rule == O.RULE_MAX else np.minimum(la, lb)
    with np.errstate(invalid="ignore"):
        lim = rho * sc
    low = np.tril(np.ones((n, n), bool))
    inner = low & (D <= lim * (1 - 1e-12))
    outer = low & (D <= lim * (1 + 1e-12))
    got = np.zeros((n, n), bool)
    cols = np.repeat(np.arange(n), np.diff(P.colptr))
    got[P.rowidx, cols] = True
    assert np.all(got[inner]) and not np.any(got & ~outer)
    assert np.all(np.diag(got))
    for b in range(n):  # rows ascending, diagonal first
        r = P.rowidx[P.colptr[b]:P.colptr[b + 1]]
        assert r[0] == b and np.all(np.diff(r) > 0)


def test_pattern_rho_to_zero():
    # rho -> 0+: the max-rule keeps the diagonal and the first column (rho*inf = inf),
    # the min-rule keeps the diagonal only
    x = W.uniform_points(200, 2, 12)
    Pmax = O.pattern(x, 1e-9, O.RULE_MAX)
    assert Pmax.nnz == 200 + 199 and Pmax.colptr[1] == 200
    Pmin = O.pattern(x, 1e-9, O.RULE_MIN)
    assert Pmin.nnz == 200


@pytest.mark.parametrize("row", [0, 1, 2])
def test_pattern_size_matches_paper(golden, row):
    """nnz(L)/N^2 printed in the Section 4.4 vary-N tables (rho=3), fresh uniform points."""
    g = golden["vary_N"][row]
    w = W.paper_uniform(g["N"], g["d"], seed=100 + row)
    P = O.pattern(w.points, g["rho"])
    ratio = P.nnz / g["N"] ** 2
    assert ratio == pytest.approx(g["nnz_over_N2"], rel=0.03)


def test_pattern_near_linear_growth():
    """#S grows like N log N (Section 2.3): nnz/N is affine in log N."""
    ns = [1000, 2000, 4000, 8000, 16000]
    per = []
    for n in ns:
        P = O.pattern(W.uniform_points(n, 2, 21), 3.0)
        per.append(P.nnz / n)
    A = np.vstack([np.ones(len(ns)), np.log(ns)]).T
    coef, res, *_ = np.linalg.lstsq(A, np.array(per), rcond=None)
    fit = A @ coef
    assert coef[1] > 0
    assert np.max(np.abs(fit - per) / np.array(per)) < 0.03
