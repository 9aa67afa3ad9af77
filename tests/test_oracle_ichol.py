"""Pins for the oracle's ICHOL(0) (Section 2.2) and its error (Section 4.4).

* a full pattern reduces ICHOL(0) to the dense Cholesky factor (LAPACK);
* the update count of a full pattern is the closed form (n-1)n(n+1)/6;
* IC(0) reproduces Theta exactly on S (columns not zeroed);
* rho -> 0+ has a closed form (first column and diagonal only);
* the nonpositive-pivot rules on a hand-made 2x2 matrix;
* the error decays exponentially in rho (Section 4.4, error-vs-rho study);
* E and E-bar agree with the values printed in the Section 4.4 tables.
"""
import numpy as np
import pytest
from scipy.spatial import distance_matrix

import oracle as O
from paper_1706_02205_amd import workloads as W


def dense_theta(xh, nu, ell):
    r = distance_matrix(xh, xh)
    if nu == 0.5:
        return np.exp(-r / ell)
    a = np.sqrt(3.0) * r / ell
    return (1 + a) * np.exp(-a)


@pytest.mark.parametrize("nu,ell", [(0.5, 0.05), (0.5, 0.3), (1.5, 0.05)])
def test_full_pattern_equals_dense_cholesky(nu, ell):
    x = W.uniform_points(80, 2, 7)
    P = O.pattern(x, 1e6)
    assert P.nnz == 80 * 81 // 2
    th = O.theta_on_pattern(P, nu, ell)
    R = O.ichol(P, th)
    assert R.nonpositive == 0
    Ld = O.dense_from_csc(P, R.L)
    T = dense_theta(P.xh, nu, ell)
    Lref = np.linalg.cholesky(T)
    tol = 1e-15 * np.linalg.cond(T) + 1e-14
    np.testing.assert_allclose(Ld, Lref, rtol=0, atol=tol)
    n = P.n
    assert R.updates == (n - 1) * n * (n + 1) // 6


@pytest.mark.parametrize("nu,rho,rule", [(0.5, 3.0, O.RULE_MAX), (1.5, 3.0, O.RULE_MAX), (2.5, 2.0, O.RULE_MAX),
                                         (1.5, 3.0, O.RULE_MIN)])
def test_ic0_reproduces_theta_on_pattern(nu, rho, rule):
    x = W.uniform_points(1500, 2, 8)
    P = O.pattern(x, rho, rule)
    th = O.theta_on_pattern(P, nu, 0.2)
    R = O.ichol(P, th)
    cols = np.repeat(np.arange(P.n), np.diff(P.colptr))
    v = O.llt_pairs(P, R.L, P.rowidx.astype(np.int64), cols.astype(np.int64))
    zeroed = np.nonzero(R.L[P.colptr[:-1]] == 0.0)[0]
    assert len(zeroed) == R.nonpositive
    keep = ~np.isin(cols, zeroed)
    assert np.max(np.abs(v - th)[keep]) < 1e-13
    # a zeroed column is zero throughout
    for j in zeroed:
        assert np.all(R.L[P.colptr[j]:P.colptr[j + 1]] == 0.0)


def test_rho_to_zero_closed_form():
    x = W.uniform_points(300, 2, 9)
    P = O.pattern(x, 1e-9, O.RULE_MAX)
    th = O.theta_on_pattern(P, 0.5, 0.2)
    R = O.ichol(P, th)
    L = O.dense_from_csc(P, R.L)
    g = np.exp(-np.linalg.norm(P.xh - P.xh[0], axis=1) / 0.2)
    np.testing.assert_allclose(L[1:, 0], g[1:], rtol=1e-15)
    np.testing.assert_allclose(np.diag(L)[1:], np.sqrt(1 - g[1:] ** 2), rtol=1e-14)
    Pm = O.pattern(x, 1e-9, O.RULE_MIN)
    Rm = O.ichol(Pm, O.theta_on_pattern(Pm, 0.5, 0.2))
    assert np.all(Rm.L == 1.0)


def hand_2x2():
    P = O.Pattern(perm=np.array([0, 1], np.int32), l=np.array([np.inf, 1.0]),
                  colptr=np.array([0, 2, 3], np.int64), rowidx=np.array([0, 1, 1], np.int32),
                  xh=np.zeros((2, 1)))
    return P, np.array([1.0, 2.0, 1.0])  # [[1, 2], [2, 1]] is indefinite


def test_pivot_rules_hand_example():
    P, th = hand_2x2()
    R = O.ichol(P, th, O.PIVOT_ZERO)
    assert R.L.tolist() == [1.0, 2.0, 0.0] and R.nonpositive == 1 and R.shifted == 0
    R = O.ichol(P, th, O.PIVOT_SHIFT, 0.5)
    assert R.L.tolist() == [1.0, 2.0, np.sqrt(0.5)] and R.shifted == 1 and R.nonpositive == 0


def test_error_decays_exponentially_in_rho():
    x = W.uniform_points(2000, 2, 5)
    o = O.maximin(x)
    errs = []
    for rho in [1.0, 2.0, 3.0, 4.0]:
        P = O.pattern(x, rho, ordering=o)
        R = O.ichol(P, O.theta_on_pattern(P, 0.5, 0.2))
        errs.append(O.frob_error(P, R.L, 0.5, 0.2))
    errs = np.array(errs)
    assert np.all(errs[1:] < errs[:-1] / 2.5)
    slope = np.polyfit([1, 2, 3, 4], np.log(errs), 1)[0]
    assert slope < -1.2


def test_sampled_error_matches_exact():
    x = W.uniform_points(3000, 2, 6)
    P = O.pattern(x, 2.0)
    R = O.ichol(P, O.theta_on_pattern(P, 0.5, 0.2))
    exact = O.frob_error(P, R.L, 0.5, 0.2)
    mc = O.mc_error(P, R.L, 0.5, 0.2, W.random_pairs(P.n, 500_000, 1))
    assert mc == pytest.approx(exact, rel=0.05)


@pytest.mark.parametrize("row", [0, 2])
def test_error_matches_paper(golden, row):
    """E, E-bar and rank printed in the Section 4.4 vary-N tables (N=20000, rho=3)."""
    g = golden["vary_N"][row]
    w = W.paper_uniform(g["N"], g["d"], seed=200 + row)
    P = O.pattern(w.points, g["rho"])
    R = O.ichol(P, O.theta_on_pattern(P, g["nu"], g["l"]))
    assert P.n - R.nonpositive == g["rank"]
    pairs = W.random_pairs(P.n, 500_000, 300 + row)
    assert O.mc_error(P, R.L, g["nu"], g["l"], pairs) == pytest.approx(g["E"], rel=0.25)
    assert O.mc_error(P, R.L, g["nu"], g["l"], pairs, box=(0.05, 0.95)) == pytest.approx(g["Ebar"], rel=0.25)
