"""Pins for the oracle's triangular solves x = P^T L^-T L^-1 P b (Section 1, task (2))."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular
from scipy.spatial import distance_matrix

import oracle as O
from paper_1706_02205_amd import workloads as W


def csc_matrix(P, L):
    return sp.csc_matrix((L, P.rowidx, P.colptr), shape=(P.n, P.n))


@pytest.mark.parametrize("nrhs", [1, 4])
def test_solve_matches_scipy_triangular(nrhs):
    x = W.uniform_points(1200, 2, 13)
    P = O.pattern(x, 3.0)
    R = O.ichol(P, O.theta_on_pattern(P, 0.5, 0.2))
    assert R.nonpositive == 0
    b = W.gaussian_rhs(P.n, nrhs, 14)
    got = O.solve(P, R.L, b)
    Ls = csc_matrix(P, R.L).tocsr()
    y = spsolve_triangular(Ls, b[P.perm], lower=True)
    xh = spsolve_triangular(Ls.T.tocsr(), y, lower=False)
    ref = np.empty_like(xh)
    ref[P.perm] = xh
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_full_pattern_solve_inverts_theta():
    x = W.uniform_points(150, 2, 15)
    P = O.pattern(x, 1e6)
    R = O.ichol(P, O.theta_on_pattern(P, 0.5, 0.1))
    b = W.gaussian_rhs(P.n, 2, 16)
    sol = O.solve(P, R.L, b)
    T = np.exp(-distance_matrix(x, x) / 0.1)  # original order
    ref = np.linalg.solve(T, b)
    np.testing.assert_allclose(sol, ref, rtol=0, atol=1e-12 * np.linalg.cond(T) * np.abs(ref).max())


def test_zeroed_column_gives_zero_component():
    # L = [[2, 0, 0], [1, 0, 0], [0.5, 0, 1]] with column 1 zeroed
    P = O.Pattern(perm=np.array([0, 1, 2], np.int32), l=np.array([np.inf, 1.0, 1.0]),
                  colptr=np.array([0, 3, 5, 6], np.int64), rowidx=np.array([0, 1, 2, 1, 2, 2], np.int32),
                  xh=np.zeros((3, 1)))
    L = np.array([2.0, 1.0, 0.5, 0.0, 0.0, 1.0])
    b = np.array([[4.0], [5.0], [3.0]])
    x = O.solve_permuted(P, L, b)
    # forward: y0 = 2, y1 = 0 (zeroed), y2 = 3 - 0.5*2 = 2; backward: x2 = 2, x1 = 0, x0 = (2 - 0.5*2)/2
    assert x[:, 0].tolist() == [0.5, 0.0, 2.0]
