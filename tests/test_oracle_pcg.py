"""Pins for the oracle's dense Theta product and preconditioned CG (Sections 4.2-4.3)."""
import numpy as np
from scipy.spatial import distance_matrix

import oracle as O
from paper_1706_02205_amd import workloads as W


def test_dense_matvec_matches_numpy():
    x = W.uniform_points(700, 3, 1)
    X = W.gaussian_rhs(700, 3, 2)
    for nu, f in ((0.5, lambda a: np.exp(-a)), (1.5, lambda a: (1 + np.sqrt(3) * a) * np.exp(-np.sqrt(3) * a)),
                  (2.5, lambda a: (1 + np.sqrt(5) * a + 5 * a * a / 3) * np.exp(-np.sqrt(5) * a))):
        T = f(distance_matrix(x, x) / 0.3)
        np.testing.assert_allclose(O.dense_matvec(x, X, nu, 0.3), T @ X, rtol=1e-12, atol=1e-12)
        rows = np.array([0, 5, 699])
        np.testing.assert_allclose(O.dense_matvec_rows(x, X, nu, 0.3, rows), (T @ X)[rows], rtol=1e-12, atol=1e-12)


def test_pcg_with_exact_factor_converges_in_one_step():
    x = W.uniform_points(300, 2, 3)
    P = O.pattern(x, 1e6)  # full pattern: ICHOL(0) is the exact Cholesky factor
    R = O.ichol(P, O.theta_on_pattern(P, 0.5, 0.1))
    b = W.gaussian_rhs(300, 2, 4)
    sol, it = O.pcg(P, R.L, x, 0.5, 0.1, b, tol=1e-10)
    assert it == 1
    T = np.exp(-distance_matrix(x, x) / 0.1)
    np.testing.assert_allclose(sol, np.linalg.solve(T, b), rtol=0, atol=1e-9 * np.abs(sol).max())


def test_pcg_reaches_tolerance_with_sparse_factor():
    w = W.large_grid_2d(40)
    P = O.pattern(w.points, w.rho)
    R = O.ichol(P, O.theta_on_pattern(P, w.nu, w.lengthscale))
    b = W.gaussian_rhs(w.n, 4, 5)
    sol, it = O.pcg(P, R.L, w.points, w.nu, w.lengthscale, b, tol=1e-10)
    res = np.linalg.norm(b - O.dense_matvec(w.points, sol, w.nu, w.lengthscale), axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(res <= 1.1e-10)
    assert it < 20
