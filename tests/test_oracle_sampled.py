"""The oracle's one-by-one functions (used on samples of large problems) agree with the full oracle."""
import numpy as np

import oracle as O
from paper_1706_02205_amd import workloads as W


def test_one_by_one_functions_match_full_oracle():
    x = W.uniform_points(1500, 2, 3)
    P = O.pattern(x, 3.0)
    th = O.theta_on_pattern(P, 1.5, 0.2)
    R = O.ichol(P, th)
    assert R.nonpositive > 0  # the zeroed-column path is exercised
    for m in (1, 17, 40, 1500):
        Ll = O.ichol_leading(P.colptr, P.rowidx, m, th[:P.colptr[m]])
        assert np.array_equal(Ll, R.L[:P.colptr[m]])
    Rs = O.ichol(P, th, O.PIVOT_SHIFT, 1e-6)
    assert np.array_equal(O.ichol_leading(P.colptr, P.rowidx, 200, th[:P.colptr[200]], O.PIVOT_SHIFT, 1e-6),
                          Rs.L[:P.colptr[200]])
    ks = np.array([1, 2, 5, 100, 777, 1499])
    assert np.array_equal(O.prefix_min_dist(P.xh, ks), P.l[ks])
    for b in (0, 1, 7, 500, 1499):
        assert np.array_equal(O.pattern_column(P.xh, P.l, 3.0, b), P.rowidx[P.colptr[b]:P.colptr[b + 1]])
    Pm = O.pattern(x, 3.0, O.RULE_MIN)
    for b in (0, 3, 900):
        assert np.array_equal(O.pattern_column(Pm.xh, Pm.l, 3.0, b, O.RULE_MIN),
                              Pm.rowidx[Pm.colptr[b]:Pm.colptr[b + 1]])
    cols = np.repeat(np.arange(P.n), np.diff(P.colptr))
    assert np.array_equal(O.theta_pairs(P.xh, 1.5, 0.2, P.rowidx.astype(np.int64), cols), th)
