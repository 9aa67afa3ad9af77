"""CPU oracle for the sparse-Cholesky path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct FP64 reference, written from the paper
(Schaefer, Sullivan, Owhadi, arXiv:1706.02205).  Only the test-suite, the
package smoke check and the benchmark's CPU-baseline leg may import this
module; the product library never calls it and shares no code with it.

The heavy loops live in ``kchol_oracle.c`` (gcc, -ffp-contract=off); this
file marshals numpy arrays through ctypes and adds the small dense helpers.
Functions and the passages they follow:

* :func:`maximin`       greedy maximin ordering, O(N^2)           -- Section 2.3
* :func:`pattern`       sparsity pattern S_rho (max or min rule)   -- Section 2.3 / Section 6.2
* :func:`theta_on_pattern`  Matern covariance on S                 -- Section 4.4 (Matern definition)
* :func:`ichol`         right-looking ICHOL(0)                     -- Section 2.2 (incomplete Cholesky)
* :func:`solve`         x = P^T L^-T L^-1 P b                      -- Section 1, task (2)
* :func:`llt_pairs`, :func:`mc_error`, :func:`frob_error`  error E -- Section 4.4

Parity status: every function above is pinned by ``tests/test_oracle_*.py``
(closed forms, library special cases, brute force on tiny inputs, and the
paper's printed nnz and error statistics).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

RULE_MAX, RULE_MIN = 0, 1
PIVOT_ZERO, PIVOT_SHIFT = 0, 1

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        I64, I32, F64 = C.c_int64, C.c_int32, C.c_double
        L.or_maximin.argtypes = [_f64p, I64, I32, _i32p, _f64p]
        L.or_pattern_count.argtypes = [_f64p, I64, I32, _f64p, F64, I32, _i64p]
        L.or_pattern_fill.argtypes = [_f64p, I64, I32, _f64p, F64, I32, _i64p, _i32p]
        L.or_matern.argtypes = [_f64p, I64, F64, F64, _f64p]
        L.or_theta.argtypes = [_f64p, I64, I32, F64, F64, _i64p, _i32p, _f64p]
        L.or_ichol.argtypes = [I64, _i64p, _i32p, _f64p, I32, F64, _f64p, _i64p]
        L.or_solve.argtypes = [I64, _i64p, _i32p, _f64p, I32, _f64p, _f64p]
        L.or_llt_pairs.argtypes = [I64, _i64p, _i32p, _f64p, I64, _i64p, _i64p, _f64p]
        L.or_frob_error.argtypes = [_f64p, I64, I32, F64, F64, _i64p, _i32p, _f64p, _f64p]
        L.or_num_threads.argtypes = []
        L.or_prefix_min_dist.argtypes = [_f64p, I32, I64, _i64p, _f64p]
        L.or_pattern_column.argtypes = [_f64p, I64, I32, _f64p, F64, I32, I64, _i32p]
        L.or_pattern_column.restype = C.c_int64
        L.or_theta_pairs.argtypes = [_f64p, I32, F64, F64, I64, _i64p, _i64p, _f64p]
        L.or_ichol_leading.argtypes = [I64, _i64p, _i32p, I64, _f64p, I32, F64, _f64p]
        L.or_dense_matvec.argtypes = [_f64p, I64, I32, F64, F64, _f64p, I32, _f64p]
        L.or_dense_matvec_rows.argtypes = [_f64p, I64, I32, F64, F64, _f64p, I32, I64, _i64p, _f64p]
        L.or_supernodes.argtypes = [_f64p, I64, I32, _f64p, F64, _i32p]
        L.or_supernodes.restype = C.c_int64
        for fn in ("or_maximin", "or_pattern_count", "or_pattern_fill", "or_matern", "or_theta", "or_ichol",
                   "or_solve", "or_llt_pairs", "or_frob_error", "or_num_threads", "or_prefix_min_dist",
                   "or_theta_pairs", "or_ichol_leading", "or_dense_matvec", "or_dense_matvec_rows"):
            getattr(L, fn).restype = C.c_int
        _LIB = L
    return _LIB


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().or_num_threads())


# --------------------------------------------------------------------------
@dataclass
class Pattern:
    perm: np.ndarray     # int32[n]: maximin position -> original index
    l: np.ndarray        # float64[n]: l[k] = distance of the k-th point to the earlier ones
    colptr: np.ndarray   # int64[n+1]
    rowidx: np.ndarray   # int32[nnz], ascending within each column, diagonal first
    xh: np.ndarray       # (n, d) points gathered into maximin order

    @property
    def n(self) -> int:
        return int(self.perm.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


def maximin(x: np.ndarray):
    """Greedy maximin ordering (Section 2.3), brute force O(N^2).

    Returns (perm, l): perm[k] is the original index of the k-th point and
    l[k] its distance to the points before it (l[0] = +inf).  First index:
    original index 0; ties: lowest original index."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, d = x.shape
    perm = np.empty(n, np.int32)
    l = np.empty(n, np.float64)
    _check(lib().or_maximin(x, n, d, perm, l), "maximin")
    return perm, l


def pattern(x: np.ndarray, rho: float, rule: int = RULE_MAX, ordering=None) -> Pattern:
    """Pattern S_rho (Section 2.3) on the maximin ordering, brute force O(N^2).

    Lower triangle in CSC over maximin positions, diagonal included."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, d = x.shape
    perm, l = ordering if ordering is not None else maximin(x)
    xh = np.ascontiguousarray(x[perm])
    colptr = np.empty(n + 1, np.int64)
    _check(lib().or_pattern_count(xh, n, d, l, float(rho), int(rule), colptr), "pattern_count")
    rowidx = np.empty(int(colptr[-1]), np.int32)
    _check(lib().or_pattern_fill(xh, n, d, l, float(rho), int(rule), colptr, rowidx), "pattern_fill")
    return Pattern(perm, l, colptr, rowidx, xh)


def matern(r: np.ndarray, nu: float, ell: float) -> np.ndarray:
    """Matern covariance at distances r (Section 4.4), nu in {1/2, 3/2, 5/2}."""
    r = np.ascontiguousarray(r, dtype=np.float64).ravel()
    out = np.empty_like(r)
    _check(lib().or_matern(r, r.size, float(nu), float(ell), out), "matern")
    return out


def theta_on_pattern(P: Pattern, nu: float, ell: float) -> np.ndarray:
    """Theta_ab = G(x_a, x_b) for every (a,b) in S, in CSC order."""
    out = np.empty(P.nnz, np.float64)
    n, d = P.xh.shape
    _check(lib().or_theta(P.xh, n, d, float(nu), float(ell), P.colptr, P.rowidx, out), "theta")
    return out


@dataclass
class IcholResult:
    L: np.ndarray          # CSC values aligned with the pattern's rowidx
    nonpositive: int
    shifted: int
    updates: int

    @property
    def rank(self) -> int:
        return -1  # filled by callers that know n


def ichol(P: Pattern, theta: np.ndarray, policy: int = PIVOT_ZERO, tau: float = 0.0) -> IcholResult:
    """ICHOL(0) (Section 2.2) in the paper's right-looking order."""
    L = np.empty(P.nnz, np.float64)
    stats = np.zeros(3, np.int64)
    _check(lib().or_ichol(P.n, P.colptr, P.rowidx, np.ascontiguousarray(theta, dtype=np.float64), int(policy),
                          float(tau), L, stats), "ichol")
    return IcholResult(L, int(stats[0]), int(stats[1]), int(stats[2]))


def solve_permuted(P: Pattern, L: np.ndarray, bh: np.ndarray) -> np.ndarray:
    """L^-T L^-1 bh for bh (n, nrhs) already in maximin order."""
    bh = np.ascontiguousarray(bh, dtype=np.float64)
    if bh.ndim == 1:
        bh = bh[:, None]
    out = np.empty_like(bh)
    _check(lib().or_solve(P.n, P.colptr, P.rowidx, np.ascontiguousarray(L), bh.shape[1], bh, out), "solve")
    return out


def solve(P: Pattern, L: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x = P^T L^-T L^-1 P b in the caller's original point order."""
    b2 = b[:, None] if b.ndim == 1 else b
    xh = solve_permuted(P, L, b2[P.perm])
    x = np.empty_like(xh)
    x[P.perm] = xh
    return x[:, 0] if b.ndim == 1 else x


def llt_pairs(P: Pattern, L: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """(L L^T)_{a,b} for arrays of maximin positions."""
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    out = np.empty(a.size, np.float64)
    _check(lib().or_llt_pairs(P.n, P.colptr, P.rowidx, np.ascontiguousarray(L), a.size, a, b, out), "llt_pairs")
    return out


def mc_error(P: Pattern, L: np.ndarray, nu: float, ell: float, pairs: np.ndarray, box=None) -> float:
    """Sampled relative Frobenius error E of Section 4.4 over index pairs.

    ``pairs`` are maximin positions; with ``box=(lo, hi)`` only pairs whose two
    points lie in [lo, hi]^d are kept (the paper's E-bar)."""
    a, b = pairs[:, 0], pairs[:, 1]
    if box is not None:
        lo, hi = box
        keep = np.all((P.xh[a] >= lo) & (P.xh[a] <= hi), axis=1) & np.all((P.xh[b] >= lo) & (P.xh[b] <= hi), axis=1)
        a, b = a[keep], b[keep]
    th = matern(np.sqrt(((P.xh[a] - P.xh[b]) ** 2).sum(axis=1)), nu, ell)
    approx = llt_pairs(P, L, a, b)
    return float(np.sqrt(((approx - th) ** 2).sum()) / np.sqrt((th ** 2).sum()))


def frob_error(P: Pattern, L: np.ndarray, nu: float, ell: float) -> float:
    """Exact ||L L^T - Theta||_F / ||Theta||_F over all N^2 pairs."""
    out = np.empty(2, np.float64)
    n, d = P.xh.shape
    _check(lib().or_frob_error(P.xh, n, d, float(nu), float(ell), P.colptr, P.rowidx, np.ascontiguousarray(L), out),
           "frob_error")
    return float(np.sqrt(out[0] / out[1]))


def dense_from_csc(P: Pattern, vals: np.ndarray) -> np.ndarray:
    """Dense lower-triangular matrix from CSC values (small n only)."""
    n = P.n
    M = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(P.colptr))
    M[P.rowidx, cols] = vals
    return M


# --------------------------------------------------------------------------
# One-by-one checks for samples of problems too large for the O(N^2) oracle.

def prefix_min_dist(xh: np.ndarray, ks: np.ndarray) -> np.ndarray:
    """min_{i<k} dist(xh_k, xh_i) for each k in ks: l[k] of the maximin ordering (Section 2.3)."""
    xh = np.ascontiguousarray(xh, dtype=np.float64)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    out = np.empty(ks.size, np.float64)
    _check(lib().or_prefix_min_dist(xh, xh.shape[1], ks.size, ks, out), "prefix_min_dist")
    return out


def pattern_column(xh: np.ndarray, l: np.ndarray, rho: float, b: int, rule: int = RULE_MAX) -> np.ndarray:
    """Rows of column b of S_rho (Section 2.3), brute force over all later points."""
    xh = np.ascontiguousarray(xh, dtype=np.float64)
    n, d = xh.shape
    rows = np.empty(n - b, np.int32)
    c = lib().or_pattern_column(xh, n, d, np.ascontiguousarray(l, dtype=np.float64), float(rho), int(rule), int(b),
                                rows)
    return rows[:c]


def theta_pairs(xh: np.ndarray, nu: float, ell: float, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Theta_ab (Section 4.4 Matern) for pairs of ordered points."""
    xh = np.ascontiguousarray(xh, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    out = np.empty(a.size, np.float64)
    _check(lib().or_theta_pairs(xh, xh.shape[1], float(nu), float(ell), a.size, a, b, out), "theta_pairs")
    return out


def ichol_leading(colptr: np.ndarray, rowidx: np.ndarray, m: int, theta_lead: np.ndarray,
                  policy: int = PIVOT_ZERO, tau: float = 0.0) -> np.ndarray:
    """The first m columns of ICHOL(0) (Section 2.2) in the same per-entry order as :func:`ichol`."""
    n = colptr.size - 1
    L = np.empty(int(colptr[m]), np.float64)
    _check(lib().or_ichol_leading(n, np.ascontiguousarray(colptr, dtype=np.int64),
                                  np.ascontiguousarray(rowidx, dtype=np.int32), int(m),
                                  np.ascontiguousarray(theta_lead, dtype=np.float64), int(policy), float(tau), L),
           "ichol_leading")
    return L


# --------------------------------------------------------------------------
# Conjugate gradients with the sparse factor as preconditioner (Sections 4.2-4.3).

def dense_matvec(x: np.ndarray, X: np.ndarray, nu: float, ell: float) -> np.ndarray:
    """Theta X with the dense Matern matrix of the points x (any order)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    X2 = np.ascontiguousarray(X[:, None] if X.ndim == 1 else X, dtype=np.float64)
    Y = np.empty_like(X2)
    _check(lib().or_dense_matvec(x, x.shape[0], x.shape[1], float(nu), float(ell), X2, X2.shape[1], Y), "dense_matvec")
    return Y[:, 0] if X.ndim == 1 else Y


def dense_matvec_rows(x: np.ndarray, X: np.ndarray, nu: float, ell: float, rows: np.ndarray) -> np.ndarray:
    """Rows `rows` of Theta X."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    X2 = np.ascontiguousarray(X[:, None] if X.ndim == 1 else X, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    Y = np.empty((rows.size, X2.shape[1]), np.float64)
    _check(lib().or_dense_matvec_rows(x, x.shape[0], x.shape[1], float(nu), float(ell), X2, X2.shape[1], rows.size,
                                      rows, Y), "dense_matvec_rows")
    return Y


def pcg(P: Pattern, L: np.ndarray, x: np.ndarray, nu: float, ell: float, b: np.ndarray, tol: float = 1e-10,
        maxit: int = 200):
    """Textbook preconditioned CG on Theta sol = b, x0 = 0, M^-1 = P^T L^-T L^-1 P, every
    right-hand side stopped once ||r||/||b|| <= tol.  Returns (sol, iterations)."""
    b2 = b[:, None] if b.ndim == 1 else b
    sol = np.zeros_like(b2)
    r = b2.copy()
    nb = np.linalg.norm(b2, axis=0)
    z = solve(P, L, r)
    p = z.copy()
    rz = (r * z).sum(axis=0)
    active = np.ones(b2.shape[1], bool)
    it = 0
    for it in range(1, maxit + 1):
        q = dense_matvec(x, p, nu, ell)
        alpha = np.where(active, rz / (p * q).sum(axis=0), 0.0)
        sol += alpha * p
        r -= alpha * q
        active &= np.linalg.norm(r, axis=0) / nb > tol
        if not active.any():
            break
        z = solve(P, L, r)
        rz_new = (r * z).sum(axis=0)
        p = np.where(active, z + (rz_new / rz) * p, p)
        rz = rz_new
    return (sol[:, 0] if b.ndim == 1 else sol), it


# --------------------------------------------------------------------------
# Supernodal ordering and pattern (Section 5, supernodal construction used for
# the stability proof; its incomplete factorization is the block algorithm of
# the same section's appendix).

def supernodal_pattern(x: np.ndarray, rho: float) -> "tuple[Pattern, np.ndarray]":
    """Supernodal ordering + block-closed pattern, built from the brute-force maximin
    ordering and pattern.  Returns (pattern in the new positions, supernode boundaries)."""
    P = pattern(x, rho, RULE_MAX)
    n, d = P.xh.shape
    node = np.empty(n, np.int32)
    ns = int(lib().or_supernodes(P.xh, n, d, P.l, float(rho), node))
    # new order: supernodes by their first point, members in maximin order (stable sort)
    order = np.argsort(node, kind="stable")
    sptr = np.concatenate([[0], np.cumsum(np.bincount(node, minlength=ns))]).astype(np.int64)
    # adjacency of supernodes: some member pair in S_rho
    cols = np.repeat(np.arange(n), np.diff(P.colptr))
    a, b = node[P.rowidx], node[cols]
    adj = set(zip(np.maximum(a, b).tolist(), np.minimum(a, b).tolist()))
    by_col = {}
    for hi, lo in adj:
        by_col.setdefault(lo, []).append(hi)
    colptr = [0]
    rows = []
    for s in range(ns):
        below = sorted(t for t in by_col.get(s, []) if t > s)
        for q in range(sptr[s], sptr[s + 1]):
            rows.extend(range(q, sptr[s + 1]))
            for t in below:
                rows.extend(range(sptr[t], sptr[t + 1]))
            colptr.append(len(rows))
    perm = P.perm[order]
    Pn = Pattern(perm=perm.astype(np.int32), l=P.l[order], colptr=np.array(colptr, np.int64),
                 rowidx=np.array(rows, np.int32), xh=np.ascontiguousarray(P.xh[order]))
    return Pn, sptr


def block_ichol(Pn: Pattern, sptr: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Supernodal incomplete Cholesky in block form: for each supernode I in order,
    L_{:,I} = K_{:,I} chol(K_{I,I})^{-T}; then K_{K,J} -= K_{K,I} K_{I,I}^{-1} K_{J,I}^T for
    supernodes J >= I and K >= J adjacent to I with (K, J) adjacent.  Dense numpy, small n only."""
    n = Pn.n
    A = dense_from_csc(Pn, theta)
    A = np.tril(A) + np.tril(A, -1).T
    mask = dense_from_csc(Pn, np.ones(Pn.nnz)) != 0
    mask = mask | mask.T
    ns = len(sptr) - 1
    L = np.zeros((n, n))
    blocks = [slice(sptr[s], sptr[s + 1]) for s in range(ns)]
    adj = np.zeros((ns, ns), bool)
    for s in range(ns):
        for t in range(ns):
            adj[s, t] = mask[sptr[s], sptr[t]]
    for i, I in enumerate(blocks):
        C = np.linalg.cholesky(A[I, I])
        rest = slice(sptr[i], n)
        Li = np.linalg.solve(C, A[rest, I].T).T  # K_{:,I} C^{-T}
        Li[:, :] *= mask[rest, I]
        L[rest, I] = Li
        kids = [t for t in range(i + 1, ns) if adj[t, i]]
        for j in kids:
            for k in kids:
                if k >= j and adj[k, j]:
                    Kb, Jb = blocks[k], blocks[j]
                    A[Kb, Jb] -= L[Kb, I] @ L[Jb, I].T
                    if k != j:
                        A[Jb, Kb] = A[Kb, Jb].T
    return L
