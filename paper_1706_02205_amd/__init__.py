"""Sparse Cholesky factors of dense Matern kernel matrices on MI355X (gfx950).

Method: Schaefer, Sullivan, Owhadi (arXiv:1706.02205).  Points + kernel + rho
give the maximin ordering and pattern S (host, :func:`analyze`), then the
covariance entries on S and their ICHOL(0) factor L (GPU, :meth:`Factor.factorize`),
then x ~ Theta^{-1} b through L and L^T (GPU, :meth:`Factor.solve`).

Every step runs in the HIP library ``libkchol.so`` through its C ABI
(``include/kchol.h``); this module only marshals arguments.  PyTorch provides
device memory and the current stream.  There is no CPU fallback: without the
built library every call raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _lib
from ._lib import KCholError

__all__ = ["analyze", "analyze_supernodal", "analyze_batched", "dense_matvec", "Plan", "Factor", "Graph", "KCholError"]

_RULES = {"max": _lib.KC_RULE_MAX, "min": _lib.KC_RULE_MIN}
_PRECS = {"fp64": _lib.KC_FP64, "mixed": _lib.KC_MIXED}
_PIVOTS = {"zero": _lib.KC_PIVOT_ZERO, "shift": _lib.KC_PIVOT_SHIFT}
_ORDERS = {"spatial": _lib.KC_ORDER_SPATIAL, "longest": _lib.KC_ORDER_LONGEST}
_ORDER_NAMES = {v: k for k, v in _ORDERS.items()}


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


class Plan:
    """Host analysis: maximin ordering, pattern S and the elimination schedule."""

    def __init__(self, handle, n: int, d: int, counts=None):
        self._h = handle
        self.n, self.d = n, d
        self.counts = counts  # points per instance for a batch plan, else None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None and _lib._LIB is not None:
            _lib._LIB.kc_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _lib.kc_plan_info_t()
        _lib.check(_lib.load().kc_plan_info(self._h, C.byref(inf)), "kc_plan_info")
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    @property
    def nnz(self) -> int:
        return int(self.info()["nnz"])

    def export(self):
        """(perm, l, colptr, rowidx) of the ordering and the CSC pattern."""
        n, nnz = self.n, self.nnz
        perm = np.empty(n, np.int32)
        l = np.empty(n, np.float64)
        colptr = np.empty(n + 1, np.int64)
        rowidx = np.empty(nnz, np.int32)
        _lib.check(_lib.load().kc_plan_export(self._h, _ptr(perm), _ptr(l), _ptr(colptr), _ptr(rowidx)),
                   "kc_plan_export")
        return perm, l, colptr, rowidx

    def supernodes(self) -> np.ndarray:
        """Supernode boundaries (positions) of a supernodal plan; empty for other plans."""
        ns = C.c_int64()
        _lib.check(_lib.load().kc_plan_supernodes(self._h, None, C.byref(ns)), "kc_plan_supernodes")
        ptr = np.empty(ns.value + 1 if ns.value else 0, np.int64)
        if ns.value:
            _lib.check(_lib.load().kc_plan_supernodes(self._h, _ptr(ptr), C.byref(ns)), "kc_plan_supernodes")
        return ptr

    def levels(self) -> np.ndarray:
        lv = np.empty(self.n, np.int32)
        _lib.check(_lib.load().kc_plan_levels(self._h, _ptr(lv)), "kc_plan_levels")
        return lv

    def set_delta_limit(self, limit: int) -> int:
        """Re-encode the 16-bit row-index gaps with escapes for gaps >= limit (1..65536; default 65536).
        The factor is the same for every limit; small limits exercise the escape path.  Returns the
        number of escapes."""
        ne = C.c_int64()
        _lib.check(_lib.load().kc_plan_set_delta_limit(self._h, int(limit), C.byref(ne)), "kc_plan_set_delta_limit")
        return int(ne.value)


def analyze(x: np.ndarray, rho: float, rule: str = "max", nthreads: int = 0) -> Plan:
    """Maximin ordering + pattern S_rho + level schedule (Section 2.3) on the host."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("x must be (n, d)")
    n, d = x.shape
    h = C.c_void_p()
    _lib.check(_lib.load().kc_analyze(_ptr(x), n, d, float(rho), _RULES[rule], int(nthreads), C.byref(h)),
               "kc_analyze")
    return Plan(h, n, d)


def analyze_supernodal(x: np.ndarray, rho: float, nthreads: int = 0) -> Plan:
    """Supernodal ordering + block-closed pattern (aggregated maximin ordering) on the host."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("x must be (n, d)")
    n, d = x.shape
    h = C.c_void_p()
    _lib.check(_lib.load().kc_analyze_supernodal(_ptr(x), n, d, float(rho), int(nthreads), C.byref(h)),
               "kc_analyze_supernodal")
    return Plan(h, n, d)


def analyze_batched(xs, rho: float, rule: str = "max", nthreads: int = 0) -> Plan:
    """Independent problems (a list of (n_i, d) arrays) analysed as one block-diagonal plan."""
    xs = [np.ascontiguousarray(x, dtype=np.float64) for x in xs]
    d = xs[0].shape[1]
    if any(x.ndim != 2 or x.shape[1] != d for x in xs):
        raise ValueError("every instance must be (n_i, d) with the same d")
    counts = np.array([x.shape[0] for x in xs], dtype=np.int64)
    allx = np.ascontiguousarray(np.concatenate(xs))
    h = C.c_void_p()
    _lib.check(_lib.load().kc_analyze_batched(_ptr(allx), _ptr(counts), len(xs), d, float(rho), _RULES[rule],
                                              int(nthreads), C.byref(h)), "kc_analyze_batched")
    return Plan(h, int(counts.sum()), d, counts)


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def dense_matvec(x_dev, X_dev, nu: float, lengthscale: float, stream=None):
    """Y = Theta X with the dense Matern matrix of the points x_dev (N x d), generated on the fly."""
    import torch
    for t in (x_dev, X_dev):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("points and X must be contiguous float64 CUDA tensors")
    n, d = x_dev.shape
    nrhs = 1 if X_dev.dim() == 1 else int(X_dev.shape[1])
    Y = torch.empty_like(X_dev)
    _lib.check(_lib.load().kc_dense_matvec(C.c_void_p(x_dev.data_ptr()), n, d, _lib.kc_kernel(nu, lengthscale),
                                           C.c_void_p(X_dev.data_ptr()), C.c_void_p(Y.data_ptr()), nrhs,
                                           _stream_ptr(stream)), "kc_dense_matvec")
    return Y


@dataclass
class PcgInfo:
    iterations: int
    converged: bool
    max_rel_residual: float
    t_matvec_ms: float
    t_precond_ms: float
    true_rel_residual: float
    restarts: int


@dataclass
class Stats:
    nonpositive: int
    shifted: int
    rank: int
    updates: int
    exp_hard: int
    nonfinite: int
    match_errors: int


class Factor:
    """A factor bound to a torch-allocated device workspace."""

    def __init__(self, plan: Plan, prec: str = "fp64", stream=None):
        import torch
        L = _lib.load()
        self.n, self.d, self.nnz, self.prec = plan.n, plan.d, plan.nnz, prec
        nbytes = C.c_size_t()
        _lib.check(L.kc_factor_bytes(plan.handle, _PRECS[prec], C.byref(nbytes)), "kc_factor_bytes")
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        _lib.check(L.kc_factor_create(plan.handle, _PRECS[prec], C.c_void_p(self.workspace.data_ptr()),
                                      nbytes.value, _stream_ptr(stream), C.byref(h)), "kc_factor_create")
        self._h = h
        self._scratch = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None and _lib._LIB is not None:
            _lib._LIB.kc_factor_destroy(h)
            self._h = None

    @property
    def workspace_bytes(self) -> int:
        return int(self.workspace.numel())

    def factorize(self, x_dev, nu: float, lengthscale: float, pivot: str = "zero", tau: float = 0.0,
                  count_updates: bool = False, stream=None) -> None:
        """Theta on S + ICHOL(0), asynchronous on the stream."""
        self._check_points(x_dev)
        _lib.check(_lib.load().kc_factorize(self._h, C.c_void_p(x_dev.data_ptr()), _lib.kc_kernel(nu, lengthscale),
                                            _PIVOTS[pivot], float(tau), int(bool(count_updates)),
                                            _stream_ptr(stream)), "kc_factorize")

    def factorize_batched(self, x_dev, nu: float, ell_dev, pivot: str = "zero", tau: float = 0.0,
                          count_updates: bool = False, stream=None) -> None:
        """Factor every instance of a batch plan; ell_dev holds one lengthscale per instance (device)."""
        self._check_points(x_dev)
        _lib.check(_lib.load().kc_factorize_batched(self._h, C.c_void_p(x_dev.data_ptr()), float(nu),
                                                    C.c_void_p(ell_dev.data_ptr()), _PIVOTS[pivot], float(tau),
                                                    int(bool(count_updates)), _stream_ptr(stream)),
                   "kc_factorize_batched")

    def tune(self, x_dev, nu: float, lengthscale: float = 0.0, ell_dev=None, pivot: str = "zero", tau: float = 0.0,
             reps: int = 3, stream=None) -> int:
        """Pick the fastest schedule (wavefronts per workgroup x level grouping x unit order) for this factor by
        timing it; returns the wavefronts per workgroup (schedule() gives all three)."""
        self._check_points(x_dev)
        w = C.c_int32()
        _lib.check(_lib.load().kc_factor_tune(self._h, C.c_void_p(x_dev.data_ptr()), float(nu), float(lengthscale),
                                              C.c_void_p(ell_dev.data_ptr()) if ell_dev is not None else None,
                                              _PIVOTS[pivot], float(tau), int(reps), _stream_ptr(stream),
                                              C.byref(w)), "kc_factor_tune")
        return int(w.value)

    def set_schedule(self, wpb: int, persist_max: int, order: Optional[str] = None) -> None:
        """Wavefronts per workgroup (1, 2, 4), the level grouping (runs of consecutive levels with at most
        persist_max work units share one persistent launch; 0: every level its own launch; 2**63 - 1: the
        whole factorization in one launch) and the order of the units within a level ("spatial" or
        "longest"; None keeps the current one)."""
        if order is None:
            order = self.schedule()[2]
        _lib.check(_lib.load().kc_factor_set_schedule(self._h, int(wpb), int(persist_max), _ORDERS[order]),
                   "kc_factor_set_schedule")

    def use_groups(self, enable: bool = True) -> None:
        """Factor a mixed-precision supernodal plan by supernodal groups on the matrix cores (the default for
        such factors) or entry by entry (enable=False)."""
        _lib.check(_lib.load().kc_factor_use_groups(self._h, int(bool(enable))), "kc_factor_use_groups")

    def set_stage_limit(self, max_parents: int = -1) -> None:
        """Rows with more than max_parents parents are read from device memory instead of staged in LDS
        (the same L); -1 restores the largest limit the LDS allows."""
        _lib.check(_lib.load().kc_factor_set_stage_limit(self._h, int(max_parents)), "kc_factor_set_stage_limit")

    def schedule(self) -> tuple:
        """(wavefronts per workgroup, persist_max, unit order) in use -- the tuner's choice after tune()."""
        w, pm, o = C.c_int32(), C.c_int64(), C.c_int()
        _lib.check(_lib.load().kc_factor_schedule(self._h, C.byref(w), C.byref(pm), C.byref(o)), "kc_factor_schedule")
        return int(w.value), int(pm.value), _ORDER_NAMES[int(o.value)]

    def capture(self, x_dev, b_dev, nu: float, lengthscale: float = 0.0, ell_dev=None, pivot: str = "zero",
                tau: float = 0.0) -> "Graph":
        """Capture factorize + solve into a HIP graph; returns the graph and its output tensor."""
        return Graph(self, x_dev, b_dev, nu, lengthscale, ell_dev, pivot, tau)

    def theta(self, x_dev, nu: float, lengthscale: float, stream=None):
        """Theta on S in CSC order (the factorization's starting entries)."""
        import torch
        self._check_points(x_dev)
        out = torch.empty(self.nnz, dtype=torch.float64, device=x_dev.device)
        _lib.check(_lib.load().kc_theta(self._h, C.c_void_p(x_dev.data_ptr()), _lib.kc_kernel(nu, lengthscale),
                                        C.c_void_p(out.data_ptr()), _stream_ptr(stream)), "kc_theta")
        return out

    def factorize_solve(self, x_dev, b_dev, nu: float, lengthscale: float = 0.0, pivot: str = "zero",
                        tau: float = 0.0, out=None, stream=None, ell_dev=None):
        """factorize() (or factorize_batched() with ell_dev) then solve() in one call, the forward sweep
        overlapped with the factorization on a second stream; bitwise the same result.  Returns x."""
        import torch
        self._check_points(x_dev)
        if b_dev.dtype != torch.float64 or not b_dev.is_cuda or not b_dev.is_contiguous():
            raise ValueError("b must be a contiguous float64 CUDA tensor")
        if b_dev.shape[0] != self.n:
            raise ValueError("b must have n rows")
        nrhs = 1 if b_dev.dim() == 1 else int(b_dev.shape[1])
        x = out if out is not None else torch.empty_like(b_dev)
        nb = C.c_size_t()
        _lib.check(_lib.load().kc_solve_bytes(self._h, nrhs, C.byref(nb)), "kc_solve_bytes")
        need = int(nb.value)
        if self._scratch is None or self._scratch.numel() < need:
            self._scratch = torch.empty(need, dtype=torch.uint8, device=b_dev.device)
        _lib.check(_lib.load().kc_factorize_solve(self._h, C.c_void_p(x_dev.data_ptr()), _lib.kc_kernel(nu, lengthscale),
                                                  C.c_void_p(ell_dev.data_ptr()) if ell_dev is not None else None,
                                                  _PIVOTS[pivot], float(tau), C.c_void_p(b_dev.data_ptr()),
                                                  C.c_void_p(x.data_ptr()), nrhs, C.c_void_p(self._scratch.data_ptr()),
                                                  self._scratch.numel(), _stream_ptr(stream)), "kc_factorize_solve")
        return x

    def solve(self, b_dev, out=None, stream=None):
        """x = P^T L^-T L^-1 P b for b of shape (n,) or (n, nrhs), original order."""
        import torch
        if b_dev.dtype != torch.float64 or not b_dev.is_cuda or not b_dev.is_contiguous():
            raise ValueError("b must be a contiguous float64 CUDA tensor")
        if b_dev.shape[0] != self.n:
            raise ValueError("b must have n rows")
        nrhs = 1 if b_dev.dim() == 1 else int(b_dev.shape[1])
        x = out if out is not None else torch.empty_like(b_dev)
        nb = C.c_size_t()
        _lib.check(_lib.load().kc_solve_bytes(self._h, nrhs, C.byref(nb)), "kc_solve_bytes")
        need = int(nb.value)
        if self._scratch is None or self._scratch.numel() < need:
            self._scratch = torch.empty(need, dtype=torch.uint8, device=b_dev.device)
        _lib.check(_lib.load().kc_solve(self._h, C.c_void_p(b_dev.data_ptr()), C.c_void_p(x.data_ptr()), nrhs,
                                        C.c_void_p(self._scratch.data_ptr()), self._scratch.numel(),
                                        _stream_ptr(stream)), "kc_solve")
        return x

    def solve_noalloc(self, b_dev, out, stream=None):
        """solve() through kc_solve_noalloc: the library's fixed per-device scratch array instead of a
        workspace, so the call allocates nothing (``out`` must be given).  Calls that overlap on one
        device race on that array."""
        import torch
        for t in (b_dev, out):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("b and out must be contiguous float64 CUDA tensors")
        if b_dev.shape[0] != self.n or out.shape != b_dev.shape:
            raise ValueError("b must have n rows and out the shape of b")
        nrhs = 1 if b_dev.dim() == 1 else int(b_dev.shape[1])
        _lib.check(_lib.load().kc_solve_noalloc(self._h, C.c_void_p(b_dev.data_ptr()), C.c_void_p(out.data_ptr()),
                                                nrhs, _stream_ptr(stream)), "kc_solve_noalloc")
        return out

    def pcg(self, x_dev, b_dev, nu: float, lengthscale: float, tol: float = 1e-10, maxit: int = 200, stream=None):
        """Solve Theta x = b by CG on the dense Theta preconditioned with this factor."""
        import torch
        if b_dev.dtype != torch.float64 or not b_dev.is_cuda or not b_dev.is_contiguous():
            raise ValueError("b must be a contiguous float64 CUDA tensor")
        self._check_points(x_dev)
        nrhs = 1 if b_dev.dim() == 1 else int(b_dev.shape[1])
        nb = C.c_size_t()
        _lib.check(_lib.load().kc_pcg_bytes(self._h, nrhs, C.byref(nb)), "kc_pcg_bytes")
        scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=b_dev.device)
        sol = torch.empty_like(b_dev)
        info = _lib.kc_pcg_info_t()
        _lib.check(_lib.load().kc_pcg(self._h, C.c_void_p(x_dev.data_ptr()), _lib.kc_kernel(nu, lengthscale),
                                      C.c_void_p(b_dev.data_ptr()), C.c_void_p(sol.data_ptr()), nrhs, float(tol),
                                      int(maxit), C.c_void_p(scratch.data_ptr()), scratch.numel(),
                                      _stream_ptr(stream), C.byref(info)), "kc_pcg")
        return sol, PcgInfo(info.iterations, bool(info.converged), info.max_rel_residual, info.t_matvec_ms,
                            info.t_precond_ms, info.true_rel_residual, info.restarts)

    def match_bytes(self, stream=None) -> int:
        """Device bytes the match masks of this factor's pattern need (counted on the device once)."""
        nb = C.c_size_t()
        _lib.check(_lib.load().kc_factor_match_bytes(self._h, _stream_ptr(stream), C.byref(nb)),
                   "kc_factor_match_bytes")
        return int(nb.value)

    def build_matches(self, stream=None) -> int:
        """Build the match masks (symbolic, once per pattern) in a torch-allocated buffer kept by this
        object; later factorizations use them and give bitwise the same L.  Returns their bytes."""
        import torch
        need = self.match_bytes(stream)
        self._matches = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        _lib.check(_lib.load().kc_factor_match_build(self._h, C.c_void_p(self._matches.data_ptr()),
                                                     self._matches.numel(), _stream_ptr(stream)),
                   "kc_factor_match_build")
        return need

    def drop_matches(self) -> None:
        """Detach and free the match masks (back to the index merge)."""
        _lib.check(_lib.load().kc_factor_match_build(self._h, None, 0, None), "kc_factor_match_build")
        self._matches = None

    def stats(self) -> Stats:
        st = _lib.kc_factor_stats_t()
        _lib.check(_lib.load().kc_factor_stats(self._h, C.byref(st)), "kc_factor_stats")
        return Stats(st.nonpositive, st.shifted, st.rank, st.updates, st.exp_hard, st.nonfinite, st.match_errors)

    def export_L(self) -> np.ndarray:
        """L in the plan's CSC order (float64; MIXED values widened)."""
        v = np.empty(self.nnz, np.float64)
        _lib.check(_lib.load().kc_factor_export_L(self._h, _ptr(v)), "kc_factor_export_L")
        return v

    def _check_points(self, x_dev):
        import torch
        if x_dev.dtype != torch.float64 or not x_dev.is_cuda or not x_dev.is_contiguous():
            raise ValueError("points must be a contiguous float64 CUDA tensor")
        if tuple(x_dev.shape) != (self.n, self.d):
            raise ValueError(f"points must have shape ({self.n}, {self.d})")


class Graph:
    """factorize + solve of one factor captured as a HIP graph (see Factor.capture)."""

    def __init__(self, factor: "Factor", x_dev, b_dev, nu, lengthscale, ell_dev, pivot, tau):
        import torch
        factor._check_points(x_dev)
        nrhs = 1 if b_dev.dim() == 1 else int(b_dev.shape[1])
        nb = C.c_size_t()
        _lib.check(_lib.load().kc_solve_bytes(factor._h, nrhs, C.byref(nb)), "kc_solve_bytes")
        self.scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=b_dev.device)
        self.out = torch.empty_like(b_dev)
        self._keep = (factor, x_dev, b_dev, ell_dev)
        h = C.c_void_p()
        _lib.check(_lib.load().kc_graph_create(factor._h, C.c_void_p(x_dev.data_ptr()), float(nu), float(lengthscale),
                                               C.c_void_p(ell_dev.data_ptr()) if ell_dev is not None else None,
                                               _PIVOTS[pivot], float(tau), C.c_void_p(b_dev.data_ptr()),
                                               C.c_void_p(self.out.data_ptr()), nrhs,
                                               C.c_void_p(self.scratch.data_ptr()), self.scratch.numel(),
                                               C.byref(h)), "kc_graph_create")
        self._h = h

    def launch(self, stream=None):
        _lib.check(_lib.load().kc_graph_launch(self._h, _stream_ptr(stream)), "kc_graph_launch")
        return self.out

    def info(self) -> dict:
        """Nodes of the recorded graph and whether the factorization was recorded with persistent launches."""
        nodes, pers = C.c_int64(), C.c_int32()
        _lib.check(_lib.load().kc_graph_info(self._h, C.byref(nodes), C.byref(pers)), "kc_graph_info")
        return {"nodes": int(nodes.value), "persistent": bool(pers.value)}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None and _lib._LIB is not None:
            _lib._LIB.kc_graph_destroy(h)
            self._h = None
