"""GPU parity: the HIP path through the C ABI against the CPU oracle.

FP64 bar: the pattern is bit-identical (host analysis), Theta on S is
bit-identical (both sides use the correctly rounded exponential), and L is
bit-identical (same per-entry update order, one fma per update, correctly
rounded sqrt and division).  Solves are bit-identical whenever every column has
at most 2048 off-diagonal entries and every forward level fewer than 1024 rows
(sequential substitution on both sides; the workloads here have at most a few
hundred rows per level).  Otherwise the backward sweep sums the columns up to
the last long one in fixed pieces (and large forward levels sum a row across a
wavefront), which changes the summation order; those solves are held to
max|x - x_oracle| <= 1e-12 max|x_oracle| for each right-hand side
(test_long_column_solve_matches_oracle).  Rows read from device memory instead
of LDS (kc_factor_set_stage_limit) give the same L bit for bit
(test_unstaged_rows_give_the_same_factor).
"""
import numpy as np
import pytest

import oracle as O
from paper_1706_02205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1706_02205_amd as K
    return K


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def oracle_factor(x, rho, rule, nu, ell, pivot=O.PIVOT_ZERO, tau=0.0):
    P = O.pattern(x, rho, O.RULE_MAX if rule == "max" else O.RULE_MIN)
    th = O.theta_on_pattern(P, nu, ell)
    return P, th, O.ichol(P, th, pivot, tau)


CASES = [
    # name, points, rho, rule, nu, ell, pivot, tau
    ("uniform2d-n2000-matern32-rho3", lambda: W.small_uniform_2d().points, 3.0, "max", 1.5, 0.2, "zero", 0.0),
    ("uniform2d-n2000-matern12-rho3", lambda: W.uniform_points(2000, 2, 21), 3.0, "max", 0.5, 0.2, "zero", 0.0),
    ("uniform3d-n1500-matern52-rho2.5", lambda: W.uniform_points(1500, 3, 22), 2.5, "max", 2.5, 0.3, "zero", 0.0),
    ("uniform2d-n1800-matern32-min-rho4", lambda: W.uniform_points(1800, 2, 23), 4.0, "min", 1.5, 0.2, "zero", 0.0),
    ("uniform2d-n2000-matern32-shift", lambda: W.small_uniform_2d().points, 3.0, "max", 1.5, 0.2, "shift", 1e-6),
    ("jittergrid-n1600-matern12-rho4", lambda: W.jittered_grid(40, 24), 4.0, "max", 0.5, 0.1, "zero", 0.0),
    ("sphere20d-n1000-matern32-rho3", lambda: W.embedded_sincos(1000, 25), 3.0, "max", 1.5, 0.2, "zero", 0.0),
    ("duplicates-n330", lambda: np.concatenate([W.uniform_points(300, 2, 26), W.uniform_points(300, 2, 26)[:30]]),
     2.0, "max", 0.5, 0.2, "zero", 0.0),
    # rows longer than 512 entries: the staged row gets a bucket directory instead of the cursor merge
    ("uniform3d-n6000-matern32-rho4.5-longrows", lambda: W.uniform_points(6000, 3, 31), 4.5, "max", 1.5, 0.2, "zero", 0.0),
    ("uniform2d-n4000-matern12-rho14-longrows", lambda: W.uniform_points(4000, 2, 31), 14.0, "max", 0.5, 0.2, "zero", 0.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_factor_bitwise_equal_to_oracle(K, case):
    name, gen, rho, rule, nu, ell, pivot, tau = case
    print(f"[gpu] factor parity {name}", flush=True)
    x = gen()
    P, th, R = oracle_factor(x, rho, rule, nu, ell, O.PIVOT_ZERO if pivot == "zero" else O.PIVOT_SHIFT, tau)
    plan = K.analyze(x, rho, rule)
    f = K.Factor(plan, "fp64")
    xd = dev(x)
    theta = f.theta(xd, nu, ell).cpu().numpy()
    assert np.array_equal(theta, th), f"Theta differs in {np.sum(theta != th)} entries"
    f.factorize(xd, nu, ell, pivot, tau, count_updates=True)
    st = f.stats()
    L = f.export_L()
    assert st.exp_hard == 0
    assert st.nonpositive == R.nonpositive and st.shifted == R.shifted
    assert st.rank == P.n - R.nonpositive
    assert st.updates == R.updates
    bad = np.nonzero(L != R.L)[0]
    assert bad.size == 0, f"{bad.size} of {L.size} entries of L differ; first at CSC position {bad[:5]}"


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_match_masks_factor_bitwise(K, case):
    """With match masks (kc_factor_match_build) the factorization finds the shared parents from bits
    instead of merging indices: L, pivot counts and the update count stay bitwise the oracle's (FP64),
    and the mixed factor stays bitwise the index merge's."""
    name, gen, rho, rule, nu, ell, pivot, tau = case
    print(f"[gpu] match masks {name}", flush=True)
    x = gen()
    P, th, R = oracle_factor(x, rho, rule, nu, ell, O.PIVOT_ZERO if pivot == "zero" else O.PIVOT_SHIFT, tau)
    plan = K.analyze(x, rho, rule)
    xd = dev(x)
    f = K.Factor(plan, "fp64")
    nbytes = f.build_matches()
    assert nbytes >= 8 * P.nnz
    f.factorize(xd, nu, ell, pivot, tau, count_updates=True)
    st = f.stats()
    assert st.match_errors == 0 and st.exp_hard == 0
    assert st.nonpositive == R.nonpositive and st.shifted == R.shifted and st.updates == R.updates
    assert np.array_equal(f.export_L(), R.L)
    mpiv, mtau = ("shift", 1e-6) if pivot == "zero" else (pivot, tau)
    fm, fi = K.Factor(plan, "mixed"), K.Factor(plan, "mixed")
    fm.build_matches()
    fm.factorize(xd, nu, ell, mpiv, mtau)
    fi.factorize(xd, nu, ell, mpiv, mtau)
    Lm, Li = fm.export_L(), fi.export_L()
    assert np.array_equal(np.isnan(Lm), np.isnan(Li)) and np.array_equal(Lm[~np.isnan(Li)], Li[~np.isnan(Li)])
    assert fm.stats().match_errors == 0
    # detaching returns to the index merge, same factor
    f.drop_matches()
    f.factorize(xd, nu, ell, pivot, tau)
    assert np.array_equal(f.export_L(), R.L)


@pytest.mark.parametrize("persist_max,order,wpb", [(2**63 - 1, "spatial", 1), (16, "longest", 2), (0, "longest", 4),
                                                   (0, "spatial", 1)])
def test_match_masks_under_every_schedule(K, persist_max, order, wpb):
    print(f"[gpu] match masks schedule persist_max={persist_max} order={order} wpb={wpb}", flush=True)
    w = W.small_uniform_2d()
    P, th, R = oracle_factor(w.points, w.rho, "max", w.nu, w.lengthscale)
    plan = K.analyze(w.points, w.rho)
    f = K.Factor(plan, "fp64")
    f.build_matches()
    f.set_schedule(wpb, persist_max, order)
    f.factorize(dev(w.points), w.nu, w.lengthscale, count_updates=True)
    st = f.stats()
    assert st.updates == R.updates and st.match_errors == 0
    assert np.array_equal(f.export_L(), R.L)


@pytest.mark.parametrize("limit", [1, 3, 40, 65536])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_index_gap_escapes_do_not_change_the_factor(K, limit, prec):
    """The factorization reads row indices as 16-bit gaps with an escape list for wide gaps.
    Lowering the gap limit forces escapes -- every entry at limit 1, more than the two a row
    keeps in registers at limits 1 and 3 -- and the factor must stay bitwise the same."""
    print(f"[gpu] index gap escapes limit={limit} prec={prec}", flush=True)
    w = W.small_uniform_2d()
    plan = K.analyze(w.points, w.rho)
    xd = dev(w.points)
    pivot, tau = ("zero", 0.0) if prec == "fp64" else ("shift", 1e-6)
    f0 = K.Factor(plan, prec)
    f0.factorize(xd, w.nu, w.lengthscale, pivot, tau)
    ref = f0.export_L()
    nesc = plan.set_delta_limit(limit)
    if limit == 1:
        assert nesc == plan.nnz
    if limit <= 3:
        assert nesc > 8 * plan.n  # most rows go beyond the register queue
    f = K.Factor(plan, prec)
    f.factorize(xd, w.nu, w.lengthscale, pivot, tau)
    assert np.array_equal(f.export_L(), ref)
    if prec == "fp64":
        P = O.pattern(w.points, w.rho)
        R = O.ichol(P, O.theta_on_pattern(P, w.nu, w.lengthscale), O.PIVOT_ZERO)
        assert np.array_equal(f.export_L(), R.L)


@pytest.mark.parametrize("persist_max,order", [(2**63 - 1, "spatial"), (16, "longest"), (0, "longest"),
                                               (0, "spatial")])
def test_schedules_factorization_bitwise(K, persist_max, order):
    """The whole factorization in one persistent launch (or its small levels grouped), with the units
    of a level in either order, equals the oracle bit for bit, update counts included."""
    print(f"[gpu] factorization schedule persist_max={persist_max} order={order}", flush=True)
    w = W.small_uniform_2d()
    P, th, R = oracle_factor(w.points, w.rho, "max", w.nu, w.lengthscale)
    plan = K.analyze(w.points, w.rho)
    f = K.Factor(plan, "fp64")
    f.set_schedule(4, persist_max, order)
    assert f.schedule() == (4, persist_max, order)
    f.factorize(dev(w.points), w.nu, w.lengthscale, count_updates=True)
    st = f.stats()
    assert st.updates == R.updates and st.nonpositive == R.nonpositive
    assert np.array_equal(f.export_L(), R.L)


def test_factor_is_deterministic(K):
    print("[gpu] determinism", flush=True)
    w = W.small_uniform_2d()
    plan = K.analyze(w.points, w.rho)
    f = K.Factor(plan, "fp64")
    xd = dev(w.points)
    f.factorize(xd, w.nu, w.lengthscale)
    a = f.export_L()
    f.factorize(xd, w.nu, w.lengthscale)
    assert np.array_equal(a, f.export_L())


def test_exponential_over_the_whole_range(K):
    """exp(-r/l) for r/l from 0 to 750 (normal and subnormal results) equals the oracle's bit for bit."""
    print("[gpu] correctly rounded exp over [-750, 0]", flush=True)
    x = W.uniform_points(1500, 1, 27)
    ell = 1.0 / 750.0
    P = O.pattern(x, 1e9)
    th = O.theta_on_pattern(P, 0.5, ell)
    assert np.sum((th > 0) & (th < 2.2250738585072014e-308)) > 1000  # subnormal results are exercised
    plan = K.analyze(x, 1e9)
    f = K.Factor(plan, "fp64")
    theta = f.theta(dev(x), 0.5, ell).cpu().numpy()
    assert np.array_equal(theta, th)
    assert f.stats().exp_hard == 0


@pytest.mark.parametrize("nrhs", [1, 3, 8, 11])
def test_solve_matches_oracle(K, nrhs):
    print(f"[gpu] solve parity nrhs={nrhs}", flush=True)
    w = W.small_uniform_2d()
    P, th, R = oracle_factor(w.points, w.rho, "max", w.nu, w.lengthscale)
    plan = K.analyze(w.points, w.rho)
    f = K.Factor(plan, "fp64")
    f.factorize(dev(w.points), w.nu, w.lengthscale)
    b = W.gaussian_rhs(P.n, nrhs, 31)
    x = f.solve(dev(b if nrhs > 1 else b[:, 0])).cpu().numpy()
    ref = O.solve(P, R.L, b if nrhs > 1 else b[:, 0])
    assert plan.info()["max_col"] - 1 <= 2048  # every column takes the sequential path
    assert np.array_equal(x, ref)


LONG_TOL = 1e-12


def assert_close_per_rhs(x, ref, what):
    """max_k |x_k - ref_k| <= LONG_TOL * max_k |ref_k| for each right-hand side (column)."""
    x2, r2 = (x, ref) if x.ndim == 2 else (x[:, None], ref[:, None])
    err = np.abs(x2 - r2).max(axis=0) / np.abs(r2).max(axis=0)
    same = np.mean(x2 == r2)
    print(f"[gpu] {what}: max error per rhs {err.max():.2e} (relative to max|x|), "
          f"{100 * same:.1f}% of components bitwise equal", flush=True)
    assert np.all(err <= LONG_TOL), f"{what}: {err}"


@pytest.mark.parametrize("nrhs", [1, 8, 11])
def test_long_column_solve_matches_oracle(K, nrhs):
    """Columns with more than 2048 off-diagonal entries: the backward sweep runs its three stages
    (columns past the last long one by reverse level, the top columns' rows below the top block in
    banded pieces, the top block by its own levels, sums in a fixed order): compared with the
    oracle's sequential substitution element by element, for kc_solve and kc_factorize_solve."""
    print(f"[gpu] long-column solve parity nrhs={nrhs}", flush=True)
    x = W.uniform_points(5000, 2, 33)
    P, th, R = oracle_factor(x, 3.0, "max", 1.5, 0.2)
    plan = K.analyze(x, 3.0)
    info = plan.info()
    assert info["max_col"] - 1 > 2048
    assert int(np.sum(np.diff(P.colptr) - 1 > 2048)) >= 2  # several columns on the piecewise path
    f = K.Factor(plan, "fp64")
    xd = dev(x)
    f.factorize(xd, 1.5, 0.2)
    assert np.array_equal(f.export_L(), R.L)
    b = W.gaussian_rhs(P.n, nrhs, 34)
    bb = b if nrhs > 1 else b[:, 0]
    ref = O.solve(P, R.L, bb)
    got = f.solve(dev(bb)).cpu().numpy()
    assert_close_per_rhs(got, ref, f"kc_solve n=5000 nrhs={nrhs}")
    fused = f.factorize_solve(xd, dev(bb), 1.5, 0.2).cpu().numpy()
    assert np.array_equal(fused, got)
    assert f.stats().nonfinite == 0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nrhs,persist_max", [(1, 0), (8, 0), (11, 0), (8, 16), (3, 2**63 - 1)])
def test_factorize_solve_overlapped_bitwise(K, prec, nrhs, persist_max):
    """The fused call (forward sweep on a second stream, overlapped with the factorization, per level
    or per persistent run of levels) gives bitwise the factor and solution of factorize then solve,
    on two calls in a row; in FP64 both equal the oracle."""
    print(f"[gpu] factorize_solve prec={prec} nrhs={nrhs} persist_max={persist_max}", flush=True)
    w = W.small_uniform_2d()
    pivot, tau = ("zero", 0.0) if prec == "fp64" else ("shift", 1e-6)
    plan = K.analyze(w.points, w.rho)
    xd = dev(w.points)
    ref_f = K.Factor(plan, prec)
    f = K.Factor(plan, prec)
    f.set_schedule(f.schedule()[0], persist_max)
    for seed in (41, 42):
        b = W.gaussian_rhs(plan.n, nrhs, seed)
        bd = dev(b if nrhs > 1 else b[:, 0])
        ref_f.factorize(xd, w.nu, w.lengthscale, pivot, tau)
        ref_x = ref_f.solve(bd).cpu().numpy()
        x = f.factorize_solve(xd, bd, w.nu, w.lengthscale, pivot, tau).cpu().numpy()
        assert np.array_equal(x, ref_x), f"seed {seed}"
        assert np.array_equal(f.export_L(), ref_f.export_L())
    if prec == "fp64":
        P, th, R = oracle_factor(w.points, w.rho, "max", w.nu, w.lengthscale)
        assert np.array_equal(f.export_L(), R.L)
        assert np.array_equal(x, O.solve(P, R.L, b if nrhs > 1 else b[:, 0]))


def test_tiny_and_degenerate_inputs(K):
    print("[gpu] tiny inputs", flush=True)
    for x in (np.array([[0.3, 0.7]]), W.uniform_points(2, 2, 40), np.ones((5, 3)),
              np.array([[0.0], [1.0], [0.4]])):
        P, th, R = oracle_factor(x, 1.0, "max", 0.5, 0.5)
        plan = K.analyze(x, 1.0)
        f = K.Factor(plan, "fp64")
        f.factorize(dev(x), 0.5, 0.5)
        assert np.array_equal(f.export_L(), R.L)
        assert f.stats().nonpositive == R.nonpositive
        b = W.gaussian_rhs(len(x), 2, 41)
        assert np.array_equal(f.solve(dev(b)).cpu().numpy(), O.solve(P, R.L, b))


def test_mixed_precision_error_against_fp64_oracle(K):
    """FP32 updates / FP64 pivots: no bitwise bar; the error against the FP64 oracle is stated and bounded."""
    print("[gpu] mixed precision", flush=True)
    x = W.uniform_points(2000, 2, 42)
    P, th, R = oracle_factor(x, 3.0, "max", 0.5, 0.2)
    plan = K.analyze(x, 3.0)
    f = K.Factor(plan, "mixed")
    f.factorize(dev(x), 0.5, 0.2, "shift", 1e-6, count_updates=True)
    st = f.stats()
    Lm = f.export_L()
    assert R.nonpositive == 0 and st.shifted == 0
    assert st.updates == R.updates
    rel = np.linalg.norm(Lm - R.L) / np.linalg.norm(R.L)
    print(f"[gpu] mixed vs fp64 oracle: ||dL||_F/||L||_F = {rel:.2e}", flush=True)
    assert rel < 1e-4
    e_fp64 = O.frob_error(P, R.L, 0.5, 0.2)
    e_mixed = O.frob_error(P, Lm, 0.5, 0.2)
    print(f"[gpu] ||LL^T-Theta||_F/||Theta||_F: fp64 {e_fp64:.3e} mixed {e_mixed:.3e}", flush=True)
    assert e_mixed < 1.5 * e_fp64


def test_errors_surface_as_exceptions(K):
    import torch
    w = W.small_uniform_2d()
    plan = K.analyze(w.points, w.rho)
    f = K.Factor(plan, "fp64")
    with pytest.raises(K.KCholError, match="call out of order"):
        f.solve(dev(np.zeros((w.n, 1))))
    with pytest.raises(K.KCholError, match="invalid argument"):
        f.factorize(dev(w.points), 1.0, 0.2)
    with pytest.raises(ValueError):
        f.factorize(dev(w.points[:10]), 1.5, 0.2)
    with pytest.raises(ValueError):
        f.solve(torch.zeros(w.n, dtype=torch.float32, device="cuda"))


def test_unstaged_rows_give_the_same_factor(K):
    """Rows with more parents than the stage limit are read from device memory instead of LDS (the path
    rows too long for LDS always take): L, pivot counts and U stay bitwise the oracle's in FP64, per level
    and in persistent launches, and the mixed factor stays bitwise its staged self.  Match masks need
    every row staged and are refused meanwhile."""
    print("[gpu] unstaged rows", flush=True)
    x = W.uniform_points(4000, 2, 31)
    rho, nu, ell = 14.0, 0.5, 0.2
    P, th, R = oracle_factor(x, rho, "max", nu, ell)
    plan = K.analyze(x, rho)
    assert plan.info()["max_row"] > 200
    xd = dev(x)
    f = K.Factor(plan, "fp64")
    wpb, pm, order = f.schedule()
    for limit in (0, 40, 200):
        f.set_stage_limit(limit)
        for persist in (0, 1 << 40):
            f.set_schedule(wpb, persist, order)
            f.factorize(xd, nu, ell, count_updates=True)
            st = f.stats()
            assert st.updates == R.updates and st.nonpositive == R.nonpositive, (limit, persist)
            assert np.array_equal(f.export_L(), R.L), (limit, persist)
    f.set_schedule(wpb, pm, order)
    with pytest.raises(RuntimeError):
        f.build_matches()
    f.set_stage_limit(-1)
    f.build_matches()
    with pytest.raises(RuntimeError):
        f.set_stage_limit(40)  # masks attached: every row must stay staged
    f.factorize(xd, nu, ell)
    assert np.array_equal(f.export_L(), R.L)
    f.drop_matches()
    fm = K.Factor(plan, "mixed")
    fm.factorize(xd, nu, ell, "shift", 1e-6)
    Lm = fm.export_L()
    fm.set_stage_limit(40)
    fm.factorize(xd, nu, ell, "shift", 1e-6)
    assert np.array_equal(fm.export_L(), Lm)
