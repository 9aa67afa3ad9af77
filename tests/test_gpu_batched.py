"""Many independent problems in one level-launch sequence: parity per instance,
HIP-graph replays, and the autotuner's choice (which must not change results)."""
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


@pytest.fixture(scope="module")
def batch():
    # the batched recipe shrunk so the oracle finishes quickly: N log-uniform in [40, 2000]
    inst = W.batched_instances(24, 40, 2000, seed=4100)
    xs = [b.points for b in inst]
    ells = np.array([b.lengthscale for b in inst])
    ref = []
    for x, ell in zip(xs, ells):
        P = O.pattern(x, 3.0)
        ref.append((P, O.ichol(P, O.theta_on_pattern(P, 1.5, ell))))
    b = np.concatenate([W.gaussian_rhs(len(x), 1, 4200 + i) for i, x in enumerate(xs)])
    return xs, ells, ref, b


def run_batch(K, xs, ells, prec="fp64", pivot="zero", tau=0.0):
    plan = K.analyze_batched(xs, 3.0)
    f = K.Factor(plan, prec)
    xd = dev(np.concatenate(xs))
    ed = dev(ells)
    f.factorize_batched(xd, 1.5, ed, pivot, tau, count_updates=True)
    return plan, f, xd, ed


def test_batched_factor_and_solve_bitwise_per_instance(K, batch):
    print("[gpu] batched parity", flush=True)
    xs, ells, ref, b = batch
    plan, f, xd, ed = run_batch(K, xs, ells)
    L = f.export_L()
    st = f.stats()
    sol = f.solve(dev(b)).cpu().numpy()
    assert st.nonpositive == sum(R.nonpositive for _, R in ref)
    assert st.updates == sum(R.updates for _, R in ref)
    e0 = o0 = 0
    for x, (P, R) in zip(xs, ref):
        assert np.array_equal(L[e0:e0 + P.nnz], R.L)
        assert np.array_equal(sol[o0:o0 + P.n], O.solve(P, R.L, b[o0:o0 + P.n]))
        e0 += P.nnz
        o0 += P.n


def test_graph_replays_match_eager(K, batch):
    print("[gpu] batched graph replays", flush=True)
    import torch
    xs, ells, ref, b = batch
    plan, f, xd, ed = run_batch(K, xs, ells)
    bd = dev(b)
    eager = f.solve(bd).cpu().numpy()
    eager_L = f.export_L()
    g = f.capture(xd, bd, 1.5, ell_dev=ed)
    for rep in range(3):
        out = g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), f"replay {rep}"
        assert np.array_equal(f.export_L(), eager_L)
        # eager work between replays
        f.factorize_batched(xd, 1.5, ed)
        assert np.array_equal(f.solve(bd).cpu().numpy(), eager)


def test_fused_factorize_solve_on_a_batch(K, batch):
    """The fused call with one lengthscale per instance gives bitwise the factor and solution of
    factorize_batched then solve; a plan/argument mismatch is rejected."""
    print("[gpu] batched factorize_solve", flush=True)
    xs, ells, ref, b = batch
    plan, f, xd, ed = run_batch(K, xs, ells)
    bd = dev(b)
    base_L = f.export_L()
    base_x = f.solve(bd).cpu().numpy()
    g = K.Factor(plan, "fp64")
    x = g.factorize_solve(xd, bd, 1.5, ell_dev=ed).cpu().numpy()
    assert np.array_equal(x, base_x) and np.array_equal(g.export_L(), base_L)
    with pytest.raises(K.KCholError):
        g.factorize_solve(xd, bd, 1.5, 0.2)  # a batch needs ell_dev


def test_tuner_choice_does_not_change_results(K, batch):
    print("[gpu] autotuner", flush=True)
    xs, ells, ref, b = batch
    plan, f, xd, ed = run_batch(K, xs, ells)
    base = f.export_L()
    wpb = f.tune(xd, 1.5, ell_dev=ed, reps=2)
    assert wpb in (1, 2, 4)
    w2, pm, order = f.schedule()
    print(f"[gpu] tuner chose wpb={w2} persist_max={pm} order={order}", flush=True)
    assert w2 == wpb and pm in (0, 256, 4096, 2**63 - 1) and order in ("spatial", "longest")
    f.factorize_batched(xd, 1.5, ed)
    assert np.array_equal(f.export_L(), base)


ALL_LEVELS = 2**63 - 1


@pytest.mark.parametrize("wpb,persist_max,order", [(1, ALL_LEVELS, "spatial"), (4, ALL_LEVELS, "longest"),
                                                   (2, 3, "longest"), (1, 40, "spatial"), (1, 0, "longest"),
                                                   (2, 0, "spatial")])
def test_persistent_schedules_bitwise(K, batch, wpb, persist_max, order):
    """Levels grouped into persistent launches (all levels in one launch, or runs of small levels
    between per-level launches), in either unit order, give the default schedule's result bit for bit;
    a graph captured from such a factor (which records per-level launches) replays the same result."""
    print(f"[gpu] schedule wpb={wpb} persist_max={persist_max} order={order}", flush=True)
    import torch
    xs, ells, ref, b = batch
    plan, f, xd, ed = run_batch(K, xs, ells)
    bd = dev(b)
    base_L = f.export_L()
    base_x = f.solve(bd).cpu().numpy()
    f.set_schedule(wpb, persist_max, order)
    assert f.schedule() == (wpb, persist_max, order)
    f.factorize_batched(xd, 1.5, ed)
    assert np.array_equal(f.export_L(), base_L)
    g = f.capture(xd, bd, 1.5, ell_dev=ed)
    info = g.info()
    print(f"[gpu] graph {info}", flush=True)
    assert not info["persistent"] and f.schedule() == (wpb, persist_max, order)
    for rep in range(2):
        out = g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), base_x), f"replay {rep}"
        f.factorize_batched(xd, 1.5, ed)  # eager work between replays
        torch.cuda.synchronize()


def test_single_problem_graph(K):
    print("[gpu] single-problem graph", flush=True)
    import torch
    w = W.small_uniform_2d()
    plan = K.analyze(w.points, w.rho)
    f = K.Factor(plan, "mixed")
    xd, bd = dev(w.points), dev(w.rhs())
    f.factorize(xd, w.nu, w.lengthscale, "shift", 1e-6)
    eager = f.solve(bd).cpu().numpy()
    g = f.capture(xd, bd, w.nu, w.lengthscale, pivot="shift", tau=1e-6)
    for _ in range(3):
        out = g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager)


def test_graph_state_without_device_synchronize(K):
    """Capturing records and runs nothing: a fresh factor stays uncomputed (kc_solve refuses it)
    and stats/export wait for nothing on the destroyed capture stream.  After a replay, stats and
    export_L wait for that replay on its own stream -- no device-wide synchronize in between --
    and see the replay's L."""
    print("[gpu] graph state after capture and replay", flush=True)
    import torch
    w = W.small_uniform_2d()
    plan = K.analyze(w.points, w.rho)
    xd, bd = dev(w.points), dev(w.rhs())
    ref = K.Factor(plan, "fp64")
    ref.factorize(xd, w.nu, w.lengthscale)
    ref_L, ref_x, ref_st = ref.export_L(), ref.solve(bd).cpu().numpy(), ref.stats()
    f = K.Factor(plan, "fp64")
    g = f.capture(xd, bd, w.nu, w.lengthscale)
    with pytest.raises(K.KCholError, match="call out of order"):
        f.solve(bd)  # nothing has computed L yet
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = g.launch(stream=s)
    st = f.stats()  # waits on s
    assert st.nonpositive == ref_st.nonpositive and st.nonfinite == 0
    assert np.array_equal(f.export_L(), ref_L)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref_x)


def test_batched_mixed_error(K, batch):
    print("[gpu] batched mixed", flush=True)
    xs, ells, ref, b = batch
    plan, f, xd, ed = run_batch(K, xs, ells, "mixed", "shift", 1e-6)
    L = f.export_L()
    e0 = 0
    worst = 0.0
    for P, R in ref:
        if R.nonpositive == 0:
            worst = max(worst, np.linalg.norm(L[e0:e0 + P.nnz] - R.L) / np.linalg.norm(R.L))
        e0 += P.nnz
    print(f"[gpu] batched mixed: worst ||dL||/||L|| over instances without zeroed columns {worst:.2e}", flush=True)
    assert worst < 1e-3


def test_batch_with_long_columns_solves_each_instance_as_alone(K):
    """Instances with columns longer than 2048 entries: each instance gets its own top block (its last long
    column bounds it), and the stages are merged across instances by level -- so every instance's solution
    is bitwise the one it gets when solved alone, and within 1e-12 max|x| of the oracle's sequential solve."""
    print("[gpu] batched long columns", flush=True)
    xs = [W.uniform_points(5000, 2, 4301), W.uniform_points(1200, 2, 4302), W.uniform_points(3000, 2, 4303)]
    ells = np.array([0.2, 0.3, 0.25])
    b = np.concatenate([W.gaussian_rhs(len(x), 3, 4400 + i) for i, x in enumerate(xs)])
    plan, f, xd, ed = run_batch(K, xs, ells)
    sol = f.solve(dev(b)).cpu().numpy()
    o0 = 0
    for i, (x, ell) in enumerate(zip(xs, ells)):
        bi = b[o0:o0 + len(x)]
        alone = K.Factor(K.analyze(x, 3.0), "fp64")
        alone.factorize(dev(x), 1.5, float(ell))
        xa = alone.solve(dev(bi)).cpu().numpy()
        assert np.array_equal(sol[o0:o0 + len(x)], xa), f"instance {i}"
        P = O.pattern(x, 3.0)
        R = O.ichol(P, O.theta_on_pattern(P, 1.5, float(ell)))
        xr = O.solve(P, R.L, bi)
        err = np.abs(xa - xr).max(axis=0) / np.abs(xr).max(axis=0)
        assert np.all(err <= 1e-12), (i, err)
        o0 += len(x)
