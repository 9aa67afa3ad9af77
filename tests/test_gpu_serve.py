"""Serving loop: requests of uneven size admitted as slots and the device-byte
budget allow, running beside each other on several streams.  Each result must be
bitwise the result of the same request served alone, and (FP64) the oracle's."""
import numpy as np
import pytest

import oracle as O
from paper_1706_02205_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1706_02205_amd import serve
    return serve


def trace(count, rate, seed):
    reqs = W.serving_trace(count, rate, n_lo=300, n_hi=2000, seed=seed)
    return [(r.arrival_s, r.points, W.gaussian_rhs(len(r.points), 4, r.rhs_seed)) for r in reqs]


def test_results_in_the_mix_equal_results_alone(serve):
    print("[gpu] serving: mix vs alone", flush=True)
    reqs = trace(24, 400.0, 5100)
    # a small budget forces admission to wait for completions and to evict resident factors
    one = max(len(p) for _, p, _ in reqs) * 400 * 12
    srv = serve.Server(1.5, 0.2, 3.0, prec="fp64", budget_bytes=3 * one, max_inflight=6, nstreams=4)
    st = srv.run(reqs)
    srv.close()
    s = st.summary()
    print(f"[gpu] serving: {s}", flush=True)
    assert s["requests"] == 24 and st.peak_resident_bytes <= st.budget_bytes
    assert st.peak_inflight >= 2  # requests overlapped on the device
    for i in (0, 7, 23):
        alone = serve.Server(1.5, 0.2, 3.0, prec="fp64", max_inflight=1, nstreams=1)
        sa = alone.run([(0.0, reqs[i][1], reqs[i][2])])
        alone.close()
        assert np.array_equal(sa.results[0].solution, st.results[i].solution)
    # and the oracle's solve with its own factor (every column <= 2048 entries: sequential sums)
    for i in (3, 11):
        _, pts, b = reqs[i]
        P = O.pattern(pts, 3.0)
        R = O.ichol(P, O.theta_on_pattern(P, 1.5, 0.2))
        assert np.array_equal(st.results[i].solution, O.solve(P, R.L, b))


def test_mixed_precision_serving_latency_report(serve):
    print("[gpu] serving: mixed precision report", flush=True)
    reqs = trace(40, 200.0, 5200)
    srv = serve.Server(1.5, 0.2, 3.0, prec="mixed", max_inflight=8, nstreams=4)
    st = srv.run(reqs)
    srv.close()
    s = st.summary()
    print(f"[gpu] serving: {s}", flush=True)
    assert s["requests"] == 40 and s["p99_ms"] >= s["p50_ms"] > 0


def test_head_of_line_bypass_is_bounded(serve):
    """A large request at the head that does not fit next to the requests in flight is passed by smaller
    ones that do, at most max_bypass times; results stay bitwise those of the request served alone."""
    print("[gpu] serving: bounded bypass", flush=True)
    big = [(0.0, W.uniform_points(3000, 2, 5300 + i), W.gaussian_rhs(3000, 4, 5400 + i)) for i in range(3)]
    small = [(0.0, W.uniform_points(300, 2, 5500 + i), W.gaussian_rhs(300, 4, 5600 + i)) for i in range(12)]
    reqs = [big[0], big[1]] + small[:6] + [big[2]] + small[6:]
    srv0 = serve.Server(1.5, 0.2, 3.0, prec="fp64", max_inflight=8, nstreams=4)
    need_big = srv0._need(__import__("paper_1706_02205_amd").analyze(big[0][1], 3.0), big[0][2])
    srv0.close()
    # room for one large request and some small ones, not for two large ones
    srv = serve.Server(1.5, 0.2, 3.0, prec="fp64", budget_bytes=int(1.6 * need_big), max_inflight=8, nstreams=4,
                       max_bypass=3)
    st = srv.run(reqs)
    srv.close()
    s = st.summary()
    print(f"[gpu] serving: {s}", flush=True)
    assert s["requests"] == len(reqs) and st.peak_resident_bytes <= st.budget_bytes
    assert s["max_bypassed"] <= 3
    for i in (1, 3, 8):
        alone = serve.Server(1.5, 0.2, 3.0, prec="fp64", max_inflight=1, nstreams=1)
        sa = alone.run([(0.0, reqs[i][1], reqs[i][2])])
        alone.close()
        assert np.array_equal(sa.results[0].solution, st.results[i].solution)
