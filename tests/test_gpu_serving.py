"""Serving loop on the GPU: continuous batching with admission by HBM
footprint.  Each run's result (diagnostics, per-step history, final
particles) must be bit-identical to the same run created and stepped alone,
whatever else shared the device with it; the arrival schedule is injected
(virtual clock), and a small budget forces admissions to wait."""
import numpy as np
import pytest

from paper_1108_1954_amd import pic as P
from paper_1108_1954_amd import serve as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    yield


def small_requests(n, seed, steps=(5, 60), rate=2000.0, np_scale=0.01):
    return S.make_requests(n, rate=rate, seed_runs=seed, seed_arrivals=seed + 1,
                           steps_range=steps, np_scale=np_scale, workers=4)


def alone(req):
    p = P.make_params(req.spec.L, req.spec.ng, req.spec.np_, req.spec.dt, history_cap=req.nsteps)
    with P.Run(p, req.x, req.v) as r:
        r.step(req.nsteps)
        d, _, _ = r.diagnostics()
        return d, (r.history() if req.nsteps else None)


def check_same_as_alone(results, requests):
    assert [r.index for r in results] == [q.index for q in requests]
    for res, req in zip(results, requests):
        d, hist = alone(req)
        assert res.diag == d, f"request {req.index}: diagnostics differ from the run alone"
        if req.nsteps:
            np.testing.assert_array_equal(res.history, hist)
        assert res.diag["step"] == req.nsteps
        assert res.diag["charge_fixed_sum"] == req.spec.np_ << 32


def test_serving_results_equal_runs_alone_under_a_tight_budget():
    reqs = small_requests(24, seed=11)
    foot = [P.pic_footprint(P.make_params(q.spec.L, q.spec.ng, q.spec.np_, q.spec.dt,
                                          history_cap=q.nsteps)) for q in reqs]
    budget = int(max(foot) * 2.2)            # two or three runs at a time
    clock = S.VirtualClock(tick=1e-3)
    with S.Server(budget, ng_max=2048, max_runs=8, chunk=4, graph_steps=4, depth=0,
                  keep_history=True, clock=clock) as srv:
        results = srv.run(reqs)
        assert srv.admit_blocked > 0, "the budget never made an admission wait"
        assert 1 < srv.max_resident < len(reqs)
        assert P.pic_batch_usage(srv.batch)[0] == 0
    check_same_as_alone(results, reqs)
    # first come, first served: admissions in arrival order
    adm = [r.admitted for r in sorted(results, key=lambda r: (r.arrival, r.index))]
    assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_serving_overlaps_runs_and_handles_zero_step_requests():
    reqs = small_requests(10, seed=21, steps=(0, 30))
    reqs[3].nsteps = 0
    clock = S.VirtualClock(tick=1e-4)
    with S.Server(1 << 30, ng_max=2048, max_runs=16, chunk=3, graph_steps=3, depth=0,
                  keep_history=True, clock=clock) as srv:
        results = srv.run(reqs)
        assert srv.max_resident > 1, "no two runs were ever resident together"
    check_same_as_alone(results, reqs)


def test_serving_wall_clock_load_with_pipelined_chunks():
    """The real-time loop (chunks in flight, completions detected by events)
    finishes every request, and results still equal the runs alone."""
    reqs = small_requests(16, seed=31, steps=(20, 120), rate=400.0)
    with S.Server(1 << 30, ng_max=2048, max_runs=32, chunk=8, graph_steps=8, depth=2,
                  keep_history=True) as srv:
        results = srv.run(reqs)
    check_same_as_alone(results, reqs)
    summary = S.summarize(results, 1 << 30)
    assert 0 < summary["p50_latency_s"] <= summary["p99_latency_s"]
    assert summary["particle_steps"] == sum(q.work for q in reqs)


def test_a_request_larger_than_the_budget_is_rejected_up_front():
    reqs = small_requests(3, seed=31, np_scale=0.05)
    biggest = max(P.pic_footprint(P.make_params(q.spec.L, q.spec.ng, q.spec.np_, q.spec.dt)) for q in reqs)
    with S.Server(budget=biggest // 2, clock=S.VirtualClock(tick=1e-3)) as srv:
        with pytest.raises(ValueError, match="budget"):
            srv.run(reqs)
