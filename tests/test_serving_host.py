"""Host-side logic of the serving loop (no GPU): the request load, the
virtual clock and the latency summary."""
import numpy as np

from paper_1108_1954_amd import serve as S


def test_requests_are_seeded_and_in_range():
    a = S.make_requests(12, rate=50.0, steps_range=(100, 2000), np_scale=1e-3, workers=2)
    b = S.make_requests(12, rate=50.0, steps_range=(100, 2000), np_scale=1e-3, workers=2)
    assert [q.nsteps for q in a] == [q.nsteps for q in b]
    for qa, qb in zip(a, b):
        np.testing.assert_array_equal(qa.x, qb.x)
        np.testing.assert_array_equal(qa.v, qb.v)
    assert all(100 <= q.nsteps <= 2000 for q in a)
    arr = [q.arrival for q in a]
    assert all(x < y for x, y in zip(arr, arr[1:]))
    for q in a:
        assert q.x.shape == (q.spec.np_,) and q.spec.ng in (64, 128, 256, 512, 1024, 2048)
        assert np.all((q.x >= 0) & (q.x < q.spec.L))


def test_arrival_gaps_have_the_poisson_mean():
    reqs = S.make_requests(2000, rate=50.0, np_scale=1e-5, steps_range=(1, 1), workers=4)
    gaps = np.diff([0.0] + [q.arrival for q in reqs])
    assert abs(gaps.mean() * 50.0 - 1.0) < 0.07        # 2000 exponential gaps: sd of mean 2.2%
    assert abs(np.median(gaps) * 50.0 - np.log(2.0)) < 0.07


def test_virtual_clock():
    c = S.VirtualClock(tick=0.5)
    c.advance()
    c.advance()
    assert c.now() == 1.0
    c.sleep_until(0.2)
    assert c.now() == 1.0
    c.sleep_until(3.0)
    assert c.now() == 3.0


def test_summary_percentiles_and_rate():
    res = [S.Result(k, 100, 64, 10, arrival=float(k), admitted=float(k), completed=k + 1.0 + 0.01 * k,
                    diag={}) for k in range(100)]
    s = S.summarize(res, 1 << 20)
    lat = np.array([1.0 + 0.01 * k for k in range(100)])
    assert np.isclose(s["p50_latency_s"], np.percentile(lat, 50), rtol=1e-12)
    assert np.isclose(s["p99_latency_s"], np.percentile(lat, 99), rtol=1e-12)
    assert s["particle_steps"] == 100 * 100 * 10
    assert np.isclose(s["aggregate_particle_steps_per_s"], 1e5 / (99 + 1.99))
