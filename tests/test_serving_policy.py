"""CPU tests of the serving policy with a simulated device on a virtual clock."""
import pytest

pytest.importorskip("torch")
from paper_2412_14973_amd.serve import Job, Server, SimBackend, percentile, summarize  # noqa: E402


def _jobs(specs):
    return [Job(rid=i, arrival=a, payload=dict(bytes=b, service=s, value=i)) for i, (a, b, s) in enumerate(specs)]


def test_fifo_one_at_a_time_latencies():
    jobs = _jobs([(0.0, 1, 1.0), (0.1, 1, 1.0), (0.2, 1, 1.0)])
    Server(SimBackend(width=1), hbm_budget=10, max_active=1).run(jobs, poll_interval=1e-3)
    fin = [j.finished for j in jobs]
    assert fin == pytest.approx([1.0, 2.0, 3.0], abs=2e-3)
    assert [j.latency for j in jobs] == pytest.approx([1.0, 1.9, 2.8], abs=2e-3)


def test_admission_respects_budget_and_order():
    # 3 jobs of 6 bytes with budget 10: at most one at a time even with 4 slots
    jobs = _jobs([(0.0, 6, 1.0), (0.0, 6, 1.0), (0.0, 6, 1.0)])
    srv = Server(SimBackend(width=4), hbm_budget=10, max_active=4)
    srv.run(jobs, poll_interval=1e-3)
    assert srv.peak_in_use <= 10
    adm = [j.admitted for j in jobs]
    assert adm == sorted(adm)
    assert jobs[1].admitted >= jobs[0].finished - 1e-9


def test_concurrency_improves_throughput_on_underfilled_device():
    specs = [(0.01 * i, 1, 1.0) for i in range(8)]
    one = _jobs(specs)
    Server(SimBackend(width=4), hbm_budget=100, max_active=1).run(one, poll_interval=1e-3)
    many = _jobs(specs)
    Server(SimBackend(width=4), hbm_budget=100, max_active=4).run(many, poll_interval=1e-3)
    s1, s4 = summarize(one), summarize(many)
    assert s4["solves_per_s"] > 3 * s1["solves_per_s"]
    assert s4["p99_latency_s"] < s1["p99_latency_s"]


def test_oversized_request_rejected_others_served():
    jobs = _jobs([(0.0, 1, 0.5), (0.0, 50, 0.5), (0.0, 1, 0.5)])
    Server(SimBackend(width=2), hbm_budget=10, max_active=2).run(jobs, poll_interval=1e-3)
    assert jobs[1].rejected and jobs[1].result is None
    assert not jobs[0].rejected and not jobs[2].rejected
    assert jobs[0].result["value"] == 0 and jobs[2].result["value"] == 2


def test_failing_request_isolated():
    jobs = _jobs([(0.0, 1, 0.3), (0.0, 1, 0.3), (0.0, 1, 0.3)])
    Server(SimBackend(width=3, fail=lambda p: p["value"] == 1), hbm_budget=10, max_active=3).run(
        jobs, poll_interval=1e-3)
    assert [j.result["ok"] for j in jobs] == [True, False, True]


def test_arrivals_in_the_future_wait():
    jobs = _jobs([(5.0, 1, 1.0)])
    Server(SimBackend(), hbm_budget=10).run(jobs, poll_interval=1e-3)
    assert jobs[0].admitted >= 5.0 and jobs[0].finished == pytest.approx(6.0, abs=2e-3)


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50 and percentile(v, 99) == 99 and percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0
