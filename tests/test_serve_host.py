"""Host logic of the served form (no GPU): arrival traces and the latency /
throughput summary."""
import numpy as np

from paper_2604_00546_amd import serve, synth


def test_poisson_trace_rate_and_order():
    arr = serve.poisson_trace(200.0, 30.0, synth.rng(5, synth.SUB_ARRIVAL, 200))
    assert np.all(np.diff(arr) > 0) and arr[0] > 0 and arr[-1] < 30.0
    # 6000 expected arrivals; the count of a Poisson process has sd sqrt(6000) ~ 77
    assert abs(len(arr) - 6000) < 5 * 77
    gaps = np.diff(arr)
    assert abs(gaps.mean() - 1 / 200.0) < 0.05 / 200.0
    # exponential gaps: coefficient of variation 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05


def test_poisson_trace_is_seeded():
    a = serve.poisson_trace(50.0, 10.0, synth.rng(5, synth.SUB_ARRIVAL, 50))
    b = serve.poisson_trace(50.0, 10.0, synth.rng(5, synth.SUB_ARRIVAL, 50))
    assert np.array_equal(a, b)


def test_summary_percentiles():
    reqs = []
    for i in range(100):
        r = serve.Request(i, arrival=0.01 * i, kind="verify", query=None, db=None)
        r.admitted = r.arrival
        r.done = r.arrival + 0.001 * (i + 1)  # latencies 1..100 ms
        reqs.append(r)
    s = serve.summarize(reqs, wall=1.1, batches=[4] * 25)
    assert abs(s["latency_ms"]["p50"] - 50.5) < 1e-6
    assert abs(s["latency_ms"]["p99"] - 99.01) < 1e-6
    assert s["latency_ms"]["max"] == 100.0 or abs(s["latency_ms"]["max"] - 100.0) < 1e-9
    assert s["batches"] == 25 and s["mean_batch"] == 4.0
    span = reqs[-1].done - reqs[0].arrival
    assert abs(s["throughput_rps"] - 100 / span) < 1e-9
