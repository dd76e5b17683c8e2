"""Host-side logic of the serving loop (no GPU): the Poisson query trace and
the latency percentiles."""
import numpy as np

from paper_2106_06889_amd import serve


def test_poisson_trace_shape_and_rate():
    tr = serve.poisson_trace(20000, rate=1000.0, num_grammars=256, seed=3)
    arr = np.array([q.arrival for q in tr])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    gaps = np.diff(arr)
    assert abs(gaps.mean() - 1e-3) < 0.05e-3            # mean inter-arrival 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05   # exponential: coefficient of variation 1
    kinds = np.array([q.kind for q in tr])
    for k, p in zip(serve.KINDS, (0.5, 0.3, 0.2)):
        assert abs((kinds == k).mean() - p) < 0.02
    gs = np.array([q.grammar for q in tr])
    assert gs.min() >= 0 and gs.max() < 256
    assert [q.qid for q in tr] == list(range(20000))


def test_poisson_trace_is_seeded():
    a = serve.poisson_trace(100, 50.0, 4, seed=9)
    b = serve.poisson_trace(100, 50.0, 4, seed=9)
    c = serve.poisson_trace(100, 50.0, 4, seed=10)
    assert a == b and a != c


def test_percentiles():
    recs = [serve.Record(i, "wc", 0, arrival=0.0, finish=(i + 1) / 1000.0) for i in range(100)]
    st = serve.percentiles(recs)
    assert st["n"] == 100
    assert abs(st["p50_ms"] - 50.5) < 1e-9 and abs(st["p99_ms"] - 99.01) < 1e-9
    assert abs(st["mean_ms"] - 50.5) < 1e-9
