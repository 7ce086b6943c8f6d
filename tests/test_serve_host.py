"""Host-side pieces of the server (no GPU): percentiles and request generation."""
import math

from paper_2103_02202_amd import workloads as wl


def test_percentile():
    from paper_2103_02202_amd.serve import percentile
    v = list(range(101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile([], 50) is None            # JSON null in the bench output, never NaN


def test_serving_requests_are_poisson_and_log_uniform():
    reqs = wl.serving_requests(4000, rate=100.0, pool_size=50, seed=0)
    gaps = [b["arrival"] - a["arrival"] for a, b in zip(reqs, reqs[1:])]
    mean = sum(gaps) / len(gaps)
    assert abs(mean - 0.01) < 0.001
    shots = [r["shots"] for r in reqs]
    assert min(shots) >= 256 and max(shots) <= 1 << 20
    logs = [math.log(s) for s in shots]
    mid = (math.log(256) + math.log(1 << 20)) / 2
    assert abs(sum(logs) / len(logs) - mid) < 0.2
    assert len({r["circuit"] for r in reqs}) == 50


def test_batch_mix_composition():
    mix = wl.batch_mix(seed=0)
    assert len(mix) == 64
    assert sum(m["kind"] == "surface" for m in mix) == 32
    for m in mix:
        assert 1024 <= m["shots"] <= 262144
        if m["kind"] == "surface":
            assert 3 <= m["d"] <= 25 and m["d"] % 2 == 1 and 1e-4 <= m["p"] <= 1e-2
        else:
            assert 8 <= m["n"] <= 512
