"""Pins for the oracle's Pauli-frame sampler (CPU only).

* Noiseless circuits: every sampled record lies in the exact state-vector
  support, and the records are uniform over it (each random stabilizer
  measurement is 50/50), chi-squared.
* Noisy circuits with few noise sites: empirical record distribution against
  the exact mixture over Pauli-error configurations, chi-squared.
* Noise rates against closed forms (two-sided, 5 sigma).
* Surface-code invariants: noiseless detection events are all zero; an
  X_ERROR(1) on a bulk data qubit between rounds fires exactly the adjacent
  Z-type detectors of the next round.
* Shot slicing: shots [a, b) sampled alone equal that slice of a larger run.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import statevector as sv
from paper_2103_02202_amd import workloads as wl
from circuit_gen import random_circuit


def records(c, shots, seed=0):
    out = c.sample(seed, 0, shots, meas=True)["meas"]
    return oracle.unpack_bits(out, shots)


def chi2_against(dist, recs):
    keys = list(dist)
    index = {k: i for i, k in enumerate(keys)}
    counts = np.zeros(len(keys))
    for r in map(tuple, recs.tolist()):
        assert r in index, "sampled record outside the exact support"
        counts[index[r]] += 1
    exp = np.array([dist[k] for k in keys]) * len(recs)
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        obs, e = obs[:-1], e[:-1]
    e *= obs.sum() / e.sum()
    if len(obs) < 2:
        return 1.0
    return stats.chisquare(obs, e).pvalue


@pytest.mark.parametrize("seed", range(12))
def test_noiseless_records_uniform_over_support(seed):
    text = random_circuit(4, 30, seed=2000 + seed)
    dist = sv.record_distribution(text)
    if len(dist) > 256:
        pytest.skip("too many outcomes for a chi-squared test")
    c = oracle.Circuit(text)
    recs = records(c, 16384, seed=seed)
    assert chi2_against(dist, recs) > 1e-4


@pytest.mark.parametrize("seed", range(12))
def test_noisy_records_match_exact_mixture(seed):
    rng = np.random.Generator(np.random.PCG64(77 + seed))
    n = 3
    while True:
        text = random_circuit(n, 12, seed=3000 + seed * 31 + int(rng.integers(1000)),
                              noise=True, p=0.15, collapse_weight=0.15)
        ops = sv.parse(text)
        sites = sum(1 for name, arg, t in ops if name in sv.NOISE)
        if 1 <= sites <= 3:
            break
    dist = sv.noisy_record_distribution(text)
    c = oracle.Circuit(text)
    recs = records(c, 32768, seed=seed)
    assert chi2_against(dist, recs) > 1e-4


def rate(text, shots, col):
    c = oracle.Circuit(text)
    r = records(c, shots)
    return r[:, col].mean() if isinstance(col, int) else np.all(r[:, col] == 1, axis=1).mean()


@pytest.mark.parametrize("p", [1e-3, 1e-2, 0.3])
@pytest.mark.parametrize("text,factor,col", [
    ("X_ERROR({p}) 0\nM 0\n", 1.0, 0),
    ("Y_ERROR({p}) 0\nM 0\n", 1.0, 0),
    ("H 0\nZ_ERROR({p}) 0\nH 0\nM 0\n", 1.0, 0),
    ("DEPOLARIZE1({p}) 0\nM 0\n", 2 / 3, 0),
    ("H 0\nDEPOLARIZE1({p}) 0\nH 0\nM 0\n", 2 / 3, 0),
    ("DEPOLARIZE2({p}) 0 1\nM 0 1\n", 8 / 15, 0),
    ("DEPOLARIZE2({p}) 0 1\nM 0 1\n", 8 / 15, 1),
    ("DEPOLARIZE2({p}) 0 1\nM 0 1\n", 4 / 15, [0, 1]),
])
def test_noise_rates(p, text, factor, col):
    shots = 1 << 17
    q = factor * p
    got = rate(text.format(p=p), shots, col)
    sigma = math.sqrt(q * (1 - q) / shots)
    assert abs(got - q) < 5 * sigma + 1e-12


def test_noise_rate_small_p_many_shots():
    shots = 1 << 20
    p = 1e-4
    got = rate(f"X_ERROR({p}) 0 1 2 3\nM 0 1 2 3\n", shots, 2)
    assert abs(got - p) < 5 * math.sqrt(p / shots)


@pytest.mark.parametrize("d", [3, 5, 7])
def test_noiseless_surface_code_detectors_are_zero(d):
    c = oracle.Circuit(wl.surface_code(d, d, 0.0))
    out = c.sample(1, 0, 1024, det=True, obs=True, meas=True)
    assert not out["det"].any()
    assert not out["obs"].any()
    # the measurement record itself is random (X-type ancillas), not all zero
    assert out["meas"].any()


def test_x_error_injection_fires_adjacent_detectors():
    d = 5
    text = wl.surface_code(d, 4, 0.0)
    data, anc, idx = wl._surface_layout(d)
    x0, y0 = 5, 5                      # a bulk data qubit
    q = idx[(x0, y0)]
    lines = text.split("\n")
    pos = lines.index(next(s for s in lines if s.startswith("REPEAT")))
    lines.insert(pos, f"X_ERROR(1) {q}")
    c = oracle.Circuit("\n".join(lines))
    out = c.sample(3, 0, 256, det=True)["det"]
    fired = [k for k in range(c.num_detectors) if out[k].any()]
    assert all(np.all(out[k] == ~np.uint64(0)) for k in fired)
    # detectors of round 2 (after the A/2 round-1 detectors) for Z ancillas adjacent to (5, 5)
    A = d * d - 1
    zs = [k for k, (x, y, is_x) in enumerate(anc) if not is_x]
    expect = []
    for k, (x, y, is_x) in enumerate(anc):
        if not is_x and abs(x - x0) == 1 and abs(y - y0) == 1:
            expect.append(len(zs) + k)
    assert fired == expect and len(expect) == 2


def test_shot_slices_equal_slices_of_a_full_run():
    c = oracle.Circuit(wl.surface_code(3, 3, 0.02))
    full = c.sample(9, 0, 1000, det=True, meas=True)
    part = c.sample(9, 256, 500, det=True, meas=True)
    for k in ("meas", "det"):
        f = oracle.unpack_bits(full[k], 1000)[256:756]
        g = oracle.unpack_bits(part[k], 500)
        assert np.array_equal(f, g)
        # tail bits beyond num_shots are zero
        assert not (part[k][:, -1] >> np.uint64(500 - 448)).any()


def test_sampling_is_deterministic_and_seed_dependent():
    c = oracle.Circuit(wl.surface_code(3, 3, 0.01))
    a = c.sample(5, 0, 640, meas=True)["meas"]
    b = c.sample(5, 0, 640, meas=True)["meas"]
    e = c.sample(6, 0, 640, meas=True)["meas"]
    assert np.array_equal(a, b)
    assert not np.array_equal(a, e)


def test_repetition_example_at_p_zero_is_all_zero():
    text = wl.repetition_code_example().replace("0.01", "0")
    c = oracle.Circuit(text)
    assert not c.sample(0, 0, 1024, meas=True)["meas"].any()


def test_teleportation_last_measurement_always_zero():
    c = oracle.Circuit(wl.teleportation_example())
    m = oracle.unpack_bits(c.sample(4, 0, 4096, meas=True)["meas"], 4096)
    assert not m[:, -1].any()
    assert 0.4 < m[:, 0].mean() < 0.6 and 0.4 < m[:, 1].mean() < 0.6
