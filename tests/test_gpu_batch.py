"""Batched launches: one persistent, graph-captured launch over many circuits
must give bit-identical results to running each request alone (and to the
oracle), on first submission (tuned), on graph replays, and in a different
mix."""
import numpy as np
import pytest

import oracle
from paper_2103_02202_amd import workloads as wl
from circuit_gen import random_circuit

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def announce(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def sg():
    from paper_2103_02202_amd import stim_gpu
    assert torch.cuda.is_available()
    return stim_gpu


def make_requests(sg, specs):
    reqs, circs = [], []
    for text, shots, seed, mode, offset in specs:
        c = sg.Circuit(text)
        circs.append(c)
        W = (shots + 63) // 64
        if mode == 0:
            out0 = torch.full((c.num_measurements, W), -1, dtype=torch.int64, device="cuda")
            out1 = None
        else:
            out0 = torch.full((c.num_detectors, W), -1, dtype=torch.int64, device="cuda")
            out1 = torch.full((max(c.num_observables, 1), W), -1, dtype=torch.int64, device="cuda")
        reqs.append({"handle": c.handle, "seed": seed, "shot_offset": offset, "num_shots": shots, "mode": mode,
                     "out0": out0, "out1": out1})
    return reqs, circs


def single(sg, c, r):
    if r["mode"] == 0:
        out = c.sample(r["seed"], r["num_shots"], shot_offset=r["shot_offset"])
        return out, None
    det, obs = c.detect(r["seed"], r["num_shots"], shot_offset=r["shot_offset"])
    return det, obs


SPECS = [
    (wl.surface_code(3, 3, 1e-3), 1024, 0, 1, 0),
    (wl.surface_code(5, 5, 3e-3), 5000, 1, 1, 0),
    (wl.surface_code(7, 7, 1e-2), 777, 2, 0, 64),
    (wl.random_clifford(64, 30, seed=3), 4096, 3, 0, 0),
    (random_circuit(20, 150, seed=77, noise=True, p=0.05), 3333, 4, 0, 128),
    (wl.surface_code(9, 9, 1e-4), 20000, 5, 1, 0),
    (wl.repetition_code_example(), 2048, 6, 0, 0),
    (wl.surface_code(25, 25, 1e-3), 3000, 7, 1, 0),
]


def check_against_single(sg, reqs, circs):
    for r, c in zip(reqs, circs):
        a, b = single(sg, c, r)
        torch.cuda.synchronize()
        assert torch.equal(r["out0"], a), f"request seed {r['seed']} differs from its single run"
        if b is not None and c.num_observables:
            assert torch.equal(r["out1"][: c.num_observables], b)


def test_batch_matches_single_requests_and_replays(sg):
    announce("batch mix", len(SPECS))
    reqs, circs = make_requests(sg, SPECS)
    sg.stim_batch_sample(reqs)
    torch.cuda.synchronize()
    check_against_single(sg, reqs, circs)
    # second submission builds the tuned, graph-captured plan; the third replays it
    for _ in range(2):
        for r in reqs:
            r["out0"].fill_(-1)
            if r["out1"] is not None:
                r["out1"].fill_(-1)
        sg.stim_batch_sample(reqs)
        torch.cuda.synchronize()
        check_against_single(sg, reqs, circs)


def test_batch_matches_oracle_on_small_requests(sg):
    announce("batch vs oracle")
    specs = [s for s in SPECS if s[1] <= 5000 and "REPEAT 24" not in s[0]][:5]
    reqs, circs = make_requests(sg, specs)
    sg.stim_batch_sample(reqs)
    torch.cuda.synchronize()
    for (text, shots, seed, mode, offset), r in zip(specs, reqs):
        o = oracle.Circuit(text)
        want = o.sample(seed, offset, shots, meas=mode == 0, det=mode == 1, obs=mode == 1)
        got = r["out0"].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want["meas" if mode == 0 else "det"])


def test_batch_without_tuning_and_order_independence(sg, monkeypatch):
    announce("batch untuned, reversed")
    monkeypatch.setenv("STIM_TUNE", "0")
    specs = list(reversed(SPECS[:6]))
    reqs, circs = make_requests(sg, specs)
    for _ in range(2):
        sg.stim_batch_sample(reqs)
        torch.cuda.synchronize()
        check_against_single(sg, reqs, circs)


def test_batch_generated_mix_sample(sg):
    """A slice of the 64-circuit generated batch (shots capped for test time)."""
    announce("generated batch mix")
    mix = wl.batch_mix(seed=0)[::8]
    specs = [(m["text"], min(m["shots"], 8192), m["seed"], 1 if m["kind"] == "surface" else 0, 0) for m in mix]
    reqs, circs = make_requests(sg, specs)
    sg.stim_batch_sample(reqs)
    torch.cuda.synchronize()
    check_against_single(sg, reqs, circs)


def test_batch_rejects_bad_requests(sg):
    announce("batch errors")
    c = sg.Circuit("M 0\n")
    out = torch.zeros((1, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(sg.StimError):
        sg.stim_batch_sample([{"handle": c.handle, "seed": 0, "shot_offset": 3, "num_shots": 64, "mode": 0,
                               "out0": out, "out1": None}])
    with pytest.raises(sg.StimError):
        sg.stim_batch_sample([{"handle": c.handle, "seed": 0, "shot_offset": 0, "num_shots": 64, "mode": 7,
                               "out0": out, "out1": None}])


def test_batch_with_feedback_requests(sg):
    """Classically controlled Paulis inside the persistent batched kernel."""
    announce("batch with feedback")
    specs = [
        (wl.surface_code(5, 5, 1e-2, feedback_reset=True), 3000, 11, 1, 0),
        (random_circuit(12, 120, seed=91, noise=True, p=0.05, feedback=0.2), 2222, 12, 0, 64),
        (wl.surface_code(3, 3, 1e-3), 1024, 13, 1, 0),
        (wl.surface_code(7, 7, 3e-3, feedback_reset=True), 4500, 14, 0, 0),
    ]
    reqs, circs = make_requests(sg, specs)
    for _ in range(3):                       # direct, tuned + captured, replay
        for r in reqs:
            r["out0"].fill_(-1)
        sg.stim_batch_sample(reqs)
        torch.cuda.synchronize()
        check_against_single(sg, reqs, circs)
    for (text, shots, seed, mode, offset), r in zip(specs, reqs):
        o = oracle.Circuit(text)
        want = o.sample(seed, offset, shots, meas=mode == 0, det=mode == 1, obs=mode == 1)
        assert np.array_equal(r["out0"].cpu().numpy().view(np.uint64), want["meas" if mode == 0 else "det"])


def test_batch_prepass_equals_inline_noise(sg, monkeypatch):
    """The per-request noise pre-pass and inline noise draw the same errors:
    batches with and without it agree bit for bit, on every submission
    (direct, tuned + captured, replay)."""
    announce("batch pre-pass vs inline")
    specs = [s for s in SPECS if "ERROR" in s[0] or "DEPOLARIZE" in s[0]]
    outs = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("STIM_NOISE_PREPASS", flag)
        reqs, circs = make_requests(sg, specs)
        got = []
        for _ in range(3):
            for r in reqs:
                r["out0"].fill_(-1)
            sg.stim_batch_sample(reqs)
            torch.cuda.synchronize()
            got.append([r["out0"].clone() for r in reqs])
        for g in got[1:]:
            assert all(torch.equal(a, b) for a, b in zip(got[0], g))
        outs[flag] = got[0]
    for a, b, s in zip(outs["1"], outs["0"], specs):
        assert torch.equal(a, b), f"request seed {s[2]} differs between pre-pass and inline noise"


def test_many_noise_executions_fall_back_to_inline(sg):
    """More noise executions than one pre-pass launch covers: sampled with
    inline noise, still equal to the oracle (single and batched)."""
    text = "REPEAT 70000 {\nX_ERROR(0.002) 0\nCX 0 1\n}\nM 0 1\n"
    announce("70000 noise executions")
    specs = [(text, 1000, 21, 0, 0), (wl.surface_code(3, 3, 1e-2), 700, 22, 0, 0)]
    reqs, circs = make_requests(sg, specs)
    sg.stim_batch_sample(reqs)
    torch.cuda.synchronize()
    o = oracle.Circuit(text)
    want = o.sample(21, 0, 1000, meas=True)["meas"]
    assert np.array_equal(reqs[0]["out0"].cpu().numpy().view(np.uint64), want)
    assert want.any()
    check_against_single(sg, reqs, circs)


def test_tuned_width_is_not_reused_where_the_frame_does_not_fit(sg, tmp_path, monkeypatch):
    """A shape class spans a factor of two in qubit count.  A tile width tuned
    for its smaller circuits (here written into the tuning cache file: 8 words,
    256 threads for the class of 1,025..2,048 qubits, 64 words, one request)
    must not be used for a 2,000-qubit circuit, whose frame needs 256 KB of
    LDS at that width: both the first (one launch) and the second (tuned,
    captured) submission succeed and equal the single call."""
    announce("tuned width vs larger circuit of the same class")
    cache = tmp_path / "tune.txt"
    cache.write_text("11/6/0 8 256\n")
    monkeypatch.setenv("STIM_TUNE_CACHE", str(cache))
    text = wl.random_clifford(2000, 5, seed=17)
    reqs, circs = make_requests(sg, [(text, 4096, 31, 0, 0)])
    for _ in range(3):
        reqs[0]["out0"].fill_(-1)
        sg.stim_batch_sample(reqs)
        torch.cuda.synchronize()
        check_against_single(sg, reqs, circs)
    # The class was tuned again (its cached width does not fit): a new line.
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and lines[1].startswith("11/6/0 ") and not lines[1].endswith(" 8 256")


def test_tuning_cache_file_round_trip(sg, tmp_path, monkeypatch):
    """Tuned classes are appended to the cache file and read back by a later
    launch: a class present in the file is not tuned again."""
    announce("tuning cache round trip")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("STIM_TUNE_CACHE", str(cache))
    # 17 requests: a shape class no other test of this process submits.
    specs = [(wl.surface_code(3, 3, 1e-3), 1024, 41 + k, 1, 0) for k in range(16)]
    specs.append((wl.random_clifford(20, 20, seed=4), 1000, 60, 0, 0))
    reqs, circs = make_requests(sg, specs)
    for _ in range(2):
        sg.stim_batch_sample(reqs)
        torch.cuda.synchronize()
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    cls, T, threads = lines[0].split()
    assert int(T) in (1, 2, 4, 8) and int(threads) in (64, 256, 512, 1024)      # 64: one wave per tile
    reqs2, circs2 = make_requests(sg, specs)         # same class, new outputs: a new plan
    for _ in range(2):
        sg.stim_batch_sample(reqs2)
        torch.cuda.synchronize()
    check_against_single(sg, reqs2, circs2)
    assert cache.read_text().splitlines() == lines


@pytest.mark.parametrize("tune", ["0", "1"])
def test_one_wave_per_tile_batches(sg, tune, monkeypatch):
    """The batched walk with one wave per tile (STIM_BATCH_WAVE=1 forces it;
    otherwise the tuner may pick it): noisy surface codes up to d=25, random
    circuits, feedback and the repetition code, equal to their single calls on
    the first submission, the captured one and a replay, and to the oracle."""
    announce("one wave per tile", tune)
    monkeypatch.setenv("STIM_BATCH_WAVE", "1")
    monkeypatch.setenv("STIM_TUNE", tune)
    specs = SPECS + [(wl.surface_code(5, 5, 1e-2, feedback_reset=True), 3000, 11, 1, 0),
                     (random_circuit(12, 120, seed=91, noise=True, p=0.05, feedback=0.2), 2222, 12, 0, 64)]
    reqs, circs = make_requests(sg, specs)
    for _ in range(3):
        for r in reqs:
            r["out0"].fill_(-1)
            if r["out1"] is not None:
                r["out1"].fill_(-1)
        sg.stim_batch_sample(reqs)
        torch.cuda.synchronize()
        check_against_single(sg, reqs, circs)
    for (text, shots, seed, mode, offset), r in list(zip(specs, reqs))[:6]:
        o = oracle.Circuit(text)
        want = o.sample(seed, offset, shots, meas=mode == 0, det=mode == 1, obs=mode == 1)
        assert np.array_equal(r["out0"].cpu().numpy().view(np.uint64), want["meas" if mode == 0 else "det"])
