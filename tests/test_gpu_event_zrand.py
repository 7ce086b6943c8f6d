"""Detector mode without the collapses' Z randomisations.

When every detector and observable of a circuit is deterministic, the Z
randomisation drawn after each collapse contributes nothing to any event (the
frame is linear in its random bits, and each such draw acts like a Z error
whose detector set is empty), so the detector-mode walk skips them.  The
events must stay the same bits: against the oracle (which draws every one),
and against the same circuit sampled with the draws kept
(STIM_EVENT_ZRAND=1).  Circuits with a random detector or observable, or with
classically controlled Paulis, keep their draws and still match the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2103_02202_amd import workloads as wl
from circuit_gen import random_detector_circuit

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sg():
    from paper_2103_02202_amd import stim_gpu
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    stim_gpu.lib()
    return stim_gpu


def events(c, seed, shots, offset=0):
    det, obs = c.detect(seed, shots, shot_offset=offset)
    torch.cuda.synchronize()
    return det.cpu().numpy().view(np.uint64), obs.cpu().numpy().view(np.uint64)


def both_ways(sg, text, seed, shots, monkeypatch, offset=0):
    """Events with the draws skipped (default) and kept, on fresh handles."""
    monkeypatch.delenv("STIM_EVENT_ZRAND", raising=False)
    a = events(sg.Circuit(text), seed, shots, offset)
    monkeypatch.setenv("STIM_EVENT_ZRAND", "1")
    b = events(sg.Circuit(text), seed, shots, offset)
    monkeypatch.delenv("STIM_EVENT_ZRAND", raising=False)
    return a, b


CASES = [
    ("surface d3 p=0.05", lambda: wl.surface_code(3, 5, 0.05), 4097),
    ("surface d5 p=0.01", lambda: wl.surface_code(5, 5, 0.01), 20000),
    ("surface d9 p=0.003", lambda: wl.surface_code(9, 9, 0.003), 65536),
    ("surface d7 r3 p=0.02", lambda: wl.surface_code(7, 3, 0.02), 1000),
]


@pytest.mark.parametrize("name,make,shots", CASES, ids=[c[0] for c in CASES])
def test_deterministic_circuits_same_events_with_and_without_draws(sg, name, make, shots, monkeypatch):
    announce("event zrand", name, shots)
    text = make()
    (da, oa), (db, ob) = both_ways(sg, text, 7, shots, monkeypatch)
    assert np.array_equal(da, db) and np.array_equal(oa, ob)
    want = oracle.Circuit(text).sample(7, 0, shots, det=True, obs=True, meas=False)
    assert np.array_equal(da, want["det"]) and np.array_equal(oa, want["obs"])
    assert np.count_nonzero(da) > 0


def test_tiled_and_global_frames_and_offsets(sg, monkeypatch):
    """Other tile widths, a global frame and a shot offset."""
    text = wl.surface_code(5, 7, 0.02)
    want = oracle.Circuit(text).sample(3, 64 * 9, 5000, det=True, obs=True, meas=False)
    for tile, placement in (("1", "lds"), ("8", "lds"), ("2", "global")):
        announce("event zrand tiling", tile, placement)
        monkeypatch.setenv("STIM_TILE_WORDS", tile)
        monkeypatch.setenv("STIM_FRAME_PLACEMENT", placement)
        (da, oa), (db, ob) = both_ways(sg, text, 3, 5000, monkeypatch, offset=64 * 9)
        assert np.array_equal(da, want["det"]) and np.array_equal(oa, want["obs"])
        assert np.array_equal(db, want["det"]) and np.array_equal(ob, want["obs"])


def test_random_outputs_and_feedback_keep_their_draws(sg):
    """A random detector (H then M), random lookbacks, and feedback resets:
    the draws stay, and the events match the oracle."""
    texts = ["H 0\nM 0\nDETECTOR rec[-1]\nX_ERROR(0.1) 1\nM 1\nDETECTOR rec[-1]\n",
             random_detector_circuit(12, 80, seed=404, reps=4),
             wl.surface_code(5, 5, 0.01, feedback_reset=True)]
    for i, text in enumerate(texts):
        announce("event zrand kept", i)
        c = sg.Circuit(text)
        det, obs = events(c, 11, 3000)
        want = oracle.Circuit(text).sample(11, 0, 3000, det=True, obs=True, meas=False)
        assert np.array_equal(det, want["det"]) and np.array_equal(obs, want["obs"]), f"case {i}"


def test_batched_requests_use_the_same_program(sg):
    """Detector-mode requests of a persistent batched launch equal their
    single calls (both without the draws) and the oracle."""
    announce("event zrand batch")
    texts = [wl.surface_code(3, 3, 0.02), wl.surface_code(5, 5, 0.005), wl.surface_code(7, 3, 0.01)]
    reqs, circs = [], []
    for i, t in enumerate(texts):
        c = sg.Circuit(t)
        circs.append(c)
        W = (3000 + 63) // 64
        reqs.append({"handle": c.handle, "seed": 20 + i, "shot_offset": 0, "num_shots": 3000, "mode": 1,
                     "out0": torch.full((c.num_detectors, W), -1, dtype=torch.int64, device="cuda"),
                     "out1": torch.full((max(c.num_observables, 1), W), -1, dtype=torch.int64, device="cuda")})
    for _ in range(3):
        sg.stim_batch_sample(reqs)
        torch.cuda.synchronize()
        for i, (r, c, t) in enumerate(zip(reqs, circs, texts)):
            want = oracle.Circuit(t).sample(20 + i, 0, 3000, det=True, obs=True, meas=False)
            assert np.array_equal(r["out0"].cpu().numpy().view(np.uint64), want["det"]), f"request {i}"
            assert np.array_equal(r["out1"][: c.num_observables].cpu().numpy().view(np.uint64), want["obs"])


MEASURE_THEN_RESET = """R 0 1 2 3 4
CX 0 1 2 3
CX 2 1 4 3
M 1 3
DETECTOR rec[-2]
DETECTOR rec[-1]
R 3 1
X_ERROR(0.05) 0 2 4
CX 0 1 2 3
CX 2 1 4 3
M 1 3
DETECTOR rec[-2] rec[-4]
DETECTOR rec[-1] rec[-3]
REPEAT 5 {
    R 1 3
    DEPOLARIZE1(0.02) 0 2 4
    CX 0 1 2 3
    CX 2 1 4 3
    X_ERROR(0.03) 1 3
    M 1 3
    DETECTOR rec[-2] rec[-4]
    DETECTOR rec[-1] rec[-3]
}
M 1
DETECTOR rec[-1] rec[-3]
R 1 3
CX 0 1 2 3
M 1 3
DETECTOR rec[-2]
DETECTOR rec[-1]
M 0 2 4
OBSERVABLE_INCLUDE(0) rec[-1]
"""


def test_measure_then_reset_done_as_one_op(sg, monkeypatch):
    """Without the draws, an M followed by an R of the same qubits (directly,
    in another order; across the start of a loop; across its back edge) resets
    them itself and the R is skipped; an R of other qubits is not.  Events
    equal the oracle's and those of the program that keeps every op."""
    announce("measure then reset")
    (da, oa), (db, ob) = both_ways(sg, MEASURE_THEN_RESET, 13, 5000, monkeypatch)
    want = oracle.Circuit(MEASURE_THEN_RESET).sample(13, 0, 5000, det=True, obs=True, meas=False)
    assert np.array_equal(da, want["det"]) and np.array_equal(oa, want["obs"])
    assert np.array_equal(db, want["det"]) and np.array_equal(ob, want["obs"])
    assert np.count_nonzero(da) > 0


ZERO_ENTRY_ERROR = """R 0 1 2
X_ERROR(0.3) 0
REPEAT 4 {
    CX 0 1
    M 1
    DETECTOR rec[-1]
    R 0 1
    X_ERROR(0.1) 2
}
M 2
DETECTOR rec[-1]
"""

ZERO_AFTER_RESET = """REPEAT 5 {
    R 0 1 2
    S 0
    CX 0 1
    S_DAG 2
    X_ERROR(0.2) 0 1
    CZ 1 2
    M 0 1 2
    DETECTOR rec[-1]
    DETECTOR rec[-2]
    DETECTOR rec[-3]
}
"""


@pytest.mark.parametrize("name,text", [("error before the loop", ZERO_ENTRY_ERROR),
                                       ("Cliffords right after resets", ZERO_AFTER_RESET)])
def test_cliffords_on_zero_qubits(sg, name, text, monkeypatch):
    """Without the draws, a Clifford op whose qubits are zero in every shot is
    skipped.  A loop body starting with CX on a qubit that an error before
    the loop made nonzero must keep it on the first pass (the analysis meets
    the state before the loop with the state at the end of the body); ops
    right after a reset are skipped.  Events equal the oracle's and those of
    the program that keeps every op."""
    announce("zero qubits", name)
    (da, oa), (db, ob) = both_ways(sg, text, 21, 4000, monkeypatch)
    want = oracle.Circuit(text).sample(21, 0, 4000, det=True, obs=True, meas=False)
    assert np.array_equal(da, want["det"]) and np.array_equal(db, want["det"])
    assert np.count_nonzero(da) > 0
