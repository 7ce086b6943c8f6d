"""Detection events formed inside the frame walk (STIM_WALK_EVENTS=1: the walk
keeps its recent measurement flips in a per-workgroup ring and writes event
and observable rows itself), against the oracle bit for bit, and against the
default flip-record path (flip record written out, events formed by a second
kernel).

The circuits put detectors of 0 to 5 lookbacks (repeats and empty detectors
included) and repeated observable includes inside REPEAT blocks, so the ring
wraps many times; tile widths, both frame placements, slot caps that make a
workgroup take several tiles in turn, ragged shot counts and shot offsets are
varied.
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


@pytest.fixture(autouse=True)
def walk_events(monkeypatch):
    monkeypatch.setenv("STIM_WALK_EVENTS", "1")


@pytest.fixture(scope="module")
def sg():
    from paper_2103_02202_amd import stim_gpu
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    stim_gpu.lib()
    return stim_gpu


def gpu_events(c, seed, shots, offset=0):
    det, obs = c.detect(seed, shots, shot_offset=offset)
    torch.cuda.synchronize()
    return det.cpu().numpy().view(np.uint64), obs.cpu().numpy().view(np.uint64)


def check(sg, text, seed, shots, offset=0):
    c, o = sg.Circuit(text), oracle.Circuit(text)
    det, obs = gpu_events(c, seed, shots, offset)
    want = o.sample(seed, offset, shots, det=True, obs=True, meas=False)
    bad = np.argwhere(det != want["det"])
    assert bad.size == 0, f"first event mismatch at (detector, word) {bad[0].tolist()}"
    bad = np.argwhere(obs != want["obs"])
    assert bad.size == 0, f"first observable mismatch at (observable, word) {bad[0].tolist()}"
    return det, obs


@pytest.mark.parametrize("seed", range(16))
def test_random_detector_circuits(sg, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(3, 40))
    text = random_detector_circuit(n, int(rng.integers(30, 160)), seed=9100 + seed,
                                   p=float(rng.choice([1e-3, 0.02, 0.3])), reps=int(rng.integers(1, 12)),
                                   feedback=0.05 if seed % 3 == 0 else 0.0)
    shots = int(rng.integers(1, 6000))
    announce("random detectors", seed, n, shots)
    check(sg, text, seed, shots)


@pytest.mark.parametrize("tile,placement", [("1", "lds"), ("2", "lds"), ("8", "lds"), ("32", "lds"),
                                            ("1", "global"), ("4", "global")])
def test_tilings_with_events_in_the_walk(sg, tile, placement, monkeypatch):
    announce("walk events tiling", tile, placement)
    monkeypatch.setenv("STIM_TILE_WORDS", tile)
    monkeypatch.setenv("STIM_FRAME_PLACEMENT", placement)
    check(sg, random_detector_circuit(20, 120, seed=77, reps=9, feedback=0.05), 5, 9000)
    check(sg, wl.surface_code(5, 7, 0.02), 6, 4500, offset=128)


@pytest.mark.parametrize("slots", ["1", "3", "7"])
def test_workgroups_taking_tiles_in_turn(sg, slots, monkeypatch):
    """Fewer ring slots than tiles: each workgroup reuses its ring for tile
    after tile."""
    announce("walk events slots", slots)
    monkeypatch.setenv("STIM_WALK_EVENT_SLOTS", slots)
    monkeypatch.setenv("STIM_TILE_WORDS", "1")
    check(sg, random_detector_circuit(16, 100, seed=31, reps=6), 2, 64 * 23 + 5)
    check(sg, wl.surface_code(3, 5, 0.05), 3, 64 * 40)


def test_flip_record_path_gives_the_same_bits(sg, monkeypatch):
    """The flip-record path and the walk's events agree on surface codes with
    feedback resets and on random circuits, at offsets."""
    cases = [(wl.surface_code(7, 7, 0.01), 1, 20000, 0),
             (wl.surface_code(5, 9, 0.003, feedback_reset=True), 4, 7000, 64 * 5),
             (random_detector_circuit(30, 200, seed=5, reps=15, feedback=0.05), 8, 3333, 1 << 30)]
    for i, (text, seed, shots, off) in enumerate(cases):
        announce("walk events vs flip record", i)
        c = sg.Circuit(text)
        monkeypatch.setenv("STIM_WALK_EVENTS", "1")
        a = gpu_events(c, seed, shots, off)
        monkeypatch.setenv("STIM_WALK_EVENTS", "0")
        b = gpu_events(c, seed, shots, off)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), f"case {i}"


def test_observables_not_requested_and_detector_only(sg):
    """out_obs = NULL skips the observable ops; a circuit with detectors and
    no observables, and one with observables only."""
    announce("walk events: obs NULL, detector-only, observable-only")
    text = random_detector_circuit(10, 80, seed=12, reps=5)
    c, o = sg.Circuit(text), oracle.Circuit(text)
    shots = 3000
    W = (shots + 63) // 64
    det = torch.full((c.num_detectors, W), -1, dtype=torch.int64, device="cuda")
    sg.stim_detector_sample(c.handle, 4, 0, shots, det, None)
    torch.cuda.synchronize()
    want = o.sample(4, 0, shots, det=True, obs=True, meas=False)
    assert np.array_equal(det.cpu().numpy().view(np.uint64), want["det"])
    check(sg, "X_ERROR(0.3) 0 1\nM 0 1\nDETECTOR rec[-1] rec[-2]\nREPEAT 3 {\n  X_ERROR(0.1) 0\n  M 0\n"
              "  DETECTOR rec[-1] rec[-3]\n}\n", 2, 999)
    check(sg, "X_ERROR(0.3) 0 1\nM 0 1\nOBSERVABLE_INCLUDE(1) rec[-1]\nOBSERVABLE_INCLUDE(1) rec[-2]\n", 3, 777)
