"""Host-side tests of the C ABI (no GPU needed).

* The library loads and exports every function declared in include/stim_gpu.h.
* stim_compile / stim_circuit_shape / stim_reference_sample (host-only calls)
  agree with the oracle: shapes, and the canonical reference bit for bit.
* Error codes for malformed input and bad sampling arguments.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2103_02202_amd import stim_gpu as sg
from paper_2103_02202_amd import workloads as wl
from circuit_gen import random_circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "stim_gpu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stim_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "stim_frame_sample" in names and "stim_batch_sample" in names
    L = sg.lib()
    for name in names:
        assert hasattr(L, name), name


def unpack_ref(words, m):
    bits = np.array(words, dtype=np.uint64)
    return np.unpackbits(bits.view(np.uint8), bitorder="little")[:m] if m else np.zeros(0, np.uint8)


CASES = {
    "surface_d3": lambda: wl.surface_code(3, 3, 1e-3),
    "surface_d7": lambda: wl.surface_code(7, 7, 1e-3),
    "surface_d15": lambda: wl.surface_code(15, 15, 1e-3),
    "repetition": wl.repetition_code_example,
    "teleport": wl.teleportation_example,
    "random_clifford_64": lambda: wl.random_clifford(64, 40, seed=3),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_shape_and_reference_match_oracle(name):
    text = CASES[name]()
    c, o = sg.Circuit(text), oracle.Circuit(text)
    assert (c.num_qubits, c.num_measurements, c.num_detectors, c.num_observables, c.num_gate_targets) == \
        (o.num_qubits, o.num_measurements, o.num_detectors, o.num_observables, o.num_gate_targets)
    assert np.array_equal(unpack_ref(c.reference(), c.num_measurements), o.reference())


@pytest.mark.parametrize("seed", range(30))
def test_reference_matches_oracle_on_random_circuits(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(2, 40))
    text = random_circuit(n, int(rng.integers(20, 300)), seed=9000 + seed, noise=True)
    c, o = sg.Circuit(text), oracle.Circuit(text)
    assert np.array_equal(unpack_ref(c.reference(), c.num_measurements), o.reference())


@pytest.mark.parametrize("seed", range(20))
def test_reference_with_feedback_matches_oracle(seed):
    rng = np.random.Generator(np.random.PCG64(300 + seed))
    n = int(rng.integers(2, 30))
    text = random_circuit(n, int(rng.integers(20, 300)), seed=9500 + seed, noise=True, feedback=0.15)
    c, o = sg.Circuit(text), oracle.Circuit(text)
    assert (c.num_qubits, c.num_measurements, c.num_gate_targets) == \
        (o.num_qubits, o.num_measurements, o.num_gate_targets)
    assert np.array_equal(unpack_ref(c.reference(), c.num_measurements), o.reference())


def test_reference_with_feedback_inside_repeat_blocks():
    # The lookback is relative to each iteration's own measurements.
    text = "X 0\nREPEAT 5 {\n  M 0\n  CX rec[-1] 1\n  M 1\n  CX rec[-1] 1\n  X 0\n}\n"
    c, o = sg.Circuit(text), oracle.Circuit(text)
    want = o.reference()
    assert want.tolist() == [1, 1, 0, 0, 1, 1, 0, 0, 1, 1]
    assert np.array_equal(unpack_ref(c.reference(), c.num_measurements), want)


def test_surface_closed_form_counts():
    for d in (3, 5, 9):
        c = sg.Circuit(wl.surface_code(d, d, 1e-3))
        k = wl.surface_code_counts(d, d)
        assert (c.num_qubits, c.num_gate_targets, c.num_measurements, c.num_detectors) == \
            (k["num_qubits"], k["num_gate_targets"], k["num_measurements"], k["num_detectors"])


@pytest.mark.parametrize("text,code", [
    ("FOO 0", sg.STIM_E_UNSUPPORTED),
    ("H 0 x", sg.STIM_E_PARSE),
    ("CX 0", sg.STIM_E_PARSE),
    ("CX 2 2", sg.STIM_E_PARSE),
    ("REPEAT 0 {\nH 0\n}", sg.STIM_E_PARSE),
    ("REPEAT 3 {\nH 0", sg.STIM_E_PARSE),
    ("}", sg.STIM_E_PARSE),
    ("X_ERROR(1.5) 0", sg.STIM_E_PARSE),
    ("DEPOLARIZE1 0", sg.STIM_E_PARSE),
    ("M 0\nDETECTOR rec[-2]", sg.STIM_E_PARSE),
    ("H(0.5) 0", sg.STIM_E_PARSE),
    ("AMPLITUDE_DAMP(0.1) 0", sg.STIM_E_UNSUPPORTED),
    ("M 0\nCX 1 rec[-1]", sg.STIM_E_PARSE),
    ("M 0\nCY 1 rec[-1]", sg.STIM_E_PARSE),
    ("M 0 1\nCZ rec[-1] rec[-2]", sg.STIM_E_PARSE),
    ("CX rec[-1] 0", sg.STIM_E_PARSE),
    ("M 0\nCX rec[-2] 1", sg.STIM_E_PARSE),
    ("M 0\nCX rec[-0] 1", sg.STIM_E_PARSE),
    ("M 0\nH rec[-1]", sg.STIM_E_PARSE),
    ("M 0\nSWAP rec[-1] 1", sg.STIM_E_PARSE),
])
def test_compile_errors(text, code):
    with pytest.raises(sg.StimError) as e:
        sg.Circuit(text)
    assert e.value.code == code
    if code == sg.STIM_E_PARSE:
        assert "line" in str(e.value)


def test_sampling_argument_errors_need_no_gpu():
    c = sg.Circuit("M 0\n")
    L = sg.lib()
    h = ctypes.c_void_p(c.handle)
    # misaligned offset, zero shots and a null handle fail before any device work
    assert L.stim_frame_sample(h, 0, 3, 64, ctypes.c_void_p(1), None) == sg.STIM_E_INVALID_ARG
    assert L.stim_frame_sample(h, 0, 0, 0, ctypes.c_void_p(1), None) == sg.STIM_E_INVALID_ARG
    assert L.stim_frame_sample(None, 0, 0, 64, ctypes.c_void_p(1), None) == sg.STIM_E_INVALID_ARG
    assert L.stim_detector_sample(h, 0, 65, 64, None, None, None) == sg.STIM_E_INVALID_ARG
    assert L.stim_batch_sample(None, 1, None) == sg.STIM_E_INVALID_ARG


def test_sample_scratch_bytes(monkeypatch):
    """stim_sample_scratch_bytes: detector mode adds one flip row per
    measurement, sparse sampling allocates nothing per call, a noiseless
    circuit whose frame fits in LDS needs no scratch, and the noise records of
    one X_ERROR execution lie between the expected number of 64-shot words an
    error lands in and its reservation bound (at fewer than 512 words a tile
    is one word)."""
    monkeypatch.delenv("STIM_NOISE_PREPASS", raising=False)
    shots = 64 * 1000
    W = shots // 64
    noiseless = sg.Circuit("H 0\nCX 0 1\nM 0 1\n")
    assert noiseless.scratch_bytes(shots, "frame") == 0
    assert noiseless.scratch_bytes(shots, "detector") == 8 * W * 2
    p, n = 0.01, 4
    c = sg.Circuit(f"X_ERROR({p}) 0 1 2 3\nM 0 1 2 3\nDETECTOR rec[-1]\n")
    f, d, s = (c.scratch_bytes(shots, m) for m in ("frame", "detector", "sparse"))
    assert s == 0 and d - f == 8 * W * 4
    hit = 1 - (1 - p) ** 64
    lo = 16 * n * hit * W
    mu_hi = n * min(1.0, hit + 2 / 256)
    hi = 16 * W * (mu_hi + 6 * mu_hi ** 0.5 + 17) + 8 * W + 12
    assert lo <= f <= hi, (lo, f, hi)
    # More noise, more records; at the same tile width, twice the tiles take
    # twice the records and meta entries (plus the per-execution tables).
    assert sg.Circuit(f"X_ERROR(0.05) 0 1 2 3\nM 0 1 2 3\n").scratch_bytes(shots, "frame") > f
    assert c.scratch_bytes(64 * 400, "frame") - 12 == 2 * (c.scratch_bytes(64 * 200, "frame") - 12)
    # Wider tiles past 1,024 words: fewer records per word.
    assert c.scratch_bytes(2 * shots, "frame") < 2 * f
    monkeypatch.setenv("STIM_NOISE_PREPASS", "0")
    assert c.scratch_bytes(shots, "frame") == 0
    with pytest.raises(sg.StimError):
        sg.stim_sample_scratch_bytes(c.handle, shots, 3)
    with pytest.raises(sg.StimError):
        sg.stim_sample_scratch_bytes(0, shots, 0)             # no circuit
    assert c.scratch_bytes(0, "detector") == 0
