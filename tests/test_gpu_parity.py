"""GPU parity: the HIP sampler against the oracle, bit for bit (tolerance 0).

Every case names itself on stdout before touching the GPU.  Sizes span several
tiles and ragged tails; large configurations are checked on sampled shot
slices the oracle computes alone (exact, because random bits are keyed by
absolute shot).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2103_02202_amd import workloads as wl
from circuit_gen import random_circuit

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


def gpu_meas(sg, c, seed, shots, offset=0):
    out = c.sample(seed, shots, shot_offset=offset)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


def gpu_det(sg, c, seed, shots, offset=0):
    det, obs = c.detect(seed, shots, shot_offset=offset)
    torch.cuda.synchronize()
    return det.cpu().numpy().view(np.uint64), obs.cpu().numpy().view(np.uint64)


def check_meas(sg, text, seed, shots, offset=0):
    c = sg.Circuit(text)
    o = oracle.Circuit(text)
    got = gpu_meas(sg, c, seed, shots, offset)
    want = o.sample(seed, offset, shots, meas=True)["meas"]
    assert got.shape == want.shape
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"first mismatch at (measurement, word) {bad[0].tolist()}"


def check_det(sg, text, seed, shots, offset=0):
    c = sg.Circuit(text)
    o = oracle.Circuit(text)
    det, obs = gpu_det(sg, c, seed, shots, offset)
    want = o.sample(seed, offset, shots, det=True, obs=True, meas=False)
    assert np.array_equal(det, want["det"])
    assert np.array_equal(obs, want["obs"])


@pytest.mark.parametrize("shots", [1024, 1000, 1, 65, 4097])
def test_surface_d3_measurements(sg, shots):
    announce("surface d3", shots)
    check_meas(sg, wl.surface_code(3, 3, 1e-3), 0, shots)


def test_surface_d3_detectors(sg):
    announce("surface d3 detectors")
    check_det(sg, wl.surface_code(3, 3, 1e-3), 0, 1024)


@pytest.mark.parametrize("p", [1e-3, 1e-2, 0.2])
def test_surface_d5_high_noise(sg, p):
    announce("surface d5", p)
    text = wl.surface_code(5, 5, p)
    check_meas(sg, text, 7, 3000)
    check_det(sg, text, 7, 3000)


@pytest.mark.parametrize("seed", range(24))
def test_random_noisy_circuits(sg, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(2, 60))
    text = random_circuit(n, int(rng.integers(20, 250)), seed=7000 + seed, noise=True,
                          p=float(rng.choice([1e-3, 0.05, 0.5, 1.0])))
    shots = int(rng.integers(1, 5000))
    announce("random", seed, n, shots)
    check_meas(sg, text, seed, shots)


def test_paper_examples(sg):
    announce("appendix examples")
    check_meas(sg, wl.repetition_code_example(), 3, 1024)
    check_meas(sg, wl.teleportation_example(), 3, 2048)


def test_repeat_nesting_and_annotations(sg):
    announce("nested repeat")
    text = ("H 0 1\nTICK\nREPEAT 3 {\n  DEPOLARIZE1(0.1) 0 1 2\n  REPEAT 2 {\n    CX 0 1 1 2\n    TICK\n"
            "    X_ERROR(0.2) 2\n  }\n  MR 2\n  DETECTOR rec[-1]\n  M 0 0\n}\nM 0 1 2\n"
            "OBSERVABLE_INCLUDE(1) rec[-1] rec[-2]\n")
    check_meas(sg, text, 11, 777)
    check_det(sg, text, 11, 777)


def test_shot_offset_slices(sg):
    announce("shot offsets")
    text = wl.surface_code(5, 3, 0.01)
    for off, shots in [(64, 100), (4096, 64), (1 << 20, 3000), ((1 << 40) + 128, 500)]:
        check_meas(sg, text, 5, shots, off)


@pytest.mark.parametrize("tile,placement", [("1", "lds"), ("4", "lds"), ("32", "lds"),
                                            ("2", "global"), ("16", "global")])
def test_tiling_does_not_change_results(sg, tile, placement, monkeypatch):
    announce("tiling", tile, placement)
    monkeypatch.setenv("STIM_TILE_WORDS", tile)
    monkeypatch.setenv("STIM_FRAME_PLACEMENT", placement)
    text = wl.surface_code(5, 5, 0.01)
    check_meas(sg, text, 2, 5000)
    check_det(sg, text, 2, 5000)


@pytest.mark.parametrize("prepass", ["0", "1"])
@pytest.mark.parametrize("p", [1e-4, 1e-3, 3e-2, 0.3])
def test_noise_prepass_and_inline_agree_with_oracle(sg, prepass, p, monkeypatch):
    """Noise drawn by the pre-pass (records) or inline in the walker; high p
    overflows the records and falls back to the inline path per op."""
    announce("noise path", prepass, p)
    monkeypatch.setenv("STIM_NOISE_PREPASS", prepass)
    text = wl.surface_code(7, 4, p)
    check_meas(sg, text, 13, 6000)
    check_det(sg, text, 13, 6000)


def test_surface_d15_slices_of_full_run(sg):
    """d=15, 2^20 shots (the full configuration) on the GPU; slices checked by
    the oracle, everything checked for all-zero tails."""
    announce("surface d15 full")
    text = wl.surface_code(15, 15, 1e-3)
    c = sg.Circuit(text)
    o = oracle.Circuit(text)
    shots = 1 << 20
    full = c.sample(0, shots)
    det, obs = c.detect(0, shots)
    torch.cuda.synchronize()
    for w0 in (0, 5000, 16383):
        sl = full[:, w0:w0 + 1].cpu().numpy().view(np.uint64)
        want = o.sample(0, 64 * w0, 64, meas=True, det=True, obs=True)
        assert np.array_equal(sl, want["meas"])
        assert np.array_equal(det[:, w0:w0 + 1].cpu().numpy().view(np.uint64), want["det"])
        assert np.array_equal(obs[:, w0:w0 + 1].cpu().numpy().view(np.uint64), want["obs"])


def test_surface_d49_noiseless_detectors_zero_and_noisy_slices(sg):
    announce("surface d49")
    shots = 65536
    c0 = sg.Circuit(wl.surface_code(49, 49, 0.0))
    det, obs = c0.detect(0, shots)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(det)) == 0
    assert int(torch.count_nonzero(obs)) == 0
    text = wl.surface_code(49, 49, 1e-3)
    c = sg.Circuit(text)
    o = oracle.Circuit(text)
    full = c.sample(0, shots)
    torch.cuda.synchronize()
    for w0 in (0, 777):
        sl = full[:, w0:w0 + 1].cpu().numpy().view(np.uint64)
        want = o.sample(0, 64 * w0, 64, meas=True)["meas"]
        assert np.array_equal(sl, want)


def test_determinism_run_twice(sg):
    announce("determinism")
    c = sg.Circuit(wl.surface_code(9, 9, 5e-3))
    a = gpu_meas(sg, c, 4, 20000)
    b = gpu_meas(sg, c, 4, 20000)
    assert np.array_equal(a, b)


def test_device_pointer_validation(sg):
    announce("pointer validation")
    import ctypes
    c = sg.Circuit("M 0\n")
    host = np.zeros(4, dtype=np.uint64)
    rc = sg.lib().stim_frame_sample(ctypes.c_void_p(c.handle), 0, 0, 64,
                                    ctypes.c_void_p(host.ctypes.data), None)
    assert rc == sg.STIM_E_INVALID_ARG


def test_kernel_timing_counts_passes_and_keeps_results(sg):
    text = wl.surface_code(5, 5, 1e-2)
    announce("kernel timing, d=5 p=1e-2 4096 shots")
    c = sg.Circuit(text)
    base = gpu_meas(sg, c, 3, 4096)
    sg.stim_kernel_timing(True)
    try:
        timed = gpu_meas(sg, c, 3, 4096)
        gpu_meas(sg, c, 3, 4096)
        gen_ms, frame_ms, passes = sg.stim_kernel_times()
        assert passes == 2
        assert gen_ms > 0 and frame_ms > 0
        assert sg.stim_kernel_times()[2] == 0            # read-out discards
    finally:
        sg.stim_kernel_timing(False)
    assert (timed == base).all()


@pytest.mark.parametrize("tile,slots,threads", [(1, 3, "256"), (2, 2, "512"), (4, 1, "1024")])
def test_global_frame_workgroups_take_tiles_in_turn(sg, tile, slots, threads, monkeypatch):
    """A global frame walked by fewer workgroups than tiles: each workgroup
    reuses its scratch slot for several tiles."""
    text = wl.surface_code(5, 4, 2e-2)
    shots = 64 * 23 + 5
    announce("global slots", tile, slots, threads, shots)
    monkeypatch.setenv("STIM_TILE_WORDS", str(tile))
    monkeypatch.setenv("STIM_FRAME_PLACEMENT", "global")
    monkeypatch.setenv("STIM_FRAME_SLOTS", str(slots))
    monkeypatch.setenv("STIM_FRAME_THREADS", threads)
    check_meas(sg, text, 21, shots)
    check_det(sg, text, 21, shots)


# --- classically controlled Paulis (Sec. 3, tracking corrections) ----------

@pytest.mark.parametrize("seed", range(16))
def test_random_feedback_circuits(sg, seed):
    rng = np.random.Generator(np.random.PCG64(500 + seed))
    n = int(rng.integers(2, 50))
    text = random_circuit(n, int(rng.integers(20, 250)), seed=8000 + seed, noise=True,
                          p=float(rng.choice([1e-3, 0.05, 0.5])), feedback=0.15)
    shots = int(rng.integers(1, 5000))
    announce("random feedback", seed, n, shots)
    check_meas(sg, text, seed, shots)


def test_feedback_teleportation_and_deterministic_cases(sg):
    announce("feedback teleportation")
    for prep, undo in [("H 0\nS 0", "S_DAG 2\nH 2"), ("X 0\nH 0", "H 2\nX 2")]:
        text = f"{prep}\nH 1\nCX 1 2\nCX 0 1\nH 0\nM 0 1\nCX rec[-1] 2\nCZ 2 rec[-2]\n{undo}\nM 2\n"
        check_meas(sg, text, 1, 3000)
        c = sg.Circuit(text)
        assert int(torch.count_nonzero(c.sample(1, 3000)[2])) == 0
    for text in ["X 0\nM 0\nH 1\nCY rec[-1] 1\nH 1\nM 1\n", "X_ERROR(1) 0\nM 0\nH 1\nCY rec[-1] 1\nH 1\nM 1\n",
                 "X 0\nM 0 1\nCX rec[-2] 2 rec[-1] 3 2 3\nM 2 3\n"]:
        check_meas(sg, text, 2, 700)


@pytest.mark.parametrize("tile,placement", [("1", "lds"), ("4", "lds"), ("2", "global"), ("16", "global")])
def test_feedback_reset_surface_code_tilings(sg, tile, placement, monkeypatch):
    announce("feedback surface d5", tile, placement)
    monkeypatch.setenv("STIM_TILE_WORDS", tile)
    monkeypatch.setenv("STIM_FRAME_PLACEMENT", placement)
    text = wl.surface_code(5, 5, 0.01, feedback_reset=True)
    check_meas(sg, text, 4, 5000)
    check_det(sg, text, 4, 5000)


def test_feedback_reset_surface_d15(sg):
    """d=15 with feedback resets: noiseless detectors are all zero at 2^16
    shots; noisy slices of a 2^18-shot run match the oracle."""
    announce("feedback surface d15")
    c0 = sg.Circuit(wl.surface_code(15, 15, 0.0, feedback_reset=True))
    det, obs = c0.detect(0, 1 << 16)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(det)) == 0 and int(torch.count_nonzero(obs)) == 0
    text = wl.surface_code(15, 15, 1e-3, feedback_reset=True)
    c, o = sg.Circuit(text), oracle.Circuit(text)
    full = c.sample(3, 1 << 18)
    det, obs = c.detect(3, 1 << 18)
    torch.cuda.synchronize()
    for w0 in (0, 1234, 4095):
        want = o.sample(3, 64 * w0, 64, meas=True, det=True, obs=True)
        assert np.array_equal(full[:, w0:w0 + 1].cpu().numpy().view(np.uint64), want["meas"])
        assert np.array_equal(det[:, w0:w0 + 1].cpu().numpy().view(np.uint64), want["det"])
        assert np.array_equal(obs[:, w0:w0 + 1].cpu().numpy().view(np.uint64), want["obs"])


def test_feedback_lookback_across_repeat_iterations(sg):
    """Controls that reach into the previous iteration of a REPEAT block."""
    announce("feedback across iterations")
    text = ("M 0 1\nREPEAT 7 {\n  H 0\n  DEPOLARIZE1(0.2) 0 1\n  M 0 1\n  CX rec[-3] 2 rec[-4] 1\n"
            "  CZ 0 rec[-2]\n  M 2\n  X_ERROR(0.1) 2\n}\nM 0 1 2\n")
    for tile, placement in [("1", "lds"), ("2", "global")]:
        import os
        os.environ["STIM_TILE_WORDS"], os.environ["STIM_FRAME_PLACEMENT"] = tile, placement
        try:
            check_meas(sg, text, 3, 3000)
        finally:
            del os.environ["STIM_TILE_WORDS"], os.environ["STIM_FRAME_PLACEMENT"]


# Controlled Paulis whose result is a plain M of the same qubit, untouched
# since, take the flip from the qubit's frame instead of the stored record;
# everything else reads the record.  Each case against the oracle, with noise
# before the measurement so that flips are frequent.
LOCALITY_CASES = {
    "local_x": "X_ERROR(0.3) 0\nM 0\nCX rec[-1] 0\nM 0\n",
    "local_y": "H 0\nX_ERROR(0.3) 0\nM 0\nCY rec[-1] 0\nH 0\nM 0\n",
    "local_z": "X_ERROR(0.3) 0\nM 0\nCZ rec[-1] 0\nH 0\nM 0\n",
    "double_measure": "X_ERROR(0.3) 0\nM 0 0\nCX rec[-2] 0\nM 0\n",
    "pauli_gate_between": "X_ERROR(0.3) 0\nM 0\nX 0\nCX rec[-1] 0\nM 0\n",
    "noise_between": "X_ERROR(0.3) 0\nM 0\nX_ERROR(0.4) 0\nCX rec[-1] 0\nM 0\n",
    "clifford_between": "X_ERROR(0.3) 0 1\nM 0\nCX 1 0\nCX rec[-1] 0\nM 0 1\n",
    "earlier_pair_same_line": "X_ERROR(0.3) 0 1\nM 0\nCX 1 0 rec[-1] 0\nM 0 1\n",
    "later_pair_same_line": "X_ERROR(0.3) 0 1\nM 0\nCX rec[-1] 0 1 0\nM 0 1\n",
    "mr_source": "X_ERROR(0.3) 0\nMR 0\nX_ERROR(0.3) 0\nCX rec[-1] 0\nM 0\n",
    "other_qubit": "X_ERROR(0.3) 0\nM 0\nCX rec[-1] 1\nM 0 1\n",
    "mixed_op": "X_ERROR(0.3) 0 1 2\nM 0 1\nX_ERROR(0.2) 1\nCX rec[-2] 0 rec[-1] 1 rec[-2] 2\nM 0 1 2\n",
    "loop_local_then_not": ("X_ERROR(0.3) 0 1\nM 0\nREPEAT 5 {\n  CX rec[-1] 0\n  X_ERROR(0.2) 0 1\n  M 1 0\n"
                            "  CX 0 1\n}\nM 0 1\n"),
}


@pytest.mark.parametrize("name", sorted(LOCALITY_CASES))
def test_feedback_local_and_global_pairs(sg, name):
    announce("feedback locality", name)
    check_meas(sg, LOCALITY_CASES[name], 21, 64 * 37 + 5)


def test_feedback_reset_surface_d49_sampled_slices(sg):
    """The feedback-reset d=49 workload at the benchmark's size (65,536
    shots, local controlled pairs throughout), checked on sampled words of
    the record and of the detection events."""
    announce("feedback reset d49")
    shots = 65536
    text = wl.surface_code(49, 49, 1e-3, feedback_reset=True)
    c = sg.Circuit(text)
    o = oracle.Circuit(text)
    full = c.sample(5, shots)
    det, obs = c.detect(5, shots)
    torch.cuda.synchronize()
    for w0 in (3, 1000):
        want = o.sample(5, 64 * w0, 64, meas=True, det=True, obs=True)
        assert np.array_equal(full[:, w0:w0 + 1].cpu().numpy().view(np.uint64), want["meas"])
        assert np.array_equal(det[:, w0:w0 + 1].cpu().numpy().view(np.uint64), want["det"])
        assert np.array_equal(obs[:, w0:w0 + 1].cpu().numpy().view(np.uint64), want["obs"])
