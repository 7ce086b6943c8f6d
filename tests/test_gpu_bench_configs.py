"""The configurations the benchmark times, checked against the oracle at their
full sizes and launch configurations.

Random bits are keyed by absolute shot, so the oracle computes any shot slice
alone: each check samples the whole configuration on the GPU and compares
chosen 64-shot words (the first and the last word, both words of one tile,
interior tiles) with the oracle's sample of the same shots, bit for bit.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2103_02202_amd import workloads as wl

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


def words(t, w0, k):
    return t[:, w0:w0 + k].cpu().numpy().view(np.uint64)


def check_slices(o, ref, seed, spans, meas=None, det=None, obs=None):
    """Compares the GPU tables on each (first word, words) span with the
    oracle's sample of the same shots."""
    for w0, k in spans:
        want = o.sample(seed, 64 * w0, 64 * k, ref=ref, meas=meas is not None, det=det is not None,
                        obs=obs is not None)
        if meas is not None:
            got = words(meas, w0, k)
            bad = np.argwhere(got != want["meas"])
            assert bad.size == 0, f"record words [{w0}, {w0 + k}): first mismatch (row, word) {bad[0].tolist()}"
        if det is not None:
            got = words(det, w0, k)
            bad = np.argwhere(got != want["det"])
            assert bad.size == 0, f"event words [{w0}, {w0 + k}): first mismatch (row, word) {bad[0].tolist()}"
        if obs is not None:
            assert np.array_equal(words(obs, w0, k), want["obs"]), f"observable words [{w0}, {w0 + k})"


def test_d49_headline_step_detection_events_and_observable(sg):
    """The benchmark's step: d=49, 49 rounds, p=1e-3, seed 0, 65,536 shots,
    detection events and the observable (stim_detector_sample, tile width 2),
    then the measurement record of the same run (stim_frame_sample)."""
    announce("d49 headline, 65536 shots, detector + measurement mode")
    text = wl.surface_code(49, 49, 1e-3)
    c, o = sg.Circuit(text), oracle.Circuit(text)
    shots = 65536
    W = shots // 64
    det = torch.empty((c.num_detectors, W), dtype=torch.int64, device="cuda")
    obs = torch.empty((max(c.num_observables, 1), W), dtype=torch.int64, device="cuda")
    sg.stim_detector_sample(c.handle, 0, 0, shots, det, obs)
    meas = c.sample(0, shots)
    torch.cuda.synchronize()
    ref = o.reference()
    assert np.array_equal(np.packbits(ref, bitorder="little").view(np.uint8)[: (len(ref) + 7) // 8],
                          np.frombuffer(np.array(c.reference(), dtype=np.uint64).tobytes(),
                                        dtype=np.uint8)[: (len(ref) + 7) // 8])
    spans = [(0, 1), (300, 1), (512, 2), (777, 1), (1023, 1)]
    check_slices(o, ref, 0, spans, meas=meas, det=det, obs=obs[: c.num_observables])
    # Some events fire at p = 1e-3 (a table of zeros would pass the slices).
    assert int(torch.count_nonzero(det[:, :8])) > 0


def test_d49_262144_shots_slices(sg):
    """d=49 at 262,144 shots: a 315 MB frame, a 3.9 GB record."""
    announce("d49, 262144 shots, detector + measurement mode")
    text = wl.surface_code(49, 49, 1e-3)
    c, o = sg.Circuit(text), oracle.Circuit(text)
    shots = 1 << 18
    det, obs = c.detect(0, shots)
    torch.cuda.synchronize()
    ref = o.reference()
    spans = [(0, 1), (2048, 2), (3001, 1), (4095, 1)]
    check_slices(o, ref, 0, spans, det=det, obs=obs)
    del det, obs
    torch.cuda.empty_cache()
    meas = c.sample(0, shots)
    torch.cuda.synchronize()
    check_slices(o, ref, 0, spans, meas=meas)


def test_d101_global_frame_walk_slices(sg):
    """d=101 (20,401 qubits): the frame does not fit in LDS, so the walk keeps
    it in global memory slots reused by about one workgroup per CU, at the
    tile width the sampler picks for 2^17 shots (8 words).  The canonical
    reference of this Z-memory circuit is all zeros (a closed form the oracle's
    reference tests pin on smaller distances); the GPU's reference must be that
    too, and the oracle samples with it."""
    announce("d101, 131072 shots, global frame, measurement + detector mode")
    text = wl.surface_code(101, 101, 1e-3)
    c, o = sg.Circuit(text), oracle.Circuit(text)
    shots = 1 << 17
    meas = c.sample(3, shots)
    torch.cuda.synchronize()
    assert not np.any(np.array(c.reference(), dtype=np.uint64)), "canonical d=101 reference is not all zeros"
    ref = np.zeros(c.num_measurements, dtype=np.uint8)
    spans = [(0, 1), (8, 8), (1000, 1), (2047, 1)]
    check_slices(o, ref, 3, spans, meas=meas)
    del meas
    torch.cuda.empty_cache()
    det, obs = c.detect(3, shots)
    torch.cuda.synchronize()
    check_slices(o, ref, 3, [(0, 1), (1000, 1), (2047, 1)], det=det, obs=obs)


def test_full_batch_mix_against_single_calls_and_oracle(sg):
    """The benchmark's 64-circuit batch at its real shot counts: every request
    of the persistent launch equals its single call on the first submission
    (one launch), the second (tuned and graph-captured) and a replay, with
    both outputs of every request poisoned before each submission; two
    interior words of every request equal the oracle's (stored as digests by
    tests/golden/make_batch_mix_digests.py, which calls only the oracle: its
    reference sample of the ~500-qubit random circuits takes minutes)."""
    announce("full 64-circuit batch mix")
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch_mix_oracle_words.json")))
    mix = wl.batch_mix(seed=0)
    assert len(golden["requests"]) == len(mix)
    circs, reqs, singles = [], [], []
    for m in mix:
        c = sg.Circuit(m["text"])
        circs.append(c)
        W = (m["shots"] + 63) // 64
        if m["kind"] == "surface":
            out0 = torch.full((c.num_detectors, W), -1, dtype=torch.int64, device="cuda")
            out1 = torch.full((max(c.num_observables, 1), W), -1, dtype=torch.int64, device="cuda")
            mode = 1
            d, ob = c.detect(m["seed"], m["shots"])
            singles.append((d, ob))
        else:
            out0 = torch.full((c.num_measurements, W), -1, dtype=torch.int64, device="cuda")
            out1, mode = None, 0
            singles.append((c.sample(m["seed"], m["shots"]), None))
        reqs.append({"handle": c.handle, "seed": m["seed"], "shot_offset": 0, "num_shots": m["shots"],
                     "mode": mode, "out0": out0, "out1": out1})
    torch.cuda.synchronize()
    for submission in range(3):
        announce("batch submission", submission)
        for r in reqs:
            r["out0"].fill_(-1)
            if r["out1"] is not None:
                r["out1"].fill_(-1)
        sg.stim_batch_sample(reqs)
        torch.cuda.synchronize()
        for i, (r, c, (a, b)) in enumerate(zip(reqs, circs, singles)):
            assert torch.equal(r["out0"], a), f"submission {submission}: request {i} differs from its single call"
            if b is not None and c.num_observables:
                assert torch.equal(r["out1"][: c.num_observables], b), f"submission {submission}: request {i} obs"
    for i, (m, r, c, g) in enumerate(zip(mix, reqs, circs, golden["requests"])):
        assert (g["kind"], g["shots"], g["seed"]) == (m["kind"], m["shots"], m["seed"])
        w0, k = g["w0"], g["words"]
        if r["mode"] == 1:
            assert digest(words(r["out0"], w0, k)) == g["det_sha256"], f"request {i}: events differ from the oracle"
            assert digest(words(r["out1"][: c.num_observables], w0, k)) == g["obs_sha256"], f"request {i}: obs"
        else:
            assert digest(words(r["out0"], w0, k)) == g["meas_sha256"], f"request {i}: record differs from the oracle"


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()
