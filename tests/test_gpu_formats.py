"""GPU parity of the shot-major output formats against the oracle's (byte for byte)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import formats as F
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


def random_table(rng, rows, shots, density):
    W = (shots + 63) // 64
    if rows == 0:
        return np.zeros((0, W), dtype=np.uint64)
    bits = rng.random((rows, W * 64)) < density
    bits[:, shots:] = False                     # tail bits of the last word are zero, as the samplers write
    words = np.packbits(bits.reshape(rows, W, 64), axis=2, bitorder="little").view(np.uint64).reshape(rows, W)
    return words


def check(sg, words, rows, shots, fmt):
    want = F.format_shots(words, rows, shots, fmt)
    t = torch.from_numpy(words.view(np.int64).copy()).cuda() if rows else torch.zeros(1, dtype=torch.int64).cuda()
    got = sg.format_shots(t, rows, shots, fmt)
    torch.cuda.synchronize()
    got = bytes(got.cpu().numpy().tobytes())
    assert len(got) == len(want), (fmt, len(got), len(want))
    if got != want:
        i = next(k for k in range(len(want)) if got[k] != want[k])
        raise AssertionError(f"{fmt}: first differing byte {i}: {got[max(0, i - 8):i + 8]!r} vs {want[max(0, i - 8):i + 8]!r}")


@pytest.mark.parametrize("fmt", ["01", "b8", "hits", "r8"])
@pytest.mark.parametrize("rows,shots,density", [(0, 5, 0.0), (1, 1, 0.5), (7, 70, 0.5), (64, 64, 0.3), (65, 200, 0.1),
                                                (130, 1000, 0.02), (300, 777, 0.001), (600, 129, 0.0),
                                                (1000, 300, 1.0), (70, 3000, 0.05), (4001, 333, 0.3),
                                                # b8 rows of a multiple of 4 bytes (written by the transpose)
                                                (32, 999, 0.2), (224, 64, 0.5), (256, 130, 0.1),
                                                (800, 257, 0.05), (2080, 1100, 0.01)])
def test_random_tables(sg, fmt, rows, shots, density):
    announce("formats random", fmt, rows, shots, density)
    rng = np.random.default_rng(rows * 1000 + shots)
    check(sg, random_table(rng, rows, shots, density), rows, shots, fmt)


@pytest.mark.parametrize("fmt", ["01", "b8", "hits", "r8"])
def test_sampler_outputs(sg, fmt):
    text = wl.surface_code(5, 5, 1e-2)
    announce("formats of sampler output d=5", fmt)
    c = sg.Circuit(text)
    shots = 1000
    meas = c.sample(7, shots)
    det, obs = c.detect(7, shots)
    torch.cuda.synchronize()
    for t, rows in ((meas, c.num_measurements), (det, c.num_detectors), (obs, c.num_observables)):
        words = t.cpu().numpy().view(np.uint64)
        check(sg, words, rows, shots, fmt)


def test_size_query_and_errors(sg):
    announce("formats size query and errors")
    rng = np.random.default_rng(5)
    words = random_table(rng, 10, 100, 0.2)
    t = torch.from_numpy(words.view(np.int64).copy()).cuda()
    for fmt in ("01", "b8", "hits", "r8"):
        n = sg.stim_format_shots(t, 10, 100, fmt)
        assert n == len(F.format_shots(words, 10, 100, fmt))
        small = torch.empty(max(n - 1, 1), dtype=torch.uint8, device="cuda")
        with pytest.raises(sg.StimError):
            sg.stim_format_shots(t, 10, 100, fmt, small)
    with pytest.raises(sg.StimError):
        sg.stim_format_shots(t, 10, 0, "b8")
    with pytest.raises(sg.StimError):
        sg.stim_format_shots(t, 10, 100, 9)
