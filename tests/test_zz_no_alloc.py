"""stim_detector_sample_noalloc: the allocation-free variant of
stim_detector_sample (its flip table and frame slots live in the library's
static device scratch).  Called through the C ABI, it must give the same
events and observables as stim_detector_sample, bit for bit, on two calls in a
row (the second smaller, so that stale scratch from the first would show)."""
import ctypes

import pytest

from paper_2103_02202_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def announce(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def sg():
    from paper_2103_02202_amd import stim_gpu
    assert torch.cuda.is_available()
    stim_gpu.lib()
    return stim_gpu


def noalloc(sg, c, seed, shots, offset=0, obs=True):
    W = (shots + 63) // 64
    det = torch.full((c.num_detectors, W), -1, dtype=torch.int64, device="cuda")
    o = torch.full((max(c.num_observables, 1), W), -1, dtype=torch.int64, device="cuda") if obs else None
    rc = sg.lib().stim_detector_sample_noalloc(ctypes.c_void_p(c.handle), seed, offset, shots,
                                               ctypes.c_void_p(det.data_ptr()),
                                               ctypes.c_void_p(o.data_ptr() if o is not None else None),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, det, o


@pytest.mark.parametrize("text,calls", [
    (wl.surface_code(7, 7, 5e-3), [(3, 64 * 301 + 17, 0), (4, 64 * 40 + 3, 128)]),
    (wl.surface_code(15, 15, 1e-3), [(0, 1 << 16, 0), (1, 5000, 64)]),
    # frame too large for LDS: global frame slots in the scratch as well
    (wl.surface_code(75, 3, 1e-3), [(2, 4096, 0), (5, 700, 0)]),
], ids=["d7", "d15", "d75_global_frame"])
def test_noalloc_equals_detector_sample_on_two_calls(sg, text, calls):
    c = sg.Circuit(text)
    announce("noalloc", c.num_qubits, calls)
    c.detect(0, 64)                       # an allocating call uploads the circuit
    torch.cuda.synchronize()
    for seed, shots, offset in calls:
        rc, det, obs = noalloc(sg, c, seed, shots, offset)
        torch.cuda.synchronize()
        assert rc == sg.STIM_OK, sg.lib().stim_last_error().decode()
        want_det, want_obs = c.detect(seed, shots, shot_offset=offset)
        torch.cuda.synchronize()
        assert torch.equal(det, want_det), f"events differ (seed {seed}, {shots} shots)"
        assert torch.equal(obs[: c.num_observables], want_obs), f"observables differ (seed {seed})"


def test_noalloc_refuses_what_it_cannot_serve(sg):
    announce("noalloc refusals")
    c = sg.Circuit(wl.surface_code(5, 5, 1e-3))
    # not yet resident on the device: refused, nothing launched
    rc, _, _ = noalloc(sg, c, 0, 1000)
    assert rc == sg.STIM_E_INVALID_ARG
    assert "resident" in sg.lib().stim_last_error().decode()
    c.detect(0, 64)
    torch.cuda.synchronize()
    # more scratch than the array holds: refused with the size in the message
    big = sg.Circuit(wl.surface_code(15, 15, 1e-3))
    big.detect(0, 64)
    torch.cuda.synchronize()
    W = (1 << 20) // 64
    det = torch.empty((big.num_detectors, W), dtype=torch.int64, device="cuda")
    rc = sg.lib().stim_detector_sample_noalloc(ctypes.c_void_p(big.handle), 0, 0, 1 << 20,
                                               ctypes.c_void_p(det.data_ptr()), ctypes.c_void_p(None),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == sg.STIM_E_UNSUPPORTED
    assert "bytes of device scratch" in sg.lib().stim_last_error().decode()
    # a fitting call still works afterwards
    rc, det, obs = noalloc(sg, c, 9, 3000)
    torch.cuda.synchronize()
    assert rc == sg.STIM_OK
    want_det, _ = c.detect(9, 3000)
    torch.cuda.synchronize()
    assert torch.equal(det, want_det)
