"""GPU: stim_sample_scratch_bytes reports what a sampling call takes.

The library allocates its per-call scratch (flip rings or flip table, noise
records and their tables, global frame slots) from the device's default stream-ordered
pool; all of it is live at once, so the pool's used-memory high-water mark
over one call, minus what was in use before, is that scratch (allocations are
rounded up by the pool, so a small slack per allocation is allowed).
"""
import ctypes

import pytest

from paper_2103_02202_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

USED_CURRENT, USED_HIGH = 7, 8          # hipMemPoolAttrUsedMemCurrent / UsedMemHigh


def announce(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def hip():
    from paper_2103_02202_amd import stim_gpu
    assert torch.cuda.is_available()
    stim_gpu.lib()
    paths = {l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l}
    assert len(paths) == 1, paths
    H = ctypes.CDLL(paths.pop())
    pool = ctypes.c_void_p()
    assert H.hipDeviceGetDefaultMemPool(ctypes.byref(pool), torch.cuda.current_device()) == 0
    return H, pool


def pool_attr(H, pool, attr):
    v = ctypes.c_uint64()
    assert H.hipMemPoolGetAttribute(pool, attr, ctypes.byref(v)) == 0
    return v.value


@pytest.mark.parametrize("d,p,shots,mode,walk_events", [
    (5, 1e-3, 65536, "frame", "0"), (9, 1e-2, 100_000, "detector", "0"), (25, 1e-3, 65536, "detector", "0"),
    (9, 1e-2, 100_000, "detector", "1"),          # flip rings of events formed in the walk
    (71, 1e-3, 8192, "frame", "0"),               # frame slice past LDS: global frame slots
    (71, 1e-3, 8192, "detector", "1"),            # global frame slots + flip rings
])
def test_scratch_query_matches_pool_use(hip, d, p, shots, mode, walk_events, monkeypatch):
    from paper_2103_02202_amd import stim_gpu as sg
    H, pool = hip
    monkeypatch.setenv("STIM_WALK_EVENTS", walk_events)
    announce("scratch", d, p, shots, mode, walk_events)
    c = sg.Circuit(wl.surface_code(d, d, p))
    W = (shots + 63) // 64
    rows = c.num_measurements if mode == "frame" else c.num_detectors
    out = torch.empty((rows, W), dtype=torch.int64, device="cuda")
    obs = torch.empty((max(c.num_observables, 1), W), dtype=torch.int64, device="cuda")

    def call():
        if mode == "frame":
            sg.stim_frame_sample(c.handle, 3, 0, shots, out, None)
        else:
            sg.stim_detector_sample(c.handle, 3, 0, shots, out, obs, None)

    call()                                        # reference, program upload
    torch.cuda.synchronize()
    before = pool_attr(H, pool, USED_CURRENT)
    zero = ctypes.c_uint64(0)
    assert H.hipMemPoolSetAttribute(pool, USED_HIGH, ctypes.byref(zero)) == 0
    call()
    torch.cuda.synchronize()
    used = pool_attr(H, pool, USED_HIGH) - before
    want = c.scratch_bytes(shots, mode)
    assert want > 0
    assert want <= used <= want + 6 * (2 << 20), (want, used)
