"""Python binding of libstimgpu.so (argument marshalling only).

Every call goes to the native library; there is no Python or CPU fallback.
The function names mirror the C ABI in include/stim_gpu.h.  Device buffers are
torch tensors (PyTorch supplies device memory and streams only).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstimgpu.so")

STIM_OK, STIM_E_PARSE, STIM_E_INVALID_ARG, STIM_E_OOM, STIM_E_DEVICE, STIM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5

_lib = None


class StimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class StimRequest(ctypes.Structure):
    _fields_ = [("c", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("shot_offset", ctypes.c_uint64),
                ("num_shots", ctypes.c_uint64), ("mode", ctypes.c_int),
                ("out0", ctypes.c_void_p), ("out1", ctypes.c_void_p)]


def lib():
    """Loads libstimgpu.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_02202_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        u64, vp = ctypes.c_uint64, ctypes.c_void_p
        P64 = ctypes.POINTER(ctypes.c_uint64)
        L.stim_last_error.restype = ctypes.c_char_p
        L.stim_compile.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.stim_circuit_free.argtypes = [vp]
        L.stim_circuit_free.restype = None
        L.stim_circuit_shape.argtypes = [vp, P64, P64, P64, P64, P64]
        L.stim_reference_sample.argtypes = [vp, vp]
        L.stim_frame_sample.argtypes = [vp, u64, u64, u64, vp, vp]
        L.stim_detector_sample.argtypes = [vp, u64, u64, u64, vp, vp, vp]
        L.stim_sparse_detector_sample.argtypes = [vp, u64, u64, u64, vp, vp, vp]
        L.stim_detector_sample_noalloc.argtypes = [vp, u64, u64, u64, vp, vp, vp]
        L.stim_reference_sample_gpu.argtypes = [vp, vp, vp]
        L.stim_error_sets.argtypes = [vp, P64, P64, vp, vp]
        L.stim_sample_scratch_bytes.argtypes = [vp, u64, ctypes.c_int, P64]
        L.stim_batch_sample.argtypes = [ctypes.POINTER(StimRequest), ctypes.c_size_t, vp]
        L.stim_format_shots.argtypes = [vp, u64, u64, ctypes.c_int, vp, u64, P64, vp]
        L.stim_kernel_timing.argtypes = [ctypes.c_int]
        L.stim_kernel_times.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), P64]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != STIM_OK:
        raise StimError(rc, lib().stim_last_error().decode())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def stim_compile(text: str) -> int:
    h = ctypes.c_void_p()
    b = text.encode()
    _check(lib().stim_compile(b, len(b), ctypes.byref(h)))
    return h.value


def stim_circuit_free(handle: int) -> None:
    lib().stim_circuit_free(ctypes.c_void_p(handle))


def stim_circuit_shape(handle: int):
    v = [ctypes.c_uint64() for _ in range(5)]
    _check(lib().stim_circuit_shape(ctypes.c_void_p(handle), *[ctypes.byref(x) for x in v]))
    keys = ("num_qubits", "num_measurements", "num_detectors", "num_observables", "num_gate_targets")
    return {k: int(x.value) for k, x in zip(keys, v)}


def stim_reference_sample(handle: int, num_measurements: int):
    """Returns the reference bits as a list of uint64 words (host)."""
    n = max((num_measurements + 63) // 64, 1)
    buf = (ctypes.c_uint64 * n)()
    _check(lib().stim_reference_sample(ctypes.c_void_p(handle), ctypes.cast(buf, ctypes.c_void_p)))
    return [int(x) for x in buf][: (num_measurements + 63) // 64]


def stim_reference_sample_gpu(handle: int, num_measurements: int, stream=None):
    """Reference bits computed on the GPU, as a list of uint64 words."""
    n = max((num_measurements + 63) // 64, 1)
    buf = (ctypes.c_uint64 * n)()
    _check(lib().stim_reference_sample_gpu(ctypes.c_void_p(handle), ctypes.cast(buf, ctypes.c_void_p),
                                           _stream_ptr(stream)))
    return [int(x) for x in buf][: (num_measurements + 63) // 64]


def stim_frame_sample(handle: int, seed: int, shot_offset: int, num_shots: int, out_meas, stream=None):
    _check(lib().stim_frame_sample(ctypes.c_void_p(handle), seed, shot_offset, num_shots,
                                   _dptr(out_meas), _stream_ptr(stream)))


def stim_detector_sample(handle: int, seed: int, shot_offset: int, num_shots: int, out_det, out_obs=None,
                         stream=None):
    _check(lib().stim_detector_sample(ctypes.c_void_p(handle), seed, shot_offset, num_shots,
                                      _dptr(out_det), _dptr(out_obs), _stream_ptr(stream)))


def stim_sparse_detector_sample(handle: int, seed: int, shot_offset: int, num_shots: int, out_det,
                                out_obs=None, stream=None):
    _check(lib().stim_sparse_detector_sample(ctypes.c_void_p(handle), seed, shot_offset, num_shots,
                                             _dptr(out_det), _dptr(out_obs), _stream_ptr(stream)))


def stim_error_sets(handle: int):
    """(offsets, lanes) as numpy uint32 arrays (host only)."""
    import numpy as np
    n_sets, n_ent = ctypes.c_uint64(), ctypes.c_uint64()
    h = ctypes.c_void_p(handle)
    _check(lib().stim_error_sets(h, ctypes.byref(n_sets), ctypes.byref(n_ent), None, None))
    off = np.zeros(n_sets.value + 1, dtype=np.uint32)
    lanes = np.zeros(max(n_ent.value, 1), dtype=np.uint32)
    _check(lib().stim_error_sets(h, ctypes.byref(n_sets), ctypes.byref(n_ent), ctypes.c_void_p(off.ctypes.data),
                                 ctypes.c_void_p(lanes.ctypes.data)))
    return off, lanes[: n_ent.value]


SCRATCH_MODES = {"frame": 0, "detector": 1, "sparse": 2}


def stim_sample_scratch_bytes(handle: int, num_shots: int, mode) -> int:
    """Device scratch one sampling call takes beyond its outputs (mode
    'frame', 'detector' or 'sparse', or 0 / 1 / 2)."""
    m = SCRATCH_MODES[mode] if isinstance(mode, str) else int(mode)
    b = ctypes.c_uint64()
    _check(lib().stim_sample_scratch_bytes(ctypes.c_void_p(handle), num_shots, m, ctypes.byref(b)))
    return int(b.value)


def stim_batch_sample(requests, stream=None):
    """requests: list of dicts with keys handle, seed, shot_offset, num_shots,
    mode (0 measurements, 1 detectors), out0, out1 (tensors or None)."""
    arr = (StimRequest * len(requests))()
    for i, r in enumerate(requests):
        arr[i].c = r["handle"]
        arr[i].seed = r["seed"]
        arr[i].shot_offset = r.get("shot_offset", 0)
        arr[i].num_shots = r["num_shots"]
        arr[i].mode = r["mode"]
        arr[i].out0 = r["out0"].data_ptr() if r.get("out0") is not None else None
        arr[i].out1 = r["out1"].data_ptr() if r.get("out1") is not None else None
    _check(lib().stim_batch_sample(arr, len(requests), _stream_ptr(stream)))


STIM_FORMAT_01, STIM_FORMAT_B8, STIM_FORMAT_HITS, STIM_FORMAT_R8 = 0, 1, 2, 3
FORMATS = {"01": STIM_FORMAT_01, "b8": STIM_FORMAT_B8, "hits": STIM_FORMAT_HITS, "r8": STIM_FORMAT_R8}


def stim_format_shots(table, rows: int, num_shots: int, fmt, out=None, stream=None) -> int:
    """Writes the shots of a [rows][W] device table in a shot-major format into
    the uint8 device tensor `out` (or, with out=None, only returns the size).
    Returns the byte length of the output."""
    f = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
    n = ctypes.c_uint64()
    cap = out.numel() if out is not None else 0
    _check(lib().stim_format_shots(_dptr(table), rows, num_shots, f, _dptr(out), cap, ctypes.byref(n),
                                   _stream_ptr(stream)))
    return int(n.value)


def format_shots(table, rows: int, num_shots: int, fmt, stream=None):
    """Allocates the output and formats; returns a uint8 device tensor."""
    import torch
    n = stim_format_shots(table, rows, num_shots, fmt, None, stream)
    out = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
    stim_format_shots(table, rows, num_shots, fmt, out, stream)
    return out[:n]


def stim_kernel_timing(enable: bool) -> None:
    _check(lib().stim_kernel_timing(1 if enable else 0))


def stim_kernel_times():
    """Returns (noise_gen_ms, frame_ms, passes) summed over the recorded passes."""
    g, f, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64()
    _check(lib().stim_kernel_times(ctypes.byref(g), ctypes.byref(f), ctypes.byref(n)))
    return g.value, f.value, int(n.value)


class Circuit:
    """A compiled circuit handle with torch-tensor sampling helpers."""

    def __init__(self, text: str):
        self.handle = stim_compile(text)
        s = stim_circuit_shape(self.handle)
        self.num_qubits = s["num_qubits"]
        self.num_measurements = s["num_measurements"]
        self.num_detectors = s["num_detectors"]
        self.num_observables = s["num_observables"]
        self.num_gate_targets = s["num_gate_targets"]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            try:
                _lib.stim_circuit_free(ctypes.c_void_p(h))
            except Exception:   # interpreter shutdown
                pass
            self.handle = None

    def reference(self):
        return stim_reference_sample(self.handle, self.num_measurements)

    def sample(self, seed: int, num_shots: int, shot_offset: int = 0, out=None, stream=None):
        import torch
        W = (num_shots + 63) // 64
        if out is None:
            out = torch.empty((self.num_measurements, W), dtype=torch.int64, device="cuda")
        stim_frame_sample(self.handle, seed, shot_offset, num_shots, out, stream)
        return out

    def detect(self, seed: int, num_shots: int, shot_offset: int = 0, obs: bool = True, stream=None):
        import torch
        W = (num_shots + 63) // 64
        det = torch.empty((self.num_detectors, W), dtype=torch.int64, device="cuda")
        o = torch.empty((self.num_observables, W), dtype=torch.int64, device="cuda") if obs else None
        stim_detector_sample(self.handle, seed, shot_offset, num_shots, det, o, stream)
        return det, o

    def detect_sparse(self, seed: int, num_shots: int, shot_offset: int = 0, obs: bool = True, stream=None):
        """Same results as detect(), by sparse detection-event sampling."""
        import torch
        W = (num_shots + 63) // 64
        det = torch.empty((self.num_detectors, W), dtype=torch.int64, device="cuda")
        o = torch.empty((self.num_observables, W), dtype=torch.int64, device="cuda") if obs else None
        stim_sparse_detector_sample(self.handle, seed, shot_offset, num_shots, det, o, stream)
        return det, o

    def error_sets(self):
        return stim_error_sets(self.handle)

    def scratch_bytes(self, num_shots: int, mode="detector") -> int:
        return stim_sample_scratch_bytes(self.handle, num_shots, mode)

    def reference_gpu(self, stream=None):
        """Canonical reference sample computed on the GPU (uint64 words)."""
        return stim_reference_sample_gpu(self.handle, self.num_measurements, stream)
