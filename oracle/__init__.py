"""Oracle for batched Pauli-frame sampling (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is an independent, plain CPU implementation of what the
sampler computes, following Gidney, "Stim: a fast stabilizer circuit simulator"
(arXiv:2103.02202): the inverse-tableau reference sample of Sec. 4, the Pauli
frame simulation of Sec. 3, geometric gap sampling of Sec. 5.5 and detection
events of Sec. 5.6.  It shares no code with the GPU sampler.

The C++ part lives in ``oracle.cpp`` and is built into ``liboracle.so`` by
:func:`build`.  ``statevector.py`` (brute-force state vectors) and ``gates.py``
(unitary matrices) are the independent checks that pin it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False, native: bool = False, path: str | None = None) -> str:
    """Compiles oracle.cpp into liboracle.so with g++ (-O2, OpenMP).

    native=True builds the same source with -O3 -march=native for the host it
    runs on (into `path`), the build the CPU baseline is timed with; the code
    is unchanged, only the compiler flags differ."""
    src = os.path.join(_HERE, "oracle.cpp")
    out = path or _LIB_PATH
    tmp = out + ".tmp"
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["g++", "-std=c++17", *opt, "-fopenmp", "-shared", "-fPIC", src, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + res.stderr)
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


def use_native_build(path: str) -> None:
    """Builds the -O3 -march=native copy at `path` and makes this process use
    it; must be called before the first Circuit is created."""
    global _lib, _LIB_PATH
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    build(native=True, path=path)
    _LIB_PATH = path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        L.oracle_last_error.restype = ctypes.c_char_p
        L.oracle_parse.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(p)]
        L.oracle_free.argtypes = [p]
        L.oracle_shape.argtypes = [p, p]
        L.oracle_reference.argtypes = [p, ctypes.c_int, u64, p]
        L.oracle_sample.argtypes = [p, p, u64, u64, u64, p, p, p, ctypes.c_int]
        L.oracle_detector.argtypes = [p, u64, p, u64]
        L.oracle_detector.restype = u64
        L.oracle_philox.argtypes = [p, p, p]
        L.oracle_key_hi.restype = u64
        L.oracle_thresholds.argtypes = [ctypes.c_double, p]
        L.oracle_zrand.argtypes = [u64, u64, u64, u64]
        L.oracle_zrand.restype = u64
        L.oracle_hits.argtypes = [u64, u64, u64, u64, ctypes.c_double, ctypes.c_int, p, p, ctypes.c_int]
        L.oracle_gate.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
        L.oracle_conjugate.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t]
        L.oracle_z_image.argtypes = [p, ctypes.c_uint32, ctypes.c_char_p, ctypes.c_size_t]
        L.oracle_error_sets.argtypes = [p, p, p, p, p]
        L.oracle_deterministic.argtypes = [p]
        L.oracle_sparse_detect.argtypes = [p, u64, u64, u64, p, p, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class OracleError(RuntimeError):
    pass


class Circuit:
    """A parsed, REPEAT-unrolled circuit held by the oracle."""

    def __init__(self, text: str):
        L = lib()
        h = ctypes.c_void_p()
        data = text.encode()
        rc = L.oracle_parse(data, len(data), ctypes.byref(h))
        if rc != 0:
            raise OracleError(L.oracle_last_error().decode())
        self._h = h
        shape = np.zeros(6, dtype=np.uint64)
        L.oracle_shape(h, _ptr(shape))
        (self.num_qubits, self.num_measurements, self.num_detectors,
         self.num_observables, self.num_gate_targets, self.num_instructions) = (int(v) for v in shape)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.oracle_free(self._h)
            self._h = None

    def reference(self, canonical: bool = True, coin_seed: int = 0) -> np.ndarray:
        """Reference sample, one uint8 per measurement (Sec. 4)."""
        out = np.zeros(max(self.num_measurements, 1), dtype=np.uint8)
        rc = lib().oracle_reference(self._h, 1 if canonical else 0, coin_seed, _ptr(out))
        if rc != 0:
            raise OracleError(lib().oracle_last_error().decode())
        return out[: self.num_measurements]

    def sample(self, seed: int, shot_offset: int, num_shots: int, ref: np.ndarray | None = None,
               meas: bool = True, det: bool = False, obs: bool = False, threads: int | None = None):
        """Frame sampling (Sec. 3); returns dict of [rows][W] uint64 arrays."""
        if ref is None:
            ref = self.reference()
        ref = np.ascontiguousarray(ref, dtype=np.uint8)
        W = (num_shots + 63) // 64
        outs = {}
        bufs = []
        for name, want, rows in (("meas", meas, self.num_measurements),
                                 ("det", det, self.num_detectors),
                                 ("obs", obs, self.num_observables)):
            if want:
                a = np.zeros((rows, W), dtype=np.uint64)
                outs[name] = a
                bufs.append(_ptr(a) if a.size else ctypes.c_void_p(None))
            else:
                bufs.append(ctypes.c_void_p(None))
        if threads is None:
            threads = os.cpu_count() or 1
        refbuf = ref if ref.size else np.zeros(1, dtype=np.uint8)
        rc = lib().oracle_sample(self._h, _ptr(refbuf), seed, shot_offset, num_shots,
                                 bufs[0], bufs[1], bufs[2], threads)
        if rc != 0:
            raise OracleError(lib().oracle_last_error().decode())
        return outs

    def detector(self, d: int) -> list:
        buf = np.zeros(64, dtype=np.uint64)
        n = lib().oracle_detector(self._h, d, _ptr(buf), 64)
        if n > 64:
            buf = np.zeros(n, dtype=np.uint64)
            lib().oracle_detector(self._h, d, _ptr(buf), n)
        return [int(v) for v in buf[:n]]

    def error_sets(self):
        """Detectors / observables flipped by each single-Pauli error (Sec. 5.6):
        (off, lanes) with generator g's lanes in lanes[off[g]:off[g + 1]];
        generators by noise instruction (p > 0), slot, then X, Z of each qubit.
        Lane d < num_detectors is detector d, lane num_detectors + o is
        observable o."""
        n_sets, n_ent = ctypes.c_uint64(), ctypes.c_uint64()
        L = lib()
        if L.oracle_error_sets(self._h, ctypes.byref(n_sets), ctypes.byref(n_ent), None, None) != 0:
            raise OracleError(L.oracle_last_error().decode())
        off = np.zeros(n_sets.value + 1, dtype=np.uint64)
        lanes = np.zeros(max(n_ent.value, 1), dtype=np.uint32)
        L.oracle_error_sets(self._h, ctypes.byref(n_sets), ctypes.byref(n_ent), _ptr(off), _ptr(lanes))
        return off, lanes[: n_ent.value]

    def deterministic(self) -> bool:
        return lib().oracle_deterministic(self._h) == 1

    def sparse_detect(self, seed: int, shot_offset: int, num_shots: int, threads: int | None = None):
        """Sparse detection-event sampling (Sec. 5.6): (det [D][W], obs [L][W])."""
        W = (num_shots + 63) // 64
        det = np.zeros((self.num_detectors, W), dtype=np.uint64)
        obs = np.zeros((self.num_observables, W), dtype=np.uint64)
        rc = lib().oracle_sparse_detect(self._h, seed, shot_offset, num_shots,
                                        _ptr(det) if det.size else None, _ptr(obs) if obs.size else None,
                                        threads or os.cpu_count() or 1)
        if rc != 0:
            raise OracleError(lib().oracle_last_error().decode())
        return det, obs

    def z_image(self, q: int) -> str:
        out = ctypes.create_string_buffer(self.num_qubits + 8)
        rc = lib().oracle_z_image(self._h, q, out, len(out))
        if rc != 0:
            raise OracleError(lib().oracle_last_error().decode())
        return out.value.decode()


def philox(counter, key):
    c = np.array(counter, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox(_ptr(c), _ptr(k), _ptr(o))
    return [int(v) for v in o]


def key_hi() -> int:
    return int(lib().oracle_key_hi())


def thresholds(p: float):
    o = np.zeros(64, dtype=np.uint64)
    lib().oracle_thresholds(p, _ptr(o))
    return [int(v) for v in o]


def zrand(seed, instr, slot, word) -> int:
    return int(lib().oracle_zrand(seed, instr, slot, word))


def hits(seed, instr, slot, word, p, K=0):
    pos = np.zeros(64, dtype=np.int32)
    ch = np.zeros(64, dtype=np.int32)
    n = lib().oracle_hits(seed, instr, slot, word, p, K, _ptr(pos), _ptr(ch), 64)
    return [(int(pos[i]), int(ch[i])) for i in range(n)]


def gate_table():
    """{name: (kind, images, inverse)} from the oracle's gate table."""
    out = {}
    i = 0
    buf = ctypes.create_string_buffer(256)
    while lib().oracle_gate(i, buf, 256) == 0:
        s = buf.value.decode()
        head, _, inv = s.partition(" | ")
        parts = head.split()
        out[parts[0]] = (int(parts[1]), parts[2:], inv or None)
        i += 1
    return out


def conjugate(gate: str, pauli: str) -> str:
    out = ctypes.create_string_buffer(64)
    rc = lib().oracle_conjugate(gate.encode(), pauli.encode(), out, 64)
    if rc != 0:
        raise OracleError("conjugate failed")
    return out.value.decode()


def unpack_bits(words: np.ndarray, num_shots: int) -> np.ndarray:
    """[rows][W] uint64 -> [num_shots][rows] uint8 (bit j of word w = shot 64w+j)."""
    rows, W = words.shape
    b = np.unpackbits(words.view(np.uint8).reshape(rows, W * 8), axis=1, bitorder="little")
    return b[:, :num_shots].T.copy()
