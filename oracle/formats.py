"""Shot-major output formats (test infrastructure only; see the package docstring).

Plain Python/numpy definitions of the per-shot output streams named in the
paper's "Output Format" subsection (Sec. 5.11):

* ``01``  -- one '0'/'1' character per result, in result order, then '\\n';
  shots one after another.
* ``b8``  -- results packed eight per byte, least significant bit first, the
  last byte of a shot padded with zeros; no separator between shots.
* ``hits`` and ``r8`` -- named by the paper as sparse formats built on the
  indices of the non-zero bits, but not spelled out.  Readings used here:
  ``hits`` writes the indices of a shot's set results in increasing order, in
  decimal, separated by ',' and followed by '\\n' (an empty line for a shot
  with none); ``r8`` writes, for each set result, the number of zero results
  since the previous set result (or the start of the shot) as a byte, a count
  of 255 or more being written as repeated 255 bytes that each stand for 255
  zeros, followed by the remainder; after the last set result the zeros up
  to the end of the shot are written the same way, as if a set result
  followed the shot.

Input is the sampler's measurement-major table: row r (a measurement,
detector or observable), word w, bit j = shot 64 w + j.
"""
from __future__ import annotations

import numpy as np


def shot_bits(table, rows: int, shots: int) -> np.ndarray:
    """bool [shots][rows] from a [rows][W] uint64 table (bit j of word w = shot 64 w + j)."""
    t = np.asarray(table, dtype=np.uint64).reshape(rows, -1) if rows else np.zeros((0, 1), np.uint64)
    out = np.zeros((shots, rows), dtype=bool)
    for s in range(shots):
        w, j = divmod(s, 64)
        out[s] = ((t[:, w] >> np.uint64(j)) & np.uint64(1)).astype(bool)
    return out


def format_01(bits: np.ndarray) -> bytes:
    """One character per result and a newline per shot (Sec. 5.11)."""
    return b"".join(bytes(ord("1") if b else ord("0") for b in shot) + b"\n" for shot in bits)


def format_b8(bits: np.ndarray) -> bytes:
    """Eight results per byte, least significant bit first, zero-padded per shot (Sec. 5.11)."""
    out = bytearray()
    rows = bits.shape[1]
    for shot in bits:
        for k in range(0, rows, 8):
            v = 0
            for i in range(8):
                if k + i < rows and shot[k + i]:
                    v |= 1 << i
            out.append(v)
    return bytes(out)


def format_hits(bits: np.ndarray) -> bytes:
    """Indices of the set results of each shot, comma-separated, one line per shot."""
    return b"".join((",".join(str(i) for i in np.flatnonzero(shot)) + "\n").encode() for shot in bits)


def _runs(n: int) -> list:
    out = [255] * (n // 255)
    out.append(n % 255)
    return out


def format_r8(bits: np.ndarray) -> bytes:
    """Zero-run lengths before each set result and before the end of the shot, as bytes."""
    out = bytearray()
    rows = bits.shape[1]
    for shot in bits:
        prev = -1
        for i in np.flatnonzero(shot):
            out.extend(_runs(int(i) - prev - 1))
            prev = int(i)
        out.extend(_runs(rows - prev - 1))
    return bytes(out)


def decode_r8(data: bytes, rows: int, shots: int) -> np.ndarray:
    """Inverse of format_r8 (used to pin it)."""
    bits = np.zeros((shots, rows), dtype=bool)
    pos = 0
    for s in range(shots):
        i = 0                      # index of the next result
        while True:
            run = 0
            while data[pos] == 255:
                run += 255
                pos += 1
            run += data[pos]
            pos += 1
            i += run
            if i == rows:          # the virtual result after the shot
                break
            bits[s, i] = True
            i += 1
    assert pos == len(data)
    return bits


def decode_hits(data: bytes, rows: int, shots: int) -> np.ndarray:
    """Inverse of format_hits (used to pin it)."""
    lines = data.decode().split("\n")
    assert lines[-1] == "" and len(lines) == shots + 1
    bits = np.zeros((shots, rows), dtype=bool)
    for s, line in enumerate(lines[:-1]):
        for tok in filter(None, line.split(",")):
            bits[s, int(tok)] = True
    return bits


def format_shots(table, rows: int, shots: int, fmt: str) -> bytes:
    bits = shot_bits(table, rows, shots)
    return {"01": format_01, "b8": format_b8, "hits": format_hits, "r8": format_r8}[fmt](bits)
