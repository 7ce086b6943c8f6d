"""Pins of the oracle's shot-major output formats (Sec. 5.11)."""
import os

import numpy as np
import pytest

from oracle import formats as F

HERE = os.path.dirname(os.path.abspath(__file__))


def _bits(s):
    return np.array([[c == "1" for c in s]], dtype=bool)


def _golden():
    out = []
    for line in open(os.path.join(HERE, "golden", "output_formats.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows, bits, f01, b8, hits, r8 = [x.strip() for x in line.split("|")]
        out.append((int(rows), bits, f01.replace("\\n", "\n").encode(), bytes.fromhex(b8.replace(" ", "")),
                    hits.replace("\\n", "\n").encode(), bytes(int(x) for x in r8.split())))
    return out


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c[1])
def test_worked_examples(case):
    rows, bits, f01, b8, hits, r8 = case
    b = _bits(bits)
    assert b.shape[1] == rows
    assert F.format_01(b) == f01
    assert F.format_b8(b) == b8
    assert F.format_hits(b) == hits
    assert F.format_r8(b) == r8


def test_b8_matches_numpy_little_endian_packbits():
    rng = np.random.default_rng(1)
    for rows in (1, 7, 8, 9, 63, 64, 65, 200):
        b = rng.random((5, rows)) < 0.3
        want = b"".join(np.packbits(shot, bitorder="little").tobytes() for shot in b)
        assert F.format_b8(b) == want


def test_sparse_formats_round_trip_and_long_runs():
    rng = np.random.default_rng(2)
    for rows in (1, 5, 254, 255, 256, 600, 1000):
        for dens in (0.0, 0.002, 0.05, 0.5, 1.0):
            b = rng.random((4, rows)) < dens
            assert (F.decode_r8(F.format_r8(b), rows, 4) == b).all()
            assert (F.decode_hits(F.format_hits(b), rows, 4) == b).all()
    # 255 zeros then a one: a continuation byte and then 0.
    b = np.zeros((1, 300), dtype=bool)
    b[0, 255] = True
    assert F.format_r8(b) == bytes([255, 0, 44])


def test_01_lengths_and_alphabet():
    rng = np.random.default_rng(3)
    b = rng.random((6, 37)) < 0.4
    s = F.format_01(b)
    assert len(s) == 6 * 38 and set(s) <= set(b"01\n")
    assert s.count(b"1") == b.sum()


def test_shot_bits_reads_the_sampler_layout():
    rows, shots = 3, 130
    W = (shots + 63) // 64
    rng = np.random.default_rng(4)
    b = rng.random((shots, rows)) < 0.5
    table = np.zeros((rows, W), dtype=np.uint64)
    for s in range(shots):
        for r in range(rows):
            if b[s, r]:
                table[r, s // 64] |= np.uint64(1) << np.uint64(s % 64)
    assert (F.shot_bits(table, rows, shots) == b).all()
