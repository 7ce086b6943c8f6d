"""Writes batch_mix_oracle_words.json: for every request of the 64-circuit
batch mix (workloads.batch_mix(seed=0), circuit i with seed i, shots [0, S_i))
the oracle's sample of two interior 64-shot words -- measurement records for
the random Clifford circuits, detection events and observables for the surface
codes -- as SHA-256 digests of the little-endian uint64 words (row-major
[rows][2]), with the last word masked to the request's own shots.

Only the oracle computes these values; the oracle's reference sample of the
~500-qubit random circuits takes minutes, which is why they are stored.

Usage: python tests/golden/make_batch_mix_digests.py [processes]
"""
import hashlib
import json
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def span(shots):
    W = (shots + 63) // 64
    w0 = W // 2
    return w0, min(2, W - w0)


def tail_mask(shots, w0, k):
    m = np.full(k, ~np.uint64(0), dtype=np.uint64)
    for j in range(k):
        lo = 64 * (w0 + j)
        if shots - lo < 64:
            m[j] = np.uint64((1 << max(shots - lo, 0)) - 1)
    return m


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def one(i):
    import oracle
    from paper_2103_02202_amd import workloads as wl
    m = wl.batch_mix(seed=0)[i]
    o = oracle.Circuit(m["text"])
    w0, k = span(m["shots"])
    surface = m["kind"] == "surface"
    want = o.sample(m["seed"], 64 * w0, 64 * k, meas=not surface, det=surface, obs=surface, threads=1)
    mask = tail_mask(m["shots"], w0, k)
    entry = {"kind": m["kind"], "shots": m["shots"], "seed": m["seed"], "w0": w0, "words": k}
    if surface:
        entry["det_sha256"] = digest(want["det"] & mask)
        entry["obs_sha256"] = digest(want["obs"] & mask)
    else:
        entry["meas_sha256"] = digest(want["meas"] & mask)
    print(i, m["kind"], flush=True)
    return entry


if __name__ == "__main__":
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    import oracle
    oracle.lib()
    from paper_2103_02202_amd import workloads as wl
    n = len(wl.batch_mix(seed=0))
    # Longest first: the large random circuits dominate.
    with Pool(procs) as pool:
        entries = pool.map(one, range(n), chunksize=1)
    with open(os.path.join(HERE, "batch_mix_oracle_words.json"), "w") as f:
        json.dump({"source": "oracle sample of workloads.batch_mix(seed=0); see make_batch_mix_digests.py",
                   "requests": entries}, f, indent=1)
        f.write("\n")
