"""Seeded synthetic circuit generators (circuit text only, no simulation).

These produce the workloads the sampler is measured and checked on.  The
paper's own benchmark circuit files are not available, so closed-form circuit
families stand in for them:

* ``surface_code(d, rounds, p)`` -- rotated surface-code Z-memory experiment
  (the family of the paper's surface-code benchmarks, Sec. 6): reset data,
  then ``rounds`` rounds of {R ancillas, H on X-type ancillas, four CX layers
  in the hook-avoiding order, H, M ancillas}, then measure the data.
  Noise: DEPOLARIZE1(p) after each H layer, DEPOLARIZE2(p) after each CX layer,
  X_ERROR(p) before every measurement.  Detectors: round 1 compares Z-type
  ancillas with their noiseless +1 value; later rounds compare every ancilla
  with its previous result; finally every Z-type ancilla's last result is
  compared with the parity of its data qubits.  Observable 0 is the logical Z
  along the first data row.
* ``random_clifford(n, depth, seed)`` -- layers of random {H, S, CX, CZ} on a
  shuffled qubit order followed by measurement of 10 % of the qubits (the
  random-circuit family of Sec. 6 with a two-qubit pairing walk), then
  measurement of every qubit.  Noiseless.
* ``repetition_code_example()`` -- the command-line example of Appendix A.1.
* ``teleportation_example()`` -- the interactive teleportation example of
  Appendix A.3 with its classically controlled corrections written as the
  equivalent coherent CX / CZ, so that its last measurement is always 0.
* ``batch_mix(seed)`` / ``serving_pool(seed)`` -- the 64-circuit batch and the
  resident serving pool.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import math

import numpy as np


def surface_code_counts(d: int, rounds: int):
    """Closed-form sizes of ``surface_code(d, rounds, p)``."""
    A = d * d - 1
    return {
        "num_qubits": 2 * d * d - 1,
        "num_gate_targets": rounds * (3 * A + 4 * d * (d - 1)) + 2 * d * d,
        "num_noise_targets": rounds * (2 * A + 4 * d * (d - 1)) + d * d,
        "num_measurements": rounds * A + d * d,
        "num_detectors": rounds * A,
    }


def _surface_layout(d: int):
    data = [(x, y) for y in range(1, 2 * d, 2) for x in range(1, 2 * d, 2)]
    anc = []
    for y in range(0, 2 * d + 1, 2):
        for x in range(0, 2 * d + 1, 2):
            is_x = ((x // 2 + y // 2) % 2) == 1
            nb = [(x + dx, y + dy) for dx in (-1, 1) for dy in (-1, 1)
                  if 0 < x + dx < 2 * d and 0 < y + dy < 2 * d]
            if len(nb) == 4:
                anc.append((x, y, is_x))
            elif len(nb) == 2:
                on_top_bottom = y in (0, 2 * d)
                if is_x == on_top_bottom:       # X-type on top/bottom, Z-type on left/right
                    anc.append((x, y, is_x))
    coords = sorted([(y, x) for (x, y) in data] + [(y, x) for (x, y, _) in anc])
    index = {(x, y): i for i, (y, x) in enumerate(coords)}
    return data, anc, index


def surface_code(d: int, rounds: int, p: float, feedback_reset: bool = False) -> str:
    """Rotated surface-code memory experiment.  feedback_reset: ancillas are
    reset after their measurement by a classically controlled X (CX rec[-k] a)
    instead of an R at the start of the next round (adaptive circuit)."""
    if d < 3 or d % 2 == 0:
        raise ValueError("d must be odd and >= 3")
    data, anc, idx = _surface_layout(d)
    A = len(anc)
    xa = [a for a in anc if a[2]]
    za = [a for a in anc if not a[2]]
    qd = [idx[c] for c in data]
    qa = [idx[(x, y)] for (x, y, _) in anc]
    qx = [idx[(x, y)] for (x, y, _) in xa]
    order_x = [(1, 1), (1, -1), (-1, 1), (-1, -1)]
    order_z = [(1, 1), (-1, 1), (1, -1), (-1, -1)]
    layers = []
    for k in range(4):
        pairs = []
        for (x, y, is_x) in anc:
            dx, dy = (order_x if is_x else order_z)[k]
            c = (x + dx, y + dy)
            if c not in idx:
                continue
            a, q = idx[(x, y)], idx[c]
            pairs += [a, q] if is_x else [q, a]
        layers.append(pairs)

    def j(v):
        return " ".join(str(t) for t in v)

    def noise(name, targets):
        return [f"{name}({p!r}) {j(targets)}"] if p > 0 and targets else []

    def round_body(first: bool):
        out = [f"R {j(qa)}", "TICK"] if first or not feedback_reset else []
        out += [f"H {j(qx)}"] + noise("DEPOLARIZE1", qx) + ["TICK"]
        for pairs in layers:
            out += [f"CX {j(pairs)}"] + noise("DEPOLARIZE2", pairs) + ["TICK"]
        out += [f"H {j(qx)}"] + noise("DEPOLARIZE1", qx) + ["TICK"]
        out += noise("X_ERROR", qa) + [f"M {j(qa)}"]
        if feedback_reset:
            out.append("CX " + " ".join(f"rec[-{A - k}] {a}" for k, a in enumerate(qa)))
        for k, (x, y, is_x) in enumerate(anc):
            back = A - k
            if first:
                if not is_x:
                    out.append(f"DETECTOR({x}, {y}, 0) rec[-{back}]")
            else:
                out.append(f"DETECTOR({x}, {y}, 0) rec[-{back}] rec[-{back + A}]")
        return out

    lines = [f"R {j(qd)}", "TICK"]
    lines += round_body(True)
    if rounds > 1:
        lines.append(f"REPEAT {rounds - 1} {{")
        lines += ["    " + s for s in round_body(False)]
        lines.append("}")
    lines += noise("X_ERROR", qd) + [f"M {j(qd)}"]
    D2 = len(qd)
    dpos = {c: k for k, c in enumerate(data)}
    for k, (x, y, is_x) in enumerate(anc):
        if is_x:
            continue
        recs = [f"rec[-{D2 + A - k}]"]
        for dx in (-1, 1):
            for dy in (-1, 1):
                c = (x + dx, y + dy)
                if c in dpos:
                    recs.append(f"rec[-{D2 - dpos[c]}]")
        lines.append(f"DETECTOR({x}, {y}, 1) " + " ".join(recs))
    row = [k for k, (x, y) in enumerate(data) if y == 1]
    lines.append("OBSERVABLE_INCLUDE(0) " + " ".join(f"rec[-{D2 - k}]" for k in row))
    return "\n".join(lines) + "\n"


def random_clifford(n: int, depth: int, seed: int) -> str:
    rng = np.random.Generator(np.random.PCG64(seed))
    lines = []
    m = max(1, int(round(0.1 * n)))
    for _layer in range(depth):
        order = rng.permutation(n)
        groups = {"H": [], "S": [], "CX": [], "CZ": []}
        k = 0
        while k < n:
            g = ["H", "S", "CX", "CZ"][int(rng.integers(4))]
            if g in ("CX", "CZ"):
                if k + 1 < n:
                    groups[g] += [int(order[k]), int(order[k + 1])]
                    k += 2
                    continue
                g = ["H", "S"][int(rng.integers(2))]
            groups[g].append(int(order[k]))
            k += 1
        for g in ("H", "S", "CX", "CZ"):
            if groups[g]:
                lines.append(g + " " + " ".join(map(str, groups[g])))
        meas = sorted(int(v) for v in rng.choice(n, size=m, replace=False))
        lines.append("M " + " ".join(map(str, meas)))
        lines.append("TICK")
    lines.append("M " + " ".join(map(str, range(n))))
    return "\n".join(lines) + "\n"


def repetition_code_example() -> str:
    """Appendix A.1: 20 rounds of X_ERROR(0.01), two CNOT sweeps and MR."""
    return ("REPEAT 20 {\n"
            "    X_ERROR(0.01) 0 1 2 3 4 5 6 7 8 9 10\n"
            "    CNOT 0 1 2 3 4 5 6 7 8 9\n"
            "    CNOT 10 9 8 7 6 5 4 3 2 1\n"
            "    MR 1 3 5 7 9\n"
            "}\n")


def teleportation_example() -> str:
    """Appendix A.3 with coherent corrections: the last result is always 0."""
    return ("H 1\nCX 1 9\n"            # share an EPR pair
            "H 0\nS 0\n"               # state to teleport
            "CX 0 1\nH 0\n"            # Alice's basis change
            "CX 1 9\nCZ 0 9\n"         # Bob's corrections, made coherent
            "M 1 0\n"                  # Alice's (now random, unused) results
            "S_DAG 9\nH 9\nM 9\n")     # uncompute the state; must give 0


def _log_uniform(rng, lo, hi):
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def batch_mix(seed: int = 0, count: int = 64):
    """The 64-circuit batch: 32 surface codes (odd d in [3, 25], rounds = d,
    p log-uniform in [1e-4, 1e-2]) and 32 random Clifford circuits (n in
    [8, 512], depth 100), each with a shot count log-uniform in
    [1024, 262144].  Returns a list of dicts with text, shots, seed, kind."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        shots = int(math.floor(_log_uniform(rng, 1024, 262144)))
        if i < count // 2:
            d = int(rng.choice(np.arange(3, 26, 2)))
            p = _log_uniform(rng, 1e-4, 1e-2)
            out.append({"kind": "surface", "d": d, "p": p, "text": surface_code(d, d, p),
                        "shots": shots, "seed": i})
        else:
            n = int(rng.integers(8, 513))
            out.append({"kind": "random", "n": n, "text": random_clifford(n, 100, seed=i),
                        "shots": shots, "seed": i})
    return out


def serving_pool(seed: int = 0, d_max: int = 101):
    """Resident serving pool: one surface code per odd d in [3, d_max], rounds =
    d, with p drawn once, log-uniform in [1e-4, 1e-2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = []
    for d in range(3, d_max + 1, 2):
        p = _log_uniform(rng, 1e-4, 1e-2)
        pool.append({"d": d, "p": p, "text": surface_code(d, d, p)})
    return pool


def serving_requests(num: int, rate: float, pool_size: int, seed: int = 0,
                     min_shots: int = 256, max_shots: int = 1 << 20):
    """Poisson arrivals at `rate` req/s; each request picks a pool entry
    uniformly and a shot count log-uniform in [min_shots, max_shots]."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    t = 0.0
    out = []
    for j in range(num):
        t += float(rng.exponential(1.0 / rate))
        out.append({"arrival": t, "circuit": int(rng.integers(pool_size)),
                    "shots": int(math.floor(_log_uniform(rng, min_shots, max_shots))),
                    "seed": j})
    return out
