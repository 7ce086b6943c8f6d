"""Brute-force state-vector checks for small circuits (test infrastructure only).

Independent of the oracle's C++ code: its own small parser, the unitary matrices
of ``gates.py``, and exact projective measurement.  Used to pin

  * the canonical reference sample (every random measurement, including the one
    hidden in a reset, takes result 0 -- the reading of Sec. 3 / Sec. 4 that
    both implementations follow), and
  * the exact distribution of measurement records of noiseless and noisy
    circuits (Pauli channels enumerated), against which the frame sampler's
    empirical distribution is compared.

Limited to about 12 qubits (4096 amplitudes).
"""
from __future__ import annotations

import itertools
import re

import numpy as np

from .gates import UNITARIES, PAULI

ALIASES = {"H_XZ": "H", "SQRT_Z": "S", "SQRT_Z_DAG": "S_DAG", "CNOT": "CX", "ZCX": "CX",
           "ZCY": "CY", "ZCZ": "CZ", "RZ": "R", "MZ": "M", "MRZ": "MR"}
TWO_QUBIT = {"CX", "CY", "CZ", "SWAP", "DEPOLARIZE2"}
NOISE = {"X_ERROR", "Y_ERROR", "Z_ERROR", "DEPOLARIZE1", "DEPOLARIZE2"}
CONTROLLED_PAULI = {"CX": "X", "CY": "Y", "CZ": "Z"}


def parse(text: str):
    """Returns a flat list of (name, arg, targets) with REPEAT blocks unrolled.
    DETECTOR / OBSERVABLE_INCLUDE targets are kept as negative lookbacks."""
    lines = text.splitlines()
    pos = 0

    def block(depth):
        nonlocal pos
        out = []
        while pos < len(lines):
            s = lines[pos].split("#")[0].strip()
            pos += 1
            if not s:
                continue
            if s == "}":
                return out
            m = re.match(r"^([A-Za-z_0-9]+)\s*(\(([^)]*)\))?\s*(.*)$", s)
            name = m.group(1).upper()
            name = ALIASES.get(name, name)
            arg = m.group(3)
            rest = m.group(4)
            if name == "REPEAT":
                reps = int(rest.rstrip("{").strip())
                body = block(depth + 1)
                out.extend(body * reps)
                continue
            toks = rest.split()
            # rec[-k] becomes -k: detector terms, or the classical control of
            # CX / CY / CZ.
            targets = [-int(t[5:-1]) if t.lower().startswith("rec[") else int(t) for t in toks]
            val = float(arg.split(",")[0]) if arg and name in NOISE else None
            out.append((name, val, targets))
        return out

    return block(0)


def num_qubits(ops) -> int:
    n = 0
    for name, _, t in ops:
        if name not in ("DETECTOR", "OBSERVABLE_INCLUDE") and t:
            n = max(n, max(t) + 1)
    return n


class State:
    def __init__(self, n: int):
        self.n = n
        self.psi = np.zeros(2 ** n, dtype=complex)
        self.psi[0] = 1

    def apply(self, u: np.ndarray, qs):
        """Applies a 2^k x 2^k unitary to qubits qs (qs[0] is the low bit of u)."""
        k = len(qs)
        t = self.psi.reshape([2] * self.n)          # axis a <-> qubit n-1-a
        axes = [self.n - 1 - q for q in reversed(qs)]   # u's high bit first
        t = np.moveaxis(t, axes, list(range(k)))
        shp = t.shape
        t = (u @ t.reshape(2 ** k, -1)).reshape(shp)
        t = np.moveaxis(t, list(range(k)), axes)
        self.psi = t.reshape(-1)

    def prob_one(self, q: int) -> float:
        idx = np.arange(2 ** self.n)
        return float(np.sum(np.abs(self.psi[(idx >> q) & 1 == 1]) ** 2))

    def project(self, q: int, v: int) -> float:
        idx = np.arange(2 ** self.n)
        mask = ((idx >> q) & 1) == v
        p = float(np.sum(np.abs(self.psi[mask]) ** 2))
        if p < 1e-12:
            raise ValueError("projection onto a zero-probability outcome")
        self.psi = np.where(mask, self.psi, 0) / np.sqrt(p)
        return p


def _run(ops, n, outcome_fn, paulis=None):
    """Runs the circuit; outcome_fn(p1) picks each measurement's outcome (also
    the hidden one in R).  paulis maps (op index, slot) -> Pauli string to
    inject at that noise site.  Returns (visible record, all outcomes including
    hidden reset ones, probability of those outcomes)."""
    st = State(n)
    rec, full = [], []
    prob = 1.0
    for i, (name, arg, t) in enumerate(ops):
        if name in UNITARIES:
            k = 2 if name in TWO_QUBIT else 1
            for s in range(0, len(t), k):
                pair = t[s:s + k]
                if k == 2 and min(pair) < 0:
                    # Classically controlled Pauli: the gate's action on the
                    # target when the control is |1>, applied when the
                    # recorded result is 1.
                    lookback = -min(pair)
                    q = max(pair)
                    if rec[len(rec) - lookback]:
                        st.apply(PAULI[CONTROLLED_PAULI[name]], [q])
                else:
                    st.apply(UNITARIES[name], pair)
        elif name in ("M", "MR", "R"):
            for q in t:
                p1 = st.prob_one(q)
                v = outcome_fn(p1)
                prob *= st.project(q, v)
                full.append(v)
                if name != "R":
                    rec.append(v)
                if name != "M" and v:
                    st.apply(PAULI["X"], [q])
        elif name in NOISE and paulis is not None:
            k = 2 if name == "DEPOLARIZE2" else 1
            for s in range(len(t) // k):
                pstr = paulis.get((i, s))
                if pstr:
                    for j, ch in enumerate(pstr):
                        if ch != "_":
                            st.apply(PAULI[ch], [t[s * k + j]])
    return rec, full, prob


def canonical_reference(text: str):
    """Every random outcome (probability 1/2) resolves to 0; deterministic
    outcomes are whatever they are.  Noise is ignored."""
    ops = parse(text)

    def pick(p1):
        if abs(p1 - 0.5) < 1e-9 or p1 < 1e-9:
            return 0
        if p1 > 1 - 1e-9:
            return 1
        raise ValueError("non-stabilizer probability %r" % p1)

    rec, _, _ = _run(ops, num_qubits(ops), pick)
    return rec


class _Branch(Exception):
    pass


def record_distribution(text: str, paulis=None):
    """Exact distribution {visible record: probability} for one fixed Pauli
    injection, by branching on every random measurement outcome."""
    ops = parse(text)
    n = num_qubits(ops)
    dist = {}

    def outcomes_until_random(prefix):
        forced = list(prefix)
        taken = []

        def pick(p1):
            if forced:
                v = forced.pop(0)
            elif 1e-9 < p1 < 1 - 1e-9:
                raise _Branch()
            else:
                v = 1 if p1 > 0.5 else 0
            taken.append(v)
            return v

        try:
            rec, _, prob = _run(ops, n, pick, paulis)
            return None, rec, prob
        except _Branch:
            return taken, None, None

    stack = [[]]
    while stack:
        prefix = stack.pop()
        taken, rec, prob = outcomes_until_random(prefix)
        if taken is None:
            dist[tuple(rec)] = dist.get(tuple(rec), 0.0) + prob
        else:
            stack.append(taken + [0])
            stack.append(taken + [1])
    return dist


def noisy_record_distribution(text: str):
    """Exact record distribution of a small noisy circuit: enumerate every
    Pauli-error configuration of its noise sites (Sec. 3: noise is a Pauli
    channel), weight it, and branch over random measurement outcomes."""
    ops = parse(text)
    sites = []
    for i, (name, arg, t) in enumerate(ops):
        if name in NOISE and arg:
            p = arg
            if name == "X_ERROR":
                choices = [("X", p)]
            elif name == "Y_ERROR":
                choices = [("Y", p)]
            elif name == "Z_ERROR":
                choices = [("Z", p)]
            elif name == "DEPOLARIZE1":
                choices = [(c, p / 3) for c in "XYZ"]
            else:
                choices = [(a + b, p / 15) for a in "_XYZ" for b in "_XYZ" if a + b != "__"]
            k = 2 if name == "DEPOLARIZE2" else 1
            for s in range(len(t) // k):
                none = ("_" * k, 1 - sum(w for _, w in choices))
                sites.append(((i, s), [none] + choices))
    dist = {}
    for combo in itertools.product(*[c for _, c in sites]):
        w = 1.0
        paulis = {}
        for (key, _), (pstr, pw) in zip(sites, combo):
            w *= pw
            paulis[key] = pstr
        if w == 0:
            continue
        for rec, pr in record_distribution(text, paulis).items():
            dist[rec] = dist.get(rec, 0.0) + w * pr
    return dist
