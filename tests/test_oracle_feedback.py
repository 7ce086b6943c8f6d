"""Pins for classically controlled Paulis in the oracle (CPU only).

Sec. 3 ("Tracking Corrections"): a Pauli applied when an earlier measurement
returned 1 can live in the Pauli frame -- the reference run applies it when the
reference result is 1, the frame where the shot's result differs from the
reference.  Written as CX / CY / CZ with a rec[-k] control.

Pinned against
  * closed forms: teleportation with its corrections returns the prepared
    state for every shot, for preparations whose X, Z or both corrections
    matter, and fails without them; deterministic records of small circuits
    whose controlling result is 1 in the reference;
  * the brute-force state vector: canonical reference samples, and the exact
    record distribution of random noiseless and noisy circuits with feedback.
"""
import numpy as np
import pytest

import oracle
from oracle import statevector as sv
from circuit_gen import random_circuit
from test_oracle_sampling import chi2_against, records

# Preparation of q0 and its undoing on q2 after teleportation.
PREPS = {
    "zero": ("", ""),
    "one": ("X 0", "X 2"),
    "plus": ("H 0", "H 2"),
    "minus": ("X 0\nH 0", "H 2\nX 2"),
    "plus_i": ("H 0\nS 0", "S_DAG 2\nH 2"),
    "minus_i": ("H 0\nS_DAG 0", "S 2\nH 2"),
}


def feedback_circuit(n, num_ops, seed, **kw):
    """random_circuit with at least one classically controlled line (the
    first seed of seed, seed + 1000, ... that gives one)."""
    while True:
        text = random_circuit(n, num_ops, seed=seed, **kw)
        if "rec[" in text:
            return text
        seed += 1000


def teleport(prep, undo, corrections=True):
    fix = "CX rec[-1] 2\nCZ rec[-2] 2\n" if corrections else ""
    return (f"{prep}\nH 1\nCX 1 2\nCX 0 1\nH 0\nM 0 1\n{fix}{undo}\nM 2\n")


@pytest.mark.parametrize("name", sorted(PREPS))
def test_teleportation_with_corrections_returns_the_state(name):
    text = teleport(*PREPS[name])
    c = oracle.Circuit(text)
    r = records(c, 4096, seed=3)
    assert not r[:, 2].any()
    # The two Bell-measurement results are uniform and independent.
    for cols in ([0], [1], [0, 1]):
        frac = (np.bitwise_xor.reduce(r[:, cols], axis=1)).mean()
        assert 0.45 < frac < 0.55


@pytest.mark.parametrize("name", ["one", "plus", "plus_i"])
def test_teleportation_without_corrections_fails(name):
    # Sanity of the pin above: the preparations need their corrections.
    text = teleport(*PREPS[name], corrections=False)
    r = records(oracle.Circuit(text), 4096, seed=3)
    assert 0.4 < r[:, 2].mean() < 0.6


def test_teleportation_pauli_forms_and_record_order_matter():
    # Swapping which record drives which correction breaks the X-basis case
    # (Y eigenstates cannot tell: X Z and Z X both act as Y on them).
    for name in ("plus", "one"):
        prep, undo = PREPS[name]
        text = f"{prep}\nH 1\nCX 1 2\nCX 0 1\nH 0\nM 0 1\nCX rec[-2] 2\nCZ rec[-1] 2\n{undo}\nM 2\n"
        r = records(oracle.Circuit(text), 4096, seed=3)
        assert 0.4 < r[:, 2].mean() < 0.6
    prep, undo = PREPS["plus_i"]
    # CZ with the record on the right acts the same as on the left.
    text = f"{prep}\nH 1\nCX 1 2\nCX 0 1\nH 0\nM 0 1\nCX rec[-1] 2\nCZ 2 rec[-2]\n{undo}\nM 2\n"
    assert not records(oracle.Circuit(text), 4096, seed=3)[:, 2].any()


@pytest.mark.parametrize("text,want", [
    ("X 0\nM 0\nCX rec[-1] 1\nM 1\n", [1, 1]),             # reference result 1 drives the X
    ("M 0\nCX rec[-1] 1\nM 1\n", [0, 0]),
    ("X 0\nM 0\nCY rec[-1] 1\nM 1\n", [1, 1]),
    ("X 0\nM 0\nCZ rec[-1] 1\nM 1\n", [1, 0]),
    ("X 0\nM 0\nH 1\nCZ rec[-1] 1\nH 1\nM 1\n", [1, 1]),
    ("X 0\nM 0\nH 1\nCY rec[-1] 1\nH 1\nM 1\n", [1, 1]),     # the Z part of Y
    ("X 0\nM 0\nH 1\nCX rec[-1] 1\nH 1\nM 1\n", [1, 0]),
    ("X 0\nM 0 1\nCX rec[-2] 2 rec[-1] 3\nM 2 3\n", [1, 0, 1, 0]),
    ("X 0\nM 0\nCX rec[-1] 1 1 2\nM 1 2\n", [1, 1, 1]),    # record pair, then a quantum pair
    ("X 0\nMR 0\nCX rec[-1] 0\nM 0\n", [1, 1]),
])
def test_deterministic_feedback_records(text, want):
    c = oracle.Circuit(text)
    assert c.reference().tolist() == want
    assert sv.canonical_reference(text) == want
    r = records(c, 256, seed=1)
    assert (r == np.array(want, dtype=bool)).all()


@pytest.mark.parametrize("gate,basis,flipped", [
    ("CX", "", True), ("CY", "", True), ("CZ", "", False),
    ("CX", "H", False), ("CY", "H", True), ("CZ", "H", True),
])
def test_noise_before_the_control_is_carried_by_the_frame(gate, basis, flipped):
    # X_ERROR(1) flips the controlling measurement in every shot, so the
    # frame must apply the Pauli the reference did not; measured in the Z or
    # (after H) the X basis.
    pre = f"{basis} 1\n" if basis else ""
    text = f"X_ERROR(1) 0\nM 0\n{pre}{gate} rec[-1] 1\n{pre}M 1\n"
    c = oracle.Circuit(text)
    assert c.reference().tolist() == [0, 0]
    r = records(c, 128)
    assert r[:, 0].all()
    assert (r[:, 1] == flipped).all()


@pytest.mark.parametrize("seed", range(16))
def test_canonical_reference_with_feedback_matches_state_vector(seed):
    rng = np.random.Generator(np.random.PCG64(900 + seed))
    n = int(rng.integers(2, 7))
    text = feedback_circuit(n, int(rng.integers(10, 60)), 4000 + seed, feedback=0.2)
    assert oracle.Circuit(text).reference().tolist() == sv.canonical_reference(text)


@pytest.mark.parametrize("seed", range(10))
def test_feedback_records_uniform_over_support(seed):
    text = feedback_circuit(4, 30, 5000 + seed, feedback=0.2)
    dist = sv.record_distribution(text)
    if len(dist) > 256:
        pytest.skip("too many outcomes for a chi-squared test")
    recs = records(oracle.Circuit(text), 16384, seed=seed)
    assert chi2_against(dist, recs) > 1e-4


@pytest.mark.parametrize("seed", range(8))
def test_noisy_feedback_records_match_exact_mixture(seed):
    rng = np.random.Generator(np.random.PCG64(177 + seed))
    while True:
        text = random_circuit(3, 14, seed=6000 + seed * 31 + int(rng.integers(1000)), noise=True,
                              p=0.15, collapse_weight=0.25, feedback=0.25)
        ops = sv.parse(text)
        sites = sum(1 for name, arg, t in ops if name in sv.NOISE)
        if 1 <= sites <= 3 and "rec[" in text:
            break
    dist = sv.noisy_record_distribution(text)
    recs = records(oracle.Circuit(text), 32768, seed=seed)
    assert chi2_against(dist, recs) > 1e-4


@pytest.mark.parametrize("text", [
    "M 0\nCX 1 rec[-1]\n",             # record as the target of CX
    "M 0\nCY 1 rec[-1]\n",
    "M 0 1\nCZ rec[-1] rec[-2]\n",     # both sides records
    "CX rec[-1] 0\n",                  # no measurement yet
    "M 0\nCX rec[-2] 1\n",             # reaches before the first measurement
    "M 0\nH rec[-1]\n",                # not a controllable gate
    "M 0\nSWAP rec[-1] 1\n",
    "M 0\nCX rec[-0] 1\n",
])
def test_bad_feedback_targets_are_rejected(text):
    with pytest.raises(oracle.OracleError):
        oracle.Circuit(text)
