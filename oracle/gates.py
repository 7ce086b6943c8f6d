"""Unitary matrices of the supported Clifford gates (test infrastructure only).

These are the textbook definitions, with the convention sqrt(Z) = diag(1, i)
that the paper fixes in Sec. 5.7, and sqrt(Y) as printed there.  They are an
independent specification of every gate: the test-suite derives each gate's
stabilizer tableau from its matrix (U g U^dagger for each generator g,
Sec. 2.3) and compares it with the oracle's hand-written table, following the
redundant-specification testing of Sec. 5.7.
"""
from __future__ import annotations

import itertools

import numpy as np

I2 = np.eye(2, dtype=complex)
X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = {"_": I2, "I": I2, "X": X, "Y": Y, "Z": Z}
s2 = 1 / np.sqrt(2)

SQRT_Z = np.diag([1, 1j])
H = (X + Z) * s2
H_XY = (X + Y) * s2
H_YZ = (Y + Z) * s2
# sqrt(Y) is fixed by the identity sqrt(Y) = H_YZ . sqrt(Z) . H_YZ that Sec. 5.7
# gives to pick the principal root consistently across axes.  The matrix
# printed next to it, 1/2 [[1 - i, 1 - i], [i - 1, 1 - i]] (with its tableau
# X -> +Z, Z -> -X), is the other root; it is kept here as PRINTED_ROOT_OF_Y
# and equals SQRT_Y_DAG up to global phase.
SQRT_Y = H_YZ @ SQRT_Z @ H_YZ
PRINTED_ROOT_OF_Y = 0.5 * np.array([[1 - 1j, 1 - 1j], [1j - 1, 1 - 1j]])
SQRT_X = H @ SQRT_Z @ H


def _controlled(u):
    m = np.zeros((4, 4), dtype=complex)
    # qubit 0 (control) is the low bit of the basis index; qubit 1 (target) the high bit.
    for b in range(4):
        c, t = b & 1, b >> 1
        for t2 in range(2):
            amp = u[t2, t] if c else (1.0 if t2 == t else 0.0)
            m[c | (t2 << 1), b] += amp
    return m


SWAP = np.zeros((4, 4), dtype=complex)
for _b in range(4):
    SWAP[((_b & 1) << 1) | (_b >> 1), _b] = 1

UNITARIES = {
    "I": I2, "X": X, "Y": Y, "Z": Z,
    "H": H, "H_XY": H_XY, "H_YZ": H_YZ,
    "S": SQRT_Z, "S_DAG": SQRT_Z.conj().T,
    "SQRT_X": SQRT_X, "SQRT_X_DAG": SQRT_X.conj().T,
    "SQRT_Y": SQRT_Y, "SQRT_Y_DAG": SQRT_Y.conj().T,
    "CX": _controlled(X), "CY": _controlled(Y), "CZ": _controlled(Z), "SWAP": SWAP,
}


def pauli_matrix(s: str) -> np.ndarray:
    """Matrix of a signed Pauli string like '-XZ'; character k acts on qubit k
    (qubit k is bit k of the basis index)."""
    sign = -1 if s[0] == "-" else 1
    m = np.array([[1]], dtype=complex)
    for ch in s[1:]:
        m = np.kron(PAULI[ch], m)   # later qubits are higher bits
    return sign * m


def all_paulis(k: int):
    for t in itertools.product("_XYZ", repeat=k):
        yield "".join(t)


def decompose(m: np.ndarray, k: int) -> str:
    """Writes +-P for a matrix equal to a signed Hermitian Pauli product."""
    for p in all_paulis(k):
        for sign in "+-":
            if np.allclose(m, pauli_matrix(sign + p), atol=1e-9):
                return sign + p
    raise ValueError("not a signed Pauli product")


def tableau_from_unitary(u: np.ndarray):
    """Images U g U^dagger of X_1, Z_1 (, X_2, Z_2) as signed Pauli strings."""
    k = 1 if u.shape[0] == 2 else 2
    out = []
    for q in range(k):
        for g in "XZ":
            s = ["_"] * k
            s[q] = g
            out.append(decompose(u @ pauli_matrix("+" + "".join(s)) @ u.conj().T, k))
    return out


def unsigned_frame_map(u: np.ndarray):
    """The xz-linear map of a gate on Pauli frames (signs dropped), as a
    dict from input (x0, z0[, x1, z1]) bit tuples to output bit tuples."""
    k = 1 if u.shape[0] == 2 else 2
    table = {}
    for bits in itertools.product((0, 1), repeat=2 * k):
        s = ""
        for q in range(k):
            x, z = bits[2 * q], bits[2 * q + 1]
            s += "Y" if x and z else "X" if x else "Z" if z else "_"
        img = decompose(u @ pauli_matrix("+" + s) @ u.conj().T, k)[1:]
        out = []
        for ch in img:
            out += [int(ch in "XY"), int(ch in "ZY")]
        table[bits] = tuple(out)
    return table
