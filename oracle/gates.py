"""Gate matrices used by the circuits (App. A, plus H/S/T of the workloads).

Convention: a k-qubit gate acting on qubits (q_0, ..., q_{k-1}) is a 2^k x 2^k
matrix whose row/column index is big-endian in that tuple: q_0 is the most
significant bit.  For CNOT, C-Y, C-Z, C-H, C-S, C-T the first qubit is the
control (App. A prints them in that convention).

Readings of App. A:
  * sqrt(W): the printed matrix has e^{-i pi/4} on the diagonal, which is not
    unitary; the principal square root of W = (X+Y)/sqrt(2) has e^{+i pi/4}
    there (W^2 = I, so sqrt(W) = (1+i)/2 I + (1-i)/2 W).  The latter is used.
  * C-S is printed without its "=" sign; it is read as diag(1, 1, 1, i).
"""
import numpy as np

_s2 = 1.0 / np.sqrt(2.0)
_w = np.exp(1j * np.pi / 4)

I2 = np.eye(2, dtype=np.complex128)
H = _s2 * np.array([[1, 1], [1, -1]], dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def P(phi: float) -> np.ndarray:
    """Phase gate P(phi) = diag(1, e^{i phi}) (App. A)."""
    return np.array([[1, 0], [0, np.exp(1j * phi)]], dtype=np.complex128)


S = P(np.pi / 2)
T = P(np.pi / 4)
P3PI4 = P(3 * np.pi / 4)
X4 = np.exp(1j * np.pi / 8) * np.array(
    [[np.cos(np.pi / 8), -1j * np.sin(np.pi / 8)],
     [-1j * np.sin(np.pi / 8), np.cos(np.pi / 8)]], dtype=np.complex128)
SQRTW = _s2 * np.array([[_w, -1j], [1, _w]], dtype=np.complex128)


def controlled(u: np.ndarray) -> np.ndarray:
    """The controlled gates of App. A: u on the second qubit when the first
    (the more significant index bit) is 1."""
    m = np.eye(4, dtype=np.complex128)
    m[2:, 2:] = u
    return m


CNOT = controlled(X)
CY = controlled(Y)
CZ = controlled(Z)
CH = controlled(H)
CS = controlled(S)
CT = controlled(T)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
SQRTSWAP = np.array([[1, 0, 0, 0],
                     [0, 0.5 * (1 + 1j), 0.5 * (1 - 1j), 0],
                     [0, 0.5 * (1 - 1j), 0.5 * (1 + 1j), 0],
                     [0, 0, 0, 1]], dtype=np.complex128)

TABLE = {
    "I": I2, "H": H, "X": X, "Y": Y, "Z": Z, "S": S, "T": T, "P3PI4": P3PI4,
    "X4": X4, "SQRTW": SQRTW,
    "CNOT": CNOT, "CY": CY, "CZ": CZ, "CH": CH, "CS": CS, "CT": CT,
    "SWAP": SWAP, "SQRTSWAP": SQRTSWAP,
}
CLIFFORD = {"I", "H", "X", "Y", "Z", "S", "CNOT", "CY", "CZ", "SWAP"}


def matrix(name: str) -> np.ndarray:
    """The matrix of a gate symbol of App. A (plus H, S, T)."""
    return TABLE[name]
