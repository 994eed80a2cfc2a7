"""Gate matrices handed to the library (App. A of arXiv:2502.19289 plus H, S, T).

Big-endian in the gate's qubit tuple; controlled gates have the control first.
sqrt(W) takes e^{+i pi/4} on its diagonal (the principal square root of
W = (X+Y)/sqrt(2)); C-S is diag(1, 1, 1, i).
"""
import cmath
import math

import numpy as np


def _c(rows):
    return np.array(rows, dtype=np.complex128)


def _phase(phi):
    return _c([[1, 0], [0, cmath.exp(1j * phi)]])


def _ctrl(u):
    m = np.eye(4, dtype=np.complex128)
    m[2:, 2:] = u
    return m


_r = 1 / math.sqrt(2)
_w = cmath.exp(1j * math.pi / 4)
_c8, _s8 = math.cos(math.pi / 8), math.sin(math.pi / 8)

ONE = {
    "I": _c([[1, 0], [0, 1]]),
    "H": _c([[_r, _r], [_r, -_r]]),
    "X": _c([[0, 1], [1, 0]]),
    "Y": _c([[0, -1j], [1j, 0]]),
    "Z": _c([[1, 0], [0, -1]]),
    "S": _phase(math.pi / 2),
    "T": _phase(math.pi / 4),
    "P3PI4": _phase(3 * math.pi / 4),
    "X4": cmath.exp(1j * math.pi / 8) * _c([[_c8, -1j * _s8], [-1j * _s8, _c8]]),
    "SQRTW": _r * _c([[_w, -1j], [1, _w]]),
}
TWO = {
    "CNOT": _ctrl(ONE["X"]), "CY": _ctrl(ONE["Y"]), "CZ": _ctrl(ONE["Z"]),
    "CH": _ctrl(ONE["H"]), "CS": _ctrl(ONE["S"]), "CT": _ctrl(ONE["T"]),
    "SWAP": _c([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]]),
    "SQRTSWAP": _c([[1, 0, 0, 0], [0, 0.5 + 0.5j, 0.5 - 0.5j, 0],
                    [0, 0.5 - 0.5j, 0.5 + 0.5j, 0], [0, 0, 0, 1]]),
}
GATES = {**ONE, **TWO}
