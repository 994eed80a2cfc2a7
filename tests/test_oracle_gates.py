"""Pins of the oracle's gate table against the matrices printed in App. A
(tests/golden/app_a_gates.json) and the identities they satisfy."""
import json
import os

import numpy as np
import pytest

from oracle import gates as G


@pytest.mark.parametrize("name", sorted(G.TABLE))
def test_unitary(name):
    u = G.matrix(name)
    assert np.abs(u.conj().T @ u - np.eye(u.shape[0])).max() < 1e-14


def test_phase_family():
    # T = P(pi/4), T^2 = S = P(pi/2), S^2 = Z
    assert np.allclose(G.T @ G.T, G.S, atol=1e-15)
    assert np.allclose(G.S @ G.S, G.Z, atol=1e-15)
    assert np.allclose(G.P(np.pi), G.Z, atol=1e-15)


def test_paulis_and_h():
    assert np.allclose(G.X @ G.Y, 1j * G.Z)
    assert np.allclose(G.H @ G.X @ G.H, G.Z)
    assert np.allclose(G.H @ G.H, np.eye(2))


def test_fourth_root_x():
    assert np.allclose(np.linalg.matrix_power(G.X4, 4), G.X, atol=1e-14)


def test_sqrt_w_reading():
    # the reading e^{+i pi/4} on the diagonal squares to W = (X+Y)/sqrt(2)
    W = (G.X + G.Y) / np.sqrt(2)
    assert np.allclose(G.SQRTW @ G.SQRTW, W, atol=1e-14)
    # the printed diagonal e^{-i pi/4} is not unitary
    w = np.exp(-1j * np.pi / 4)
    printed = np.array([[w, -1j], [1, w]]) / np.sqrt(2)
    assert np.abs(printed.conj().T @ printed - np.eye(2)).max() > 0.5


def test_sqrt_swap():
    assert np.allclose(G.SQRTSWAP @ G.SQRTSWAP, G.SWAP, atol=1e-15)


def test_controlled_convention():
    # control is the first (most significant) qubit: |10> -> |11>
    e = np.zeros(4); e[2] = 1
    assert np.allclose(G.CNOT @ e, np.eye(4)[3])
    assert np.allclose(G.CS, np.diag([1, 1, 1, 1j]))
    assert np.allclose(G.CT, np.diag([1, 1, 1, np.exp(1j * np.pi / 4)]))
    assert np.allclose(G.CZ, np.diag([1, 1, 1, -1]))
    assert np.allclose(G.CH[2:, 2:], G.H)


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "app_a_gates.json")


def _printed(entry):
    env = {"sqrt": np.sqrt, "exp": np.exp, "cos": np.cos, "sin": np.sin, "pi": np.pi, "i": 1j}
    return np.array([[complex(eval(x, {"__builtins__": {}}, env)) for x in row] for row in entry["m"]])


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("name", sorted(_golden()["gates"]))
def test_printed_matrix(name):
    assert np.abs(G.matrix(name) - _printed(_golden()["gates"][name])).max() < 1e-15


def test_printed_sqrt_w_is_garbled_and_read_as_principal_root():
    p = _printed(_golden()["garbled"]["SQRTW"])
    assert np.abs(p.conj().T @ p - np.eye(2)).max() > 0.5
    # the reading differs from the print only on the diagonal, by conjugation
    assert np.allclose(np.diag(G.SQRTW), np.conj(np.diag(p)), atol=1e-15)
    assert np.allclose(G.SQRTW - np.diag(np.diag(G.SQRTW)), p - np.diag(np.diag(p)), atol=1e-15)
