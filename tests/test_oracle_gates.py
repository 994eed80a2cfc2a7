"""Pins of the oracle's gate table against App. A identities."""
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
