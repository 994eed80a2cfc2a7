"""Pins of the oracle's MPS read-outs (Sec. II.B: the exact fidelity
F = |<psi_a|psi_b>|^2 of two normalised states).

`mps_tools.overlap` contracts a transfer matrix site by site.  It is checked
here against the definition of an MPS amplitude written out as a plain loop
over bit strings (psi(s_0..s_{n-1}) = B_0[:, s_0, :] B_1[:, s_1, :] ... as a
1 x 1 matrix product) on random complex, unnormalised MPS with ragged bond
dimensions, and against closed forms: a global phase leaves the infidelity at
zero, orthogonal product states give one, a product state's overlap is the
product of its one-site overlaps, and the overlap is conjugate-symmetric and
linear in its second argument.
"""
import itertools

import numpy as np
import pytest

from oracle import mps_tools as MT


def _random_mps(n, dims, seed):
    """Complex Gaussian site tensors (no canonical form, no normalisation)."""
    rng = np.random.default_rng(seed)
    full = [1] + list(dims) + [1]
    return [(rng.standard_normal((full[j], 2, full[j + 1])) +
             1j * rng.standard_normal((full[j], 2, full[j + 1]))) for j in range(n)]


def _amplitude_by_definition(B, bits):
    m = np.ones((1, 1), dtype=np.complex128)
    for t, s in zip(B, bits):
        m = m @ t[:, s, :]
    return m[0, 0]


def _state_by_definition(B):
    n = len(B)
    # qubit 0 is the most significant bit of the index
    return np.array([_amplitude_by_definition(B, bits) for bits in itertools.product((0, 1), repeat=n)])


RAGGED = [(5, [2, 3, 3, 2]), (7, [2, 4, 5, 3, 4, 2]), (8, [1, 3, 7, 2, 5, 3, 2]), (10, [2, 4, 8, 5, 9, 6, 7, 4, 2])]


@pytest.mark.parametrize("n,dims", RAGGED)
def test_overlap_equals_brute_force_inner_product(n, dims):
    A = _random_mps(n, dims, seed=n)
    B = _random_mps(n, [max(1, d - 1) for d in dims], seed=100 + n)
    a = _state_by_definition(A)
    b = _state_by_definition(B)
    exp = np.vdot(a, b)  # sum conj(a) b
    got = MT.overlap(A, B)
    assert abs(got - exp) <= 1e-12 * np.linalg.norm(a) * np.linalg.norm(b)
    # the amplitude read-out agrees with the definition too
    assert np.allclose(MT.amplitudes(A), a, rtol=0, atol=1e-12 * np.abs(a).max())
    inf = 1 - abs(exp) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)
    assert abs(MT.infidelity(A, B) - inf) < 1e-12


@pytest.mark.parametrize("n,dims", RAGGED[:3])
def test_overlap_conjugate_symmetric_and_linear(n, dims):
    A = _random_mps(n, dims, seed=1)
    B = _random_mps(n, dims, seed=2)
    C = _random_mps(n, dims, seed=3)
    scale = np.sqrt(abs(MT.overlap(A, A)) * abs(MT.overlap(B, B)))
    assert abs(MT.overlap(A, B) - np.conj(MT.overlap(B, A))) < 1e-13 * scale
    # <A|x B + y C>: a sum of two MPS is the block-diagonal MPS (first and last
    # sites concatenated along the open bond)
    x, y = 0.3 - 1.1j, -0.7 + 0.2j
    S = []
    for j in range(n):
        b, c = B[j], C[j]
        if j == 0:
            S.append(np.concatenate([x * b, y * c], axis=2))
        elif j == n - 1:
            S.append(np.concatenate([b, c], axis=0))
        else:
            t = np.zeros((b.shape[0] + c.shape[0], 2, b.shape[2] + c.shape[2]), dtype=np.complex128)
            t[: b.shape[0], :, : b.shape[2]] = b
            t[b.shape[0]:, :, b.shape[2]:] = c
            S.append(t)
    lhs = MT.overlap(A, S)
    rhs = x * MT.overlap(A, B) + y * MT.overlap(A, C)
    scale_c = np.sqrt(abs(MT.overlap(A, A)) * abs(MT.overlap(C, C)))
    assert abs(lhs - rhs) < 1e-13 * (abs(x) + abs(y)) * max(scale, scale_c)


def test_global_phase_gives_zero_infidelity():
    A = _random_mps(8, [2, 4, 6, 5, 4, 3, 2], seed=7)
    B = [t.copy() for t in A]
    B[3] = B[3] * np.exp(1j * 0.913) * 2.5  # phase and scale on one site
    assert abs(MT.infidelity(A, B)) < 1e-14
    assert abs(MT.infidelity(A, A)) < 1e-14


def _product(bits, phases=None):
    out = []
    for j, s in enumerate(bits):
        t = np.zeros((1, 2, 1), dtype=np.complex128)
        t[0, s, 0] = 1.0 if phases is None else np.exp(1j * phases[j])
        out.append(t)
    return out


def test_orthogonal_product_states_give_one():
    a = _product([0, 1, 1, 0, 1, 0])
    b = _product([0, 1, 1, 0, 1, 1])  # differs in the last qubit only
    assert MT.overlap(a, b) == 0
    assert MT.infidelity(a, b) == 1.0
    c = _product([1, 1, 1, 0, 1, 0])  # differs in the first qubit only
    assert MT.infidelity(a, c) == 1.0


def test_product_state_overlap_is_product_of_site_overlaps():
    rng = np.random.default_rng(5)
    n = 9
    u = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    v = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    A = [u[j].reshape(1, 2, 1) for j in range(n)]
    B = [v[j].reshape(1, 2, 1) for j in range(n)]
    exp = np.prod([np.vdot(u[j], v[j]) for j in range(n)])
    assert abs(MT.overlap(A, B) - exp) < 1e-12 * abs(exp)
    # a single-qubit rotation by theta on one site of |0...0>: F = cos^2(theta/2)
    th = 0.731
    a = _product([0] * n)
    b = _product([0] * n)
    b[4] = np.array([np.cos(th / 2), np.sin(th / 2)], dtype=np.complex128).reshape(1, 2, 1)
    assert abs(MT.infidelity(a, b) - np.sin(th / 2) ** 2) < 1e-15


def test_schmidt_and_entropy_readouts():
    # Bell pair on qubits (1, 2) of 4: one bond with two values 1/sqrt(2)
    psi = np.zeros(16, dtype=np.complex128)
    psi[0b0000] = psi[0b0110] = 2 ** -0.5
    s = MT.schmidt_from_state(psi, 4, 2)
    assert np.allclose(s[:2], [2 ** -0.5, 2 ** -0.5]) and np.allclose(s[2:], 0)
    assert abs(MT.entropy_bits(s) - 1.0) < 1e-14
    assert MT.entropy_bits(np.array([1.0])) == 0.0
    # GHZ-like flat spectrum of 2^k values carries k bits
    assert abs(MT.entropy_bits(np.full(8, 8 ** -0.5)) - 3.0) < 1e-14
