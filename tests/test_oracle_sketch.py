"""Pins of the learned-sketch oracle: network gradients against central finite
differences, the pinball loss against its quantile property, the first Adam
step in closed form, and the randomized range finder against LAPACK SVDs."""
import numpy as np
import pytest

from oracle import sketch as SK


def test_gelu_values_and_derivative():
    x = np.linspace(-6, 6, 101)
    assert abs(SK.gelu(np.array([0.0]))[0]) == 0.0
    assert np.allclose(SK.gelu(np.array([8.0])), 8.0, atol=1e-12)
    assert np.allclose(SK.gelu(np.array([-8.0])), 0.0, atol=1e-12)
    h = 1e-6
    fd = (SK.gelu(x + h) - SK.gelu(x - h)) / (2 * h)
    assert np.abs(fd - SK.gelu_grad(x)).max() < 1e-8


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = SK.init_params(3)
    for k in P:
        P[k] = P[k] + 0.05 * rng.standard_normal(P[k].shape)
    X = rng.standard_normal((7, SK.N_IN))
    t = rng.standard_normal(7) * 2
    tau = 0.9
    y, cache = SK.mlp_forward(P, X)
    G = SK.mlp_backward(P, cache, y, t, tau)
    h = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = SK.pinball(SK.mlp_forward(P, X)[0], t, tau)
            flat[i] = old - h
            lm = SK.pinball(SK.mlp_forward(P, X)[0], t, tau)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            g = G[k].reshape(-1)[i]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, g)


def test_pinball_minimiser_is_the_quantile():
    rng = np.random.default_rng(1)
    t = rng.standard_normal(1001)
    cs = np.linspace(-3, 3, 6001)
    losses = [SK.pinball(np.full_like(t, c), t, 0.9) for c in cs]
    c_best = cs[int(np.argmin(losses))]
    assert abs(c_best - np.quantile(t, 0.9, method="inverted_cdf")) < 2e-3


def test_first_adam_step_is_sign_step():
    P = {"w": np.array([1.0, -2.0, 0.5])}
    G = {"w": np.array([0.3, -4.0, 1e-3])}
    st = {}
    SK.adam_step(P, G, st, lr=0.01)
    assert np.allclose(P["w"], [1.0 - 0.01, -2.0 + 0.01, 0.5 - 0.01], atol=1e-7)


def _low_rank(m, n, r, seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r)))[0]
    V = np.linalg.qr(rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r)))[0]
    s = np.sort(rng.random(r) + 0.1)[::-1]
    return (U * s) @ V.conj().T, s


def _gauss(shape, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


@pytest.mark.parametrize("r,s", [(5, 5), (5, 12), (17, 30)])
def test_range_finder_exact_when_sketch_covers_rank(r, s):
    A, sv = _low_rank(80, 40, r, seed=r)
    sigma, V, est = SK.range_finder(A, _gauss((80, s), 2), _gauss((40, 8), 3))
    assert np.abs(sigma[:r] - sv).max() < 1e-12
    assert est < 1e-12
    # V spans the row space: A V V^H = A
    assert np.abs(A @ V[:, :r] @ V[:, :r].conj().T - A).max() < 1e-12


def test_range_finder_tail_and_estimate():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((60, 50)) + 1j * rng.standard_normal((60, 50))
    s_full = np.linalg.svd(A, compute_uv=False)
    s = 20
    sigma, V, est = SK.range_finder(A, _gauss((60, s), 6), _gauss((50, 8), 7))
    Q = V
    true = np.linalg.norm(A - A @ Q @ Q.conj().T)
    # no rank-s projection beats the truncated SVD (Eckart-Young)
    assert true >= np.sqrt(np.sum(s_full[s:] ** 2)) - 1e-9
    # the probe estimate tracks the true residual
    assert 0.3 * true < est < 3.0 * true


def _gram(n, rank, decay, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((3 * n, rank)) + 1j * rng.standard_normal((3 * n, rank))
    Qx, _ = np.linalg.qr(X)
    Z = rng.standard_normal((rank, n)) + 1j * rng.standard_normal((rank, n))
    Qz, _ = np.linalg.qr(Z.conj().T)
    s = np.exp(-decay * np.arange(rank))
    A = (Qx * s) @ Qz.conj().T
    return A.conj().T @ A


def _cgauss(rows, cols, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))) / np.sqrt(2)


def test_gram_range_finder_exact_when_sketch_covers_rank():
    """G of rank 20 and a sketch of 28 columns: the eigenvalues are G's, the
    vectors span its range and the residual estimate vanishes."""
    n, r = 96, 20
    G = _gram(n, r, 0.3, seed=1)
    mu, V, est, Q = SK.gram_range_finder(G, _cgauss(n, r + 8, 2), _cgauss(n, 8, 3))
    lam = np.sort(np.linalg.eigvalsh(G))[::-1]
    assert np.abs(mu[:r] - lam[:r]).max() < 1e-12 * lam[0]
    assert np.abs(G @ V[:, :r] - V[:, :r] * mu[:r]).max() < 1e-12 * lam[0]
    assert est < 1e-12 * np.trace(G).real


def test_gram_range_finder_residual_estimate_and_tail():
    """Rank above the sketch: the estimate is an unbiased Frobenius estimate
    (many probes) and lies between the first missed eigenvalue's scale and the
    Frobenius norm of the tail; the kept eigenvalues underestimate G's."""
    n, r, s = 96, 60, 24
    G = _gram(n, r, 0.15, seed=4)
    omega = _cgauss(n, s, 5)
    mu, V, est, Q = SK.gram_range_finder(G, omega, _cgauss(n, 4000, 6))
    Rf = np.linalg.norm(G - G @ Q @ Q.conj().T)
    assert abs(est - Rf) < 0.05 * Rf
    lam = np.sort(np.linalg.eigvalsh(G))[::-1]
    assert lam[s] * 0.99 <= Rf <= np.sqrt(np.sum(lam[s:] ** 2)) * 100
    assert np.all(mu <= lam[:s] * (1 + 1e-12))
