"""Oracle of the learned-sketch truncated SVD (FP64, CPU).

The paper says nothing about sketching; this is an addition to the method: a
small network predicts the rank a truncated SVD will keep, and that prediction
sets the size of a randomized range finder (N. Halko, P.-G. Martinsson,
J. A. Tropp, SIAM Rev. 53, 217 (2011), Algs. 4.1 and 5.1, a-posteriori error
estimate of Sec. 4.3).  The exact truncated SVD remains the fallback and the
reference.

Contents
  mlp_forward / mlp_backward : 12 -> 64 -> 64 -> 1 network with GELU (tanh form),
                               pinball (quantile) loss; pinned by central finite
                               differences.
  adam_step                  : Kingma & Ba (2015) update.
  range_finder               : Y = A^H Omega, Q = orth(Y), eigen of (A Q)^H (A Q),
                               probe estimate of ||A (I - Q Q^H)||_F; pinned by
                               exactness when the sketch covers the rank.
Parity of the trained network itself is unpinned (its weights come from data).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 12, 64
SQ2PI = np.sqrt(2.0 / np.pi)


def gelu(x):
    """GELU, tanh approximation: 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))."""
    return 0.5 * x * (1.0 + np.tanh(SQ2PI * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    t = np.tanh(SQ2PI * (x + 0.044715 * x ** 3))
    dt = (1.0 - t ** 2) * SQ2PI * (1.0 + 3 * 0.044715 * x ** 2)
    return 0.5 * (1.0 + t) + 0.5 * x * dt


def init_params(seed: int = 0):
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((N_H, N_IN)) * np.sqrt(2.0 / N_IN),
        "b1": np.zeros(N_H),
        "W2": rng.standard_normal((N_H, N_H)) * np.sqrt(2.0 / N_H),
        "b2": np.zeros(N_H),
        "w3": rng.standard_normal(N_H) * np.sqrt(1.0 / N_H),
        "b3": np.zeros(1),
    }


def mlp_forward(P, X):
    """X: (B, 12) -> (y (B,), cache)."""
    z1 = X @ P["W1"].T + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(z2)
    y = h2 @ P["w3"] + P["b3"][0]
    return y, (X, z1, h1, z2, h2)


def pinball(y, t, tau):
    """Mean quantile loss: tau (t - y) if t >= y else (1 - tau)(y - t)."""
    d = t - y
    return float(np.mean(np.where(d >= 0, tau * d, (tau - 1.0) * d)))


def mlp_backward(P, cache, y, t, tau):
    """Gradients of the mean pinball loss w.r.t. every parameter."""
    X, z1, h1, z2, h2 = cache
    B = X.shape[0]
    d = t - y
    gy = np.where(d >= 0, -tau, 1.0 - tau) / B
    g = {"w3": h2.T @ gy, "b3": np.array([gy.sum()])}
    gh2 = np.outer(gy, P["w3"])
    gz2 = gh2 * gelu_grad(z2)
    g["W2"] = gz2.T @ h1
    g["b2"] = gz2.sum(0)
    gh1 = gz2 @ P["W2"]
    gz1 = gh1 * gelu_grad(z1)
    g["W1"] = gz1.T @ X
    g["b1"] = gz1.sum(0)
    return g


def adam_step(P, G, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in P:
        m = state.setdefault("m_" + k, np.zeros_like(P[k]))
        v = state.setdefault("v_" + k, np.zeros_like(P[k]))
        m[:] = b1 * m + (1 - b1) * G[k]
        v[:] = b2 * v + (1 - b2) * G[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        P[k] -= lr * mh / (np.sqrt(vh) + eps)


def range_finder(A, omega, probes):
    """Right range finder of A (rows x cols): Y = A^H omega (cols x s),
    Q = orthonormal basis of Y (eigen-decomposition of Y^H Y, directions with
    eigenvalue below 1e-24 of the largest dropped), then the SVD of A Q through
    the eigen-decomposition of (A Q)^H (A Q).  Returns sigma (descending),
    right vectors V = Q W (cols x s'), and the probe estimate
    sqrt(mean_i ||A (I - Q Q^H) g_i||^2) of ||A (I - Q Q^H)||_F."""
    Y = A.conj().T @ omega
    lam, U = np.linalg.eigh(Y.conj().T @ Y)
    keep = lam > 1e-24 * max(lam.max(), 1e-300)
    Q = Y @ (U[:, keep] / np.sqrt(lam[keep]))
    Z = A @ Q
    mu, W = np.linalg.eigh(Z.conj().T @ Z)
    order = np.argsort(mu)[::-1]
    mu, W = mu[order], W[:, order]
    sigma = np.sqrt(np.maximum(mu, 0.0))
    Pg = probes - Q @ (Q.conj().T @ probes)
    est = np.sqrt(np.mean(np.sum(np.abs(A @ Pg) ** 2, axis=0)))
    return sigma, Q @ W, est


def gram_range_finder(G, omega, probes):
    """The same range finder with the Hermitian Gram matrix G (n x n) as the
    operator, as the split sweep uses it: Y = G omega, Q an orthonormal basis
    of Y (Householder QR here), H = Q^H G Q = W diag(mu) W^H, V = Q W, and the
    probe estimate sqrt(mean_i ||G (I - Q Q^H) g_i||^2) of ||G (I - Q Q^H)||_F.
    Returns (mu descending, V, est, Q)."""
    Y = G @ omega
    Q, _ = np.linalg.qr(Y)
    H = Q.conj().T @ G @ Q
    H = (H + H.conj().T) / 2
    mu, W = np.linalg.eigh(H)
    order = np.argsort(mu)[::-1]
    mu, W = mu[order], W[:, order]
    Pg = probes - Q @ (Q.conj().T @ probes)
    est = np.sqrt(np.mean(np.sum(np.abs(G @ Pg) ** 2, axis=0)))
    return mu, Q @ W, est, Q
