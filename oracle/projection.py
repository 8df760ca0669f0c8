"""SVD projection to d reduced dimensions (section 4.1, stage 1: dimensionality reduction).

The paper factors X = U S V^T, keeps the d right singular vectors with the
largest singular values and stores x_primary = (U S)_{1..d}, which equals
x^T V_d; V^T V = I means distances split exactly into a primary part and a
residual part.

Readings where the paper is silent:
* centring: the subspace is chosen from the covariance about the mean for the
  L2 metric (it best preserves pairwise distances) and from the raw second
  moment X^T X / N for inner product (the literal "SVD of X").  Vectors are
  never shifted, so the primary + residual split holds for both.
* sign: each kept column is flipped so that its entry of largest magnitude is
  positive (ties up to rounding: the lowest row index).
"""

from __future__ import annotations

import numpy as np


def second_moment(X, center: bool):
    """(matrix whose eigenvectors are the right singular vectors, mean) in fp64."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    G = X.T @ X
    mu = X.sum(0) / n
    if center:
        return G / n - np.outer(mu, mu), mu
    return G / n, mu


def fit_projection(X, d_r: int, metric: str = "l2", center: bool | None = None):
    """Return (V_d [D][d_r], eigenvalues [D] descending, mean [D]), all fp64."""
    if center is None:
        center = metric == "l2"
    M, mu = second_moment(X, center)
    w, V = np.linalg.eigh(M)
    order = np.argsort(-w, kind="stable")
    w = w[order]
    V = V[:, order]
    for j in range(V.shape[1]):
        mag = np.abs(V[:, j])
        # the first row whose magnitude equals the maximum up to rounding
        i = int(np.nonzero(mag >= mag.max() * (1.0 - 1e-12))[0][0])
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V[:, :d_r].copy(), w, mu


def project(X, V) -> np.ndarray:
    """x_primary = x^T V_d for every row (fp64)."""
    return np.asarray(X, dtype=np.float64) @ np.asarray(V, dtype=np.float64)
