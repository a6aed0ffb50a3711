"""Accuracy measures for computed eigenpairs -- test infrastructure.

Residual and orthogonality follow the thesis' accuracy goals (Sec. 3.1: a
residual of O(n eps ||T||) and |z_i^* z_j| = O(n eps)); eps = 2^-53, the unit
roundoff; ||T|| is the spectral norm, max(|lambda_1|, |lambda_n|).
"""
from __future__ import annotations

import numpy as np

EPS = 2.0 ** -53


def tmatvec(d, e, X):
    """T @ X for T = tridiag(e, d, e), X of shape (n,) or (n, m)."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    Y = d[:, None] * X
    if len(e):
        Y[:-1] += e[:, None] * X[1:]
        Y[1:] += e[:, None] * X[:-1]
    return Y[:, 0] if vec else Y


def residuals(d, e, w, Z):
    """||T z_i - w_i z_i||_2 for every column."""
    R = tmatvec(d, e, Z) - Z * np.asarray(w)[None, :]
    return np.linalg.norm(R, axis=0)


def orthogonality(Z):
    """||Z^T Z - I||_max."""
    G = Z.T @ Z
    G[np.diag_indices_from(G)] -= 1.0
    return float(np.max(np.abs(G))) if G.size else 0.0


def tnorm_of(w):
    return float(np.max(np.abs(w))) if len(w) else 0.0


def scaled(d, e, w, Z, tnorm=None):
    """(max residual / (n eps ||T||), orthogonality / (n eps))."""
    n = len(d)
    if tnorm is None:
        tnorm = tnorm_of(w)
    if tnorm == 0.0:
        tnorm = 1.0
    r = float(np.max(residuals(d, e, w, Z))) if Z.shape[1] else 0.0
    return r / (n * EPS * tnorm), orthogonality(Z) / (n * EPS)


def subspace_sigma_min(Za, Zb):
    """Smallest singular value of Za^T Zb (1 when the spans agree)."""
    s = np.linalg.svd(Za.T @ Zb, compute_uv=False)
    return float(np.min(s)) if s.size else 1.0


def sign_normalize(Z):
    """Entry of largest magnitude positive (ties to the lowest index)."""
    Z = np.array(Z, dtype=np.float64, copy=True)
    if Z.size == 0:
        return Z
    idx = np.argmax(np.abs(Z), axis=0)
    s = np.sign(Z[idx, np.arange(Z.shape[1])])
    s[s == 0] = 1.0
    return Z * s[None, :]
