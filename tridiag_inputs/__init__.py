"""Seeded synthetic symmetric tridiagonal inputs.

This module only *draws* inputs; it holds none of the eigensolver's
arithmetic.  Both the GPU path and the CPU oracle are fed from here so that
they see bit-identical (d, e).

Families follow the thesis' test-matrix appendix (App. D, "Test Matrices"):
1-2-1, Clement, Wilkinson W_n^+, Hermite, Legendre; plus the glued
Wilkinson matrices named in the mixed-precision chapter (Sec. 5.3, "clusters
within clusters") and i.i.d. uniform random tridiagonals.  Every generator is
deterministic in (n, seed): numpy's PCG64 via ``default_rng(seed)``, drawing d
first, then e.
"""
from __future__ import annotations

import math

import numpy as np

#: glue between W21+ blocks: sqrt of numpy's machine epsilon, 2**-26.
GLUE = 2.0 ** -26
#: size of the Wilkinson blocks in the glued family.
WBLOCK = 21


def random_uniform(n: int, seed: int = 0, lo: float = -1.0, hi: float = 1.0,
                   elo: float | None = None, ehi: float | None = None):
    """d_i, e_i i.i.d. uniform; e defaults to the same range as d."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(lo, hi, n)
    e = rng.uniform(lo if elo is None else elo, hi if ehi is None else ehi,
                    max(n - 1, 0))
    return d.astype(np.float64), e.astype(np.float64)


def one_two_one(n: int, offdiag: float = -1.0):
    """1-2-1 matrix: diagonal 2, off-diagonal +-1 (App. D)."""
    return np.full(n, 2.0), np.full(max(n - 1, 0), float(offdiag))


def clement(n: int):
    """Clement matrix: zero diagonal, beta_k = sqrt(k (n - k)) (App. D)."""
    k = np.arange(1, n, dtype=np.float64)
    return np.zeros(n), np.sqrt(k * (n - k))


def wilkinson_plus(n: int):
    """W_n^+: diagonal (m, m-1, ..., 1, 0, 1, ..., m), m = (n-1)/2, e = 1."""
    if n % 2 != 1:
        raise ValueError("W_n^+ needs odd n")
    m = (n - 1) // 2
    return np.abs(np.arange(n, dtype=np.float64) - m), np.ones(n - 1)


def glued_wilkinson(n: int, block: int = WBLOCK, glue: float = GLUE):
    """W21+ blocks (d = |10 - j|, e = 1) glued by e = glue between blocks.

    If ``block`` does not divide n the last block is the first n mod block
    rows of W21+ (a truncated block).
    """
    m = (block - 1) // 2
    j = np.arange(n) % block
    d = np.abs(j - m).astype(np.float64)
    e = np.ones(max(n - 1, 0))
    if n > 1:
        pos = np.arange(block - 1, n - 1, block)
        e[pos] = glue
    return d, e


def hermite(n: int):
    """Hermite matrix: zero diagonal, beta_k = sqrt(k) (App. D)."""
    return np.zeros(n), np.sqrt(np.arange(1, n, dtype=np.float64))


def legendre(n: int):
    """Legendre (Gauss) Jacobi matrix: zero diagonal, beta_k = k/sqrt(4k^2-1).

    The appendix indexes beta from 2; this is the same list shifted to the
    usual 1-based k = 1..n-1 (the Gauss-Legendre nodes are its eigenvalues).
    """
    k = np.arange(1, n, dtype=np.float64)
    return np.zeros(n), k / np.sqrt(4.0 * k * k - 1.0)


FAMILIES = {
    "random": lambda n, seed=0: random_uniform(n, seed),
    "121": lambda n, seed=0: one_two_one(n),
    "clement": lambda n, seed=0: clement(n),
    "glued_wilkinson": lambda n, seed=0: glued_wilkinson(n),
    "hermite": lambda n, seed=0: hermite(n),
    "legendre": lambda n, seed=0: legendre(n),
}


def family(name: str, n: int, seed: int = 0):
    return FAMILIES[name](n, seed)


def batch_sizes(batch: int, seed: int = 0, nmin: int = 32, nmax: int = 2048):
    """Sizes log-uniform in [nmin, nmax]: clip(floor(exp(U[ln nmin, ln nmax])))."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(math.log(nmin), math.log(nmax), batch)
    return np.clip(np.floor(np.exp(x)), nmin, nmax).astype(np.int64)


def batch_uniform(batch: int, seed: int = 0, nmin: int = 32, nmax: int = 2048,
                  dlo=-1.0, dhi=1.0, elo=0.1, ehi=1.0, sizes=None):
    """Concatenated batch of unreduced tridiagonals.

    Returns (sizes, n_offsets, d_cat, e_cat) where matrix b occupies
    [n_offsets[b], n_offsets[b+1]) of d_cat and e_cat; e_cat keeps one pad
    slot per matrix (its last entry, set to 0) so that both arrays share the
    offsets.
    """
    if sizes is None:
        sizes = batch_sizes(batch, seed, nmin, nmax)
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    rng = np.random.default_rng(seed + 1)
    d = rng.uniform(dlo, dhi, int(off[-1]))
    e = rng.uniform(elo, ehi, int(off[-1]))
    e[off[1:] - 1] = 0.0
    return sizes, off, d, e


def grad_weights(n: int, seed: int = 0, with_matrix: bool = True):
    """Loss weights c ~ N(0,1)^n and G ~ N(0,1)^{n x n} (column-major use)."""
    rng = np.random.default_rng(seed + 7)
    c = rng.standard_normal(n)
    G = rng.standard_normal((n, n)) if with_matrix else None
    return c, G
