"""CPU oracle for the symmetric tridiagonal eigenproblem -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this package.  It shares no code with the GPU library
(``paper_1401_4950_amd``) and neither imports the other.

The solver itself is plain C (``tridiag_oracle.c``: Gershgorin, Sturm-count
bisection, inverse iteration with Gram-Schmidt inside clusters, cyclic
Jacobi); this module builds it with gcc and wraps it with ctypes/numpy.  The
backward formulas (``grad``) are numpy on top of the oracle's (w, Z).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .metrics import EPS  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tridiag_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

RANGE = {"all": 0, "a": 0, "value": 1, "v": 1, "index": 2, "i": 2}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fno-fast-math",
                               "-ffp-contract=off", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, dp, ip = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        lib.orc_gershgorin.argtypes = [i64, dp, dp, dp]
        lib.orc_split.argtypes = [i64, dp, ctypes.c_double, ip]
        lib.orc_split.restype = i64
        lib.orc_negcount.argtypes = [i64, dp, dp, ctypes.c_double, ctypes.c_double]
        lib.orc_negcount.restype = i64
        lib.orc_negcount_many.argtypes = [i64, dp, dp, i64, dp, ip]
        lib.orc_negcount_many.restype = None
        lib.orc_solve.argtypes = [i64, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  i64, i64, dp, dp, i64, ctypes.c_uint64, ctypes.c_double]
        lib.orc_solve.restype = i64
        lib.orc_eigval_index.argtypes = [i64, dp, dp, i64]
        lib.orc_eigval_index.restype = ctypes.c_double
        lib.orc_sign_fix.argtypes = [i64, dp]
        lib.orc_sign_fix.restype = None
        lib.orc_jacobi.argtypes = [i64, dp, i64, dp, dp, i64]
        lib.orc_jacobi.restype = ctypes.c_int
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    _load().orc_set_num_threads(int(t))


def gershgorin(d, e):
    """(g_l, g_u, bnorm) per App. B, Alg. B.3 (inflated interval)."""
    d, e = _c(d), _c(e)
    out = np.zeros(3)
    _load().orc_gershgorin(len(d), _p(d), _p(e if len(e) else np.zeros(1)), _p(out))
    return float(out[0]), float(out[1]), float(out[2])


def split_points(d, e):
    """Block start rows (plus n at the end) under |e_i| <= eps sqrt(n) bnorm."""
    d, e = _c(d), _c(e)
    n = len(d)
    bnorm = gershgorin(d, e)[2]
    starts = np.zeros(n + 1, dtype=np.int64)
    nb = _load().orc_split(n, _p(e if len(e) else np.zeros(1)), bnorm,
                           starts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return starts[: nb + 1].copy()


def negcount(d, e, sigma, pivmin=None):
    """Sturm count of T (App. B, Alg. B.1): #eigenvalues < sigma."""
    d, e = _c(d), _c(e)
    if pivmin is None:
        pivmin = np.finfo(np.float64).tiny * max(1.0, float(np.max(e * e)) if len(e) else 1.0)
    return int(_load().orc_negcount(len(d), _p(d), _p(e if len(e) else np.zeros(1)),
                                    float(sigma), float(pivmin)))


def negcounts(d, e, shifts):
    """Sturm counts of T (App. B, Alg. B.1) at every shift, in parallel."""
    d, e = _c(d), _c(e)
    shifts = _c(shifts)
    out = np.zeros(len(shifts), dtype=np.int64)
    _load().orc_negcount_many(len(d), _p(d), _p(e if len(e) else np.zeros(1)), len(shifts), _p(shifts),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def solve(d, e, select="all", vl=0.0, vu=0.0, il=1, iu=None, vectors=True,
          seed=0, orfac=1e-3):
    """Eigenpairs of tridiag(e, d, e): (w ascending, Z column-major n x m).

    select: 'all', 'value' ([vl, vu) half-open) or 'index' (il..iu, 1-based).
    """
    d, e = _c(d), _c(e)
    n = len(d)
    if iu is None:
        iu = n
    w = np.zeros(max(n, 1))
    Z = np.zeros((max(n, 1), max(n, 1)), order="F") if vectors else None
    m = _load().orc_solve(n, _p(d), _p(e if len(e) else np.zeros(1)), RANGE[select],
                          float(vl), float(vu), int(il), int(iu), _p(w),
                          _p(Z) if vectors else None, max(n, 1), int(seed), float(orfac))
    if m < 0:
        raise ValueError("oracle: invalid arguments")
    w = w[:m].copy()
    if vectors:
        return w, np.asfortranarray(Z[:n, :m])
    return w


def eigval_index(d, e, k):
    """k-th smallest eigenvalue (1-based) of T, to full accuracy: bisection
    on the Sturm count of T after the same splitting as ``solve``."""
    d, e = _c(d), _c(e)
    return float(_load().orc_eigval_index(len(d), _p(d), _p(e if len(e) else np.zeros(1)), int(k)))


def sign_fix(x):
    """The oracle's sign convention applied to a copy of the vector x."""
    x = np.array(x, dtype=np.float64, copy=True)
    _load().orc_sign_fix(len(x), _p(x))
    return x


def jacobi(A):
    """Cyclic Jacobi on a dense symmetric matrix: (w ascending, V)."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), order="F")
    _load().orc_jacobi(n, _p(A), n, _p(w), _p(V), n)
    return w, V


def dense(d, e):
    d, e = _c(d), _c(e)
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def jacobi_tridiag(d, e):
    return jacobi(dense(d, e))


def grad(w, Z, wbar=None, Zbar=None, tnorm=None, gap_mask_rel=1e-8):
    """Reverse-mode gradient of a loss L(w, Z) w.r.t. (d, e).

    Eigenvalue part: dbar_j = sum_i wbar_i z_ji^2, ebar_j = 2 sum_i wbar_i
    z_ji z_j+1,i.  Eigenvector part: M = diag(wbar) + F o (Z^T Zbar) with
    F_ab = 1/(w_b - w_a) (zero on the diagonal and where |w_b - w_a| <
    gap_mask_rel*||T||, those pairs counted); Tbar = Z M Z^T; dbar =
    diag(Tbar), ebar_j = Tbar_{j,j+1} + Tbar_{j+1,j}.  Returns (dbar, ebar,
    n_masked).
    """
    w = np.asarray(w, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    n = Z.shape[0]
    if tnorm is None:
        tnorm = float(np.max(np.abs(w))) if len(w) else 0.0
    m = Z.shape[1]
    M = np.zeros((m, m))
    if wbar is not None:
        M[np.arange(m), np.arange(m)] += np.asarray(wbar, dtype=np.float64)
    n_masked = 0
    if Zbar is not None:
        C = Z.T @ np.asarray(Zbar, dtype=np.float64)
        diff = w[None, :] - w[:, None]            # diff[a, b] = w_b - w_a
        off = ~np.eye(m, dtype=bool)
        mask = off & (np.abs(diff) < gap_mask_rel * tnorm)
        n_masked = int(mask.sum())
        F = np.zeros((m, m))
        ok = off & ~mask
        F[ok] = 1.0 / diff[ok]
        M += F * C
    Y = Z @ M                                       # Tbar = Y Z^T
    dbar = np.einsum("ja,ja->j", Y, Z)
    ebar = np.einsum("ja,ja->j", Y[:-1], Z[1:]) + np.einsum("ja,ja->j", Z[:-1], Y[1:])
    return dbar, ebar, n_masked
