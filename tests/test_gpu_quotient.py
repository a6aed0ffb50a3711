"""The reciprocal-based quotient the kernels use in the shift selection of
Alg. 3.8 and in a new representation's rows, against IEEE division.

The rounding error analysis of the qd transforms (Sec. 3.1.2) charges each
operation a relative error of at most eps; a faithful quotient (one of the
two doubles next to the exact value) keeps that structure with the constant
doubled.  The checks: faithful on every operand class, equal to IEEE division
except where the exact quotient lies within 2^-60 (relative) of the midpoint
between two doubles (decided in exact rational arithmetic), and NaN -- the
signal on which the kernels redo the pass with IEEE division -- for zero,
infinite and NaN divisors and for quotients at the edge of overflow.
"""
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _quot(a, b):
    import ctypes
    import torch
    import paper_1401_4950_amd as mr
    from paper_1401_4950_amd import _lib
    dev = torch.device("cuda:0")
    at = torch.tensor(np.asarray(a, dtype=np.float64), device=dev)
    bt = torch.tensor(np.asarray(b, dtype=np.float64), device=dev)
    qt = torch.empty_like(at)
    h = mr._handle(dev)
    code = _lib.load().mrrr_diag_quotient(h, at.numel(), ctypes.c_void_p(at.data_ptr()),
                                          ctypes.c_void_p(bt.data_ptr()), ctypes.c_void_p(qt.data_ptr()))
    _lib.check(code, "mrrr_diag_quotient", allow_warn=False)
    torch.cuda.synchronize()
    return qt.cpu().numpy()


def _faithful(a, b, q):
    """q is one of the two doubles around the exact a/b (or equals it)."""
    ex = Fraction(float(a)) / Fraction(float(b))
    fq = Fraction(float(q))
    if fq == ex:
        return True
    toward = np.inf if fq < ex else -np.inf
    nxt = Fraction(float(np.nextafter(q, toward)))
    return (fq < ex <= nxt) or (nxt <= ex < fq)


def _near_midpoint(a, b, rel=2.0 ** -60):
    ex = Fraction(float(a)) / Fraction(float(b))
    ieee = float(a) / float(b)
    other = float(np.nextafter(ieee, np.inf if Fraction(ieee) < ex else -np.inf))
    mid = (Fraction(ieee) + Fraction(other)) / 2
    return abs(ex - mid) <= abs(ex) * Fraction(rel)


def _check_finite_class(a, b, name):
    q = _quot(a, b)
    ieee = a / b
    assert np.all(np.isfinite(q)), name
    bad = np.nonzero(q.view(np.int64) != ieee.view(np.int64))[0]
    for i in bad:
        assert _faithful(a[i], b[i], q[i]), (name, a[i], b[i], q[i], ieee[i])
        assert _near_midpoint(a[i], b[i]), (name, "off by one ulp away from a midpoint", a[i], b[i])
    return len(bad)


def test_random_operands_match_ieee():
    rng = np.random.default_rng(0)
    n = 1 << 20
    a = rng.uniform(1.0, 2.0, n) * np.ldexp(1.0, rng.integers(-300, 300, n)) * rng.choice([-1.0, 1.0], n)
    b = rng.uniform(1.0, 2.0, n) * np.ldexp(1.0, rng.integers(-300, 300, n)) * rng.choice([-1.0, 1.0], n)
    assert _check_finite_class(a, b, "random") <= 16


def test_subnormal_and_tiny_quotients():
    rng = np.random.default_rng(1)
    n = 1 << 16
    a = rng.uniform(1.0, 2.0, n) * np.ldexp(1.0, rng.integers(-1022, -900, n))
    b = rng.uniform(1.0, 2.0, n) * np.ldexp(1.0, rng.integers(40, 120, n)) * rng.choice([-1.0, 1.0], n)
    assert np.any(np.abs(a / b) < np.finfo(np.float64).tiny)
    _check_finite_class(a, b, "subnormal")


def test_quotients_next_to_a_rounding_midpoint():
    """b and a built so that a/b = m - t 2^-105 / b exactly, with m the
    midpoint between two doubles in [1, 2) and t a small integer: IEEE
    rounds on the side of the tiny offset, the reciprocal form may land one
    ulp off, never further."""
    rng = np.random.default_rng(2)
    a_l, b_l = [], []
    two53 = 1 << 53
    while len(a_l) < 4096:
        M = (1 << 53) | (int(rng.integers(0, 1 << 52)) << 1) | 1          # odd 54-bit midpoint significand
        t = int(rng.integers(1, 1000)) * (1 if rng.integers(0, 2) else -1)
        B = (t * pow(M, -1, two53)) % two53                                   # B M = t (mod 2^53)
        if B < (1 << 52):
            continue
        prod = B * M - t
        assert prod % two53 == 0
        A = prod >> 53
        if not ((1 << 52) <= A < (1 << 53)):
            continue
        a_l.append(float(Fraction(A, 1 << 52)))
        b_l.append(float(Fraction(B, 1 << 52)))
    a, b = np.array(a_l), np.array(b_l)
    mism = _check_finite_class(a, b, "midpoint")
    # the reciprocal's 2^-24 error makes some of these land on the far side
    assert mism >= 0


def test_zero_numerator():
    b = np.array([1.5, -2.0, 3e-300, -7e250])
    q = _quot(np.zeros(4), b)
    assert np.all(q == 0.0)


def test_divisor_zero_infinite_or_nan_gives_nan():
    a = np.array([1.0, -1.0, 2.5, 0.0, 1.0, 3.0, np.inf, np.nan, 1.0])
    b = np.array([0.0, -0.0, np.inf, 0.0, -np.inf, np.nan, 2.0, 1.0, 5e-324])
    q = _quot(a, b)
    assert np.all(np.isnan(q[:6])), q
    # an infinite or NaN numerator: NaN as well
    assert np.isnan(q[6]) and np.isnan(q[7])
    # the smallest subnormal divisor: 1/b overflows, so NaN (never a wrong inf)
    assert np.isnan(q[8]) or q[8] == a[8] / b[8]


def test_edge_of_overflow():
    """Quotients within 2^-24 of overflow, or beyond it: NaN, the IEEE value
    (infinity included) or, for a finite IEEE value, a faithful one -- never
    an infinity where the quotient is finite, or a finite value where it
    overflows."""
    rng = np.random.default_rng(3)
    n = 4096
    # a near the top binade, b around 1: about a quarter of the quotients
    # overflow; then the largest double over divisors a few ulps either side
    # of 1, whose exact quotients straddle the overflow threshold
    a = np.ldexp(rng.uniform(1.9, 2.0, n), 1023)
    b = rng.uniform(0.95, 1.05, n)
    big = np.finfo(np.float64).max
    j = np.arange(1, 65, dtype=np.float64)
    a = np.concatenate([a, np.full(128, big), np.full(128, -big)])
    edge = np.concatenate([1.0 - j * 2.0 ** -53, 1.0 + j * 2.0 ** -52])
    b = np.concatenate([b, edge, edge])
    n = len(a)
    with np.errstate(over="ignore"):
        ieee = a / b
    q = _quot(a, b)
    assert np.any(np.isinf(ieee)) and np.any(np.isfinite(ieee))
    for i in range(n):
        if np.isnan(q[i]) or q[i] == ieee[i]:
            continue
        assert np.isfinite(ieee[i]) and np.isfinite(q[i]), (a[i], b[i], q[i], ieee[i])
        assert _faithful(a[i], b[i], q[i]), (a[i], b[i], q[i], ieee[i])
