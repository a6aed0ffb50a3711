"""Pins for the CPU oracle against facts fixed outside it.

Every check compares the oracle with something it does not compute itself:
closed-form spectra and eigenvectors (App. D), brute-force dense Jacobi,
trace/Frobenius invariants, Weyl's bound for glued matrices, Sturm counts
against the returned spectrum, and finite differences for the gradient.
"""
import json
import os

import numpy as np
import pytest

import tridiag_inputs as ti
from oracle import metrics as M

EPS = M.EPS
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def test_golden_closed_forms(orc):
    cases = json.load(open(GOLDEN))["cases"]
    assert len(cases) >= 10
    for c in cases:
        n = c["n"]
        if c["family"] == "121":
            d, e = np.full(n, c["d"]), np.full(n - 1, c["e"])
        else:
            d, e = ti.clement(n)
        w = orc.solve(d, e, vectors=False)
        ref = np.array(c["eigenvalues"])
        tn = max(np.max(np.abs(ref)), 1.0)
        assert np.max(np.abs(w - ref)) <= 4 * EPS * tn * max(n, 1), (c["family"], n)


@pytest.mark.parametrize("n", [1, 2, 3, 64, 1000])
def test_121_closed_form_values_and_vectors(orc, n):
    d, e = ti.one_two_one(n, -1.0)
    w, Z = orc.solve(d, e)
    k = np.arange(1, n + 1)
    lam = 2.0 - 2.0 * np.cos(np.pi * k / (n + 1))
    assert np.max(np.abs(w - lam)) <= 4 * n * EPS * 4.0
    # sine eigenvectors for e = -1: z_j(i) = sqrt(2/(n+1)) sin(i j pi/(n+1))
    i = np.arange(1, n + 1)[:, None]
    S = np.sqrt(2.0 / (n + 1)) * np.sin(i * k[None, :] * np.pi / (n + 1))
    S = M.sign_normalize(S)
    gaps = np.diff(lam)
    gap = np.minimum(np.r_[np.inf, gaps], np.r_[gaps, np.inf])
    sep = gap >= 1e-3 * 4.0
    dots = np.abs(np.sum(Z * S, axis=0))
    assert np.all(dots[sep] >= 1 - 1e-10)
    # the whole basis spans the same space; cluster members per subspace
    assert M.subspace_sigma_min(Z, S) >= 1 - 1e-8


@pytest.mark.parametrize("n", [1, 2, 3, 64, 1000])
def test_clement_integer_spectrum(orc, n):
    d, e = ti.clement(n)
    w = orc.solve(d, e, vectors=False)
    ref = -(n - 1) + 2.0 * np.arange(n)
    assert np.max(np.abs(w - ref)) <= 4 * n * EPS * max(n - 1, 1)
    # symmetry lambda <-> -lambda
    assert np.max(np.abs(w + w[::-1])) <= 8 * n * EPS * max(n - 1, 1)


@pytest.mark.parametrize("fam", ["random", "121", "clement", "glued_wilkinson", "hermite", "legendre"])
@pytest.mark.parametrize("n", [2, 5, 17, 64])
def test_against_jacobi(orc, fam, n):
    for seed in (0, 1):
        d, e = ti.family(fam, n, seed)
        w, Z = orc.solve(d, e)
        wj, V = orc.jacobi_tridiag(d, e)
        tn = max(M.tnorm_of(wj), 1e-300)
        # Jacobi is accurate to O(sweeps * n * eps * ||T||_F)
        assert np.max(np.abs(w - wj)) <= 20 * n * EPS * np.linalg.norm(orc.dense(d, e)), (fam, n)
        gaps = np.diff(wj)
        gap = np.minimum(np.r_[np.inf, gaps], np.r_[gaps, np.inf])
        sep = gap >= 1e-3 * tn
        dots = np.abs(np.sum(Z * V, axis=0))
        assert np.all(dots[sep] >= 1 - 1e-9), (fam, n)
        r, o = M.scaled(d, e, w, Z)
        assert r <= 10 and o <= 100


@pytest.mark.parametrize("fam", ["random", "121", "clement", "glued_wilkinson"])
def test_accuracy_n1000(orc, fam):
    n = 1000
    d, e = ti.family(fam, n, 0)
    w, Z = orc.solve(d, e)
    assert np.all(np.diff(w) >= 0)
    r, o = M.scaled(d, e, w, Z)
    assert r <= 10, r
    assert o <= 100, o
    # invariants: trace and Frobenius norm
    assert abs(np.sum(w) - np.sum(d)) <= 1e-10 * max(1.0, np.sum(np.abs(w)))
    fro2 = np.sum(d * d) + 2 * np.sum(e * e)
    assert abs(np.sum(w * w) - fro2) <= 1e-10 * fro2


@pytest.mark.slow
def test_random_n1000_against_jacobi(orc):
    n = 1000
    d, e = ti.random_uniform(n, 0)
    w = orc.solve(d, e, vectors=False)
    wj, _ = orc.jacobi_tridiag(d, e)
    assert np.max(np.abs(w - wj)) <= 20 * n * EPS * np.linalg.norm(orc.dense(d, e))


def test_sturm_counts_match_spectrum(orc):
    rng = np.random.default_rng(3)
    for fam in ("random", "clement", "glued_wilkinson"):
        d, e = ti.family(fam, 300, 0)
        w = orc.solve(d, e, vectors=False)
        for s in rng.uniform(w[0] - 1, w[-1] + 1, 40):
            # away from eigenvalues the count is exactly #(w < s)
            if np.min(np.abs(w - s)) > 1e-9 * max(1.0, abs(s)):
                assert orc.negcount(d, e, s) == int(np.sum(w < s))


def test_glued_wilkinson_weyl(orc):
    n = 21 * 10 + 8
    d, e = ti.glued_wilkinson(n)
    w = orc.solve(d, e, vectors=False)
    blocks = []
    for b0 in range(0, n, 21):
        b1 = min(b0 + 21, n)
        wb, _ = orc.jacobi_tridiag(d[b0:b1], e[b0:b1 - 1])
        blocks.append(wb)
    ref = np.sort(np.concatenate(blocks))
    # T = blockdiag + E with ||E||_2 = glue; Jacobi adds O(n eps ||W||_F)
    assert np.max(np.abs(w - ref)) <= ti.GLUE + 1e-12


def test_splitting_union_of_blocks(orc):
    d, e = ti.random_uniform(120, 5)
    e[39] = 0.0
    e[79] = 1e-300
    starts = orc.split_points(d, e)
    assert list(starts) == [0, 40, 80, 120]
    w, Z = orc.solve(d, e)
    parts = [orc.solve(d[a:b], e[a:b - 1], vectors=False) for a, b in zip(starts[:-1], starts[1:])]
    assert np.max(np.abs(w - np.sort(np.concatenate(parts)))) <= 1e-14
    # every vector lives in one block
    for j in range(Z.shape[1]):
        nz = np.nonzero(np.abs(Z[:, j]) > 0)[0]
        blk = np.searchsorted(starts, nz, side="right") - 1
        assert len(set(blk)) == 1
    r, o = M.scaled(d, e, w, Z)
    assert r <= 10 and o <= 100


def test_subsets_consistent(orc):
    d, e = ti.random_uniform(400, 2)
    w, Z = orc.solve(d, e)
    wi, Zi = orc.solve(d, e, "index", il=37, iu=120)
    assert np.max(np.abs(wi - w[36:120])) == 0.0
    dots = np.abs(np.sum(Zi * Z[:, 36:120], axis=0))
    gaps = np.diff(w)
    gap = np.minimum(np.r_[np.inf, gaps], np.r_[gaps, np.inf])[36:120]
    assert np.all(dots[gap > 1e-3 * M.tnorm_of(w)] >= 1 - 1e-10)
    vl, vu = 0.5 * (w[9] + w[10]), 0.5 * (w[99] + w[100])
    wv = orc.solve(d, e, "value", vl=vl, vu=vu, vectors=False)
    assert len(wv) == 90 and np.max(np.abs(wv - w[10:100])) == 0.0
    # empty ranges
    assert len(orc.solve(d, e, "value", vl=1e3, vu=2e3, vectors=False)) == 0
    assert len(orc.solve(d, e, "index", il=5, iu=4, vectors=False)) == 0


def _loss(orc, d, e, c, G):
    w, Z = orc.solve(d, e)
    return float(c @ w + (np.sum(G * Z) if G is not None else 0.0))


@pytest.mark.parametrize("with_vec", [False, True])
def test_gradient_vs_central_fd(orc, with_vec):
    n = 9
    d, e = ti.random_uniform(n, 11)
    c, G = ti.grad_weights(n, 4, with_matrix=with_vec)
    w, Z = orc.solve(d, e)
    dbar, ebar, nm = orc.grad(w, Z, c, G)
    assert nm == 0
    h = 1e-6
    for j in range(n):
        dp, dm = d.copy(), d.copy()
        dp[j] += h
        dm[j] -= h
        fd = (_loss(orc, dp, e, c, G) - _loss(orc, dm, e, c, G)) / (2 * h)
        assert abs(fd - dbar[j]) <= 1e-6 * max(1.0, abs(dbar[j])), (j, fd, dbar[j])
    for j in range(n - 1):
        ep, em = e.copy(), e.copy()
        ep[j] += h
        em[j] -= h
        fd = (_loss(orc, d, ep, c, G) - _loss(orc, d, em, c, G)) / (2 * h)
        assert abs(fd - ebar[j]) <= 1e-6 * max(1.0, abs(ebar[j])), (j, fd, ebar[j])


def test_gradient_identities(orc):
    n = 50
    d, e = ti.random_uniform(n, 3)
    w, Z = orc.solve(d, e)
    # d lambda_i / d d_j = z_ij^2: rows and columns of the squared-Z matrix sum to one
    for i in (0, 17, 49):
        wbar = np.zeros(n)
        wbar[i] = 1.0
        dbar, ebar, _ = orc.grad(w, Z, wbar)
        assert abs(np.sum(dbar) - 1.0) <= 1e-12
        # degree-1 homogeneity (Euler): sum d_j dl/dd_j + sum e_j dl/de_j = lambda_i
        assert abs(d @ dbar + e @ ebar - w[i]) <= 1e-12 * max(1.0, abs(w[i]))
    dbar, _, _ = orc.grad(w, Z, np.ones(n))
    assert np.max(np.abs(dbar - 1.0)) <= 1e-12


def test_gradient_gap_mask_counts(orc):
    d, e = ti.glued_wilkinson(42)
    w, Z = orc.solve(d, e)
    c, G = ti.grad_weights(42, 0)
    _, _, nm = orc.grad(w, Z, c, G, gap_mask_rel=1e-8)
    # the two glued W21+ copies have pairs closer than 1e-8 ||T||
    assert nm > 0 and nm % 2 == 0


# ------------------------------------------- single eigenvalues by index


@pytest.mark.parametrize("n", [1, 2, 7, 64, 401])
def test_eigval_index_closed_forms(orc, n):
    """The k-th eigenvalue by itself against the closed forms of App. D:
    1-2-1 (2 - 2 cos(k pi/(n+1))) and Clement (-(n-1) + 2(k-1))."""
    ks = sorted({1, 2, n // 2, n - 1, n} & set(range(1, n + 1)))
    d, e = ti.one_two_one(n)
    for k in ks:
        lam = 2.0 - 2.0 * np.cos(np.pi * k / (n + 1))
        assert abs(orc.eigval_index(d, e, k) - lam) <= 4 * n * EPS * 4.0, (n, k)
    d, e = ti.clement(n)
    for k in ks:
        assert abs(orc.eigval_index(d, e, k) - (-(n - 1) + 2.0 * (k - 1))) <= 4 * n * EPS * max(n - 1, 1), (n, k)


@pytest.mark.parametrize("fam", ["random", "121", "clement", "glued_wilkinson", "hermite"])
def test_eigval_index_against_jacobi(orc, fam):
    """Every index of a 40 x 40 matrix against brute-force Jacobi."""
    n = 40
    d, e = ti.family(fam, n, 3)
    wj, _ = orc.jacobi_tridiag(d, e)
    got = np.array([orc.eigval_index(d, e, k) for k in range(1, n + 1)])
    assert np.max(np.abs(got - wj)) <= 20 * n * EPS * np.linalg.norm(orc.dense(d, e)), fam


@pytest.mark.parametrize("fam", ["random", "121", "clement", "glued_wilkinson"])
def test_eigval_index_equals_solve_bit_for_bit(orc, fam):
    """On a matrix that does not split, the sampled eigenvalue takes exactly
    the steps of the whole solve (same interval, same bisection), so the two
    agree bit for bit at every index, first and last included."""
    n = 630
    d, e = ti.family(fam, n, 0)
    assert len(orc.split_points(d, e)) == 2
    w = orc.solve(d, e, vectors=False)
    for k in (1, 2, 17, n // 2, n - 1, n):
        assert orc.eigval_index(d, e, k) == w[k - 1], (fam, k)


def test_eigval_index_on_split_matrices(orc):
    """Blocks separated by an exact zero coupling and by a coupling below
    the splitting threshold: the k-th eigenvalue of T is the k-th of the
    sorted union of the blocks' spectra (Jacobi on each block), and it
    agrees with the whole solve, which bisects block by block, to within the
    stopping width of the bisection."""
    d1, e1 = ti.random_uniform(30, 4)
    d2, e2 = ti.random_uniform(25, 5)
    d3, e3 = ti.glued_wilkinson(21)
    d = np.concatenate([d1, d2 + 0.01, d3 * 0.1])
    e = np.concatenate([e1, [0.0], e2, [1e-300], e3])
    n = len(d)
    assert list(orc.split_points(d, e)) == [0, 30, 55, 76]
    ref = np.sort(np.concatenate([orc.jacobi_tridiag(d1, e1)[0], orc.jacobi_tridiag(d2 + 0.01, e2)[0],
                                  orc.jacobi_tridiag(d3 * 0.1, e3)[0]]))
    got = np.array([orc.eigval_index(d, e, k) for k in range(1, n + 1)])
    tn = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 20 * n * EPS * tn
    w = orc.solve(d, e, vectors=False)
    assert np.all(np.abs(got - w) <= 4 * EPS * np.maximum(np.abs(w), 1e-300) + 1e-300)


# ----------------------------------------------------------- sign convention


def test_sign_fix_convention(orc):
    """Largest magnitude made positive; among equal magnitudes the lowest row
    decides; a vector already in the convention, and the zero vector, are
    left alone."""
    assert np.array_equal(orc.sign_fix([0.5, -0.7, 0.7, 0.1]), [-0.5, 0.7, -0.7, -0.1])
    assert np.array_equal(orc.sign_fix([0.5, 0.7, -0.7, 0.1]), [0.5, 0.7, -0.7, 0.1])
    assert np.array_equal(orc.sign_fix([-3.0, 1.0, 2.0]), [3.0, -1.0, -2.0])
    assert np.array_equal(orc.sign_fix([-0.25, 0.25, -0.25]), [0.25, -0.25, 0.25])
    assert np.array_equal(orc.sign_fix([0.0, 0.0]), [0.0, 0.0])
    assert np.array_equal(orc.sign_fix([-1e-300]), [1e-300])
    # the Python helper used on closed-form vectors follows the same rule
    X = np.array([[0.5, -0.2, -3.0], [-0.7, 0.2, 1.0], [0.7, 0.1, 2.0]])
    assert np.array_equal(M.sign_normalize(X), np.stack([orc.sign_fix(X[:, j]) for j in range(3)], axis=1))


@pytest.mark.parametrize("fam", ["random", "clement", "glued_wilkinson"])
def test_solve_vectors_follow_sign_convention(orc, fam):
    d, e = ti.family(fam, 200, 2)
    _, Z = orc.solve(d, e)
    idx = np.argmax(np.abs(Z), axis=0)
    assert np.all(Z[idx, np.arange(Z.shape[1])] > 0)


def test_negcounts_many_shifts(orc):
    """The many-shift count equals the one-shift count at every shift, and
    away from eigenvalues it is exactly #(w < s) for the returned spectrum."""
    d, e = ti.random_uniform(250, 8)
    w = orc.solve(d, e, vectors=False)
    rng = np.random.default_rng(5)
    s = np.concatenate([rng.uniform(w[0] - 1, w[-1] + 1, 200), w, [w[0] - 10, w[-1] + 10]])
    c = orc.negcounts(d, e, s)
    assert np.array_equal(c, [orc.negcount(d, e, x) for x in s])
    far = np.array([np.min(np.abs(w - x)) > 1e-9 for x in s])
    assert np.array_equal(c[far], [int(np.sum(w < x)) for x in s[far]])
    assert c[-2] == 0 and c[-1] == 250
