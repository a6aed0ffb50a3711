"""Batched solves and the backward kernels against the CPU oracle."""
import numpy as np
import pytest

import tridiag_inputs as ti
from oracle import metrics as M

pytestmark = pytest.mark.gpu

from _gpu_util import EPS, check_pairs, gpu_residual_orth, to_dev  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _split_batch(sizes, off, d_cat, e_cat, w_cat, Z_cat):
    out, zo = [], 0
    for b, nb in enumerate(sizes):
        r0 = off[b]
        d = d_cat[r0:r0 + nb]
        e = e_cat[r0:r0 + nb - 1]
        w = w_cat[r0:r0 + nb]
        Z = Z_cat[zo:zo + nb * nb].reshape(nb, nb).T
        zo += nb * nb
        out.append((d, e, w, Z))
    return out


def test_batched_small(orc):
    import torch
    import paper_1401_4950_amd as mr
    sizes = [1, 2, 3, 5, 17, 64, 65, 100, 200, 31, 1, 129, 300, 7]
    sizes, off, d_cat, e_cat = ti.batch_uniform(len(sizes), seed=3, sizes=sizes)
    w_cat, Z_cat = mr.eigh_tridiagonal_batched(to_dev(d_cat), to_dev(e_cat), off)
    torch.cuda.synchronize()
    parts = _split_batch(sizes, off, d_cat, e_cat, w_cat.cpu().numpy(), Z_cat.cpu().numpy())
    for d, e, w, Z in parts:
        wo, Zo = orc.solve(d, e)
        check_pairs(d, e, w, Z, wo, Zo)
    # the second call replays the captured graph: identical results
    w2, Z2 = mr.eigh_tridiagonal_batched(to_dev(d_cat), to_dev(e_cat), off)
    torch.cuda.synchronize()
    assert torch.equal(w_cat, w2) and torch.equal(Z_cat, Z2)


def test_batched_with_splits_and_families(orc):
    import torch
    import paper_1401_4950_amd as mr
    mats = [ti.glued_wilkinson(84), ti.one_two_one(70), ti.clement(33), ti.random_uniform(90, 2)]
    d2, e2 = ti.random_uniform(60, 5)
    e2[20] = 0.0
    mats.append((d2, e2))
    sizes = [len(d) for d, _ in mats]
    off = np.concatenate([[0], np.cumsum(sizes)])
    d_cat = np.concatenate([d for d, _ in mats])
    e_cat = np.concatenate([np.concatenate([e, [0.0]]) for _, e in mats])
    w_cat, Z_cat = mr.eigh_tridiagonal_batched(to_dev(d_cat), to_dev(e_cat), off)
    torch.cuda.synchronize()
    for d, e, w, Z in _split_batch(sizes, off, d_cat, e_cat, w_cat.cpu().numpy(), Z_cat.cpu().numpy()):
        wo, Zo = orc.solve(d, e)
        check_pairs(d, e, w, Z, wo, Zo)


def test_batched_glued_unverified_clusters_checked(orc):
    """The check of unverified clusters inside the captured graph: glued
    Wilkinson with 400 and 300 blocks in one batch (orthogonality 235 and
    137 n eps without the check), residual and orthogonality of all pairs
    of each, sampled eigenvalues against the oracle, and a replay of the
    graph bitwise equal to the first run."""
    import torch
    import paper_1401_4950_amd as mr
    mats = [ti.glued_wilkinson(8400), ti.glued_wilkinson(6300)]
    sizes = [len(d) for d, _ in mats]
    off = np.concatenate([[0], np.cumsum(sizes)])
    d_cat = np.concatenate([d for d, _ in mats])
    e_cat = np.concatenate([np.concatenate([e, [0.0]]) for _, e in mats])
    w_cat, Z_cat = mr.eigh_tridiagonal_batched(to_dev(d_cat), to_dev(e_cat), off)
    torch.cuda.synchronize()
    zo = 0
    for (d, e), nb, r0 in zip(mats, sizes, off[:-1]):
        w = w_cat[r0:r0 + nb]
        Z = Z_cat[zo:zo + nb * nb].reshape(nb, nb).T
        zo += nb * nb
        idx = np.unique(np.linspace(1, nb, 12).astype(int))
        wo = np.array([orc.eigval_index(d, e, int(k)) for k in idx])
        tn = max(abs(orc.eigval_index(d, e, 1)), abs(orc.eigval_index(d, e, nb)))
        assert np.max(np.abs(w.cpu().numpy()[idx - 1] - wo)) <= 4 * nb * EPS * tn
        res, orth = gpu_residual_orth(d, e, w, Z, tn)
        assert res <= 10 and orth <= 100, (nb, res, orth)
    w2, Z2 = mr.eigh_tridiagonal_batched(to_dev(d_cat), to_dev(e_cat), off)
    torch.cuda.synchronize()
    assert torch.equal(w_cat, w2) and torch.equal(Z_cat, Z2)


def _grad_case(orc, d, e, c, G, gap=1e-8):
    import torch
    from paper_1401_4950_amd import EighTridiagonal
    dt = to_dev(d).requires_grad_(True)
    et = to_dev(e).requires_grad_(True)
    w, Z = EighTridiagonal.apply(dt, et, gap)
    loss = (to_dev(c) * w).sum()
    if G is not None:
        loss = loss + (to_dev(G) * Z).sum()
    loss.backward()
    torch.cuda.synchronize()
    wo, Zo = orc.solve(d, e)
    gd, ge, _ = orc.grad(wo, Zo, c, G, gap_mask_rel=gap)
    return dt.grad.cpu().numpy(), et.grad.cpu().numpy(), gd, ge


@pytest.mark.parametrize("with_vec", [False, True])
@pytest.mark.parametrize("n", [2, 3, 17, 64, 65, 200])
def test_backward_vs_oracle(orc, n, with_vec):
    d, e = ti.random_uniform(n, 40 + n)
    c, G = ti.grad_weights(n, n, with_matrix=with_vec)
    gd, ge, od, oe = _grad_case(orc, d, e, c, G)
    scale = max(np.max(np.abs(od)), np.max(np.abs(oe)) if len(oe) else 0.0)
    assert np.max(np.abs(gd - od)) <= 1e-6 * scale
    if n > 1:
        assert np.max(np.abs(ge - oe)) <= 1e-6 * scale


def test_backward_central_fd():
    """Directional central difference of the loss (h = 1e-6) on n = 60."""
    import torch
    import paper_1401_4950_amd as mr
    from paper_1401_4950_amd import EighTridiagonal
    n = 60
    d, e = ti.random_uniform(n, 77)
    c, G = ti.grad_weights(n, 3)
    dt, et = to_dev(d).requires_grad_(True), to_dev(e).requires_grad_(True)
    w, Z = EighTridiagonal.apply(dt, et)
    ((to_dev(c) * w).sum() + (to_dev(G) * Z).sum()).backward()
    rng = np.random.default_rng(0)
    vd, ve = rng.standard_normal(n), rng.standard_normal(n - 1)

    def loss(dd, ee):
        ww, ZZ = mr.eigh_tridiagonal(to_dev(dd), to_dev(ee))
        return float((to_dev(c) * ww).sum() + (to_dev(G) * ZZ).sum())

    h = 1e-6
    fd = (loss(d + h * vd, e + h * ve) - loss(d - h * vd, e - h * ve)) / (2 * h)
    an = float(dt.grad.cpu().numpy() @ vd + et.grad.cpu().numpy() @ ve)
    assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)


def test_backward_identities():
    import torch
    from paper_1401_4950_amd import eigh_tridiagonal, eigh_tridiagonal_backward
    n = 300
    d, e = ti.random_uniform(n, 12)
    w, Z = eigh_tridiagonal(to_dev(d), to_dev(e))
    # sum_i dlambda_i/dd_j = 1 for every j
    dbar, ebar = eigh_tridiagonal_backward(w, Z, wbar=torch.ones(n, dtype=torch.float64, device="cuda:0"))
    assert float((dbar - 1.0).abs().max()) <= 1e-12
    assert float(ebar.abs().max()) <= 1e-12


def test_backward_gap_mask_counts():
    import torch
    from paper_1401_4950_amd import eigh_tridiagonal, eigh_tridiagonal_backward
    d, e = ti.glued_wilkinson(84)
    w, Z = eigh_tridiagonal(to_dev(d), to_dev(e))
    G = to_dev(ti.grad_weights(84, 0)[1])
    _, _, nm = eigh_tridiagonal_backward(w, Z, None, G, gap_mask_rel=1e-8, count_masked=True)
    ws = w.cpu().numpy()
    diff = np.abs(ws[None, :] - ws[:, None])
    expect = int(((diff < 1e-8 * np.max(np.abs(ws))) & ~np.eye(84, dtype=bool)).sum())
    assert nm == expect and nm > 0


def test_backward_batched_vs_single():
    import torch
    import paper_1401_4950_amd as mr
    sizes, off, d_cat, e_cat = ti.batch_uniform(6, seed=4, sizes=[40, 64, 65, 10, 128, 3])
    w_cat, Z_cat = mr.eigh_tridiagonal_batched(to_dev(d_cat), to_dev(e_cat), off)
    rng = np.random.default_rng(2)
    wbar = to_dev(rng.standard_normal(len(d_cat)))
    Zbar = to_dev(rng.standard_normal(Z_cat.numel()))
    db, eb = mr.eigh_tridiagonal_backward_batched(w_cat, Z_cat, off, wbar, Zbar)
    zo = 0
    for b, nb in enumerate(sizes):
        r0 = int(off[b])
        Zb = Z_cat[zo:zo + nb * nb].view(nb, nb).T
        Zbb = Zbar[zo:zo + nb * nb].view(nb, nb).T
        d1, e1 = mr.eigh_tridiagonal_backward(w_cat[r0:r0 + nb], Zb, wbar[r0:r0 + nb], Zbb)
        assert torch.allclose(d1, db[r0:r0 + nb], rtol=1e-12, atol=1e-12)
        if nb > 1:
            assert torch.allclose(e1, eb[r0:r0 + nb - 1], rtol=1e-12, atol=1e-12)
        zo += nb * nb


def test_launch_shapes_plain(orc):
    """Unusual launch shapes (one lane per eigenvalue, small bundles and
    slices) give the same parity on the plain solve."""
    for fam, n in (("random", 700), ("glued_wilkinson", 420), ("121", 500)):
        d, e = ti.family(fam, n, 0)
        for lanes, bundle, smax in ((1, 8, 2), (2, 64, 16), (64, 1, 64)):
            from _gpu_util import gpu_solve
            w, Z = gpu_solve(d, e, lanes_per_eig=lanes, bundle=bundle, slice_max=smax)
            wo, Zo = orc.solve(d, e)
            check_pairs(d, e, w, Z, wo, Zo)


def test_batched_tuned_table(orc):
    """A tuned per-matrix table (from the autotuner on the device) and a
    hand-made mixed table both give oracle parity."""
    import torch
    import paper_1401_4950_amd as mr
    from paper_1401_4950_amd import autotune
    sizes, off, d_cat, e_cat = ti.batch_uniform(48, seed=9)
    grid = {"lanes_per_eig": (1, 64), "bundle": (16, 64), "slice_max": (64,)}
    table, rep = autotune.tune_batched(d_cat, e_cat, off, grid=grid, reps=1, rows_per_sample=6000)
    assert table.shape == (48, 3) and rep.buckets
    rng = np.random.default_rng(4)
    mixed = np.stack([rng.choice([1, 2, 8, 64], 48), rng.choice([1, 7, 32, 64], 48),
                      rng.choice([2, 5, 64], 48)], axis=1).astype(np.int32)
    for tab in (table, mixed):
        w_cat, Z_cat = mr.eigh_tridiagonal_batched(to_dev(d_cat), to_dev(e_cat), off, tune=tab)
        torch.cuda.synchronize()
        parts = _split_batch(sizes, off, d_cat, e_cat, w_cat.cpu().numpy(), Z_cat.cpu().numpy())
        for b in range(0, 48, 6):
            d, e, w, Z = parts[b]
            wo, Zo = orc.solve(d, e)
            check_pairs(d, e, w, Z, wo, Zo)
