"""Helpers shared by the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import numpy as np
import torch

from oracle import metrics as M

EPS = M.EPS


def dev():
    return torch.device("cuda:0")


def to_dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device=dev())


def gpu_solve(d, e, select="a", select_range=None, eigvals_only=False, **opts):
    import paper_1401_4950_amd as mr
    out = mr.eigh_tridiagonal(to_dev(d), to_dev(e) if len(e) else to_dev(np.zeros(1)), select=select,
                              select_range=select_range, eigvals_only=eigvals_only, options=opts or None)
    torch.cuda.synchronize()
    if eigvals_only:
        return out.cpu().numpy()
    w, Z = out
    return w.cpu().numpy(), Z.cpu().numpy()


def oracle_clusters(w, tn, rel=1e-3):
    """Maximal chains of eigenvalues closer than rel * ||T||."""
    groups, start = [], 0
    for i in range(1, len(w) + 1):
        if i == len(w) or w[i] - w[i - 1] >= rel * tn:
            groups.append((start, i))
            start = i
    return groups


def check_pairs(d, e, w, Z, wo, Zo=None, tnorm=None, eig_tol=4.0, res_tol=10.0, orth_tol=100.0,
                full=None):
    """The parity bar: eigenvalues within eig_tol * n eps ||T|| of the
    oracle, residual <= res_tol n eps ||T||, orthogonality <= orth_tol n eps;
    vectors against the oracle individually where the oracle gap is >=
    1e-3 ||T|| and as subspaces inside oracle clusters.

    full = (w_all, Z_all, first) for a subset starting at 0-based index
    first: clusters are then taken over the whole spectrum, and the part of
    a cluster that the subset cuts must lie in that whole cluster's span
    (a cut through a cluster of nearly equal eigenvalues has no unique
    subspace of its own)."""
    n = len(d)
    assert w.shape == wo.shape, (w.shape, wo.shape)
    tn = tnorm if tnorm is not None else max(M.tnorm_of(wo), np.finfo(float).tiny)
    if len(w) == 0:
        return {}
    err = float(np.max(np.abs(w - wo))) / (n * EPS * tn)
    assert err <= eig_tol, f"eigenvalue error {err:.3f} n eps ||T||"
    assert np.all(np.diff(w) >= 0), "eigenvalues not ascending"
    r, o = M.scaled(d, e, w, Z, tn)
    assert r <= res_tol, f"residual {r:.3f} n eps ||T||"
    assert o <= orth_tol, f"orthogonality {o:.3f} n eps"
    out = {"eig": err, "res": r, "orth": o}
    if full is not None:
        w_all, Z_all, first = full
        m = len(w)
        for (a, b) in oracle_clusters(w_all, tn):
            lo, hi = max(a, first), min(b, first + m)
            if lo >= hi:
                continue
            if b - a == 1:
                dot = abs(float(Z[:, lo - first] @ Z_all[:, a]))
                assert dot >= 1 - 1e-10, f"vector {a}: |z.z_oracle| = {dot}"
            else:
                smin = M.subspace_sigma_min(Z[:, lo - first:hi - first], Z_all[:, a:b])
                assert smin >= 1 - 1e-8, f"cluster [{a},{b}) part [{lo},{hi}): sigma_min = {smin}"
        return out
    if Zo is not None:
        for (a, b) in oracle_clusters(wo, tn):
            if b - a == 1:
                dot = abs(float(Z[:, a] @ Zo[:, a]))
                assert dot >= 1 - 1e-10, f"vector {a}: |z.z_oracle| = {dot}"
            else:
                smin = M.subspace_sigma_min(Z[:, a:b], Zo[:, a:b])
                assert smin >= 1 - 1e-8, f"cluster [{a},{b}): sigma_min = {smin}"
    return out


def gpu_residual_orth(d, e, w, Z, tn, ncols_orth=None):
    """Residual (all columns) and orthogonality on the GPU for large n;
    torch (rocBLAS) does the Z^T Z check product."""
    dd, ee = to_dev(d), to_dev(e)
    wt = w if isinstance(w, torch.Tensor) else to_dev(w)
    R = dd[:, None] * Z
    R[:-1] += ee[:, None] * Z[1:]
    R[1:] += ee[:, None] * Z[:-1]
    R -= Z * wt[None, :]
    n = Z.shape[0]
    res = float(R.norm(dim=0).max()) / (n * EPS * tn)
    del R
    G = Z.T @ Z
    G.diagonal().sub_(1.0)
    orth = float(G.abs().max()) / (n * EPS)
    del G
    return res, orth
