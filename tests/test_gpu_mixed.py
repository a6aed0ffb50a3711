"""Single/double MRRR (Ch. 5): FP32 data in and out, FP64 inside.

Parity against the FP64 oracle run on the FP64 values of the same FP32
inputs (widening is exact): every eigenvalue within 4 eps_s ||T|| (rounding
the result to FP32 alone costs eps_s |lambda|); residual and orthogonality of
the FP32 vectors, measured in FP64, at most eps_s sqrt(n) ||T|| and
eps_s sqrt(n) -- the accuracy goal of Sec. 5.1.1.  The depth of the
representation tree and the clustering rho = largest cluster / n are printed
beside those of the FP64 form on the same data, the two quantities the
thesis reports for its single/double solver (Table 5.3, Sec. 5.2.1).
"""
import numpy as np
import pytest

import tridiag_inputs as ti
from oracle import metrics as M

pytestmark = pytest.mark.gpu

from _gpu_util import EPS, gpu_residual_orth, to_dev  # noqa: E402

EPS_S = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _f32_dev(x):
    import torch
    return torch.tensor(np.asarray(x, dtype=np.float32), device="cuda:0")


def _check_mixed(orc, d32, e32, w, Z, select="all", il=1, iu=None, vl=0.0, vu=0.0):
    """The parity bar of the single/double form; returns (eig, res, orth) in
    units of eps_s ||T||, eps_s sqrt(n) ||T|| and eps_s sqrt(n)."""
    import torch
    d64 = np.asarray(d32, dtype=np.float64)
    e64 = np.asarray(e32, dtype=np.float64)
    n = len(d64)
    assert w.dtype == torch.float32 and (Z is None or Z.dtype == torch.float32)
    wo = orc.solve(d64, e64, select, il=il, iu=iu if iu is not None else n, vl=vl, vu=vu, vectors=False)
    tn = max(abs(orc.eigval_index(d64, e64, 1)), abs(orc.eigval_index(d64, e64, n)))
    wh = w.cpu().numpy().astype(np.float64)
    assert wh.shape == wo.shape, (wh.shape, wo.shape)
    assert np.all(np.diff(wh) >= 0)
    eig = float(np.max(np.abs(wh - wo))) / (EPS_S * tn) if len(wo) else 0.0
    assert eig <= 4.0, f"eigenvalue error {eig:.2f} eps_s ||T||"
    if Z is None or len(wo) == 0:
        return eig, 0.0, 0.0
    res, orth = gpu_residual_orth(d64, e64, w.double(), Z.double(), tn)
    # gpu_residual_orth scales by n eps ||T|| and n eps (eps = 2^-53)
    res_s = res * n * EPS / (np.sqrt(n) * EPS_S)
    orth_s = orth * n * EPS / (np.sqrt(n) * EPS_S)
    assert res_s <= 1.0 and orth_s <= 1.0, (res_s, orth_s)
    return eig, res_s, orth_s


@pytest.mark.parametrize("fam,n", [("random", 1000), ("121", 2500), ("121", 20000), ("clement", 20000),
                                   ("glued_wilkinson", 20000), ("random", 20000)])
def test_mixed_all_pairs(orc, fam, n):
    import torch
    import paper_1401_4950_amd as mr
    d, e = ti.family(fam, n, 0)
    d32, e32 = np.float32(d), np.float32(e)
    w, Z = mr.eigh_tridiagonal(_f32_dev(d32), _f32_dev(e32))
    torch.cuda.synchronize()
    st = mr.last_stats()
    assert w.shape == (n,) and Z.shape == (n, n)
    eig, res, orth = _check_mixed(orc, d32, e32, w, Z)
    del Z
    # the FP64 form on the same data, for the tree statistics
    mr.eigh_tridiagonal(to_dev(np.float64(d32)), to_dev(np.float64(e32)), eigvals_only=False)
    sd = mr.last_stats()
    print(f"single/double {fam} n={n}: eig {eig:.2f} eps_s||T||, res {res:.3f}, orth {orth:.3f} "
          f"(units eps_s sqrt(n)); d_max {st['dmax']}, rho {st['largest_cluster'] / n:.2e}, "
          f"nodes {st['n_nodes']}, blocks {st['n_blocks']}, unverified {st['n_unverified_rrr']} | "
          f"FP64 form: d_max {sd['dmax']}, rho {sd['largest_cluster'] / n:.2e}, nodes {sd['n_nodes']}")
    # the reduced clustering the single/double form is for (Sec. 5.1.1)
    assert st["dmax"] <= sd["dmax"]
    assert st["largest_cluster"] <= sd["largest_cluster"]


def test_mixed_subsets(orc):
    import torch
    import paper_1401_4950_amd as mr
    n = 5000
    d, e = ti.random_uniform(n, 3)
    d32, e32 = np.float32(d), np.float32(e)
    w, Z = mr.eigh_tridiagonal(_f32_dev(d32), _f32_dev(e32), select="i", select_range=(100, 600))
    torch.cuda.synchronize()
    assert Z.shape == (n, 501)
    _check_mixed(orc, d32, e32, w, Z, "index", il=100, iu=600)
    vl, vu = -0.5, 0.25
    w, Z = mr.eigh_tridiagonal(_f32_dev(d32), _f32_dev(e32), select="v", select_range=(vl, vu))
    torch.cuda.synchronize()
    _check_mixed(orc, d32, e32, w, Z, "value", vl=vl, vu=vu)
    w = mr.eigh_tridiagonal(_f32_dev(d32), _f32_dev(e32), eigvals_only=True)
    _check_mixed(orc, d32, e32, w, None)


def test_mixed_splitting_follows_the_single_precision_threshold(orc):
    """Off-diagonals of 1e-9 (below eps_s sqrt(n) ||T||, above the FP64
    threshold) split the matrix in the single/double form only; the results
    still meet the bar (the dropped entries are far below eps_s ||T||)."""
    import torch
    import paper_1401_4950_amd as mr
    n = 3000
    d, e = ti.random_uniform(n, 4)
    e = e.copy()
    e[[499, 1499, 2199]] = 1e-9
    d32, e32 = np.float32(d), np.float32(e)
    w, Z = mr.eigh_tridiagonal(_f32_dev(d32), _f32_dev(e32))
    torch.cuda.synchronize()
    assert mr.last_stats()["n_blocks"] == 4
    _check_mixed(orc, d32, e32, w, Z)
    mr.eigh_tridiagonal(to_dev(np.float64(d32)), to_dev(np.float64(e32)))
    assert mr.last_stats()["n_blocks"] == 1


def test_mixed_defaults_and_arguments():
    import torch
    import paper_1401_4950_amd as mr
    from paper_1401_4950_amd import _lib
    o = _lib.default_options(mixed=True)
    assert o.gaptol == 1e-5 and o.rtol_class == 1e-7 and o.perturb_xi == 2.0 ** 29
    d = _f32_dev(np.ones(10))
    with pytest.raises(TypeError):
        mr.eigh_tridiagonal(d, to_dev(np.ones(9)))        # mixed dtypes
    w, Z = mr.eigh_tridiagonal(d[:1], d[:0])
    assert float(w[0]) == 1.0 and float(Z[0, 0]) == 1.0
