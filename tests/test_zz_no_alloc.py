"""mrrr_dstemr_backward_noalloc, the backward that keeps its work in the
library's fixed per-GPU array, against mrrr_dstemr_backward (the entry point
with a growing workspace), both called through the C ABI on the same device
buffers: the results must agree bit for bit (same kernels, same order of
operations), on consecutive calls with a smaller problem second, so that the
second call cannot profit from what the first left in the array."""
import ctypes
import os
import re

import numpy as np
import pytest

import tridiag_inputs as ti

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _backward(entry, h, n, w, Zc, wb, Zb, rel=1e-8):
    import torch
    from paper_1401_4950_amd import _lib
    dbar = torch.full((n,), np.nan, dtype=torch.float64, device="cuda:0")
    ebar = torch.full((max(n - 1, 1),), np.nan, dtype=torch.float64, device="cuda:0")
    nm = ctypes.c_int64(-1)
    code = getattr(_lib.load(), entry)(h, n, _p(w), _p(Zc), n, _p(wb), _p(Zb), n, rel, _p(dbar), _p(ebar),
                                       ctypes.byref(nm))
    torch.cuda.synchronize()
    return code, dbar, ebar[: n - 1], nm.value


def _problem(n, seed):
    import torch
    import paper_1401_4950_amd as mr
    d, e = ti.random_uniform(n, seed)
    w, Z = mr.eigh_tridiagonal(torch.tensor(d, device="cuda:0"), torch.tensor(e, device="cuda:0"))
    rng = np.random.default_rng(100 + seed)
    wb = torch.tensor(rng.standard_normal(n), device="cuda:0")
    Zb = torch.tensor(rng.standard_normal(n * n), device="cuda:0")   # column-major n x n
    return w, Z.t().contiguous(), wb, Zb                               # Z.t() storage = column-major


def test_noalloc_backward_matches_the_allocating_entry_point():
    import torch
    import paper_1401_4950_amd as mr
    h = mr._handle(torch.device("cuda:0"))
    for n, seed in ((1500, 1), (333, 2)):
        w, Zc, wb, Zb = _problem(n, seed)
        # eigenvalue and eigenvector cotangents; a mask wide enough to count pairs
        for rel in (1e-8, 1e-3):
            ca, da, ea, ma = _backward("mrrr_dstemr_backward", h, n, w, Zc, wb, Zb, rel)
            cb, db, eb, mb = _backward("mrrr_dstemr_backward_noalloc", h, n, w, Zc, wb, Zb, rel)
            assert ca == 0 and cb == 0, (ca, cb)
            assert torch.equal(da, db) and torch.equal(ea, eb), (n, rel)
            assert ma == mb, (ma, mb)
            assert bool(torch.isfinite(db).all()) and bool(torch.isfinite(eb).all())
        assert mb > 0                     # the 1e-3 mask left pairs out, counted alike
        # eigenvalue cotangent only
        ca, da, ea, _ = _backward("mrrr_dstemr_backward", h, n, w, Zc, wb, None)
        cb, db, eb, mb = _backward("mrrr_dstemr_backward_noalloc", h, n, w, Zc, wb, None)
        assert ca == 0 and cb == 0 and mb == 0
        assert torch.equal(da, db) and torch.equal(ea, eb)
        # no cotangent at all: zeros
        cb, db, eb, _ = _backward("mrrr_dstemr_backward_noalloc", h, n, w, Zc, None, None)
        assert cb == 0 and float(db.abs().max()) == 0.0 and float(eb.abs().max()) == 0.0


def test_noalloc_backward_size_limit():
    """An eigenvector cotangent beyond MRRR_BACKWARD_NOALLOC_MAX_N is refused
    (argument 2) before anything runs; the eigenvalue-only form has no limit."""
    import torch
    import paper_1401_4950_amd as mr
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mrrr.h")).read()
    limit = int(re.search(r"#define MRRR_BACKWARD_NOALLOC_MAX_N (\d+)", hdr).group(1))
    h = mr._handle(torch.device("cuda:0"))
    n = limit + 1
    w, Zc, wb, Zb = _problem(n, 3)
    code, db, _, _ = _backward("mrrr_dstemr_backward_noalloc", h, n, w, Zc, wb, Zb)
    assert code == -2
    assert bool(torch.isnan(db).all())      # nothing was written
    ca, da, ea, _ = _backward("mrrr_dstemr_backward", h, n, w, Zc, wb, None)
    cb, db, eb, _ = _backward("mrrr_dstemr_backward_noalloc", h, n, w, Zc, wb, None)
    assert ca == 0 and cb == 0
    assert torch.equal(da, db) and torch.equal(ea, eb)
