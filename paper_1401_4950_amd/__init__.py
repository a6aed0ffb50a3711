"""MRRR symmetric tridiagonal eigensolver for AMD MI355X (gfx950).

Python face of libmrrr.so (``include/mrrr.h``).  Every step of the method
runs in the HIP kernels; this module only hands torch tensors' device
pointers and the current stream to the C ABI.  There is no CPU fallback: the
calls raise when the library or a GPU is missing.

    w, Z = eigh_tridiagonal(d, e)                      # all pairs
    w, Z = eigh_tridiagonal(d, e, select="i", select_range=(1, 100))
    w, Z = eigh_tridiagonal(d, e, select="v", select_range=(vl, vu))
    w_cat, Z_cat = eigh_tridiagonal_batched(d_cat, e_cat, n_offsets)
    w, Z = EighTridiagonal.apply(d, e)                 # differentiable
"""
from __future__ import annotations

import ctypes
import threading

import numpy as np

import torch

from . import _lib
from ._lib import MrrrError, Options, Stats, default_options  # noqa: F401

__all__ = [
    "eigh_tridiagonal", "eigh_tridiagonal_batched", "eigh_tridiagonal_backward",
    "eigh_tridiagonal_backward_batched", "eigh_tridiagonal_backward_noalloc", "EighTridiagonal",
    "EighTridiagonalBatched", "eigh_symmetric",
    "default_options", "MrrrError", "last_stats", "library_path", "batched_layout",
]

_tls = threading.local()


def library_path() -> str:
    return _lib.LIB_PATH


def _handle(device: torch.device):
    hs = getattr(_tls, "handles", None)
    if hs is None:
        hs = _tls.handles = {}
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = hs.get(idx)
    if h is None:
        h = ctypes.c_void_p()
        _lib.check(_lib.load().mrrr_create(ctypes.byref(h), idx), "mrrr_create", allow_warn=False)
        hs[idx] = h
    stream = torch.cuda.current_stream(idx).cuda_stream
    _lib.load().mrrr_set_stream(h, ctypes.c_void_p(stream))
    return h


def _dev_f64(x, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    return x.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _check_len(t, need, name):
    if t.numel() < need:
        raise ValueError(f"{name} holds {t.numel()} entries, needs at least {need}")


def batched_layout(n_offsets, z_offsets=None):
    """Validated batch layout: (row offsets, z offsets, rows, Z entries).

    n_offsets must start at 0 and never decrease; z_offsets (one per matrix,
    default packed) must be non-negative, and the n_b x n_b blocks they
    start may not overlap.  The Z entries needed are max_b(z_offsets[b] +
    n_b^2)."""
    noff = [int(x) for x in n_offsets]
    if len(noff) < 1 or noff[0] != 0:
        raise ValueError("n_offsets must start at 0")
    batch = len(noff) - 1
    sizes = [noff[b + 1] - noff[b] for b in range(batch)]
    if any(nb < 0 for nb in sizes):
        raise ValueError("n_offsets must not decrease")
    if z_offsets is None:
        zoff, acc = [], 0
        for nb in sizes:
            zoff.append(acc)
            acc += nb * nb
        return noff, None, noff[-1], acc
    zoff = [int(x) for x in z_offsets]
    if len(zoff) != batch:
        raise ValueError(f"z_offsets must hold one entry per matrix ({batch}), got {len(zoff)}")
    if any(z < 0 for z in zoff):
        raise ValueError("z_offsets must be non-negative")
    spans = sorted((zoff[b], zoff[b] + sizes[b] * sizes[b]) for b in range(batch) if sizes[b] > 0)
    for (a0, a1), (b0, _) in zip(spans, spans[1:]):
        if b0 < a1:
            raise ValueError("the Z blocks of two matrices overlap")
    ztot = max((z1 for _, z1 in spans), default=0)
    return noff, zoff, noff[-1], ztot


def last_stats() -> dict:
    """Statistics of the most recent solve on this thread, with the status it
    returned (0, or MRRR_WARN_UNVERIFIED = 1) under "status"."""
    st = getattr(_tls, "stats", None)
    if st is None:
        return {}
    out = st.as_dict()
    out["status"] = int(getattr(_tls, "status", 0))
    return out


def _options(options, jobz):
    if isinstance(options, Options):
        o = options
    else:
        o = default_options(**(options or {}))
    o.jobz = 1 if jobz else 0
    return o


def _dev_real(x, name, dtype):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} like d")
    return x.contiguous()


def eigh_tridiagonal(d, e, select="a", select_range=None, eigvals_only=False, options=None):
    """Eigenpairs of tridiag(e, d, e) by MRRR on the GPU.

    select: 'a' (all), 'v' (values in the half-open [vl, vu)), 'i' (indices
    il..iu, 1-based inclusive).  Returns (w, Z) with Z n x m column-major as
    a torch tensor of shape (n, m) -- or w alone when eigvals_only.

    float64 d, e: mrrr_dstemr.  float32 d, e: mrrr_sstemr, the
    single/double form (FP32 in and out, FP64 inside; its options default to
    mrrr_default_options_mixed).
    """
    if not isinstance(d, torch.Tensor) or d.dtype not in (torch.float64, torch.float32):
        raise TypeError("d must be a float64 or float32 CUDA tensor")
    mixed = d.dtype == torch.float32
    dt = d.dtype
    d = _dev_real(d, "d", dt)
    n = d.numel()
    e = _dev_real(e, "e", dt) if n > 1 else d.new_zeros(1)
    if n > 1 and e.numel() != n - 1:
        raise ValueError("e must have n-1 entries")
    rng = {"a": 0, "all": 0, "v": 1, "value": 1, "i": 2, "index": 2}[select]
    vl = vu = 0.0
    il = iu = 0
    if rng == 1:
        vl, vu = (float(x) for x in select_range)
    elif rng == 2:
        il, iu = (int(x) for x in select_range)
    ncols = n if rng != 2 else max(iu - il + 1, 0)
    if isinstance(options, Options):
        o = options
    else:
        o = default_options(mixed=mixed, **(options or {}))
    o.jobz = 0 if eigvals_only else 1
    w = d.new_empty(max(n, 1))
    # column-major n x ncols: a (ncols, n) row-major buffer, transposed view
    Zbuf = d.new_empty((max(ncols, 1), max(n, 1))) if not eigvals_only else None
    m = ctypes.c_int64(0)
    st = Stats()
    h = _handle(d.device)
    entry = "mrrr_sstemr" if mixed else "mrrr_dstemr"
    code = getattr(_lib.load(), entry)(h, n, _ptr(d), _ptr(e), rng, vl, vu, il, iu, ctypes.byref(o),
                                       ctypes.byref(m), _ptr(w), _ptr(Zbuf), max(n, 1), ctypes.byref(st))
    _tls.stats = st
    _tls.status = code
    _lib.check(code, entry)
    k = m.value
    w = w[:k]
    if eigvals_only:
        return w
    return w, Zbuf[:k].t()


def eigh_symmetric(A, select="a", select_range=None, eigvals_only=False, options=None):
    """Eigenpairs of a dense real symmetric matrix A (n x n float64 CUDA
    tensor) through mrrr_dsyevr: reduction to tridiagonal form, MRRR,
    back-transformation.  Only one triangle is read (A must be symmetric);
    select and the outputs are as for eigh_tridiagonal."""
    if not isinstance(A, torch.Tensor) or not A.is_cuda or A.dtype != torch.float64:
        raise TypeError("A must be a float64 CUDA (HIP) tensor")
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError(f"A must be square, got {tuple(A.shape)}")
    A = A.contiguous()            # row-major storage of a symmetric matrix = its column-major storage
    n = A.shape[0]
    rng = {"a": 0, "all": 0, "v": 1, "value": 1, "i": 2, "index": 2}[select]
    vl = vu = 0.0
    il = iu = 0
    if rng == 1:
        vl, vu = (float(x) for x in select_range)
    elif rng == 2:
        il, iu = (int(x) for x in select_range)
    ncols = n if rng != 2 else max(iu - il + 1, 0)
    o = _options(options, not eigvals_only)
    w = A.new_empty(max(n, 1))
    Zbuf = A.new_empty((max(ncols, 1), max(n, 1))) if not eigvals_only else None
    m = ctypes.c_int64(0)
    st = Stats()
    h = _handle(A.device)
    code = _lib.load().mrrr_dsyevr(h, n, _ptr(A), max(n, 1), rng, vl, vu, il, iu, ctypes.byref(o), ctypes.byref(m),
                                   _ptr(w), _ptr(Zbuf), max(n, 1), ctypes.byref(st))
    _tls.stats = st
    _tls.status = code
    _lib.check(code, "mrrr_dsyevr")
    k = m.value
    w = w[:k]
    if eigvals_only:
        return w
    return w, Zbuf[:k].t()


def eigh_tridiagonal_batched(d_cat, e_cat, n_offsets, z_offsets=None, eigvals_only=False,
                             options=None, out=None, tune=None):
    """All eigenpairs of many tridiagonals in one persistent launch.

    n_offsets: host sequence of batch+1 row offsets; matrix b occupies rows
    [n_offsets[b], n_offsets[b+1]) of d_cat and e_cat (e_cat keeps one
    padding slot per matrix).  Returns (w_cat, Z_cat) with matrix b's n_b x
    n_b eigenvectors column-major at z_offsets[b] (packed by default).
    tune: optional (batch, 3) integer table of per-matrix launch shapes
    (lanes per eigenvalue, singleton bundle, slice cap), e.g. from
    ``autotune.tune_batched``.
    """
    d_cat = _dev_f64(d_cat, "d_cat")
    e_cat = _dev_f64(e_cat, "e_cat")
    noff, zoff, rows, ztot = batched_layout(n_offsets, z_offsets)
    batch = len(noff) - 1
    _check_len(d_cat, rows, "d_cat")
    _check_len(e_cat, rows, "e_cat")
    arr = (ctypes.c_int64 * (batch + 1))(*noff)
    zarr = (ctypes.c_int64 * batch)(*zoff) if zoff is not None else None
    o = _options(options, not eigvals_only)
    tune_arr = None
    if tune is not None:
        tune_arr = np.ascontiguousarray(np.asarray(tune, dtype=np.int32).reshape(-1))
        if tune_arr.size != 3 * batch:
            raise ValueError(f"tune must hold 3 entries per matrix ({3 * batch}), got {tune_arr.size}")
        o.tune = tune_arr.ctypes.data
    if out is not None:
        w_cat, Z_cat = out
        w_cat = _dev_f64(w_cat, "out[0]")
        _check_len(w_cat, rows, "out[0] (w_cat)")
        if not eigvals_only:
            Z_cat = _dev_f64(Z_cat, "out[1]")
            _check_len(Z_cat, ztot, "out[1] (Z_cat)")
        if (w_cat.data_ptr() != out[0].data_ptr()
                or (not eigvals_only and Z_cat.data_ptr() != out[1].data_ptr())):
            raise ValueError("out buffers must be contiguous")
    else:
        w_cat = d_cat.new_empty(max(noff[-1], 1))
        Z_cat = d_cat.new_empty(max(ztot, 1)) if not eigvals_only else None
    st = Stats()
    h = _handle(d_cat.device)
    code = _lib.load().mrrr_dstemr_batched(h, batch, arr, _ptr(d_cat), _ptr(e_cat), zarr, ctypes.byref(o),
                                           _ptr(w_cat), _ptr(Z_cat), ctypes.byref(st))
    _tls.stats = st
    _tls.status = code
    _lib.check(code, "mrrr_dstemr_batched")
    return (w_cat, Z_cat) if not eigvals_only else w_cat


def _backward_single(entry, w, Z, wbar, Zbar, gap_mask_rel, count_masked):
    w = _dev_f64(w, "w")
    n = w.numel()
    Z = _dev_f64(Z, "Z")
    if tuple(Z.shape) != (n, n):
        raise ValueError(f"Z must be ({n}, {n}) (all eigenpairs), got {tuple(Z.shape)}")
    Zc = Z.t().contiguous()          # column-major storage: (columns, rows)
    wb = _dev_f64(wbar, "wbar") if wbar is not None else None
    if wb is not None and wb.numel() != n:
        raise ValueError(f"wbar must hold {n} entries, got {wb.numel()}")
    if Zbar is not None:
        Zbar = _dev_f64(Zbar, "Zbar")
        if tuple(Zbar.shape) != (n, n):
            raise ValueError(f"Zbar must be ({n}, {n}), got {tuple(Zbar.shape)}")
    Zb = Zbar.t().contiguous() if Zbar is not None else None
    dbar = w.new_empty(max(n, 1))
    ebar = w.new_empty(max(n - 1, 1))
    nm = ctypes.c_int64(0)
    h = _handle(w.device)
    code = getattr(_lib.load(), entry)(h, n, _ptr(w), _ptr(Zc), max(n, 1), _ptr(wb), _ptr(Zb), max(n, 1),
                                       float(gap_mask_rel), _ptr(dbar), _ptr(ebar),
                                       ctypes.byref(nm) if count_masked else None)
    _lib.check(code, entry)
    out = (dbar[:n], ebar[: max(n - 1, 0)])
    return out + (nm.value,) if count_masked else out


def eigh_tridiagonal_backward(w, Z, wbar=None, Zbar=None, gap_mask_rel=1e-8, count_masked=False):
    """(dbar, ebar[, n_masked]) for cotangents (wbar, Zbar) of (w, Z) where Z
    is the (n, n) tensor returned by eigh_tridiagonal (column-major view)."""
    return _backward_single("mrrr_dstemr_backward", w, Z, wbar, Zbar, gap_mask_rel, count_masked)


def eigh_tridiagonal_backward_noalloc(w, Z, wbar=None, Zbar=None, gap_mask_rel=1e-8, count_masked=False):
    """As eigh_tridiagonal_backward, through the C entry point that keeps its
    work in the library's fixed per-GPU array (n <= 2048 with Zbar).  The
    C call allocates nothing; this wrapper still makes the column-major copies
    and the outputs as torch tensors."""
    return _backward_single("mrrr_dstemr_backward_noalloc", w, Z, wbar, Zbar, gap_mask_rel, count_masked)


def eigh_tridiagonal_backward_batched(w_cat, Z_cat, n_offsets, wbar_cat=None, Zbar_cat=None,
                                      z_offsets=None, gap_mask_rel=1e-8, count_masked=False):
    w_cat = _dev_f64(w_cat, "w_cat")
    Z_cat = _dev_f64(Z_cat, "Z_cat")
    noff, zoff, rows, ztot = batched_layout(n_offsets, z_offsets)
    batch = len(noff) - 1
    _check_len(w_cat, rows, "w_cat")
    _check_len(Z_cat, ztot, "Z_cat")
    arr = (ctypes.c_int64 * (batch + 1))(*noff)
    zarr = (ctypes.c_int64 * batch)(*zoff) if zoff is not None else None
    wb = _dev_f64(wbar_cat, "wbar_cat") if wbar_cat is not None else None
    Zb = _dev_f64(Zbar_cat, "Zbar_cat") if Zbar_cat is not None else None
    if wb is not None:
        _check_len(wb, rows, "wbar_cat")
    if Zb is not None:
        _check_len(Zb, ztot, "Zbar_cat")
    dbar = w_cat.new_empty(max(noff[-1], 1))
    ebar = w_cat.new_empty(max(noff[-1], 1))
    nm = ctypes.c_int64(0)
    h = _handle(w_cat.device)
    code = _lib.load().mrrr_dstemr_backward_batched(h, batch, arr, _ptr(w_cat), _ptr(Z_cat), zarr, _ptr(wb),
                                                    _ptr(Zb), float(gap_mask_rel), _ptr(dbar), _ptr(ebar),
                                                    ctypes.byref(nm) if count_masked else None)
    _lib.check(code, "mrrr_dstemr_backward_batched")
    return (dbar, ebar, nm.value) if count_masked else (dbar, ebar)


class EighTridiagonal(torch.autograd.Function):
    """(w, Z) = eigh(tridiag(e, d, e)) with the hand-written backward kernels.

    Z is returned as an (n, n) tensor (column j = eigenvector j); the sign
    convention (largest entry positive) makes it a smooth function of (d, e)
    wherever the eigenvalues are distinct.
    """

    @staticmethod
    def forward(ctx, d, e, gap_mask_rel=1e-8, options=None):
        w, Z = eigh_tridiagonal(d, e, options=options)
        ctx.gap_mask_rel = gap_mask_rel
        ctx.set_materialize_grads(False)
        ctx.save_for_backward(w, Z)
        return w, Z

    @staticmethod
    def backward(ctx, wbar, Zbar):
        w, Z = ctx.saved_tensors
        dbar, ebar = eigh_tridiagonal_backward(w, Z, wbar, Zbar, ctx.gap_mask_rel)
        return dbar, ebar, None, None


class EighTridiagonalBatched(torch.autograd.Function):
    """Batched (w_cat, Z_cat) with the batched backward kernels."""

    @staticmethod
    def forward(ctx, d_cat, e_cat, n_offsets, gap_mask_rel=1e-8, options=None):
        w, Z = eigh_tridiagonal_batched(d_cat, e_cat, n_offsets, options=options)
        ctx.noff = list(n_offsets)
        ctx.gap_mask_rel = gap_mask_rel
        ctx.set_materialize_grads(False)
        ctx.save_for_backward(w, Z)
        return w, Z

    @staticmethod
    def backward(ctx, wbar, Zbar):
        w, Z = ctx.saved_tensors
        dbar, ebar = eigh_tridiagonal_backward_batched(
            w, Z, ctx.noff, wbar.contiguous() if wbar is not None else None,
            Zbar.contiguous() if Zbar is not None else None, gap_mask_rel=ctx.gap_mask_rel)
        return dbar, ebar, None, None, None
