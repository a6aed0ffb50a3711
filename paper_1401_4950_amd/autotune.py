"""Autotuner of the batched launch shape.

The batched form runs many tridiagonals in one persistent launch.  How a
matrix's work is cut into device tasks is a trade between latency (many lanes
on one eigenvalue, small tasks that spread over many workers) and throughput
(one lane per eigenvalue, large tasks with little scheduling traffic).  The
best point depends on the matrix size and on what else shares the launch, so
it is chosen per size bucket (powers of two) by measurement in context:

* lanes_per_eig: most multisection points one refinement gives an eigenvalue;
* bundle:        singletons per S-task (one per lane);
* slice_max:     largest refinement slice (R-task) in eigenvalues.

and, for the whole launch,

* waves per CU:  persistent workers per compute unit (1..4; the tree kernel
                 holds one wave per SIMD, four per CU), i.e. options.workers.

A stratified sample of the batch (every bucket in its proportion, about
rows_per_sample rows) is solved as one batch; each bucket's three parameters
are then set by coordinate descent over a small grid while the other buckets
keep their current best, largest bucket first, keeping a change only when it
shortens the device time of the sample by more than `min_gain`; the waves per
CU come last, with the bucket shapes fixed.  The result is a (batch, 3) table
for ``eigh_tridiagonal_batched(tune=...)`` and a worker count for its options.

Results are kept in a JSON cache on disk (``MRRR_TUNE_CACHE``, default
``~/.cache/mrrr/tune.json``) keyed by the batch's size-bucket histogram, the
grid, the device and the library build, so a batch of the same make-up is
tuned once per machine.  Host-side orchestration only: every solve runs in
the library's kernels.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time
from dataclasses import dataclass, field

import numpy as np

DEFAULT = (64, 64, 64)                     # lanes_per_eig, bundle, slice_max
GRID = {
    "lanes_per_eig": (1, 4, 16, 64),
    "bundle": (16, 32, 64),
    "slice_max": (16, 32, 64),
}
PARAMS = ("lanes_per_eig", "bundle", "slice_max")
WAVES_PER_CU = (4, 3, 2, 1)                # the default (a full GPU) first


def bucket_of(n: int) -> int:
    """Size bucket: floor(log2 n) (n >= 1), so [2^k, 2^(k+1)) share one."""
    return int(math.floor(math.log2(max(int(n), 1))))


@dataclass
class TuneReport:
    buckets: dict = field(default_factory=dict)   # bucket -> dict(config, count, sample)
    seconds: float = 0.0
    sample_ms: float = 0.0           # device time of the sample with the chosen shapes
    default_sample_ms: float = 0.0   # ... and with the defaults everywhere
    tried: int = 0
    waves_per_cu: int = 4
    workers: int = 0                 # options.workers to use (0: the library's default, a full GPU)
    cached: bool = False             # taken from the on-disk cache, nothing measured
    key: str = ""

    def as_dict(self):
        return {"seconds": self.seconds, "sample_ms": self.sample_ms,
                "default_sample_ms": self.default_sample_ms, "tried": self.tried,
                "waves_per_cu": self.waves_per_cu, "workers": self.workers, "cached": self.cached,
                "buckets": {str(k): v for k, v in sorted(self.buckets.items())}}


def cache_path() -> str:
    return os.environ.get("MRRR_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "mrrr",
                                                             "tune.json")


def cache_key(sizes, grid, device_tag: str) -> str:
    """The batch's size-bucket histogram, the grid, the device and the
    library build: batches of the same make-up share a tuning."""
    from . import _lib
    hist = np.bincount([bucket_of(n) for n in sizes], minlength=32).tolist() if len(sizes) else []
    try:
        st = os.stat(_lib.LIB_PATH)
        build = f"{st.st_size}-{int(st.st_mtime)}"
    except OSError:
        build = "none"
    blob = json.dumps({"hist": hist, "grid": {k: list(v) for k, v in sorted(grid.items())},
                       "waves": list(WAVES_PER_CU), "device": device_tag, "build": build}, sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()[:24]


def _cache_load(key):
    try:
        with open(cache_path()) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def _cache_store(key, entry):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
        data[key] = entry
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(data, f)
        os.replace(tmp, path)
    except OSError:
        pass   # an unwritable cache only costs a retune


def _sub_batch(sizes, offs, d_cat, e_cat, idx):
    """Rows of matrices idx gathered into a new concatenated batch."""
    parts_d, parts_e, noff = [], [], [0]
    for b in idx:
        r0, nb = int(offs[b]), int(sizes[b])
        parts_d.append(d_cat[r0:r0 + nb])
        parts_e.append(e_cat[r0:r0 + nb])
        noff.append(noff[-1] + nb)
    return np.concatenate(parts_d), np.concatenate(parts_e), noff


def _device_timer(solve, reps):
    """Median device time (hipEvents around the graph launch, ms -> s) of
    `reps` calls after one untimed call, which builds and captures the plan."""
    from . import last_stats
    solve()
    ts = []
    for _ in range(reps):
        solve()
        ts.append(float(last_stats()["ms"]) * 1e-3)
    return float(np.median(ts))


def stratified_sample(sizes, rows, rng):
    """Indices of about `rows` rows of matrices, every size bucket in its
    proportion (at least one matrix of each), in batch order."""
    sizes = np.asarray(sizes)
    frac = min(1.0, rows / max(1, int(sizes.sum())))
    bk = np.array([bucket_of(n) for n in sizes])
    pick = []
    for k in sorted(set(bk.tolist())):
        members = np.nonzero(bk == k)[0]
        m = max(1, int(round(frac * len(members))))
        pick.append(rng.choice(members, size=min(m, len(members)), replace=False))
    return np.sort(np.concatenate(pick))


def tune_batched(d_cat, e_cat, n_offsets, *, rows_per_sample=250000, reps=3, grid=None, min_gain=0.01,
                 seed=0, measure=None, options=None, log=None, ncu=None, use_cache=None):
    """Per-bucket launch shapes and the waves per CU for the batch (d_cat,
    e_cat, n_offsets).

    d_cat / e_cat: host arrays or device tensors in the batched layout.
    measure(d_sub, e_sub, noff_sub, table_sub, workers) -> seconds may replace
    the device measurement (tests use it); table_sub is the (m, 3) shape table
    of the sample, workers the persistent worker count (0: a full GPU).
    ncu: compute units (default: the device's).  use_cache: read and write
    the on-disk cache (default: only when measuring on the device).
    Returns (table int32 (batch, 3), TuneReport); report.workers goes into
    the options of the solve.
    """
    grid = grid or GRID
    t_start = time.perf_counter()
    noff = np.asarray([int(x) for x in n_offsets], dtype=np.int64)
    sizes = np.diff(noff)
    batch = len(sizes)
    if use_cache is None:
        use_cache = measure is None
    device_tag = "injected"
    if measure is None:
        import torch
        dev = d_cat.device if isinstance(d_cat, torch.Tensor) and d_cat.is_cuda else torch.device("cuda:0")
        props = torch.cuda.get_device_properties(dev)
        device_tag = f"{props.name}/{props.multi_processor_count}"
        if ncu is None:
            ncu = int(props.multi_processor_count)
    if ncu is None:
        ncu = 256
    key = cache_key(sizes, grid, device_tag)
    if use_cache:
        hit = _cache_load(key)
        if hit is not None:
            cfg = {int(k): tuple(v) for k, v in hit["buckets"].items()}
            table = np.array([cfg.get(bucket_of(n), DEFAULT) for n in sizes], dtype=np.int32).reshape(-1, 3)
            rep = TuneReport(sample_ms=hit["sample_ms"], default_sample_ms=hit["default_sample_ms"],
                             tried=0, waves_per_cu=hit["waves_per_cu"], workers=hit["workers"], cached=True,
                             key=key)
            for k, v in cfg.items():
                rep.buckets[k] = {"config": dict(zip(PARAMS, v)),
                                  "count": int(sum(1 for n in sizes if bucket_of(n) == k))}
            rep.seconds = time.perf_counter() - t_start
            if log:
                log(f"[tune] cached shapes for this batch make-up ({key})")
            return table, rep

    def host(x):
        return x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x, dtype=np.float64)

    dh, eh = host(d_cat), host(e_cat)
    rng = np.random.default_rng(seed)
    idx = stratified_sample(sizes, rows_per_sample, rng)
    ds, es, nos = _sub_batch(sizes, noff, dh, eh, idx)
    if measure is None:
        import torch

        from . import eigh_tridiagonal_batched
        dt = torch.tensor(ds, device=dev)
        et = torch.tensor(es, device=dev)

        def measure(d_sub, e_sub, noff_sub, table_sub, workers):
            opts = dict(options or {})
            opts["workers"] = int(workers)
            return _device_timer(lambda: eigh_tridiagonal_batched(dt, et, noff_sub, options=opts,
                                                                  tune=table_sub), reps)

    sub_bk = np.array([bucket_of(n) for n in sizes[idx]])
    buckets = sorted(set(sub_bk.tolist()), reverse=True)
    best = {k: tuple(DEFAULT) for k in buckets}

    def table_for(cfgs):
        return np.array([cfgs[k] for k in sub_bk], dtype=np.int32).reshape(-1, 3)

    seen = {}

    def cost(cfgs, workers=0):
        ck = (tuple(cfgs[k] for k in buckets), workers)
        if ck not in seen:
            seen[ck] = measure(ds, es, nos, table_for(cfgs), workers)
        return seen[ck]

    default_t = best_t = cost(best)
    for k in buckets:
        for pi, name in enumerate(PARAMS):
            for v in grid[name]:
                trial = dict(best)
                trial[k] = tuple(v if i == pi else best[k][i] for i in range(3))
                if trial[k] == best[k]:
                    continue
                t = cost(trial)
                if t < best_t * (1.0 - min_gain):
                    best, best_t = trial, t
        if log:
            log(f"[tune] bucket 2^{k}: {dict(zip(PARAMS, best[k]))}, sample time {best_t * 1e3:.1f} ms "
                f"(all defaults {default_t * 1e3:.1f} ms)")
    # waves per CU (the whole launch), with the bucket shapes fixed
    best_w, best_workers = WAVES_PER_CU[0], 0
    for wv in WAVES_PER_CU[1:]:
        t = cost(best, ncu * wv)
        if t < best_t * (1.0 - min_gain):
            best_w, best_workers, best_t = wv, ncu * wv, t
    if log:
        log(f"[tune] waves per CU: {best_w}, sample time {best_t * 1e3:.1f} ms")
    table = np.zeros((batch, 3), dtype=np.int32)
    report = TuneReport(waves_per_cu=best_w, workers=best_workers, key=key)
    for k in buckets:
        members = np.nonzero(np.array([bucket_of(n) for n in sizes]) == k)[0]
        table[members] = best[k]
        report.buckets[k] = {"config": dict(zip(PARAMS, best[k])), "count": int(len(members)),
                             "sample": int((sub_bk == k).sum())}
    # buckets without a sampled matrix cannot occur (each gets at least one)
    report.sample_ms = best_t * 1e3
    report.default_sample_ms = default_t * 1e3
    report.tried = len(seen)
    report.seconds = time.perf_counter() - t_start
    if use_cache:
        _cache_store(key, {"buckets": {str(k): list(best[k]) for k in buckets}, "waves_per_cu": best_w,
                           "workers": best_workers, "sample_ms": report.sample_ms,
                           "default_sample_ms": report.default_sample_ms})
    return table, report
