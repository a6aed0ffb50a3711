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

A stratified sample of the batch (every bucket in its proportion, about
rows_per_sample rows) is solved as one batch; each bucket's three parameters
are then set by coordinate descent over a small grid while the other buckets
keep their current best, largest bucket first, keeping a change only when it
shortens the device time of the sample by more than `min_gain`.  The result is
a (batch, 3) table for ``eigh_tridiagonal_batched(tune=...)``.  Host-side
orchestration only: every solve runs in the library's kernels.
"""
from __future__ import annotations

import math
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

    def as_dict(self):
        return {"seconds": self.seconds, "sample_ms": self.sample_ms,
                "default_sample_ms": self.default_sample_ms, "tried": self.tried,
                "buckets": {str(k): v for k, v in sorted(self.buckets.items())}}


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
                 seed=0, measure=None, options=None, log=None):
    """Per-bucket launch shapes for the batch (d_cat, e_cat, n_offsets).

    d_cat / e_cat: host arrays or device tensors in the batched layout.
    measure(d_sub, e_sub, noff_sub, table_sub) -> seconds may replace the
    device measurement (tests use it); table_sub is the (m, 3) shape table of
    the sample.  Returns (table int32 (batch, 3), TuneReport).
    """
    grid = grid or GRID
    t_start = time.perf_counter()
    noff = np.asarray([int(x) for x in n_offsets], dtype=np.int64)
    sizes = np.diff(noff)
    batch = len(sizes)

    def host(x):
        return x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x, dtype=np.float64)

    dh, eh = host(d_cat), host(e_cat)
    rng = np.random.default_rng(seed)
    idx = stratified_sample(sizes, rows_per_sample, rng)
    ds, es, nos = _sub_batch(sizes, noff, dh, eh, idx)
    if measure is None:
        import torch

        from . import eigh_tridiagonal_batched
        dev = d_cat.device if isinstance(d_cat, torch.Tensor) and d_cat.is_cuda else torch.device("cuda:0")
        dt = torch.tensor(ds, device=dev)
        et = torch.tensor(es, device=dev)

        def measure(d_sub, e_sub, noff_sub, table_sub):
            return _device_timer(lambda: eigh_tridiagonal_batched(dt, et, noff_sub, options=options,
                                                                  tune=table_sub), reps)

    sub_bk = np.array([bucket_of(n) for n in sizes[idx]])
    buckets = sorted(set(sub_bk.tolist()), reverse=True)
    best = {k: tuple(DEFAULT) for k in buckets}

    def table_for(cfgs):
        return np.array([cfgs[k] for k in sub_bk], dtype=np.int32).reshape(-1, 3)

    seen = {}

    def cost(cfgs):
        key = tuple(cfgs[k] for k in buckets)
        if key not in seen:
            seen[key] = measure(ds, es, nos, table_for(cfgs))
        return seen[key]

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
    table = np.zeros((batch, 3), dtype=np.int32)
    report = TuneReport()
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
    return table, report
