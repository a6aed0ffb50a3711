"""Autotuner logic on the host with an injected cost model (no GPU)."""
import numpy as np

import tridiag_inputs as ti
from paper_1401_4950_amd import autotune


def test_bucket_of():
    assert [autotune.bucket_of(n) for n in (1, 2, 3, 32, 63, 64, 2047, 2048)] == [0, 1, 1, 5, 5, 6, 10, 11]


def test_stratified_sample_keeps_the_mix():
    sizes, _, _, _ = ti.batch_uniform(4096, seed=0)
    idx = autotune.stratified_sample(sizes, 250000, np.random.default_rng(0))
    assert np.all(np.diff(idx) > 0)
    rows = sizes[idx].sum()
    assert 0.8 * 250000 <= rows <= 1.2 * 250000
    full = np.bincount([autotune.bucket_of(n) for n in sizes], minlength=12) / len(sizes)
    part = np.bincount([autotune.bucket_of(n) for n in sizes[idx]], minlength=12) / len(idx)
    assert np.max(np.abs(full - part)) < 0.02


def test_coordinate_descent_finds_each_buckets_optimum():
    sizes, off, d_cat, e_cat = ti.batch_uniform(300, seed=1)
    # a separable cost whose optimum depends on the bucket: small matrices
    # want few lanes and small bundles, large ones the opposite
    want = {k: ((1, 16, 16) if k < 8 else (64, 64, 32)) for k in range(12)}

    def measure(ds, es, nos, table, workers):
        assert len(ds) == nos[-1] and len(es) == nos[-1] and table.shape == (len(nos) - 1, 3)
        tot = 0.0
        for (a, b), cfg in zip(zip(nos[:-1], nos[1:]), table):
            w = want[autotune.bucket_of(b - a)]
            tot += 1.0 + 10.0 * sum(abs(np.log2(c) - np.log2(x)) for c, x in zip(cfg, w))
        return tot

    table, rep = autotune.tune_batched(d_cat, e_cat, off, measure=measure, rows_per_sample=10**9,
                                       min_gain=0.0)
    assert table.shape == (300, 3) and table.dtype == np.int32
    for b, n in enumerate(sizes):
        assert tuple(table[b]) == want[autotune.bucket_of(n)]
    assert set(rep.buckets) == {autotune.bucket_of(n) for n in sizes}
    assert rep.sample_ms < rep.default_sample_ms
    assert rep.tried <= len(autotune.WAVES_PER_CU) + len(rep.buckets) * sum(len(g) for g in autotune.GRID.values())
    assert rep.workers == 0 and rep.waves_per_cu == 4       # the cost does not depend on the workers


def test_no_gain_keeps_defaults():
    sizes, off, d_cat, e_cat = ti.batch_uniform(100, seed=2)
    table, rep = autotune.tune_batched(d_cat, e_cat, off, measure=lambda *a: 1.0)
    assert (table == np.array(autotune.DEFAULT, dtype=np.int32)).all()


def test_waves_per_cu_axis():
    """A cost that prefers two waves per CU: the tuner returns that many
    workers (ncu * 2) and keeps the bucket shapes."""
    sizes, off, d_cat, e_cat = ti.batch_uniform(60, seed=3)
    calls = []

    def measure(ds, es, nos, table, workers):
        calls.append(workers)
        return 1.0 if workers != 2 * 100 else 0.5

    table, rep = autotune.tune_batched(d_cat, e_cat, off, measure=measure, ncu=100)
    assert rep.waves_per_cu == 2 and rep.workers == 200
    assert (table == np.array(autotune.DEFAULT, dtype=np.int32)).all()
    assert set(calls) == {0, 300, 200, 100}


def test_cache_round_trip(tmp_path, monkeypatch):
    """The second tuning of a batch with the same bucket histogram is read
    from the cache without a single measurement."""
    monkeypatch.setenv("MRRR_TUNE_CACHE", str(tmp_path / "tune.json"))
    sizes, off, d_cat, e_cat = ti.batch_uniform(80, seed=4)
    want = {k: (16, 32, 16) for k in range(12)}

    def measure(ds, es, nos, table, workers):
        return 1.0 + sum(float(np.sum(np.abs(np.log2(cfg) - np.log2(want[autotune.bucket_of(b - a)]))))
                         for (a, b), cfg in zip(zip(nos[:-1], nos[1:]), table)) + (0.0 if workers == 0 else 5.0)

    t1, r1 = autotune.tune_batched(d_cat, e_cat, off, measure=measure, use_cache=True, min_gain=0.0)
    assert not r1.cached and r1.tried > 0

    def forbidden(*a):
        raise AssertionError("measured although cached")

    t2, r2 = autotune.tune_batched(d_cat, e_cat, off, measure=forbidden, use_cache=True)
    assert r2.cached and r2.key == r1.key and r2.workers == r1.workers
    assert np.array_equal(t1, t2)
    # another make-up of sizes is a different key
    sizes3, off3, d3, e3 = ti.batch_uniform(80, seed=4, nmin=32, nmax=64)
    assert autotune.cache_key(sizes3, autotune.GRID, "injected") != r1.key
