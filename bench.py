#!/usr/bin/env python3
"""Throughput of the MRRR tridiagonal eigensolver on one MI355X.

One step = all eigenpairs (w and Z) of four seeded n = 20000 FP64
tridiagonals shaped like the thesis's test matrices (App. D): 1-2-1 Toeplitz,
Clement, glued Wilkinson W21+ and uniform random d, e.  Every row of the
method runs inside each call: splitting, root representation, bisection,
classification, cluster representations, Rayleigh-quotient iteration on
twisted factorizations, eigenvector solves and output assembly.  Inputs are
resident in device memory before the timed region starts.

Beside the headline the same run measures the two further forms:
  * batched: 4096 tridiagonals, sizes log-uniform in [32, 2048], in one
    captured persistent launch with the autotuned per-bucket launch shape,
    against 4096 plain per-matrix calls;
  * differentiation: forward + backward for 256 matrices of n = 512 (batched
    against per-matrix), one n = 8192 random matrix with an eigenvalue and
    eigenvector loss, and an eigenvalue-only loss on glued Wilkinson n = 8192.

The roofline object is for the persistent tree kernel, which dominates the
solve: the method's algorithmic FP64 work, 200 k n flops for k eigenpairs of
an order-n matrix (the practical bound on MRRR's work quoted where the thesis
introduces the method, Sec. 2.3.1; 8.0e10 per n = 20000 matrix), over the
kernel's mean launch time from hipEvents recorded on its own stream.  Beside
it, "issued" counts 4 flops per lane-step of the qd / Sturm recurrences the
kernel actually ran (speculative multisection points included).  The
cpu_baseline leg times the CPU oracle (test infrastructure,
never tuned) on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
N_MAIN = 20000
FAMILIES = ("121", "clement", "glued_wilkinson", "random")
FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X published FP64 vector peak
FP64_MFMA_PEAK_TFLOPS = 78.6       # MI355X published dense FP64 matrix peak
FLOPS_PER_QD_STEP = 4.0            # per lane-step: the two multiply-adds and the multiply of a
                                   # division-free row, counted as the add, divide and multiply-add
                                   # of the quotient form they replace
ALGO_FLOPS_PER_PAIR_PER_ROW = 200.0  # MRRR's work bound: fewer than 200 k n flops
TRAFFIC_FILE = os.path.join(HERE, "profiles", "mrrr_tree_kernel_n20000_traffic.md")
TREE_SOURCE = os.path.join(HERE, "paper_1401_4950_amd", "csrc", "mrrr_tree.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sections", default="plain,mixed,batched,grad,cpu",
                    help="comma list of plain, mixed, batched, grad, cpu (without plain the headline "
                         "fields are null: for profiling the other legs alone)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES bytes device to device three times and exit (a copy of known "
                         "size, to scale the HBM byte counters of a profiler)")
    return ap.parse_args(argv)


def copy_calibration(nbytes):
    import torch
    n = max(1, nbytes // 8)
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] copied {n * 8} bytes three times")
    return 0


def tree_source_digest() -> str:
    with open(TREE_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic():
    """HBM bytes per tree-kernel launch from the committed counter summary,
    or None when it is missing or was taken on a different kernel source."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m_src = re.search(r"kernel source sha256\[:16\]:\s*([0-9a-f]{16})", text)
    m_b = re.search(r"HBM bytes per launch:\s*([0-9.eE+]+)", text)
    if not (m_src and m_b) or m_src.group(1) != tree_source_digest():
        return None
    return float(m_b.group(1))


def bench_plain(mr, torch, steps, warmup):
    import tridiag_inputs as ti
    dev = torch.device("cuda:0")
    mats = []
    for fam in FAMILIES:
        d, e = ti.family(fam, N_MAIN, 0)
        mats.append((fam, torch.tensor(d, device=dev), torch.tensor(e, device=dev)))
    torch.cuda.synchronize()

    def one_step(record):
        for fam, d, e in mats:
            t0 = time.perf_counter()
            w, Z = mr.eigh_tridiagonal(d, e)
            st = mr.last_stats()
            if record is not None:
                record.append((fam, time.perf_counter() - t0, st))
            del w, Z

    for i in range(warmup):
        one_step(None)
        log(f"[bench] warmup step {i + 1}/{warmup} done")
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        one_step(recs)
        log(f"[bench] timed step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return elapsed, recs


def bench_mixed(mr, torch, reps=3):
    """The single/double form (Ch. 5): the four n = 20000 matrices rounded to
    FP32, all pairs, FP32 results; per matrix the median time, the tree depth
    and the clustering rho = largest cluster / n."""
    import tridiag_inputs as ti
    dev = torch.device("cuda:0")
    out, total = {}, 0.0
    for fam in FAMILIES:
        d, e = ti.family(fam, N_MAIN, 0)
        d32 = torch.tensor(np.float32(d), device=dev)
        e32 = torch.tensor(np.float32(e), device=dev)
        w, Z = mr.eigh_tridiagonal(d32, e32)
        del w, Z
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            w, Z = mr.eigh_tridiagonal(d32, e32)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            del w, Z
        st = mr.last_stats()
        t = float(np.median(ts))
        total += t
        out[fam] = {"ms": 1e3 * t, "tree_ms": float(st["tree_ms"]), "dmax": int(st["dmax"]),
                    "rho": int(st["largest_cluster"]) / N_MAIN, "n_nodes": int(st["n_nodes"]),
                    "n_blocks": int(st["n_blocks"]), "unverified": int(st["n_unverified_rrr"])}
        log(f"[bench] single/double {fam}: {1e3 * t:.1f} ms, d_max {st['dmax']}, "
            f"rho {int(st['largest_cluster']) / N_MAIN:.2e}")
    return {"workload": "the four n=20000 matrices rounded to FP32, all pairs, FP32 in and out, FP64 inside "
                        "(gaptol 1e-5)",
            "eigenpairs_per_s": len(FAMILIES) * N_MAIN / total, "ms_per_step": 1e3 * total,
            "per_family": out}


def bench_batched(mr, torch, reps=5):
    import tridiag_inputs as ti
    dev = torch.device("cuda:0")
    sizes, off, d_cat, e_cat = ti.batch_uniform(4096, seed=0)
    dc = torch.tensor(d_cat, device=dev)
    ec = torch.tensor(e_cat, device=dev)
    pairs = int(off[-1])

    def replay_median(tune, workers=0):
        # first call builds and captures the plan; the timed calls replay it
        opts = {"workers": int(workers)}
        w, Z = mr.eigh_tridiagonal_batched(dc, ec, off, tune=tune, options=opts)
        del w, Z
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            w, Z = mr.eigh_tridiagonal_batched(dc, ec, off, tune=tune, options=opts)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            del w, Z
        return float(np.median(times))

    default_s = replay_median(None)
    log(f"[bench] batched graph replay, default launch shape {default_s * 1e3:.1f} ms")
    from paper_1401_4950_amd import autotune
    # tuning (or reading the cached tuning of this batch make-up) happens
    # before, and outside, the timed replays
    table, rep = autotune.tune_batched(dc, ec, off, log=log)
    graph_s = replay_median(table, rep.workers)
    log(f"[bench] batched graph replay, tuned {graph_s * 1e3:.1f} ms (tuning took {rep.seconds:.1f} s, "
        f"{'cached' if rep.cached else 'measured'})")
    # plain: one call per matrix on the same stream
    views = [(dc[int(off[b]):int(off[b + 1])], ec[int(off[b]):int(off[b + 1]) - 1]) for b in range(len(sizes))]
    for d, e in views[:16]:
        mr.eigh_tridiagonal(d, e)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, e in views:
        mr.eigh_tridiagonal(d, e)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    log(f"[bench] batched as 4096 plain calls {plain_s * 1e3:.1f} ms")
    return {
        "workload": "4096 tridiagonals, n log-uniform in [32, 2048], d U[-1,1], e U[0.1,1], all pairs",
        "eigenpairs": pairs,
        "sum_n2": int(np.sum(np.asarray(sizes, dtype=np.int64) ** 2)),
        "graph_ms": graph_s * 1e3,
        "graph_ms_default_shape": default_s * 1e3,
        "plain_ms": plain_s * 1e3,
        "eigenpairs_per_s": pairs / graph_s,
        "speedup_vs_plain": plain_s / graph_s,
        "autotune": {"seconds": rep.seconds, "cached": rep.cached, "sample_ms": rep.sample_ms,
                     "default_sample_ms": rep.default_sample_ms, "tried": rep.tried,
                     "waves_per_cu": rep.waves_per_cu, "workers": rep.workers,
                     "buckets": {f"2^{k}": v["config"] for k, v in sorted(rep.buckets.items())}},
    }


def bench_grad(mr, torch, reps=3):
    import tridiag_inputs as ti
    from paper_1401_4950_amd import EighTridiagonal, EighTridiagonalBatched
    dev = torch.device("cuda:0")
    out = {}
    # (i) 256 x n = 512: fused batched forward+backward against per-matrix calls
    B, n = 256, 512
    sizes, off, d_cat, e_cat = ti.batch_uniform(B, seed=5, sizes=[n] * B, elo=-1.0, ehi=1.0)
    rng = np.random.default_rng(11)
    c = torch.tensor(rng.standard_normal(B * n), device=dev)
    G = torch.tensor(rng.standard_normal(B * n * n), device=dev)

    def fused():
        d = torch.tensor(d_cat, device=dev, requires_grad=True)
        e = torch.tensor(e_cat, device=dev, requires_grad=True)
        w, Z = EighTridiagonalBatched.apply(d, e, off)
        ((c * w).sum() + (G * Z).sum()).backward()
        return d.grad

    leaves = []
    for b in range(B):
        r0 = int(off[b])
        leaves.append((torch.tensor(d_cat[r0:r0 + n], device=dev, requires_grad=True),
                       torch.tensor(e_cat[r0:r0 + n - 1], device=dev, requires_grad=True),
                       c[r0:r0 + n], G[b * n * n:(b + 1) * n * n].view(n, n).t()))

    def plain():
        for d, e, cb, Gb in leaves:
            d.grad = None
            e.grad = None
            w, Z = EighTridiagonal.apply(d, e)
            ((cb * w).sum() + (Gb * Z).sum()).backward()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    f_s = timed(fused)
    p_s = timed(plain)
    log(f"[bench] fwd+bwd 256x512 fused {f_s * 1e3:.1f} ms, per-matrix {p_s * 1e3:.1f} ms")
    out["batch256_n512"] = {"fused_ms": f_s * 1e3, "plain_ms": p_s * 1e3, "speedup_vs_plain": p_s / f_s}

    # (ii) n = 8192 random: eigenvalue + eigenvector loss; backward alone timed
    n = 8192
    d0, e0 = ti.random_uniform(n, 0)
    c8 = torch.tensor(np.random.default_rng(12).standard_normal(n), device=dev)
    G8 = torch.tensor(np.random.default_rng(13).standard_normal((n, n)), device=dev)

    def fb8():
        d = torch.tensor(d0, device=dev, requires_grad=True)
        e = torch.tensor(e0, device=dev, requires_grad=True)
        w, Z = EighTridiagonal.apply(d, e)
        loss = (c8 * w).sum() + (G8 * Z).sum()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    fb8()
    ts, bw = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        bw.append(fb8())
        ts.append(time.perf_counter() - t0)
    fb_s, bwd_s = float(np.median(ts)), float(np.median(bw))
    flops = 4.0 * n ** 3   # the two n x n x n FP64 products of the backward
    out["n8192"] = {"fwd_bwd_ms": fb_s * 1e3, "bwd_ms": bwd_s * 1e3,
                    "bwd_mfma_tflops": flops / bwd_s / 1e12,
                    "bwd_mfma_frac": flops / bwd_s / 1e12 / FP64_MFMA_PEAK_TFLOPS}
    log(f"[bench] fwd+bwd n=8192 {fb_s * 1e3:.1f} ms (bwd {bwd_s * 1e3:.1f} ms)")

    # (iii) glued Wilkinson n = 8192, eigenvalue-only loss
    dg, eg = ti.glued_wilkinson(n)

    def fbg():
        d = torch.tensor(dg, device=dev, requires_grad=True)
        e = torch.tensor(eg, device=dev, requires_grad=True)
        w, _ = EighTridiagonal.apply(d, e)
        (c8 * w).sum().backward()

    g_s = timed(fbg)
    out["glued8192_values"] = {"fwd_bwd_ms": g_s * 1e3}
    log(f"[bench] fwd+bwd glued n=8192 values-only {g_s * 1e3:.1f} ms")
    return out


def cpu_baseline(k=400):
    """The oracle (bisection + inverse iteration + Gram-Schmidt) on k
    consecutive middle eigenpairs of each n = 20000 matrix."""
    import oracle
    import tridiag_inputs as ti
    il = N_MAIN // 2 - k // 2 + 1
    total = 0.0
    for fam in FAMILIES:
        d, e = ti.family(fam, N_MAIN, 0)
        t0 = time.perf_counter()
        oracle.solve(d, e, "index", il=il, iu=il + k - 1)
        total += time.perf_counter() - t0
    log(f"[bench] oracle sample {total:.1f} s")
    return {"value": 4 * k / total, "unit": "eigenpairs/s", "cores": int(oracle.num_threads()), "kind": "oracle",
            "sample": f"indices {il}..{il + k - 1} ({k} pairs) of each of the four n={N_MAIN} matrices, "
                      f"{total:.1f} s; Gram-Schmidt cost grows with the cluster size, so the oracle's "
                      f"rate on all 20000 pairs would be lower"}


def main(argv=None):
    args = parse_args(argv)
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path; use --gpus 1", file=sys.stderr)
        return 2
    sections = set(s.strip() for s in args.sections.split(",") if s.strip())
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    sys.path.insert(0, HERE)
    import paper_1401_4950_amd as mr

    if "plain" not in sections:
        out = {"metric": "FP64 eigenpairs/s at n=20000 all pairs; batched & fwd+bwd speedup vs plain",
               "value": None, "unit": "eigenpairs/s", "n_gpus": 1, "note": "plain leg not run"}
        if "mixed" in sections:
            out["mixed_single_double"] = bench_mixed(mr, torch)
        if "batched" in sections:
            out["batched"] = bench_batched(mr, torch)
        if "grad" in sections:
            out["fwd_bwd"] = bench_grad(mr, torch)
        print(json.dumps(out), flush=True)
        return 0
    elapsed, recs = bench_plain(mr, torch, args.steps, args.warmup)
    pairs = sum(int(st["m"]) for _, _, st in recs)
    value = pairs / elapsed
    tree_ms = [float(st["tree_ms"]) for _, _, st in recs]
    qd = [float(st["qd_steps"]) for _, _, st in recs]
    mean_ms = float(np.mean(tree_ms))
    algo_flops = ALGO_FLOPS_PER_PAIR_PER_ROW * N_MAIN * N_MAIN          # per launch: k = n = 20000
    achieved = algo_flops / (mean_ms * 1e-3) / 1e12
    issued = FLOPS_PER_QD_STEP * sum(qd) / (sum(tree_ms) * 1e-3) / 1e12
    traffic = read_traffic()
    per_family = {}
    for fam in FAMILIES:
        rs = [(t, st) for f, t, st in recs if f == fam]
        per_family[fam] = {"ms": 1e3 * float(np.median([t for t, _ in rs])),
                           "tree_ms": float(np.median([st["tree_ms"] for _, st in rs])),
                           "qd_steps": int(rs[0][1]["qd_steps"]), "dmax": int(rs[0][1]["dmax"]),
                           "n_nodes": int(rs[0][1]["n_nodes"]),
                           "largest_cluster": int(rs[0][1]["largest_cluster"]),
                           # representations accepted without passing max|D+| <= 8 spdiam, those of
                           # them checked (and failed) for conditional element growth, and the
                           # returned status (1 = MRRR_WARN_UNVERIFIED)
                           "unverified": int(rs[0][1]["n_unverified_rrr"]),
                           "cond_checked": int(rs[0][1]["n_cond_checked"]),
                           "cond_failed": int(rs[0][1]["n_cond_failed"]),
                           "status": int(rs[0][1].get("status", 0))}
    out = {
        "metric": "FP64 eigenpairs/s at n=20000 all pairs; batched & fwd+bwd speedup vs plain",
        "value": value,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / max(args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "all eigenpairs of four n=20000 tridiagonals per step: 1-2-1 (d=2, e=-1), "
                               "Clement, glued Wilkinson W21+ (glue 2^-26), random d,e U[-1,1] (seed 0)",
                   "n": N_MAIN, "matrices_per_step": len(FAMILIES)},
        "per_family": per_family,
        "roofline": {"bound": "alu", "kernel": "mrrr_tree_kernel", "achieved": achieved,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "mean_launch_ms": mean_ms, "flops_per_launch": algo_flops,
                     "work": "200 k n algorithmic flops per n = 20000 matrix (k = n)",
                     "issued": {"tflops": issued, "frac": issued / FP64_VECTOR_PEAK_TFLOPS,
                                "flops_per_launch": FLOPS_PER_QD_STEP * float(np.mean(qd)),
                                "note": "4 flops per executed lane-step of the recurrences"}},
    }
    if "mixed" in sections:
        out["mixed_single_double"] = bench_mixed(mr, torch)
    if "batched" in sections:
        out["batched"] = bench_batched(mr, torch)
    if "grad" in sections:
        out["fwd_bwd"] = bench_grad(mr, torch)
    if "cpu" in sections:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
