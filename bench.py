"""Time-to-tolerance benchmark of IterativeCUR on one MI355X.

Default workload (the metric's headline comparison): the uneven batch, 512 planted FP32
matrices A = P diag(sigma) Q^T with m, n uniform in [500, 8000], sigma_i = exp(-i / r0),
r0 uniform in [10, 400], per-matrix tolerance log-uniform in [1e-6, 1e-2], block 32,
Gaussian sketch.  One step is one icur_run_batched call on the whole batch (the grouped
form: every matrix advanced together, one launch per step of Alg. 1), with all matrices
resident in HBM.  Beside it, in the same line:
  plain_loop_s          the same 512 matrices through one icur_run call each (the plain
                        FP32 form, one matrix at a time), and the speed-up over it;
  precision_form        the 60000 x 40000 precision-form matrix (block 128, Gaussian
                        sketch) at tol 1e-3 and 1e-5, BF16-split against plain FP32.
  roofline              the grouped FP64 product kernel of the batched loop (the kernel
                        with the most device time: its P1-P3 launches), algorithmic bytes
                        over its duration from device events inside the timed calls,
                        against HBM;
  cpu_baseline          the FP64 NumPy oracle on randomly drawn matrices of the batch
                        (about 20 s of host time), scaled by count / drawn.
Other workloads (--workload): rbf (40000 x 40000 RBF kernel, tol 1e-4, block 100,
sparse-sign sketch, plain FP32), precision (the 60000 x 40000 form alone), csr (the
200000 x 100000 sparse form), x1 (the paper's 30000 x 30000 rank-2000 Low-Rank matrix,
tol 1e-6, block 250), each printing its own line with the same fields.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--workload batched|rbf|precision|csr|x1] [--count N] [--workers W]
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-tol (s) + sketch TFLOP/s|GB/s, BF16-split/batched vs FP32 plain"
HBM_PEAK_GBS = 8000.0


SKETCH_SOURCES = ("icur_sketch.hip", "icur_wide_kernel.h")
GROUPED_SOURCES = ("icur_group_kernels.hip", "icur_batched.h")


def kernel_source_hash(files=SKETCH_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2509_21963_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name, files=SKETCH_SOURCES):
    """HBM bytes per launch of a kernel from committed rocprofv3 counter runs
    (profiles/<name>_traffic.json), if they were taken on the current source of the
    kernel; else None."""
    path = os.path.join(ROOT, "profiles", "%s_traffic.json" % name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash(files):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(A_dev, tol=1e-4, b=100):
    """The FP64 oracle on the same matrix the GPU runs: A copied from the device to the host
    and widened to FP64, then one complete oracle run (sketch, selections, residual
    iterations and core) with the same tolerance, block and sketch family."""
    import numpy as np
    from oracle.icur import iterative_cur
    cores = oracle_threads()
    A64 = A_dev.cpu().numpy().astype(np.float64)
    m, n = A64.shape
    t0 = time.perf_counter()
    out = iterative_cur(A64, tol, b, kind=1, seed=0)
    dt = time.perf_counter() - t0
    del A64
    return {"value": dt, "unit": "s", "cores": int(cores), "kind": "oracle",
            "sample": ("one FP64 NumPy oracle run on the full %dx%d RBF matrix of the timed workload "
                       "(copied from the device, widened to FP64; tol %g, b %d, sparse-sign sketch): "
                       "rank %d, rho %.2e; no extrapolation" % (m, n, tol, b, out["rank"], out["rho"]))}


def oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def precision_runs(A, steps, warmup, b=128):
    """The precision-form matrix at tol 1e-3 and 1e-5: BF16-split against plain FP32."""
    import torch
    from paper_2509_21963_amd import icur
    runs = {}
    for tol in (1e-3, 1e-5):
        for form, prec in (("bf16", icur.BF16_SPLIT), ("fp32", icur.FP32)):
            for i in range(warmup):
                icur.run(A, tol, b, icur.GAUSSIAN, seed=i, precision=prec, device_outputs=True)
            torch.cuda.synchronize()
            times, outs = [], []
            for i in range(steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = icur.run(A, tol, b, icur.GAUSSIAN, seed=i, precision=prec, device_outputs=True)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                outs.append(out)
            last = outs[-1]
            key = "%s@%g" % (form, tol)
            runs[key] = {
                "s": statistics.median(times), "rank": last["rank"], "rho": last["rho"],
                "iterations": last["info"]["iterations"], "split_terms": last["info"]["split_terms"],
                "sketch_ms": statistics.mean(o["info"]["ms_sketch_product"] for o in outs),
                "select_ms": statistics.mean(o["info"]["ms_select"] for o in outs),
                "residual_ms": statistics.mean(o["info"]["ms_residual"] for o in outs),
                "core_ms": statistics.mean(o["info"]["ms_core"] for o in outs)}
            print("precision form %s tol %g: %.2f ms, rank %d, rho %.3e" % (
                form, tol, runs[key]["s"] * 1e3, last["rank"], last["rho"]), file=sys.stderr, flush=True)
    return runs


def bench_batched(a):
    """The uneven batch through icur_run_batched (grouped form), beside one icur_run per
    matrix (the plain FP32 loop) and the precision form's BF16-split / FP32 pair."""
    import random
    import numpy as np
    import torch
    from paper_2509_21963_amd import icur
    from paper_2509_21963_amd import workloads as W

    icur.load()
    b = 32
    c = (11 * b) // 10
    specs = W.batch_specs(a.count, seed=0)
    print("generating %d planted matrices on the device" % a.count, file=sys.stderr, flush=True)
    As = []
    for i, sp in enumerate(specs):
        As.append(W.planted_device(sp["m"], sp["n"], W.batch_sigma(sp["r0"], sp["K"]), seed=i))
        if (i + 1) % 128 == 0:
            torch.cuda.synchronize()
            print("  %d generated" % (i + 1), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tols = [sp["tol"] for sp in specs]
    seeds = list(range(a.count))
    elems = float(sum(sp["m"] * sp["n"] for sp in specs))
    # the timed calls write their indices and cores to device pools (inputs and outputs
    # resident in HBM); one more call with host pools gives the rate with the results
    # copied over PCIe
    got = None
    for w in range(a.warmup):
        got = None
        got = icur.run_batched(As, tols, b, icur.GAUSSIAN, seeds, workers=a.workers, check=False,
                               device_outputs=True)
        print("batched warm-up %d done" % w, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tb, infos = [], []
    for s in range(a.steps):
        got = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got = icur.run_batched(As, tols, b, icur.GAUSSIAN, seeds, workers=a.workers, check=False,
                               device_outputs=True)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        infos.append(icur.last_info())
        print("batched step %d: %.3f s" % (s, tb[-1]), file=sys.stderr, flush=True)
    got = [{"I": g["I"].cpu().numpy(), "J": g["J"].cpu().numpy(), "rank": g["rank"], "status": g["status"]}
           for g in got]
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hp = icur.run_batched(As, tols, b, icur.GAUSSIAN, seeds, workers=a.workers, check=False)
    t_host = time.perf_counter() - t0
    host_info = icur.last_info()
    same_host = sum(1 for g, h in zip(got, hp) if np.array_equal(g["I"], h["I"]) and np.array_equal(g["J"], h["J"]))
    del hp
    print("batched, host pools: %.3f s" % t_host, file=sys.stderr, flush=True)
    # the plain FP32 loop: one icur_run per matrix, once (its workspace is sized by a first
    # call on the largest matrix)
    if a.no_plain:
        plain, t_plain = got, float("nan")
    else:
        big = max(range(a.count), key=lambda i: specs[i]["m"] * specs[i]["n"])
        icur.run(As[big], tols[big], b, icur.GAUSSIAN, seeds[big], device_outputs=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = [icur.run(As[i], tols[i], b, icur.GAUSSIAN, seeds[i], device_outputs=True) for i in range(a.count)]
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        plain = [{"I": p["I"].cpu().numpy(), "J": p["J"].cpu().numpy(), "rank": p["rank"]} for p in plain]
        print("plain loop: %.3f s" % t_plain, file=sys.stderr, flush=True)
    ranks = [g["rank"] for g in got]
    same_rank = sum(1 for g, p in zip(got, plain) if g["rank"] == p["rank"])
    same_idx = sum(1 for g, p in zip(got, plain) if np.array_equal(g["I"], p["I"]) and np.array_equal(g["J"], p["J"]))
    value = statistics.median(tb)
    inf = infos[-1]
    # roofline of the loop's large FP64 products (stages P1-P3: the row residual, the
    # new-row residual with the (Q^-1)^T block row, the row factors with the P^-1 block
    # row; one gemm_kernel launch each per iteration): algorithmic bytes over their device
    # time, from events around every launch of the timed calls
    shapes = ["16x128", "32x128", "48x128", "64x128", "32x256", "64x256", "w32x32", "w16x64", "w32x64",
              "32x128/2", "64x128/2", "32x128/3"]
    prod_ms = statistics.mean(sum(i["ms_stage"][:3]) for i in infos)
    prod_bytes = statistics.mean(sum(i["stage_bytes"][:3]) for i in infos)
    launches = 3 * inf["group_iterations"]
    achieved = prod_bytes / (prod_ms * 1e-3) / 1e9 if prod_ms > 0 else None
    line = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": "uneven batch: %d planted FP32 matrices, m,n ~ U{500..8000}, sigma_i = exp(-i/r0), "
                        "r0 ~ U[10,400], tol ~ 10^U[-6,-2], block 32, Gaussian sketch; grouped batched form "
                        "(every matrix advanced together) against one icur_run per matrix" % a.count,
            "count": a.count, "elements": elems, "block": b, "form": "grouped" if not a.workers else "workers",
            "outputs": "device pools (indices and cores stay in HBM)",
            "plain_loop_s": t_plain, "speedup_vs_plain_loop": t_plain / value,
            "host_pools_s": t_host, "host_pools_results_copy_ms": host_info["ms_results"],
            "same_indices_host_vs_device_pools": same_host,
            "same_rank_as_plain_loop": same_rank, "same_indices_as_plain_loop": same_idx,
            "rank_min": min(ranks), "rank_median": statistics.median(ranks), "rank_max": max(ranks),
            "statuses": {k: sum(1 for g in got if g["status"] == k) for k in set(g["status"] for g in got)},
            "grouped_iterations": inf["group_iterations"], "sketch_phase_ms": inf["ms_sketch"],
            "select_ms": inf["ms_select"], "products_ms": inf["ms_products"],
            "buffer_setup_ms": inf["ms_setup"], "iterations_host_ms": inf["ms_residual"],
            "core_products_ms": inf["ms_core"], "results_copy_ms": inf["ms_results"],
            "stage_ms": dict(zip(("P1", "P2", "P3", "P4", "FIN"), inf["ms_stage"])),
            "stage_gbytes": dict(zip(("P1", "P2", "P3", "P4", "FIN"), [x / 1e9 for x in inf["stage_bytes"]])),
            "tiles": dict(zip(("P1", "P2", "P3", "FIN"), [shapes[t] for t in inf["tiles"]])),
        },
        "roofline": {
            "kernel": "grouped FP64 product kernel of the batched loop, stages P1-P3 (gemm_kernel<%s>: row "
                      "residual, new-row residual and the two inverses' block rows; %d launches per call)"
                      % (shapes[inf["tiles"][0]], launches),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": measured_traffic("batched_products_uneven%d" % a.count, GROUPED_SOURCES),
            "avg_ms": prod_ms / max(launches, 1),
            "algorithmic_bytes": prod_bytes / max(launches, 1),
        },
    }
    cpu = None
    if not a.no_cpu:
        from oracle.icur import iterative_cur
        print("timing the CPU oracle on randomly drawn matrices of the batch", file=sys.stderr, flush=True)
        order = list(range(a.count))
        random.Random(0).shuffle(order)
        spent, k = 0.0, 0
        for i in order:
            A64 = As[i].cpu().numpy().astype(np.float64)
            t0 = time.perf_counter()
            iterative_cur(A64, tols[i], b, kind=0, seed=seeds[i])
            spent += time.perf_counter() - t0
            k += 1
            if spent > 20.0:
                break
        cpu = {"value": spent * a.count / k, "unit": "s", "cores": int(oracle_threads()), "kind": "oracle",
               "sample": "FP64 NumPy oracle on %d matrices drawn at random from the batch (%.1f s measured), "
                         "scaled by count / drawn to the whole batch" % (k, spent)}
    line["cpu_baseline"] = cpu
    if not a.no_precision:
        del As, got, plain
        torch.cuda.empty_cache()
        m, n = 60000, 40000
        print("generating the %dx%d precision-form matrix on the device" % (m, n), file=sys.stderr, flush=True)
        A = W.precision_form_device(m, n, seed=0)
        torch.cuda.synchronize()
        runs = precision_runs(A, min(a.steps, 3), min(a.warmup, 1))
        line["config"]["precision_form"] = {
            "matrix": "A = P diag((1+i)^-2) Q^T + E, %dx%d FP32, K=4096, ||E||_F = 1e-9 ||A||_F, block 128, "
                      "Gaussian sketch" % (m, n),
            "runs": runs,
            "speedup_bf16_vs_fp32": {t: runs["fp32@%s" % t]["s"] / runs["bf16@%s" % t]["s"] for t in ("0.001", "1e-05")}}
    print(json.dumps(line), flush=True)


def bench_precision(a):
    """The precision form against the plain FP32 form on the 60000 x 40000 planted matrix."""
    import numpy as np
    import torch
    from paper_2509_21963_amd import icur
    from paper_2509_21963_amd import workloads as W

    icur.load()
    m, n, b = 60000, 40000, 128
    c = (11 * b) // 10
    print("generating the %dx%d planted matrix on the device" % (m, n), file=sys.stderr, flush=True)
    A = W.precision_form_device(m, n, seed=0)
    torch.cuda.synchronize()
    runs = precision_runs(A, a.steps, a.warmup, b)
    head = runs["bf16@0.001"]
    # the sketch kernel in the BF16-split form at tol 1e-3 (2 pieces of A): algorithmic
    # bytes read A once, the BF16 G, and write X0 in FP64
    alg_bytes = 4.0 * m * n + 2.0 * c * m + 8.0 * c * n
    achieved = alg_bytes / (head["sketch_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": head["s"], "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": head["s"] * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {
            "workload": "precision form: A = P diag((1+i)^-2) Q^T + E, %dx%d FP32, K=4096, ||E||_F = 1e-9 ||A||_F, "
                        "block %d, Gaussian sketch; value = BF16-split at tol 1e-3" % (m, n, b),
            "m": m, "n": n, "block": b, "sketch_rows": c, "runs": runs,
            "speedup_bf16_vs_fp32": {t: runs["fp32@%s" % t]["s"] / runs["bf16@%s" % t]["s"] for t in ("0.001", "1e-05")},
        },
        "roofline": {
            "kernel": "sketch product G A, BF16-split form at tol 1e-3 (sketch_kernel, %d BF16 pieces of A)"
                      % head["split_terms"],
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_ms": head["sketch_ms"],
            "algorithmic_bytes": alg_bytes,
        },
    }
    if not a.no_cpu:
        from oracle.icur import iterative_cur
        print("timing the CPU oracle on the same matrix at tol 1e-3", file=sys.stderr, flush=True)
        A64 = A.cpu().numpy().astype(np.float64)
        del A
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        ora = iterative_cur(A64, 1e-3, b, kind=0, seed=0)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {
            "value": dt, "unit": "s", "cores": int(oracle_threads()), "kind": "oracle",
            "sample": "one FP64 NumPy oracle run on the full %dx%d matrix at tol 1e-3 (copied from the device, "
                      "widened to FP64): rank %d, rho %.2e" % (m, n, ora["rank"], ora["rho"])}
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def bench_x1(a):
    """The paper's rank-adaptive Low-Rank matrix (§5.1): A = G1 G2^T, G_i 30000 x 2000
    standard Gaussian, FP32, tol 1e-6, block 250, Gaussian sketch, plain form."""
    import numpy as np
    import torch
    from paper_2509_21963_amd import icur
    from paper_2509_21963_amd import workloads as W

    icur.load()
    m = n = 30000
    rk, b, tol = 2000, 250, 1e-6
    c = (11 * b) // 10
    print("generating the %dx%d rank-%d matrix on the device" % (m, n, rk), file=sys.stderr, flush=True)
    A = W.low_rank_device(m, n, rk, seed=0)
    torch.cuda.synchronize()
    for i in range(a.warmup):
        icur.run(A, tol, b, icur.GAUSSIAN, seed=i, device_outputs=True)
    torch.cuda.synchronize()
    times, outs = [], []
    for i in range(a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = icur.run(A, tol, b, icur.GAUSSIAN, seed=i, device_outputs=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        outs.append(out)
        print("step %d: %.2f ms, rank %d, rho %.3e, %d iterations" % (
            i, times[-1] * 1e3, out["rank"], out["rho"], out["info"]["iterations"]), file=sys.stderr, flush=True)
    value = statistics.median(times)
    last = outs[-1]
    sk = statistics.mean(o["info"]["ms_sketch_product"] for o in outs)
    # the sketch kernel: c = 275 rows run as two slices of G, each reading A once
    slices = -(-c // 160)
    alg_bytes = 4.0 * m * n * slices + 2.0 * c * m + 8.0 * c * n
    achieved = alg_bytes / (sk * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": "Low-Rank (rank-adaptive experiment): A = G1 G2^T, G_i %dx%d standard Gaussian (device "
                        "generator), FP32 %dx%d, tol %g, block %d, Gaussian sketch, plain form" % (m, rk, m, n, tol, b),
            "rank": last["rank"], "rho": last["rho"], "iterations": last["info"]["iterations"],
            "sketch_ms": sk, "select_ms": statistics.mean(o["info"]["ms_select"] for o in outs),
            "residual_ms": statistics.mean(o["info"]["ms_residual"] for o in outs),
            "core_ms": statistics.mean(o["info"]["ms_core"] for o in outs),
            "paper_context": "the paper reports a 12 s median for IterativeCUR on this matrix on its CPU machine "
                             "(48 cores); context, not the target",
        },
        "roofline": {
            "kernel": "sketch product G A (sketch_kernel, 3 BF16 pieces of A, %d slices of G)" % slices,
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_ms": sk, "algorithmic_bytes": alg_bytes,
        },
    }
    if not a.no_cpu:
        from oracle.icur import iterative_cur
        print("timing the CPU oracle on the same matrix", file=sys.stderr, flush=True)
        A64 = A.cpu().numpy().astype(np.float64)
        del A
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        ora = iterative_cur(A64, tol, b, kind=0, seed=0)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {
            "value": dt, "unit": "s", "cores": int(oracle_threads()), "kind": "oracle",
            "sample": "one FP64 NumPy oracle run on the full %dx%d matrix (copied from the device, widened to "
                      "FP64): rank %d, rho %.2e" % (m, n, ora["rank"], ora["rho"])}
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def bench_csr(a):
    """The sparse form through icur_run_csr, BF16-split and plain FP32."""
    import numpy as np
    import torch
    from paper_2509_21963_amd import icur
    from paper_2509_21963_amd import workloads as W

    icur.load()
    m, n, b, tol = 200000, 100000, 64, 1e-6
    c = (11 * b) // 10
    print("generating the %dx%d sparse matrix on the host" % (m, n), file=sys.stderr, flush=True)
    rowptr, colind, vals = W.csr_to_f32(W.sparse_lowrank(m, n, seed=0))
    nnz = int(colind.size)
    d = [torch.from_numpy(x).cuda() for x in (rowptr, colind, vals)]
    torch.cuda.synchronize()
    runs = {}
    for form, prec in (("bf16", icur.BF16_SPLIT), ("fp32", icur.FP32)):
        for i in range(a.warmup):
            icur.run_csr(*d, (m, n), tol, b, icur.SPARSE_SIGN, seed=i, precision=prec, device_outputs=True)
        torch.cuda.synchronize()
        times, outs = [], []
        for i in range(a.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = icur.run_csr(*d, (m, n), tol, b, icur.SPARSE_SIGN, seed=i, precision=prec, device_outputs=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            outs.append(out)
        last = outs[-1]
        runs[form] = {"s": statistics.median(times), "rank": last["rank"], "rho": last["rho"],
                      "iterations": last["info"]["iterations"],
                      "sketch_ms": statistics.mean(o["info"]["ms_sketch_product"] for o in outs)}
        print("%s: %.2f ms, rank %d, rho %.3e, %d iterations" % (form, runs[form]["s"] * 1e3, last["rank"],
                                                                 last["rho"], last["info"]["iterations"]),
              file=sys.stderr, flush=True)
    head = runs["bf16"]
    # the CSR sketch reads every stored entry once from the column-compressed copy
    # (4-byte value + 4-byte row index) and writes X0 in FP64
    alg_bytes = 8.0 * nnz + 8.0 * c * n
    achieved = alg_bytes / (head["sketch_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": head["s"], "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": head["s"] * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {
            "workload": "sparse form: A = P Q + E, CSR FP32 %dx%d (nnz %d), 300 latent dims, tol %g, block %d, "
                        "sparse-sign sketch zeta=8; value = BF16-split" % (m, n, nnz, tol, b),
            "m": m, "n": n, "nnz": nnz, "block": b, "sketch_rows": c, "runs": runs,
            "speedup_bf16_vs_fp32": runs["fp32"]["s"] / head["s"],
        },
        "roofline": {
            "kernel": "CSR sketch X0 = G A (column-compressed copy, FP64 accumulation)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_ms": head["sketch_ms"],
            "algorithmic_bytes": alg_bytes,
        },
    }
    if not a.no_cpu:
        # the dense oracle cannot hold the full matrix: time it on a smaller instance of
        # the same recipe and scale by the stored entries
        from oracle.icur import iterative_cur
        ms_, ns_ = 20000, 10000
        print("timing the CPU oracle on a %dx%d instance of the recipe" % (ms_, ns_), file=sys.stderr, flush=True)
        rp, ci, vv = W.csr_to_f32(W.sparse_lowrank(ms_, ns_, seed=0))
        A64 = W.csr_dense64(rp, ci, vv, (ms_, ns_))
        t0 = time.perf_counter()
        ora = iterative_cur(A64, tol, b, kind=1, seed=0)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {
            "value": dt * nnz / float(ci.size), "unit": "s", "cores": int(oracle_threads()), "kind": "oracle",
            "sample": "dense FP64 NumPy oracle on a %dx%d instance of the same recipe (nnz %d): %.2f s, rank %d, "
                      "rho %.2e; scaled by the ratio of stored entries to the full matrix" % (
                          ms_, ns_, ci.size, dt, ora["rank"], ora["rho"])}
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--form", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--size", type=int, default=40000)
    ap.add_argument("--workload", choices=["rbf", "batched", "precision", "csr", "x1"], default="batched")
    ap.add_argument("--no-precision", action="store_true", help="batched: skip the precision-form comparison")
    ap.add_argument("--no-plain", action="store_true", help="batched: skip the plain loop (profiling runs)")
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--workers", type=int, default=0)
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path (requested %d)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.workload != "rbf":
        import torch
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            sys.exit(1)
        return {"batched": bench_batched, "precision": bench_precision, "csr": bench_csr,
                "x1": bench_x1}[a.workload](a)

    import torch
    from paper_2509_21963_amd import icur
    from paper_2509_21963_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    icur.load()
    m = n = a.size
    tol, b, kind, zeta = 1e-4, 100, icur.SPARSE_SIGN, 8
    precision = icur.FP32 if a.form == "fp32" else icur.BF16_SPLIT
    print("generating RBF %dx%d on the device" % (m, n), file=sys.stderr, flush=True)
    A = W.rbf_torch(m, n, seed=0)
    torch.cuda.synchronize()

    results = []
    for i in range(a.warmup):
        icur.run(A, tol, b, kind, seed=i, precision=precision, zeta=zeta, device_outputs=True)
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, sketch_ms = [], []
    t_all = time.perf_counter()
    for i in range(a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = icur.run(A, tol, b, kind, seed=i, precision=precision, zeta=zeta, device_outputs=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        sketch_ms.append(out["info"]["ms_sketch_product"])
        results.append(out)
        print("step %d: %.2f ms, rank %d, rho %.3e, %d iterations" % (
            i, times[-1] * 1e3, out["rank"], out["rho"], out["info"]["iterations"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    value = sum(times) / len(times)
    last = results[-1]
    # roofline of the sketch product: algorithmic bytes = read A once (4 m n), read the
    # dense BF16 G (2 c m), write X0 in FP64 (8 c n)
    c = (11 * b) // 10
    alg_bytes = 4.0 * m * n + 2.0 * c * m + 8.0 * c * n
    avg_ms = statistics.mean(sketch_ms)
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None
    traffic = measured_traffic("sketch_product_rbf%d" % m)
    info = last["info"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": value * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "RBF kernel matrix %dx%d FP32 (h=0.5, x,y ~ U[0,1]^3 seed 0), tol %g, block %d, "
                        "sparse-sign sketch zeta=%d, %s form" % (m, n, tol, b, zeta, a.form),
            "m": m, "n": n, "tol": tol, "block": b, "sketch_rows": c, "sketch": "sparse-sign",
            "zeta": zeta, "form": a.form, "rank": last["rank"], "rho": last["rho"],
            "iterations": info["iterations"], "timed_wall_s": wall,
            "phase_ms": {"sketch": info["ms_sketch"], "select": info["ms_select"],
                         "residual": info["ms_residual"], "core": info["ms_core"],
                         "total_host": info["ms_total"]},
        },
        "roofline": {
            "kernel": "sketch product G A (sketch_kernel: 3 BF16 pieces of A on bf16 MFMA, FP64 output)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "avg_ms": avg_ms, "algorithmic_bytes": alg_bytes,
        },
    }
    if not a.no_cpu:
        print("timing the CPU oracle on the same matrix", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(A, tol=tol, b=b)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
