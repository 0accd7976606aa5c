"""Time-to-tolerance benchmark of IterativeCUR on one MI355X.

Default workload: the dense RBF kernel matrix A_ij = exp(-||x_i - y_j||^2 / (2 * 0.5^2)),
40000 x 40000, x_i, y_j seeded U[0,1]^3, stored FP32 in HBM; tolerance 1e-4, block
b = 100 (c = 110 sketch rows), sparse-sign sketch with 8 nonzeros per column, plain FP32
form.  One step is one complete icur_run call (sketch, every selection and residual
iteration until rho <= tol, and the FP64 core), with A already resident on the device.

Prints one JSON line (the contract described in the repository's design doc):
  value        mean time-to-tolerance over the timed steps, seconds (lower is better)
  roofline     the sketch product (the dominant kernel) against HBM bandwidth, from
               device events around its launches inside the timed calls
  cpu_baseline the FP64 NumPy oracle timed on the host cores, one run on the same
               matrix (copied from the device and widened to FP64)
Other workloads (each prints its own line; the default is the one above):
  --workload batched   the uneven batch: 512 planted FP32 matrices, m, n uniform in
                       [500, 8000], sigma_i = exp(-i / r0) with r0 uniform in [10, 400],
                       tol log-uniform in [1e-6, 1e-2], block 32, Gaussian sketch; value =
                       time-to-tolerance of the whole batch through icur_run_batched, beside
                       the same matrices through one icur_run call each (plain FP32 loop)
  --workload precision the precision form: A = P diag((1+i)^-2) Q^T + E, 60000 x 40000
                       FP32 (K = 4096 planted terms, ||E||_F = 1e-9 ||A||_F), block 128,
                       Gaussian sketch, tol 1e-3 and 1e-5; value = BF16-split time-to-tol at
                       1e-3, beside the plain FP32 form and both forms at 1e-5
  --workload csr       the sparse form: A = P Q + E as CSR FP32, 200000 x 100000 (P with 5,
                       Q with 100 Gaussian entries per row over 300 latent dimensions, E with
                       20 entries of size 1e-8 per row), tol 1e-6, block 64, sparse-sign
                       sketch; value = BF16-split time-to-tol, beside the plain FP32 form
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--form fp32|bf16]
                       [--workload rbf|batched|precision|csr] [--count N]
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


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("icur_sketch.hip", "icur_wide_kernel.h"):
        with open(os.path.join(ROOT, "paper_2509_21963_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_key):
    """HBM bytes per launch of the sketch product from committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "sketch_product_%s_traffic.json" % workload_key)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
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


def bench_batched(a):
    """The uneven batch through icur_run_batched, and through one icur_run per matrix."""
    import numpy as np
    import torch
    from paper_2509_21963_amd import icur
    from paper_2509_21963_amd import workloads as W

    icur.load()
    b = 32
    specs = W.batch_specs(a.count, seed=0)
    print("generating %d planted matrices on the device" % a.count, file=sys.stderr, flush=True)
    As = []
    for i, sp in enumerate(specs):
        As.append(W.planted_device(sp["m"], sp["n"], W.batch_sigma(sp["r0"], sp["K"]), seed=i))
        if (i + 1) % 64 == 0:
            torch.cuda.synchronize()
            print("  %d generated" % (i + 1), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tols = [sp["tol"] for sp in specs]
    seeds = list(range(a.count))
    elems = float(sum(sp["m"] * sp["n"] for sp in specs))
    # warm-up: one batched call (sizes every worker's workspace) and single calls on the
    # four largest matrices (sizes the single-call workspace)
    for _ in range(a.warmup):
        icur.run_batched(As, tols, b, icur.GAUSSIAN, seeds, workers=a.workers, check=False)
        print("batched warm-up done", file=sys.stderr, flush=True)
    order = sorted(range(a.count), key=lambda i: -specs[i]["m"] * specs[i]["n"])
    if a.warmup:
        for i in order[:4]:
            icur.run(As[i], tols[i], b, icur.GAUSSIAN, seeds[i])
    torch.cuda.synchronize()
    tb = []
    for s in range(a.steps):
        t0 = time.perf_counter()
        got = icur.run_batched(As, tols, b, icur.GAUSSIAN, seeds, workers=a.workers, check=False)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        print("batched step %d: %.3f s" % (s, tb[-1]), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plain, sk_ms, sk_bytes = [], 0.0, 0.0
    for i in range(a.count):
        out = icur.run(As[i], tols[i], b, icur.GAUSSIAN, seeds[i])
        plain.append(out)
        sk_ms += out["info"]["ms_sketch_product"]
        m, n = As[i].shape
        c = (11 * b) // 10
        sk_bytes += 4.0 * m * n + 2.0 * c * m + 8.0 * c * n
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    print("plain loop: %.3f s" % t_plain, file=sys.stderr, flush=True)
    same = all(g["rank"] == p["rank"] and np.array_equal(g["I"], p["I"]) and np.array_equal(g["J"], p["J"])
               for g, p in zip(got, plain))
    ranks = [g["rank"] for g in got]
    value = statistics.median(tb)
    achieved = sk_bytes / (sk_ms * 1e-3) / 1e9 if sk_ms > 0 else None
    line = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": value * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": "uneven batch: %d planted FP32 matrices, m,n ~ U{500..8000}, sigma_i = exp(-i/r0), "
                        "r0 ~ U[10,400], tol ~ 10^U[-6,-2], block 32, Gaussian sketch, fp32 form" % a.count,
            "count": a.count, "elements": elems, "block": b, "workers": a.workers or 16,
            "plain_loop_s": t_plain, "speedup_vs_plain_loop": t_plain / value,
            "identical_to_plain_loop": bool(same),
            "rank_min": min(ranks), "rank_median": statistics.median(ranks), "rank_max": max(ranks),
            "statuses": {k: sum(1 for g in got if g["status"] == k) for k in set(g["status"] for g in got)},
        },
        "roofline": {
            "kernel": "sketch product G A over the batch (sketch_kernel, from the plain loop's device events)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": None,
            "avg_ms": sk_ms / a.count, "algorithmic_bytes": sk_bytes / a.count,
        },
    }
    if not a.no_cpu:
        from oracle.icur import iterative_cur
        print("timing the CPU oracle on a sample of the batch", file=sys.stderr, flush=True)
        spent, done_elems, k = 0.0, 0.0, 0
        for i in sorted(range(a.count), key=lambda q: specs[q]["m"] * specs[q]["n"]):
            A64 = As[i].cpu().numpy().astype(np.float64)
            t0 = time.perf_counter()
            iterative_cur(A64, tols[i], b, kind=0, seed=seeds[i])
            spent += time.perf_counter() - t0
            done_elems += A64.size
            k += 1
            if spent > 15.0:
                break
        line["cpu_baseline"] = {
            "value": spent * elems / done_elems, "unit": "s", "cores": int(oracle_threads()), "kind": "oracle",
            "sample": "FP64 NumPy oracle on the %d smallest matrices of the batch (%.1f s measured), scaled by "
                      "total m n / sampled m n to the whole batch" % (k, spent)}
    else:
        line["cpu_baseline"] = None
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
    runs = {}
    for tol in (1e-3, 1e-5):
        for form, prec in (("bf16", icur.BF16_SPLIT), ("fp32", icur.FP32)):
            for i in range(a.warmup):
                icur.run(A, tol, b, icur.GAUSSIAN, seed=i, precision=prec)
            torch.cuda.synchronize()
            times, outs = [], []
            for i in range(a.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = icur.run(A, tol, b, icur.GAUSSIAN, seed=i, precision=prec)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                outs.append(out)
            last = outs[-1]
            runs["%s@%g" % (form, tol)] = {
                "s": statistics.median(times), "rank": last["rank"], "rho": last["rho"],
                "iterations": last["info"]["iterations"], "split_terms": last["info"]["split_terms"],
                "sketch_ms": statistics.mean(o["info"]["ms_sketch_product"] for o in outs)}
            print("%s tol %g: %.2f ms, rank %d, rho %.3e, %d iterations" % (
                form, tol, runs["%s@%g" % (form, tol)]["s"] * 1e3, last["rank"], last["rho"],
                last["info"]["iterations"]), file=sys.stderr, flush=True)
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
            icur.run_csr(*d, (m, n), tol, b, icur.SPARSE_SIGN, seed=i, precision=prec)
        torch.cuda.synchronize()
        times, outs = [], []
        for i in range(a.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = icur.run_csr(*d, (m, n), tol, b, icur.SPARSE_SIGN, seed=i, precision=prec)
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
    ap.add_argument("--workload", choices=["rbf", "batched", "precision", "csr"], default="rbf")
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
        return {"batched": bench_batched, "precision": bench_precision, "csr": bench_csr}[a.workload](a)

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
        icur.run(A, tol, b, kind, seed=i, precision=precision, zeta=zeta)
        print("warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, sketch_ms = [], []
    t_all = time.perf_counter()
    for i in range(a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = icur.run(A, tol, b, kind, seed=i, precision=precision, zeta=zeta)
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
    traffic = measured_traffic("rbf%d" % m)
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
