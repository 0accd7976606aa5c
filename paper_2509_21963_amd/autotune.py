"""Tile-shape autotuner of the grouped batched products (icur_run_batched, grouped form).

The grouped loop has four product stages whose tile shape is free: the row residual (P1),
the new-row residual with the (Q^{-1})^T block (P2), the row factors with the P^{-1} block
(P3) and the closing core products (FIN).  Every shape gives bit-identical results (the
depth chunks start at fixed multiples, so each element's sum is the same), so the choice is
speed only.  This script runs one uneven batch once per shape, with every stage on that
shape (ICUR_BATCH_TILES), reads each stage's device time from icur_last_info, checks that
the results are identical, and writes the fastest shape per stage to a JSON file that the
library reads at its first grouped call (tune_gfx950.json beside libicur.so, or
ICUR_TUNE_FILE):

    {"device": ..., "batched_tiles": {"<block>": {"p1": s, "p2": s, "p3": s, "fin": s}},
     "measured_ms": {"<block>": {"<shape>": [P1, P2, P3, P4, FIN]}}}

Usage (on the GPU): python -m paper_2509_21963_amd.autotune [--count 192] [--block 32]
"""
import argparse
import json
import os
import sys
import time

SHAPES = ["16x128", "32x128", "48x128", "64x128", "32x256", "64x256", "w32x32", "w16x64", "w32x64",
          "32x128/2", "64x128/2", "32x128/3"]
STAGES = ["p1", "p2", "p3", "p4", "fin"]


def tune(count, block, seed=0, out=None, repeats=1):
    import numpy as np
    import torch
    from . import icur
    from . import workloads as W

    icur.load()
    specs = W.batch_specs(count, seed=seed)
    mats = [W.planted_device(sp["m"], sp["n"], W.batch_sigma(sp["r0"], sp["K"]), seed=i)
            for i, sp in enumerate(specs)]
    torch.cuda.synchronize()
    tols = [sp["tol"] for sp in specs]
    seeds = list(range(count))
    measured, first = {}, None
    old = os.environ.get("ICUR_BATCH_TILES")
    try:
        for v in range(len(SHAPES)):
            os.environ["ICUR_BATCH_TILES"] = "%d,%d,%d,%d" % (v, v, v, v)
            best = None
            for _ in range(repeats + 1):  # the first run warms the arena and the kernels
                got = icur.run_batched(mats, tols, block, icur.GAUSSIAN, seeds, check=False)
                inf = icur.last_info()
                if inf["tiles"] != [v, v, v, v]:
                    raise RuntimeError("tile override not applied: %s" % inf["tiles"])
                st = inf["ms_stage"]
                best = st if best is None else [min(x, y) for x, y in zip(best, st)]
            measured[SHAPES[v]] = best
            print("shape %-7s stage ms %s" % (SHAPES[v], " ".join("%8.1f" % x for x in best)), flush=True)
            # every shape must give the same results
            if first is None:
                first = got
            else:
                for a, b in zip(first, got):
                    same = (a["rank"] == b["rank"] and a["status"] == b["status"] and
                            np.array_equal(a["I"], b["I"]) and np.array_equal(a["J"], b["J"]) and
                            np.array_equal(a["U"], b["U"]) and a["rho"] == b["rho"])
                    if not same:
                        raise RuntimeError("shape %s changed a result" % SHAPES[v])
    finally:
        if old is None:
            os.environ.pop("ICUR_BATCH_TILES", None)
        else:
            os.environ["ICUR_BATCH_TILES"] = old
    choice = {}
    for q, name in enumerate(STAGES):
        if name == "p4":
            continue  # its shape follows c
        choice[name] = min(range(len(SHAPES)), key=lambda v: measured[SHAPES[v]][q])
    path = out or os.path.join(os.path.dirname(os.path.abspath(icur.LIB_PATH)), "tune_gfx950.json")
    doc = {}
    if os.path.exists(path):
        with open(path) as f:
            doc = json.load(f)
    doc["device"] = torch.cuda.get_device_name(0)
    doc.setdefault("batched_tiles", {})[str(block)] = choice
    doc.setdefault("measured_ms", {})[str(block)] = measured
    doc.setdefault("workload", {})[str(block)] = (
        "uneven batch: %d planted matrices, m,n ~ U{500..8000}, sigma_i = exp(-i/r0), r0 ~ U[10,400], "
        "tol ~ 10^U[-6,-2], seed %d, Gaussian sketch; stage times are device events, best of %d" %
        (count, seed, repeats))
    doc["tuned_at"] = time.strftime("%Y-%m-%d %H:%M:%S")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    print("chosen", choice, "->", path, flush=True)
    return choice


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--count", type=int, default=192)
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--repeats", type=int, default=1)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    tune(a.count, a.block, a.seed, a.out, a.repeats)
    return 0


if __name__ == "__main__":
    sys.exit(main())
