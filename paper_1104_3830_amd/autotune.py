"""Tile-shape autotuner for the column sweep (run on the GPU).

The column sweep splits an instance's rows into segments; each segment of
each column tile is one work unit, and the finalise kernel adds one partial
per segment and column. Short segments give more parallel units, long ones
fewer partials to add. The tuner times whole iterations (row sweep, column
sweep, finalise, end of iteration; int16 weights uniform on 0..1000, p = 32)
as the difference between a long and a short fixed-iteration run (best of a
few repeats each), so the per-call work cancels:
  - the size buckets of the batched workload (512 instances, n log-uniform
    on [32, 1024]) on that batch itself, one bucket at a time with the others
    held (coordinate descent from the built-in rule), since the table serves
    mixed batches;
  - the larger buckets on a single instance of the bucket's largest size.
The table is written as JSON next to the library; the binding loads it at
import, so every later process uses the same shapes (the shape is a function
of n only, which keeps results independent of batch mixes).

    python -m paper_1104_3830_amd.autotune [--out PATH] [--iters K]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

BUCKETS = [64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
CANDIDATES = [16, 32, 64, 128, 256, 512, 1024]


def main():
    ap = argparse.ArgumentParser()
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--out", default=os.path.join(here, "tile_table_gfx950.json"))
    ap.add_argument("--iters", type=int, default=400)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args()
    os.environ["SK_NO_TILE_TABLE"] = "1"
    sys.path.insert(0, os.path.dirname(here))
    import torch

    import paper_1104_3830_amd as sk
    import skgen

    ctx = sk.Context(0)
    lo = max(1, args.iters // 10)
    prm_hi = sk.make_params([32], tol=0.0, max_iters=args.iters, check_every=64)
    prm_lo = sk.make_params([32], tol=0.0, max_iters=lo, check_every=64)

    def per_iter(Ws, table):
        # (time of iters iterations - time of iters / 10) / the difference:
        # the per-call work (plan, input scan, FP64 checks) cancels
        sk.set_tile_table(table)
        ctx.scale_batch(Ws, prm_lo)  # warm-up (sizes the arena)

        def run(prm):
            best = float("inf")
            for _ in range(args.repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.scale_batch(Ws, prm)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            return best
        return (run(prm_hi) - run(prm_lo)) / (args.iters - lo)

    report = {}
    # buckets of the batched workload, tuned on the batch
    ns = skgen.sizes_loguniform(512, 32, 1024, 1)
    batch = [torch.from_numpy(skgen.uniform_weights(int(n), 0, 1000, seed=100003 + k)).cuda()
             for k, n in enumerate(ns)]
    small = [b for b in BUCKETS if b <= 1024]
    choice = {b: min(128, b) for b in small}  # the built-in rule's height at these sizes
    for b in small:
        for seg in CANDIDATES:
            if seg > b:
                continue
            trial = {**choice, b: seg}
            t = per_iter(batch, [(k, trial[k]) for k in small])
            report.setdefault(b, {})[seg] = round(t * 1e6, 2)
        choice[b] = min(report[b], key=report[b].get)
        print(json.dumps({"n": b, "on": "batch", "best": choice[b], "us_per_iter": report[b]}), flush=True)
    del batch
    entries = [{"n_max": b, "seg_rows": choice[b], "tuned_on": "batch of 512, n in [32, 1024]",
                "us_per_iter": report[b][choice[b]]} for b in small]
    # larger buckets on one instance of the bucket's largest size
    for n in [b for b in BUCKETS if b > 1024]:
        W = [torch.from_numpy(skgen.uniform_weights(n, 0, 1000, seed=n)).cuda()]
        for seg in CANDIDATES:
            table = [(e["n_max"], e["seg_rows"]) for e in entries] + [(n, seg)]
            report.setdefault(n, {})[seg] = round(per_iter(W, table) * 1e6, 2)
        best = min(report[n], key=report[n].get)
        entries.append({"n_max": n, "seg_rows": best, "tuned_on": f"one instance, n = {n}",
                        "us_per_iter": report[n][best]})
        print(json.dumps({"n": n, "on": "single", "best": best, "us_per_iter": report[n]}), flush=True)
        del W
    sk.set_tile_table([])
    ctx.close()
    with open(args.out, "w") as f:
        json.dump({"arch": "gfx950", "measured": "whole iterations (row sweep, column sweep, "
                   "finalise, end of iteration), best of the repeats",
                   "workload": "int16 w uniform 0..1000, p=32", "entries": entries,
                   "us_per_iter": report}, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
