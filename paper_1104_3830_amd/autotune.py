"""Tile-shape autotuner for the column sweep (run on the GPU).

For each size bucket it times the column-sweep kernel with every candidate
segment height on a synthetic instance of the bucket's largest size (int16
weights uniform on 0..1000, a fixed number of iterations at p = 32) and keeps
the fastest. The table is written as JSON next to the library; the binding
loads it at import, so every later process uses the same shapes (the shape is
a function of n only, which keeps results independent of batch mixes).

    python -m paper_1104_3830_amd.autotune [--out PATH] [--iters K]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

BUCKETS = [64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
CANDIDATES = [16, 32, 64, 128, 256, 512, 1024]


def main():
    ap = argparse.ArgumentParser()
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--out", default=os.path.join(here, "tile_table_gfx950.json"))
    ap.add_argument("--iters", type=int, default=20)
    args = ap.parse_args()
    os.environ["SK_NO_TILE_TABLE"] = "1"
    sys.path.insert(0, os.path.dirname(here))
    import torch

    import paper_1104_3830_amd as sk
    import skgen

    ctx = sk.Context(0)
    entries, report = [], {}
    for n in BUCKETS:
        W = torch.from_numpy(skgen.uniform_weights(n, 0, 1000, seed=n)).cuda()
        best = None
        for seg in CANDIDATES:
            if seg > max(16, n):
                continue
            sk.set_tile_table([(n, seg)])
            prm = sk.make_params([32], tol=0.0, max_iters=args.iters, check_every=args.iters)
            ctx.scale(W, prm)  # warm-up
            ctx.profile(True)
            ctx.scale(W, prm)
            prof = ctx.profile_read()
            ctx.profile(False)
            col = prof.get("col_sweep", (1, float("inf")))
            fin = prof.get("finalize", (1, 0.0))
            t = col[1] / max(col[0], 1) + fin[1] / max(fin[0], 1)  # ms per iteration
            report.setdefault(n, {})[seg] = round(t * 1e3, 2)
            if best is None or t < best[1]:
                best = (seg, t)
        entries.append({"n_max": n, "seg_rows": best[0], "us_per_iter": round(best[1] * 1e3, 2)})
        print(json.dumps({"n": n, "best": entries[-1], "us": report[n]}), flush=True)
    sk.set_tile_table([])
    ctx.close()
    with open(args.out, "w") as f:
        json.dump({"arch": "gfx950", "kernel": "col_sweep+finalize",
                   "workload": "int16 w uniform 0..1000, p=32", "entries": entries,
                   "measured_us": report}, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
