"""Benchmark: Sinkhorn sweep HBM bandwidth at n = 16384 on one MI355X.

One step = one pass of the whole path over one synthetic instance (n = 16384,
int16 log-weights uniform on 0..1000, seed 0; input resident in HBM before the
timed region), one sk_solve call: continuation over the p ladder 1, 2, 4, 8,
16, 32 (tolerance 1e-5, a fixed per-stage iteration budget), FP64 recheck and
certificate, reduction at t = 1e-4 to CSR, copy of the CSR to the host, exact
solve of the reduced instance, and the gamma decision. phases_ms times the
same path once more in its separate calls.

value = algorithmic sweep bytes of the step (n^2 * element bytes per sweep,
two sweeps per iteration) / wall time of the step, i.e. whole-job throughput of
the scaling phase with everything else of the path counted as overhead.

roofline: the dominant kernel (most total time), its algorithmic bytes per
launch / its average launch duration from HIP events recorded around every
launch on the library's stream during the timed region. `traffic` is the HBM
bytes per launch of that kernel measured with rocprofv3 FETCH_SIZE and
WRITE_SIZE counters (each scaled by what the same counter reads for a plain
1 GiB copy), taken from the committed summary in profiles/ only while the
kernel sources still hash to the value recorded there; otherwise null.

cpu_baseline: the FP64 oracle, as it stands, timed on this host's cores on a
bounded sample of the same workload (median of 5 runs of 2 full iterations at
n = 16384 on every core; median of 5 one-core runs of a 1/16 sample), converted
to the same unit, with the CPU model.

single_pass: the main leg's step through the single-pass iteration (one
matrix read per iteration), with the single-pass kernel's launch duration.

precision: the same workload with int16 W, BF16 K and FP32 K: whole steps,
sweep launch durations and roofline fractions, and the error of each against
the FP64 oracle after a fixed number of iterations from identical potentials.

batched: 512 independent instances, n log-uniform on [32, 1024], weights
uniform 0..1000; sk_scale_batch (one launch per sweep across all instances)
against 512 sequential sk_scale calls with the same parameters (scalings per
second; the number of instances that reached the tolerance is reported).

algorithm1: Algorithm 1 with the paper's defaults (p0 = 100, +50 per round on
the prescaled matrix, eps = t = 1/n, required ratio 2) on real-valued
log-weights at n = 1000: the random matrix (entries uniform on (0, 1]) and
the Euclidean random assignment matrix (2n points uniform in the unit cube,
a_ij = exp(-d), not quantised), through sk_solve_real: gamma, p, iterations,
kept entries beside Table 1's rows (context); and the real-valued sweeps'
launch durations at n = 16384.

dominant: the diagonally dominant 5% pattern at n = 16384 (w_ii uniform
800..1000, off-diagonal entries present with probability 0.05 with values
0..600, the sentinel elsewhere) through sk_solve with the main leg's
parameters: time per solve, sweep rate over the dense-stored int16 matrix
and over the non-zeros only (2 B value + 4 B column index each), and whether
the unique optimum (the identity) is recovered with its exact weight.

served: 1000 Poisson arrivals of distinct planted instances (row permutations
of 32 base instances) with n log-uniform on
[64, 8192], tolerance 1e-5, at offered loads of 0.5, 0.9 and 1.5 times the
FIFO loop's measured capacity; requests through sk_submit/sk_poll (continuous
batching) against a plain FIFO loop that solves one request at a time
(host-to-device copy, scale, prune, exact solve) on the same GPU; solves/s
and p50/p99 latency (completion minus arrival) for both at each load.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Sinkhorn sweep HBM GB/s at n=16384; served solves/s + p99 vs plain loop"
ELEM_BYTES = {"i16": 2, "bf16": 2, "f32": 4}
SWEEP_KERNELS = {"i16": ("row_sweep", "col_sweep", "fused"),
                 "bf16": ("row_sweep_k", "col_sweep_k", "fused"),
                 "f32": ("row_sweep_k", "col_sweep_k", "fused")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--storage", default="i16", choices=sorted(ELEM_BYTES))
    ap.add_argument("--ladder", default="1,2,4,8,16,32")
    ap.add_argument("--cap", type=int, default=60, help="iterations per stage")
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--threshold", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--precision-steps", type=int, default=3)
    ap.add_argument("--no-single-pass", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-algorithm1", action="store_true")
    ap.add_argument("--no-dominant", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--served-requests", type=int, default=1000)
    ap.add_argument("--served-loads", default="0.5,0.9,1.5",
                    help="arrival rates as multiples of the FIFO loop's measured capacity")
    ap.add_argument("--method", default="sinkhorn", choices=["sinkhorn", "newton"],
                    help="scaling iteration of the sweep leg")
    ap.add_argument("--fused", action="store_true",
                    help="single-pass iteration (one matrix read per iteration)")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="only summarise a rocprofv3 kernel-trace CSV: per kernel, all dispatches "
                         "and those longer than 20 us (launches that did work)")
    ap.add_argument("--counter-summary", metavar="CSV",
                    help="only summarise a rocprofv3 --pmc counter CSV: per kernel and counter, the "
                         "mean over full-work dispatches (value at least half the kernel's max)")
    ap.add_argument("--traffic-report", nargs=6,
                    metavar=("KERNEL", "WORKLOAD", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                             "COPY_WRITE_CSV"),
                    help="only write the HBM traffic summary of one kernel from two --pmc runs of "
                         "the benchmark and two of --calibrate-copy")
    ap.add_argument("--traffic-table", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                         "COPY_WRITE_CSV"),
                    help="only print, per kernel instantiation, the HBM bytes per launch (FETCH_SIZE + "
                         "WRITE_SIZE scaled by the copy calibration) over launches that did work")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (the reference "
                         "kernel for scaling HBM byte counters)")
    return ap.parse_args()


def trace_summary(path):
    import csv
    per = {}
    for r in csv.DictReader(open(path)):
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per.setdefault(r["Kernel_Name"].split("(")[0], []).append(d)
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        big = [x for x in v if x > 20000]
        print(f"{k} calls={len(v)} avg_ns={sum(v) / len(v):.0f} calls_over_20us={len(big)} "
              f"avg_over_20us_ns={(sum(big) / len(big) if big else 0):.0f}")


def counter_summary(path):
    """Per kernel instantiation, the mean of every counter over its full-work
    dispatches: those whose SQ_INSTS_VALU (else the first counter) is at
    least half the kernel's largest, so launches that only detected a
    stage's end or skipped a finished instance are left out."""
    import csv
    per = {}
    for r in csv.DictReader(open(path)):
        k = r["Kernel_Name"].split("(")[0]
        d = per.setdefault(k, {}).setdefault(r["Dispatch_Id"], {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    for k, disp in sorted(per.items()):
        names = sorted({c for d in disp.values() for c in d})
        ref = "SQ_INSTS_VALU" if "SQ_INSTS_VALU" in names else names[0]
        hi = max(d.get(ref, 0.0) for d in disp.values())
        full = [d for d in disp.values() if d.get(ref, 0.0) >= 0.5 * hi]
        means = {c: sum(d.get(c, 0.0) for d in full) / len(full) for c in names}
        cells = " ".join(f"{c}={means[c]:.4g}" for c in names)
        print(f"{k} | dispatches={len(disp)} full_work={len(full)} | {cells}")


def source_hash():
    """sha256 over the library's kernel and runtime sources."""
    import hashlib
    d = os.path.join(ROOT, "paper_1104_3830_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def _kernel_key(name):
    """'void sk::k_row_sweep<true>(...)' -> 'sk::k_row_sweep'."""
    import re
    k = name.split("(")[0]
    k = re.sub(r"<[^<>]*>$", "", k)
    return k[5:] if k.startswith("void ") else k


def _counter_means(path, counter):
    import csv
    per = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = _kernel_key(r["Kernel_Name"])
        per.setdefault(k, {}).setdefault(r["Dispatch_Id"], 0.0)
        per[k][r["Dispatch_Id"]] += float(r["Counter_Value"])
    out = {}
    for k, d in per.items():
        v = list(d.values())
        hi = max(v) if v else 0.0
        # full-work dispatches: at least half the kernel's largest (launches
        # that only detected a stage's end read a few MB at most)
        work = [x for x in v if x >= 0.5 * hi]
        out[k] = (sum(work) / len(work) if work else 0.0, len(work), len(v))
    return out


def traffic_report(kernel, workload, fcsv, wcsv, cfcsv, cwcsv):
    copy_kib = (1 << 30) / 1024.0
    cf = _counter_means(cfcsv, "FETCH_SIZE")["__amd_rocclr_copyBuffer"][0]
    cw = _counter_means(cwcsv, "WRITE_SIZE")["__amd_rocclr_copyBuffer"][0]
    fs, ws = copy_kib / cf, copy_kib / cw
    kname = {"finalize": "sk::k_col_finalize"}.get(kernel, "sk::k_" + kernel)
    f = _counter_means(fcsv, "FETCH_SIZE")[kname]
    w = _counter_means(wcsv, "WRITE_SIZE")[kname]
    total = (f[0] * fs + w[0] * ws) * 1024.0
    print(f"kernel: {kernel}")
    print(f"workload: {workload}")
    print(f"source_sha256: {source_hash()}")
    print(f"copy_bytes_read_and_written: {1 << 30}")
    print(f"copy_fetch_kib: {cf:.1f}")
    print(f"copy_write_kib: {cw:.1f}")
    print(f"fetch_scale: {fs:.4f}")
    print(f"write_scale: {ws:.4f}")
    print(f"fetch_kib_per_launch_raw: {f[0]:.1f} (mean over the {f[1]} full-work dispatches of {f[2]})")
    print(f"write_kib_per_launch_raw: {w[0]:.1f} (mean over the {w[1]} full-work dispatches of {w[2]})")
    print(f"bytes_per_launch: {total:.0f}")


def _counter_means_full(path, counter):
    """As _counter_means, keyed by the full kernel name with its template
    arguments (instantiations apart)."""
    import csv
    per = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = r["Kernel_Name"].split("(")[0]
        k = k[5:] if k.startswith("void ") else k
        per.setdefault(k, {}).setdefault(r["Dispatch_Id"], 0.0)
        per[k][r["Dispatch_Id"]] += float(r["Counter_Value"])
    out = {}
    for k, d in per.items():
        v = list(d.values())
        hi = max(v) if v else 0.0
        # full-work dispatches: at least half the kernel's largest (launches
        # that only detected a stage's end read a few MB at most)
        work = [x for x in v if x >= 0.5 * hi]
        out[k] = (sum(work) / len(work) if work else 0.0, len(work), len(v))
    return out


def traffic_table(fcsv, wcsv, cfcsv, cwcsv):
    copy_kib = (1 << 30) / 1024.0
    cf = _counter_means(cfcsv, "FETCH_SIZE")["__amd_rocclr_copyBuffer"][0]
    cw = _counter_means(cwcsv, "WRITE_SIZE")["__amd_rocclr_copyBuffer"][0]
    fs, ws = copy_kib / cf, copy_kib / cw
    f = _counter_means_full(fcsv, "FETCH_SIZE")
    w = _counter_means_full(wcsv, "WRITE_SIZE")
    print(f"source_sha256: {source_hash()}")
    print(f"copy calibration: 1 GiB copy reads {cf:.1f} KiB (fetch x {fs:.4f}), writes {cw:.1f} KiB "
          f"(write x {ws:.4f})")
    print("| kernel | working launches | fetch MB/launch | write MB/launch | HBM MB/launch |")
    print("|---|---|---|---|---|")
    for k in sorted(f, key=lambda k: -f[k][0]):
        fb = f[k][0] * fs * 1024.0
        wb = w.get(k, (0.0, 0, 0))[0] * ws * 1024.0
        print(f"| {k} | {f[k][1]} of {f[k][2]} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {(fb + wb) / 1e6:.1f} |")


def committed_traffic(kernel, storage, n):
    """HBM bytes per launch from profiles/, or None if the sources changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{kernel}_{storage}_n{n}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash():
        return None
    try:
        return int(float(kv["bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def calibrate_copy():
    """A plain copy kernel of known size: 1 GiB read + 1 GiB written per launch."""
    import torch
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes": 1 << 30, "launches": 5, "avg_ms": round(el * 1e3, 3),
                      "gbs_read_plus_write": round(2 * (1 << 30) / el / 1e9, 1)}), flush=True)


def batched_leg(sk, torch, seed=1, cap=500, planted=False):
    """512 ragged instances: one batched scaling run vs 512 sequential runs
    with the same parameters (scaling only: no reduction or exact solve, so
    the rates are scalings per second). Uniform weights on 0..1000 at p = 1
    converge slowly (the oracle needs more than 1e5 iterations for some of
    these instances), so stages stop at the cap; the leg reports how many
    instances reached the tolerance in every stage and the worst FP64
    residual, which are the same for both forms (bitwise equal results).
    planted: the same sizes with a planted optimum (w_i sigma(i) = 1050),
    which every instance scales to the tolerance."""
    import skgen
    ns = skgen.sizes_loguniform(512, 32, 1024, seed)
    gen = ((lambda n, s: skgen.planted(n, s)[0]) if planted
           else (lambda n, s: skgen.uniform_weights(n, 0, 1000, s)))
    Ws = [torch.from_numpy(gen(int(n), seed * 100003 + k)).cuda() for k, n in enumerate(ns)]
    prm = sk.make_params([1, 2, 4, 8, 16, 32], tol=1e-5, max_iters=cap, check_every=32)
    ctx = sk.Context(0)
    # warm-up over the whole batch (2 iterations per stage): the arena is
    # sized and touched before the timed run
    ctx.scale_batch(Ws, sk.make_params([1, 2, 4, 8, 16, 32], tol=1e-5, max_iters=2, check_every=2))
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    res_b = ctx.scale_batch(Ws, prm)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    t0 = time.perf_counter()
    res_s = [ctx.scale(W, prm) for W in Ws]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    same = all(torch.equal(a.potentials, b.potentials) for a, b in zip(res_b, res_s))
    ctx.close()
    elems = int(sum(int(n) * int(n) for n in ns))
    reps = [r.report for r in res_b]
    return {"instances": 512, "n_range": [32, 1024], "matrix_MB": round(elems * 2 / 1e6, 1),
            "weights": "planted (w_i sigma(i) = 1050)" if planted else "uniform 0..1000",
            "tol": 1e-5, "cap_per_stage": cap,
            "instances_reached_tol": int(sum(r["stages_capped"] == 0 for r in reps)),
            "stages_capped_total": int(sum(r["stages_capped"] for r in reps)),
            "max_residual_fp64": float(max(max(r["residual_fp64"], r["col_residual_fp64"])
                                           for r in reps)),
            "batched_scalings_per_s": round(512 / tb, 1),
            "sequential_scalings_per_s": round(512 / ts, 1),
            "speedup": round(ts / tb, 2), "batched_s": round(tb, 3), "sequential_s": round(ts, 3),
            "iters_total": int(sum(r["iters_total"] for r in reps)),
            "iters_max": int(max(r["iters_total"] for r in reps)),
            "identical_to_sequential": bool(same),
            "kernels": {k: {"launches": v[0], "avg_us": round(v[1] / max(v[0], 1) * 1e3, 2)}
                        for k, v in prof.items()}}


def served_leg(sk, torch, n_requests, loads, seed=2):
    """Poisson arrivals; continuous batching vs a FIFO one-at-a-time loop."""
    import skgen
    # 32 planted base instances with log-uniform sizes; request k is a base
    # instance with its rows permuted by a seeded permutation, so every
    # request is a distinct matrix with the known optimum 1050 n
    pool_n = skgen.sizes_loguniform(32, 64, 8192, seed)
    pool = [skgen.planted(int(n), seed * 100003 + k) for k, n in enumerate(pool_n)]
    pick = skgen.bounded(skgen.stream(seed, 99, n_requests), len(pool)).astype(np.int64)
    reqs = []
    for r, k in enumerate(pick):
        base = pool[int(k)][0]
        reqs.append(np.ascontiguousarray(base[skgen.permutation(base.shape[0], seed * 7919 + r)]))
    prm = sk.make_params([1, 2, 4, 8, 16, 32], tol=1e-5, max_iters=2000, check_every=32,
                         threshold=1e-4)
    fifo = sk.Context(0)

    def fifo_one(W):
        # a request arrives as host memory, like sk_submit's input
        return fifo.solve(torch.from_numpy(W).cuda(), prm)

    for W, _ in pool[:4] + [max(pool, key=lambda e: e[0].shape[0])]:
        fifo_one(W)  # warm-up (the largest instance sizes the arena once)
    # FIFO capacity: back-to-back service time over the first 64 requests
    m = min(64, n_requests)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for W in reqs[:m]:
        fifo_one(W)
    torch.cuda.synchronize()
    mu = m / (time.perf_counter() - t0)
    q = lambda v, pc: round(float(np.percentile(np.asarray(v), pc)) * 1e3, 2)

    def run_fifo(arrivals):
        lat, ok = [], 0
        t_start = time.perf_counter()
        for W, a in zip(reqs, arrivals):
            now = time.perf_counter() - t_start
            if now < a:
                time.sleep(a - now)
            out = fifo_one(W)
            ok += out["weight"] == 1050 * W.shape[0]
            lat.append(time.perf_counter() - t_start - a)
        return time.perf_counter() - t_start, lat, ok

    srv = sk.Context(0, arena_bytes=4 << 30)
    t = srv.submit(pool[0][0], prm)  # warm-up request
    while srv.poll(t, pool[0][0].shape[0]) is None:
        time.sleep(0.0005)

    def run_served(arrivals):
        pending = {}
        lat = [None] * n_requests
        ok = 0
        t_start = time.perf_counter()
        nxt = 0
        while nxt < n_requests or pending:
            now = time.perf_counter() - t_start
            while nxt < n_requests and arrivals[nxt] <= now:
                W = reqs[nxt]
                try:
                    pending[srv.submit(W, prm)] = (nxt, W.shape[0])
                except sk.SkError as e:
                    if e.status != sk.SK_EAGAIN:
                        raise
                    break  # queue full: poll, then submit again
                nxt += 1
            # finished requests from the completion queue, then collected
            for tk in srv.completed():
                idx, n = pending.pop(tk)
                r = srv.poll(tk, n)
                lat[idx] = time.perf_counter() - t_start - arrivals[idx]
                ok += r[2] == 1050 * n
            time.sleep(0.0002)
        return time.perf_counter() - t_start, lat, ok

    per_load = []
    for load in loads:
        arrivals = skgen.poisson_arrivals(load * mu, n_requests, seed)
        span_f, lat_f, ok_f = run_fifo(arrivals)
        span_s, lat_s, ok_s = run_served(arrivals)
        per_load.append({
            "load": load, "arrival_rate_per_s": round(load * mu, 2),
            "served": {"solves_per_s": round(n_requests / span_s, 2), "p50_ms": q(lat_s, 50),
                       "p99_ms": q(lat_s, 99), "optimal": int(ok_s)},
            "fifo": {"solves_per_s": round(n_requests / span_f, 2), "p50_ms": q(lat_f, 50),
                     "p99_ms": q(lat_f, 99), "optimal": int(ok_f)},
            "speedup_solves_per_s": round(span_f / span_s, 2)})
    # saturation: every request arrives at time 0 (peak solves/s of each)
    zero = np.zeros(n_requests)
    span_f, _, ok_f = run_fifo(zero)
    span_s, _, ok_s = run_served(zero)
    saturated = {"served_solves_per_s": round(n_requests / span_s, 2),
                 "fifo_solves_per_s": round(n_requests / span_f, 2),
                 "speedup_solves_per_s": round(span_f / span_s, 2),
                 "optimal": [int(ok_s), int(ok_f)]}
    fifo.close()
    srv.close()
    return {"requests": n_requests, "n_range": [64, 8192], "distinct_matrices": n_requests,
            "base_instances": len(pool),
            "fifo_capacity_solves_per_s": round(mu, 2), "loads": per_load,
            "saturated": saturated}


def table1_rows():
    """Table 1 of the paper (Section 5.1) from the committed context fixture:
    {name: (gamma, p, iterations, kept %)}."""
    out = {}
    path = os.path.join(ROOT, "tests", "golden", "table1_sinkhorn.txt")
    for line in open(path):
        parts = line.split()
        if len(parts) == 5 and not line.startswith("#"):
            out[parts[0]] = tuple(float(x) for x in parts[1:])
    return out


def algorithm1_leg(sk, torch, n=1000, seed=0, sweep_n=16384, sweep_iters=20):
    """Algorithm alg:alg1 with the paper's defaults (p0 = 100, +50 per round on
    the prescaled matrix, eps = t = 1/n, required ratio 2) on real-valued
    log-weights at the paper's n = 1000: the random matrix (entries uniform
    on (0, 1]) and the Euclidean random assignment matrix (-d, not
    quantised), through sk_solve_real: gamma, p, iterations, kept entries and
    time per solve, beside Table 1's rand and euclidean rows (another
    machine, MATLAB, other random draws: context only). Also the real-valued
    sweeps at n = sweep_n (float32 W, 4 bytes per element): average launch
    durations over sweep_iters iterations at the prescaled p = 200."""
    import math
    import skgen
    ref = table1_rows()
    ctx = sk.Context(0)
    out = {"n": n, "defaults": "p0=100, +50 per round (prescaled), eps=t=1/n, opt_ratio=2"}
    for name, W in (("rand", skgen.uniform_real(n, seed)), ("euclidean", skgen.euclidean_real(n, seed))):
        Wd = torch.from_numpy(W).cuda()
        prm = sk.paper_params(n)
        ctx.solve_real(Wd, prm)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = ctx.solve_real(Wd, prm)
        el = time.perf_counter() - t0
        r = o["report"]
        g, pp, it, kept = ref[name]
        out[name] = {"gamma": round(math.exp(o["log_gamma"]), 4), "p": r["p_final"],
                     "p_on_W": r["p_final"] * r["p_scale"], "iterations": r["iters_total"],
                     "iters_per_round": r["iters_stage"][:r["stages_evaluated"]],
                     "kept_percent": round(100.0 * o["nnz"] / n / n, 3), "status": o["status"],
                     "ms_per_solve": round(el * 1e3, 2), "weight": o["weight"],
                     "table1": {"gamma": g, "p": int(pp), "iterations": int(it), "kept_percent": kept}}
    W = skgen.uniform_real(sweep_n, seed)
    Wd = torch.from_numpy(W).cuda()
    del W
    prm = sk.make_params([200], tol=0.0, max_iters=sweep_iters, check_every=sweep_iters, prescale=True)
    ctx.scale_real(Wd, prm)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.scale_real(Wd, prm)
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    us = {k: prof[k][1] / prof[k][0] * 1e3 for k in ("row_sweep", "col_sweep") if k in prof}
    bytes_sweep = sweep_n * sweep_n * 4
    out["sweeps"] = {"n": sweep_n, "element_bytes": 4, "iterations": sweep_iters,
                     **{f"{k}_us": round(v, 2) for k, v in us.items()},
                     **{f"{k}_frac": round(bytes_sweep / (v * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                        for k, v in us.items()}}
    return out


def dominant_leg(sk, torch, prm, n=16384, seed=5, solves=8):
    """Diagonally dominant 5% pattern at n = 16384 (sentinel-heavy input)."""
    import skgen
    W = skgen.dominant(n, seed)
    diag = int(np.diag(W).astype(np.int64).sum())
    nz = int(np.count_nonzero(W != skgen.SENTINEL))
    Wd = torch.from_numpy(W).cuda()
    del W
    ctx = sk.Context(0)
    ctx.solve(Wd, prm)  # warm-up
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(solves):
        out = ctx.solve(Wd, prm)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / solves
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    r = out["report"]
    sweeps = 2 * r["iters_total"]
    kern = {k: round(v[1] / max(v[0], 1) * 1e3, 2) for k, v in prof.items()
            if k in ("row_sweep", "col_sweep")}
    return {"n": n, "density": round(nz / n / n, 4), "ms_per_solve": round(el * 1e3, 3),
            "iterations": r["iters_total"],
            "sweep_GBps_dense": round(sweeps * n * n * 2 / el / 1e9, 1),
            "sweep_GBps_nonzeros": round(sweeps * nz * 6 / el / 1e9, 1),
            "sweep_avg_us": kern, "nnz_kept": out["nnz"],
            "optimal": bool(np.array_equal(out["perm"], np.arange(n)) and out["weight"] == diag)}


def large_leg(sk, torch, ladder, cap, tol, threshold, n=32768, seed=0, solves=3):
    """One instance above the LDS limit (n = 32768, w uniform on 0..1000, the
    main leg's parameters): the sweeps read the column entries from the
    packed global buffer. Whole sk_solve steps, the sweeps' average launch
    durations and their fraction of the HBM peak (n^2 * 2 bytes each)."""
    import skgen
    Wd = torch.from_numpy(skgen.uniform_weights(n, 0, 1000, seed=seed)).cuda()
    prm = sk.make_params(ladder, tol=tol, max_iters=cap, check_every=32, threshold=threshold)
    ctx = sk.Context(0)
    ctx.solve(Wd, prm)  # warm-up
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(solves):
        out = ctx.solve(Wd, prm)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / solves
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    del Wd
    r = out["report"]
    kern = {k: round(v[1] / max(v[0], 1) * 1e3, 2) for k, v in prof.items() if k in ("row_sweep", "col_sweep")}
    return {"n": n, "ms_per_step": round(el * 1e3, 3), "iters_per_step": r["iters_total"],
            "stages_capped": r["stages_capped"], "weight": out["weight"],
            "optimal_proved": bool(r["optimal_proved"]), "sweep_avg_us": kern,
            "frac": {k: round(n * n * 2 / (v * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) for k, v in kern.items()},
            "value_GBps": round(2 * r["iters_total"] * n * n * 2 / el / 1e9, 1)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# One repetition of the 1-core sample, run in a child process started with
# OMP_NUM_THREADS=1 (the oracle is OpenMP-parallel over rows and columns): a
# row step over a block of rows and a column step over a block of columns of
# the same instance (handed over in an .npz file), printed as seconds per
# full iteration.
_ONE_CORE = """
import sys, time, numpy as np
sys.path.insert(0, {root!r})
import oracle
d = np.load({path!r})
n, p = {n}, {p}
Br = oracle.log_weights(d["rows"])
Bc = oracle.log_weights(d["cols"])
z = np.zeros(n)
t0 = time.perf_counter()
oracle.row_step(Br, p, z)
oracle.col_step(Bc, p, z)
print((time.perf_counter() - t0) * n / Br.shape[0])
"""


def cpu_baseline(W, B, p, runs=5, iters=2, blk=1024):
    """The oracle's Sinkhorn at the same n and p, timed on the host cores:
    the median of `runs` runs of `iters` full iterations (row step, column
    step, residual) with every core OpenMP gives it, and the median of `runs`
    one-core runs of a 1/16 sample (a row step over `blk` rows and a column
    step over `blk` columns, scaled to a full iteration)."""
    import statistics
    import subprocess
    import tempfile

    import oracle
    n = W.shape[0]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    per_iter = []
    for _ in range(runs):
        t0 = time.perf_counter()
        _, _, m, _ = oracle.sinkhorn(B, p, 0.0, iters)
        per_iter.append((time.perf_counter() - t0) / m)
    med = statistics.median(per_iter)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = []
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "blocks.npz")
        np.savez(path, rows=W[:blk], cols=np.ascontiguousarray(W[:, :blk]))
        code = _ONE_CORE.format(root=ROOT, path=path, n=n, p=p)
        for _ in range(runs):
            r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                               text=True, check=True)
            one.append(float(r.stdout.strip().splitlines()[-1]))
    med1 = statistics.median(one)
    gbs = lambda t: round(2 * n * n * 2 / t / 1e9, 3)
    return {"value": gbs(med), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "runs": runs,
            "sweeps_per_s": round(2 / med, 3),
            "one_core": {"value": gbs(med1), "unit": "GB/s", "sweeps_per_s": round(2 / med1, 4)},
            "sample": f"FP64 oracle Sinkhorn at n={n}, p={p}, w uniform 0..1000: median of {runs} "
                      f"runs of {iters} full iterations (row step, column step, residual) on "
                      f"{threads} threads ({med:.2f} s per iteration); 1 core: median of {runs} "
                      f"runs of a row step over {blk} rows and a column step over {blk} columns, "
                      f"scaled to a full iteration ({med1:.1f} s per iteration); counted at "
                      f"n^2*2 bytes per sweep"}


def single_pass_leg(sk, torch, Wd, ladder, cap, tol, threshold, steps=3):
    """The main leg's step through the single-pass iteration (one read of the
    matrix per iteration instead of two): step time and the single-pass
    kernel's average launch duration against one matrix read, for int16 W
    and for the stored BF16 and FP32 K (whose steps include the absorb pass
    of every stage)."""
    n = int(Wd.shape[0])
    out = {"n": n, "matrix_reads_per_iter": 1}
    ctx = sk.Context(0)
    for st, eb in (("i16", 2), ("bf16", 2), ("f32", 4)):
        prm = sk.make_params(ladder, tol=tol, max_iters=cap, check_every=32, threshold=threshold,
                             fused=True, storage=st)
        ctx.solve(Wd, prm)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        its = 0
        for _ in range(steps):
            o = ctx.solve(Wd, prm)
            its += o["report"]["iters_total"]
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        prof = ctx.profile_read()
        ctx.profile(False)
        us = prof["fused"][1] / prof["fused"][0] * 1e3 if "fused" in prof else None
        leg = {"ms_per_step": round(el * 1e3, 3), "iters_per_step": its // steps,
               "weight": o["weight"], "stages_capped": o["report"]["stages_capped"],
               "kernel_us": round(us, 2) if us else None,
               "frac": round(n * n * eb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if us else None}
        if st == "i16":
            out.update(leg)
        else:
            out[st] = leg
    ctx.close()
    return out


def precision_leg(sk, torch, W, Wd, B, ladder, cap, tol, threshold, p=32, iters=3, steps=3):
    """The n = 16384 workload with the matrix read three ways: int16 W with
    exp recomputed in every sweep, K stored in BF16, K stored in FP32.
    Per storage: whole sk_solve steps (the main leg's parameters) with the
    sweeps' average launch durations and their fraction of the HBM peak; and
    the error against the FP64 oracle at a fixed sweep count: from identical
    potentials (20 int16 iterations at p), `iters` iterations of the storage
    (the first of a stored-K stage is the exact log-domain one, the others
    sweep K) against the oracle's `iters` iterations from the same start,
    as max |log u - log u*| and max |log v - log v*| over all rows and
    columns, and the FP64 residual of the matrix the storage balances."""
    import oracle
    n = W.shape[0]
    ctx = sk.Context(0)
    warm = ctx.scale(Wd, sk.make_params([p], tol=0.0, max_iters=20, check_every=20))
    lu0, lv0 = sk.split_potentials(warm.potentials, n)
    ub_o, vb_o, m, _ = oracle.sinkhorn(B, p, 0.0, iters, lu0 / p, lv0 / p)
    assert m == iters
    out = {"n": n, "p_error": p, "iterations_from_identical_start": iters}
    for storage in ("i16", "bf16", "f32"):
        es = ELEM_BYTES[storage]
        prm = sk.make_params(ladder, tol=tol, max_iters=cap, check_every=32, threshold=threshold,
                             storage=storage)
        ctx.solve(Wd, prm)  # warm-up (sizes the arena)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        its = 0
        for _ in range(steps):
            o = ctx.solve(Wd, prm)
            its += o["report"]["iters_total"]
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        prof = ctx.profile_read()
        ctx.profile(False)
        r = o["report"]
        rk, ck = SWEEP_KERNELS[storage][:2]
        us = {k: prof[k][1] / prof[k][0] * 1e3 for k in (rk, ck) if k in prof}
        res = ctx.scale(Wd, sk.make_params([p], tol=0.0, max_iters=iters, warm_start=True,
                                           storage=storage), potentials=warm.potentials.clone())
        lu, lv = sk.split_potentials(res.potentials, n)
        out[storage] = {
            "ms_per_step": round(el * 1e3, 3), "iters_per_step": its // steps,
            "step_sweep_GBps": round(2 * its / steps * n * n * es / el / 1e9, 1),
            "row_sweep_us": round(us.get(rk, 0.0), 2), "col_sweep_us": round(us.get(ck, 0.0), 2),
            "row_sweep_frac": round(n * n * es / (us[rk] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
            if rk in us else None,
            "col_sweep_frac": round(n * n * es / (us[ck] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
            if ck in us else None,
            "absorbs_per_step": r["absorbs"], "weight": o["weight"],
            "residual_fp64": r["residual_fp64"], "col_residual_fp64": r["col_residual_fp64"],
            "residual_exact_fp64": r["residual_exact_fp64"],
            "max_abs_err_log_u": float(np.abs(lu - p * ub_o).max()),
            "max_abs_err_log_v": float(np.abs(lv - p * vb_o).max()),
        }
    ctx.close()
    return out


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary)
        return
    if args.traffic_report:
        traffic_report(*args.traffic_report)
        return
    if args.traffic_table:
        traffic_table(*args.traffic_table)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1104_3830_amd as sk
    import skgen

    n = args.n
    ladder = [int(x) for x in args.ladder.split(",")]
    W = skgen.uniform_weights(n, 0, 1000, seed=args.seed)
    Wd = torch.from_numpy(W).cuda()
    prm = sk.make_params(ladder, tol=args.tol, max_iters=args.cap, check_every=32,
                         threshold=args.threshold, storage=args.storage, fused=args.fused,
                         method=args.method)
    ctx = sk.Context(0)
    torch.cuda.synchronize()

    def step():
        # the whole path in one library call (sk_solve)
        out = ctx.solve(Wd, prm)
        return out["report"], out["nnz"], out["weight"], out["log_gamma"]

    def phases():
        """One untimed pass through the same path in its separate calls,
        with the time of each (milliseconds)."""
        t = [time.perf_counter()]
        res = ctx.scale(Wd, prm)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        row_ptr, col, w = ctx.prune(Wd, res.potentials, prm)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        rp, cc, ww = row_ptr.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy()
        t.append(time.perf_counter())
        sk.solve_reduced(rp, cc, ww, n)
        t.append(time.perf_counter())
        names = ["scale_and_recheck", "prune", "csr_to_host", "exact_solve_host"]
        return {k: round((t[i + 1] - t[i]) * 1e3, 3) for i, k in enumerate(names)}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    iters = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rep, nnz, weight, lg = step()
        iters += rep["iters_total"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    phase_ms = phases()

    es = ELEM_BYTES[args.storage]
    # matrix reads per iteration: two sweeps, or one single-pass launch
    reads = 1 if args.fused else 2
    sweep_bytes = reads * iters * n * n * es
    value = sweep_bytes / el / 1e9
    # dominant kernel (full-work launches only; launches that only detected
    # convergence or came after the ladder finished are tagged apart)
    full = {k: v for k, v in prof.items() if ":" not in k}
    dom = max(full.items(), key=lambda kv: kv[1][1])
    dom_name, (dom_launches, dom_ms) = dom
    avg_s = dom_ms / dom_launches / 1e3
    # a Newton product with S = [[0, X], [X^T, 0]] reads the matrix twice
    per_launch = (n * n * es if dom_name in SWEEP_KERNELS[args.storage]
                  else 2 * n * n * es if dom_name == "nt_product" else None)
    achieved = per_launch / avg_s / 1e9 if per_launch else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": committed_traffic(dom_name, args.storage, n), "kernel": dom_name,
                "avg_us": round(avg_s * 1e6, 2), "launches": dom_launches}
    kernels = {k: {"launches": v[0], "avg_us": round(v[1] / max(v[0], 1) * 1e3, 2)}
               for k, v in prof.items()}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"i16": "int16->f32", "bf16": "bf16->f32", "f32": "f32"}[args.storage],
        "data": "synthetic",
        "config": {"workload": f"dense n={n}, int16 w uniform 0..1000 (seed {args.seed}), "
                               f"ladder {ladder}, tol {args.tol}, {args.cap} iterations/stage cap, "
                               f"t={args.threshold}, storage {args.storage}"
                               f"{', single-pass iteration' if args.fused else ''}"
                               f"{', Newton scaling' if args.method == 'newton' else ''}; scale+recheck+"
                               f"prune+exact solve per step", "n": n, "storage": args.storage,
                   "fused": bool(args.fused), "method": args.method},
        "iters_per_step": iters // args.steps, "iters_per_s": round(iters / el, 1),
        "matrix_reads_per_iter": reads,
        "stages_capped": rep["stages_capped"],
        "iters_stage": rep["iters_stage"][:len(ladder)],
        "nnz_kept": nnz, "weight": weight, "log_gamma": lg,
        "optimal_proved": bool(rep["optimal_proved"]),
        "residual_fp32": rep["residual_fp32"],
        "residual_fp64": rep["residual_fp64"], "col_residual_fp64": rep["col_residual_fp64"],
        "phases_ms": phase_ms,
        "roofline": roofline, "kernels": kernels,
    }
    ctx.close()
    B = None
    if not (args.no_precision and args.no_cpu_baseline):
        import oracle
        B = oracle.log_weights(W)
    if not args.no_precision:
        out["precision"] = precision_leg(sk, torch, W, Wd, B, ladder, args.cap, args.tol,
                                         args.threshold, steps=args.precision_steps)
    if not args.no_single_pass and not args.fused:
        out["single_pass"] = single_pass_leg(sk, torch, Wd, ladder, args.cap, args.tol, args.threshold,
                                             steps=args.precision_steps)
    del Wd
    if not args.no_batched:
        out["batched"] = batched_leg(sk, torch)
        out["batched_planted"] = batched_leg(sk, torch, planted=True)
    if not args.no_algorithm1:
        out["algorithm1"] = algorithm1_leg(sk, torch)
    if not args.no_dominant:
        out["dominant"] = dominant_leg(sk, torch, prm)
    if not args.no_large:
        out["large"] = large_leg(sk, torch, ladder, args.cap, args.tol, args.threshold)
    if not args.no_served:
        out["served"] = served_leg(sk, torch, args.served_requests,
                                   [float(x) for x in args.served_loads.split(",")])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, B, ladder[-1])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
