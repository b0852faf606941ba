#!/usr/bin/env python3
"""Snapshot GB/s ingested by the streaming randomized ID on one MI355X.

One step = one pass of the whole method over one synthetic stream resident in
HBM: every snapshot is pushed (borrowed, no copy), sketched, and every update
of Alg. 3 runs (scores, prune/fill, basis copy and Gram, Alg. 4 coefficients,
NA-Hutch++ estimate), ending with the final partial update.

Default workload: the channel-flow-shaped stream (4 fields u, v, w, p on a
192 x 129 x 192 grid: m = 19 021 824 binary32 rows per snapshot, n = 1000
snapshots), l = 300, k = t = 150, bfloat16 sketch.  The binary32 and the fp8
(e4m3, block-scaled) sketch forms are measured beside it; every form reports
the relative Frobenius error of its reconstruction (exact on sampled
snapshots, and the NA-Hutch++ estimate).

Prints one JSON line (rank 0).  `--gpus N` with N > 1 exits: this benchmark
runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "snapshot GB/s ingested (and % HBM roofline) at stated rel. Frobenius error"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(HERE, "profiles", "sketch_bf16_channel_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_2405_16076_amd", "csrc")
    for f in ("sketch.hip", "rid_internal.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(small):
    if small:
        return dict(nx=48, ny=33, nz=48, fields=4, n=300, ell=300, t=150, n_modes=300)
    return dict(nx=192, ny=129, nz=192, fields=4, n=1000, ell=300, t=150, n_modes=300)


def run_form(D, m, wl, sketch, steps, warmup, push, seeds):
    import torch
    from paper_2405_16076_amd import OnlineRID, StreamConfig
    n = wl["n"]
    cfg = StreamConfig(m=m, ell=wl["ell"], k=wl["t"], t=wl["t"], n_max=n, dtype=torch.float32, sketch=sketch,
                       omega_seed=seeds[0], select_seed=seeds[1], lookahead=1024)
    s = OnlineRID(cfg)
    X = D[:, :m]

    def step():
        s.reset()
        for j0 in range(0, n, push):
            s.push(X[j0:j0 + push], borrow=True)
        s.finalize()

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"  [{sketch}] warmup step {i + 1}/{warmup} done")
    s.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile_read()
    s.profile_enable(False)
    ms = (t1 - t0) * 1000.0 / steps
    log(f"  [{sketch}] {steps} steps: {ms:.2f} ms/step; sketch {prof['sketch_ms'] / steps:.2f} ms, "
        f"reduce {prof['reduce_ms'] / steps:.2f} ms, updates {prof['update_ms'] / steps:.2f} ms "
        f"(gram {prof['gram_ms'] / steps:.2f} ms); coefficient phases on the second stream "
        f"{prof['coeff_ms'] / steps:.2f} ms (beside the next pass's sketch)")
    return s, ms, prof


def sampled_exact_error(s, D, m, n, blocks=8, width=16):
    """Exact ||A - A_J P||_F / ||A||_F over `blocks` blocks of `width` snapshots."""
    import torch
    num = den = 0.0
    for b in range(blocks):
        j0 = (b * (n - width)) // max(blocks - 1, 1)
        R = s.reconstruct(j0, width)
        A = D[j0:j0 + width, :m]
        num += float(torch.sum((R.double() - A.double()) ** 2))
        den += float(torch.sum(A.double() ** 2))
        del R
    return math.sqrt(num / den)


def cpu_baseline(wl, seeds, operand, rows=1 << 19, cols=None):
    """The oracle timed on the host on a bounded sample of the same stream."""
    import numpy as np
    import synth
    from oracle.rid import Config, OnlineRID as OracleRID
    cols = cols or wl["t"]
    modes = synth.channel_modes(synth.data_seed(3), n_modes=wl["n_modes"], fields=wl["fields"])
    B = synth.channel_spatial_rows(modes, (wl["nx"], wl["ny"], wl["nz"]), 0, np.arange(rows))
    A = (B @ synth.channel_temporal(modes, cols)).astype(np.float32)
    cfg = Config(m=rows, ell=wl["ell"], k=wl["t"], t=wl["t"], omega_seed=seeds[0], select_seed=seeds[1],
                 operand=operand)
    o = OracleRID(cfg, n_max=cols)
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    o.push(A)
    o.finalize()
    dt = time.perf_counter() - t0
    return {"value": A.nbytes / dt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"rows 0..{rows} of field u, snapshots 0..{cols} (one full update of the method, "
                      f"{operand} operands, binary64 sums) in {dt:.1f} s on {threads} BLAS threads"}


def batched_bench(steps, warmup, n=1000, push=100, tile="auto"):
    """64 image streams of uneven m (log-uniform in [1e4, 1e6]), l = 200,
    k = t = 100, bf16 sketch, lookahead 512 (two full 256-column tiles),
    pushed 100 frames per round as one batch (persistent sketch launch,
    batched updates, one graph per round).  n = 1000 of the configuration's 5000 frames per stream keeps the
    stream resident in HBM (49.6 GB)."""
    import torch
    import synth
    from paper_2405_16076_amd import StreamBatch, StreamConfig
    shapes = synth.batch_frame_shapes(64, synth.data_seed(4))
    ms = [h * w for h, w in shapes]
    log(f"generating 64 image streams, sum m = {sum(ms)}, n = {n} ({sum(ms) * n * 4 / 1e9:.1f} GB)")
    X = [synth.blobs_torch(h, w, n, synth.data_seed(4) + 31 * i) for i, (h, w) in enumerate(shapes)]
    torch.cuda.synchronize()
    cfgs = [StreamConfig(m=m, ell=200, k=100, t=100, n_max=n, dtype=torch.float32, sketch="bf16",
                         omega_seed=1004 + i, select_seed=2004 + i, lookahead=512, tile=tile)
            for i, m in enumerate(ms)]
    B = StreamBatch(cfgs)

    def step():
        B.reset()
        for j0 in range(0, n, push):
            B.push([x[j0:j0 + push, :m] for x, m in zip(X, ms)], borrow=True)
        B.finalize()

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"  [batch] warmup step {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1000.0 / steps
    info = B.info()
    tune_table = B.tune_table()
    # one more pass with every launch timed by events (direct launches)
    B.profile_enable(True)
    step()
    prof = B.profile_read()
    B.profile_enable(False)
    B_snap = float(sum(ms)) * n * 4
    per_launch = prof["sketch_bytes"] / max(prof["sketch_launches"], 1)
    per_ms = prof["sketch_ms"] / max(prof["sketch_launches"], 1)
    achieved = per_launch / (per_ms / 1000.0) / 1e9
    est = [mbr.error_estimate()["rel"] for mbr in B.members]
    log(f"  [batch] {steps} steps: {ms_step:.2f} ms/step; timed pass: sketch {prof['sketch_ms']:.2f} ms in "
        f"{prof['sketch_launches']} launches, reduce {prof['reduce_ms']:.2f} ms, updates {prof['update_ms']:.2f} ms")
    out = {
        "workload": f"64 image streams (advected Gaussian blobs, m log-uniform in [1e4, 1e6], sum m = {sum(ms)}), "
                    f"n = {n} each, l = 200, k = t = 100, bf16 sketch, lookahead 512, pushed {push} frames per round",
        "value": round(B_snap / (ms_step / 1000.0) / 1e9, 2), "unit": "GB/s", "ms_per_step": round(ms_step, 3),
        "steps": steps, "warmup": warmup, "rounds_per_step": info["rounds"] // max(1, steps + warmup),
        "graph_launches": info["graph_launches"], "graph_instantiations": info["graph_instantiations"],
        "graph_updates": info["graph_updates"], "slab_rows": info["slab_rows"],
        "tile": "wide" if info["wide"] else "narrow", "tune_ms": round(info["tune_ms"], 2),
        "tune_table_ms": tune_table,
        "timed_pass_ms": {k: round(prof[k], 3) for k in ("sketch_ms", "reduce_ms", "update_ms", "gram_ms")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "sketch_bf16_multi", "bytes_per_launch": per_launch,
                     "ms_per_launch": round(per_ms, 4)},
        "nahutchpp_rel_estimate": {"min": min(est), "median": sorted(est)[len(est) // 2], "max": max(est)},
    }
    B.close()
    del X
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sketch", default="bf16", choices=["bf16", "f32", "fp8"])
    ap.add_argument("--push", type=int, default=100, help="snapshots per push call")
    ap.add_argument("--small", action="store_true", help="a small stream (quick check)")
    ap.add_argument("--no-compare", action="store_true", help="skip the other sketch forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched image-stream measurement")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched image-stream measurement (prints its JSON object)")
    ap.add_argument("--batch-tile", default="auto", choices=["auto", "narrow", "wide"],
                    help="bf16 work split of the batched streams (auto: the tuner picks)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the stream is row-sharded across GPUs only in the design "
              f"(no multi-GPU path is built); got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2405_16076_amd import _lib
    _lib.lib()  # fails loudly without the HIP library
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.batch_only:
        print(json.dumps(batched_bench(args.steps, args.warmup, tile=args.batch_tile)), flush=True)
        return
    wl = workload(args.small)
    seeds = (1003, 2003)
    m = wl["fields"] * wl["nx"] * wl["ny"] * wl["nz"]
    n = wl["n"]
    log(f"generating the channel stream m={m} n={n} ({m * n * 4 / 1e9:.1f} GB) on the GPU")
    t0 = time.perf_counter()
    D = synth.channel_torch(wl["nx"], wl["ny"], wl["nz"], n, synth.data_seed(3), fields=wl["fields"],
                            n_modes=wl["n_modes"])
    torch.cuda.synchronize()
    log(f"  generated in {time.perf_counter() - t0:.1f} s")

    s, ms, prof = run_form(D, m, wl, args.sketch, args.steps, args.warmup, args.push, seeds)
    B_snap = float(m) * n * 4
    value = B_snap / (ms / 1000.0) / 1e9
    est = s.error_estimate()
    exact = sampled_exact_error(s, D, m, n)
    log(f"  [{args.sketch}] estimate rel {est['rel']:.4e}, exact (sampled) rel {exact:.4e}")
    # roofline of the dominant kernel: the sketch contraction reads each
    # snapshot once (m x 4 bytes per column)
    per_launch_bytes = prof["sketch_bytes"] / max(prof["sketch_launches"], 1)
    per_launch_ms = prof["sketch_ms"] / max(prof["sketch_launches"], 1)
    achieved = per_launch_bytes / (per_launch_ms / 1000.0) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tr = json.load(open(TRAFFIC_FILE))
            if tr.get("source_hash") == source_hash() and tr.get("sketch") == args.sketch and not args.small:
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"sketch_{args.sketch}_kernel", "bytes_per_launch": per_launch_bytes,
                "ms_per_launch": round(per_launch_ms, 4)}
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.sketch, "data": "synthetic",
        "config": {"workload": f"channel-flow-shaped stream: 4 fields on {wl['nx']}x{wl['ny']}x{wl['nz']} "
                               f"(m={m}) fp32, n={n}, l={wl['ell']}, k=t={wl['t']}, {args.sketch} sketch",
                   "m": m, "n": n, "ell": wl["ell"], "k": wl["t"], "t": wl["t"], "sketch": args.sketch,
                   "push": args.push, "parallelism": "single GPU"},
        "rel_frobenius_error": {"nahutchpp_estimate": est["rel"], "exact_sampled": exact},
        "hbm_frac_whole_step": round((B_snap + prof["gram_bytes"] / args.steps) / (ms / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
        "phase_ms": {k: round(prof[k] / args.steps, 3) for k in ("sketch_ms", "reduce_ms", "update_ms", "gram_ms",
                                                                  "coeff_ms")},
        "roofline": roofline,
    }
    J_main, P_main = s.select(), None
    s.close()
    for other in ([] if args.no_compare else [f for f in ("f32", "bf16", "fp8") if f != args.sketch]):
        s2, ms2, prof2 = run_form(D, m, wl, other, max(1, min(2, args.steps)), 1, args.push, seeds)
        est2 = s2.error_estimate()
        exact2 = sampled_exact_error(s2, D, m, n)
        pl = prof2["sketch_ms"] / max(prof2["sketch_launches"], 1)
        line[f"compare_{other}"] = {
            "value": round(B_snap / (ms2 / 1000.0) / 1e9, 2), "ms_per_step": round(ms2, 3),
            "sketch_ms_per_launch": round(pl, 4),
            "sketch_frac": round(prof2["sketch_bytes"] / max(prof2["sketch_launches"], 1) / (pl / 1000.0) / 1e9
                                 / HBM_PEAK_GBS, 4),
            "rel_frobenius_error": {"nahutchpp_estimate": est2["rel"], "exact_sampled": exact2},
            f"same_J_as_{args.sketch}": bool((s2.select() == J_main).all())}
        log(f"  [{other}] estimate rel {est2['rel']:.4e}, exact (sampled) rel {exact2:.4e}")
        s2.close()
    del D
    torch.cuda.empty_cache()
    if not args.no_batch and not args.small:
        line["batched"] = batched_bench(max(1, min(3, args.steps)), 1, tile=args.batch_tile)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)")
        line["cpu_baseline"] = cpu_baseline(wl, seeds, args.sketch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
