#!/usr/bin/env python3
"""Snapshot GB/s ingested by the streaming randomized ID on one MI355X.

One step = one pass of the whole method over one synthetic stream resident in
HBM: every snapshot is pushed (borrowed, no copy), sketched, and every update
of Alg. 3 runs (scores, prune/fill, basis copy and Gram, Alg. 4 coefficients,
NA-Hutch++ estimate), ending with the final partial update; the step ends
when the last update's estimate is complete (a device synchronisation), so
the step time is the latency of one pass from its first push to its last
Alg. 8.  `value` = snapshot bytes / step time.

Default workload: the channel-flow-shaped stream (4 fields u, v, w, p on a
192 x 129 x 192 grid: m = 19 021 824 binary32 rows per snapshot, n = 1000
snapshots), l = 300, k = t = 150, bfloat16 sketch, lookahead 1024.  Beside it
the line reports:
* the same passes run back to back (each pass's coefficient phases overlap
  the next pass's sketch: an amortised figure, not the latency of a pass);
* lookaheads 300 and 600 with the device memory they need;
* the binary32 and fp8 sketch forms on the same stream, and the relative
  difference of their reconstructions from the binary32 form's;
* the low-rank binary32 stream (m = 2^20, n = 2000, pushes of 32, l = 200),
  with the sketch's fraction of the FP32 matrix-core peak;
* 64 batched image streams (n = 5000 each) and the ignition-shaped fp8 stream
  (m = 50 012 325, n = 10 000, l = 400), both generated round by round into
  borrowed buffers outside the timed work;
* the oracle timed on the host on a bounded sample.

Prints one JSON line.  `--gpus N` with N > 1 exits: this benchmark runs on
one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "snapshot GB/s ingested (and % HBM roofline) at stated rel. Frobenius error"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(HERE, "profiles", "sketch_bf16_channel_traffic.json")
GRAM_TRAFFIC_FILE = os.path.join(HERE, "profiles", "gram_split_channel_traffic.json")
SKETCH_SOURCES = ("sketch.hip", "rid_internal.h", "omega_table.h")
GRAM_SOURCES = ("update.hip", "capi.hip", "rid_internal.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(files=SKETCH_SOURCES):
    """Hash of the kernel sources a stored traffic figure was measured on."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_2405_16076_amd", "csrc")
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def host_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        libs = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if libs:
            blas = f"{libs[0].get('internal_api')} {libs[0].get('version')}"
    except Exception:
        pass
    return model, blas


def channel_workload(small):
    if small:
        return dict(nx=48, ny=33, nz=48, fields=4, n=300, ell=300, t=150, n_modes=300)
    return dict(nx=192, ny=129, nz=192, fields=4, n=1000, ell=300, t=150, n_modes=300)


def open_stream(m, n_max, ell, t, sketch, seeds, lookahead, k=None):
    import torch
    from paper_2405_16076_amd import OnlineRID, StreamConfig
    cfg = StreamConfig(m=m, ell=ell, k=k or t, t=t, n_max=n_max, dtype=torch.float32, sketch=sketch,
                       omega_seed=seeds[0], select_seed=seeds[1], lookahead=lookahead)
    return OnlineRID(cfg)


# --------------------------------------------------------------------------
# method quality from the stream's Gram matrix A^T A (binary64)
# --------------------------------------------------------------------------

def stream_gram(X, rows_per_chunk=1 << 20):
    """A^T A of the n snapshots X (n x m, binary32 on the GPU), accumulated in
    binary64 over row chunks."""
    import torch
    n, m = X.shape
    G = torch.zeros((n, n), dtype=torch.float64, device=X.device)
    for r0 in range(0, m, rows_per_chunk):
        Y = X[:, r0:r0 + rows_per_chunk].double()
        G += Y @ Y.T
        del Y
    return G


def subset_rel_error(G, S):
    """min over C of ||A - A_S C||_F / ||A||_F from A^T A (G: numpy, binary64;
    the least-squares coefficients on the columns S)."""
    import numpy as np
    S = np.asarray(S, dtype=np.int64)
    GS = G[:, S]
    proj = float(np.sum(GS * np.linalg.lstsq(G[np.ix_(S, S)], GS.T, rcond=None)[0].T))
    tot = float(np.trace(G))
    return math.sqrt(max((tot - proj) / tot, 0.0))


def coeff_rel_error(G, J, P):
    """||A - A_J P||_F / ||A||_F from A^T A for the stream's own J and P."""
    import numpy as np
    J = np.asarray(J)
    occ = np.flatnonzero(J >= 0)
    Jo, Po = J[occ], np.asarray(P, dtype=np.float64)[occ]
    tot = float(np.trace(G))
    cross = float(np.sum(Po * G[Jo]))
    quad = float(np.sum(Po * (G[np.ix_(Jo, Jo)] @ Po)))
    return math.sqrt(max((tot - 2.0 * cross + quad) / tot, 0.0))


def method_quality(G, k, t, J, P, draws=5, seed=7):
    """The stream's ID against the rank-k SVD and random t-column subsets
    (G = A^T A as a numpy binary64 array)."""
    import numpy as np
    ev = np.clip(np.linalg.eigvalsh(G)[::-1], 0.0, None)
    tot = float(ev.sum())
    svd = lambda r: math.sqrt(max(float(ev[r:].sum()) / tot, 0.0))
    rng = np.random.default_rng(seed)
    n = G.shape[0]
    rnd = [subset_rel_error(G, rng.permutation(n)[:t]) for _ in range(draws)]
    J = np.asarray(J)
    return {"svd_rank_k": svd(k), "svd_rank_t": svd(t), "random_t_subset_mean": sum(rnd) / len(rnd),
            "id_basis_best_coefficients": subset_rel_error(G, J[J >= 0]), "id_exact_all_columns": coeff_rel_error(G, J, P)}


def one_pass(s, X, n, push):
    s.reset()
    for j0 in range(0, n, push):
        s.push(X[j0:j0 + push], borrow=True)
    s.finalize()


def timed_passes(s, X, n, push, steps, warmup, tag):
    """`steps` passes, each ended by a device synchronisation; returns ms per
    pass and the library's per-phase profile summed over the timed passes."""
    import torch
    for i in range(warmup):
        one_pass(s, X, n, push)
        torch.cuda.synchronize()
        log(f"  [{tag}] warmup pass {i + 1}/{warmup} done")
    s.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_pass(s, X, n, push)
        torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    prof = s.profile_read()
    s.profile_enable(False)
    log(f"  [{tag}] {steps} passes: {ms:.2f} ms per pass; sketch {prof['sketch_ms'] / steps:.2f} ms, "
        f"reduce {prof['reduce_ms'] / steps:.2f}, main-stream updates {prof['update_ms'] / steps:.2f} "
        f"(Gram {prof['gram_ms'] / steps:.2f}), coefficient phases {prof['coeff_ms'] / steps:.2f}")
    return ms, prof


def back_to_back(s, X, n, push, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_pass(s, X, n, push)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / steps


def sketch_roofline(prof, kernel, traffic=None):
    per_launch = prof["sketch_bytes"] / max(prof["sketch_launches"], 1)
    per_ms = prof["sketch_ms"] / max(prof["sketch_launches"], 1)
    achieved = per_launch / (per_ms / 1000.0) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "bytes_per_launch": per_launch, "ms_per_launch": round(per_ms, 4)}


def stored_traffic(path, sources, small, sketch):
    """Per-launch HBM bytes from a committed counter summary, while the
    kernel sources it was measured on are unchanged (else None)."""
    if small or not os.path.exists(path):
        return None
    try:
        tr = json.load(open(path))
        if tr.get("source_hash") == source_hash(sources) and tr.get("sketch") == sketch:
            return tr.get("bytes_per_launch")
    except Exception:
        return None
    return None


def gram_roofline(prof, kernel, traffic=None):
    """The basis Gram's launches: the algorithmic bytes are the occupied
    columns each launch reads (the method's B_basis; the pool copy of new
    columns is listed apart, as it is not the method's own traffic), over the
    average duration of the update's Gram phase (the Gram kernel and its small
    slab reduction)."""
    n = max(prof.get("gram_launches", 0), 1)
    per_launch = prof["gram_bytes"] / n
    per_ms = prof["gram_ms"] / n
    achieved = per_launch / (per_ms / 1000.0) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "bytes_per_launch": per_launch, "pool_copy_bytes_per_launch": prof["pool_copy_bytes"] / n,
            "ms_per_launch": round(per_ms, 4), "launches_per_pass": None}


SAMPLE_BLOCKS, SAMPLE_WIDTH = 8, 16


def sample_starts(n):
    return [(b * (n - SAMPLE_WIDTH)) // max(SAMPLE_BLOCKS - 1, 1) for b in range(SAMPLE_BLOCKS)]


def sampled_reconstructions(s, n):
    return [s.reconstruct(j0, SAMPLE_WIDTH) for j0 in sample_starts(n)]


def rel_error(R, A):
    import torch
    num = den = 0.0
    for r, a in zip(R, A):
        num += float(torch.sum((r.double() - a.double()) ** 2))
        den += float(torch.sum(a.double() ** 2))
    return math.sqrt(num / den) if den > 0 else 0.0


# --------------------------------------------------------------------------
# the headline: channel stream, bf16, single-pass latency
# --------------------------------------------------------------------------

def channel_bench(args):
    import torch
    import synth
    wl = channel_workload(args.small)
    seeds = (1003, 2003)
    m = wl["fields"] * wl["nx"] * wl["ny"] * wl["nz"]
    n, ell, t = wl["n"], wl["ell"], wl["t"]
    log(f"generating the channel stream m={m} n={n} ({m * n * 4 / 1e9:.1f} GB) on the GPU")
    t0 = time.perf_counter()
    D = synth.channel_torch(wl["nx"], wl["ny"], wl["nz"], n, synth.data_seed(3), fields=wl["fields"],
                            n_modes=wl["n_modes"])
    torch.cuda.synchronize()
    log(f"  generated in {time.perf_counter() - t0:.1f} s")
    X = D[:, :m]
    B_snap = float(m) * n * 4
    push = args.push

    s = open_stream(m, n, ell, t, args.sketch, seeds, 1024)
    ms, prof = timed_passes(s, X, n, push, args.steps, args.warmup, args.sketch)
    ms_b2b = back_to_back(s, X, n, push, max(2, args.steps))
    est = s.error_estimate()
    R_main = sampled_reconstructions(s, n)
    A_smp = [X[j0:j0 + SAMPLE_WIDTH] for j0 in sample_starts(n)]
    exact = rel_error(R_main, A_smp)
    J_main = s.select()
    P_main = s.coefficients()
    dev_bytes = int(s.info().device_bytes)
    s.close()
    log(f"  [{args.sketch}] {ms:.2f} ms per pass, back to back {ms_b2b:.2f}; estimate rel {est['rel']:.4e}, "
        f"exact (sampled) {exact:.4e}")
    traffic = None
    traffic = stored_traffic(TRAFFIC_FILE, SKETCH_SOURCES, args.small, sketch=args.sketch)
    gram_traffic = stored_traffic(GRAM_TRAFFIC_FILE, GRAM_SOURCES, args.small, sketch=args.sketch)
    steps = args.steps
    basis = prof["gram_bytes"] / steps
    line = {
        "metric": METRIC, "value": round(B_snap / (ms / 1000.0) / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.sketch, "data": "synthetic",
        "config": {"workload": f"channel-flow-shaped stream: 4 fields on {wl['nx']}x{wl['ny']}x{wl['nz']} "
                               f"(m={m}) fp32, n={n}, l={ell}, k=t={t}, {args.sketch} sketch, one pass per step "
                               f"(first push to the last update's estimate)",
                   "m": m, "n": n, "ell": ell, "k": t, "t": t, "sketch": args.sketch, "push": push,
                   "lookahead": 1024, "parallelism": "single GPU"},
        "rel_frobenius_error": {"nahutchpp_estimate": est["rel"], "exact_sampled": exact},
        "hbm_frac_whole_step": round((B_snap + basis) / (ms / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
        "bytes_per_pass": {"snapshots": B_snap, "basis_reads": basis,
                           "pool_copy_writes": prof["pool_copy_bytes"] / steps},
        "phase_ms": {k: round(prof[k] / steps, 3) for k in ("sketch_ms", "reduce_ms", "update_ms", "gram_ms",
                                                              "coeff_ms")},
        "amortised_back_to_back": {
            "ms_per_pass": round(ms_b2b, 3), "value": round(B_snap / (ms_b2b / 1000.0) / 1e9, 2),
            "note": "passes enqueued back to back: each pass's coefficient phases run beside the next "
                    "pass's sketch"},
        "device_bytes": dev_bytes,
    }
    # the roofline of the kernel that takes the larger share of the pass; the
    # other one beside it
    rf_sketch = sketch_roofline(prof, f"sketch_{args.sketch}_kernel", traffic)
    rf_gram = gram_roofline(prof, "gram_split_kernel", gram_traffic)
    rf_gram["launches_per_pass"] = round(prof.get("gram_launches", 0) / steps, 2)
    if prof["gram_ms"] > prof["sketch_ms"]:
        line["roofline"], line["roofline_other"] = rf_gram, rf_sketch
    else:
        line["roofline"], line["roofline_other"] = rf_sketch, rf_gram

    # lookahead variants of the same form
    if not args.small and not args.no_lookahead:
        rows = []
        for la in (300, 600):
            s2 = open_stream(m, n, ell, t, args.sketch, seeds, la)
            ms2, _ = timed_passes(s2, X, n, push, 2, 1, f"{args.sketch} lookahead {la}")
            rows.append({"lookahead": la, "ms_per_pass": round(ms2, 3),
                         "value": round(B_snap / (ms2 / 1000.0) / 1e9, 2),
                         "device_bytes": int(s2.info().device_bytes),
                         "borrowed_window_bytes": float(la + push) * m * 4})
            s2.close()
        rows.append({"lookahead": 1024, "ms_per_pass": round(ms, 3), "value": line["value"],
                     "device_bytes": dev_bytes, "borrowed_window_bytes": float(min(n, 1024 + push)) * m * 4})
        line["lookahead"] = rows

    # what the selection is worth: the rank-k SVD and random t-column subsets
    # on the same stream, and a run with k < t (the basis size of Sec. 2.2.2's
    # bound against a smaller target rank)
    if not args.small and not args.no_quality:
        G = stream_gram(X).cpu().numpy()
        q = method_quality(G, t, t, J_main, P_main)
        k2 = t // 3
        s2 = open_stream(m, n, ell, t, args.sketch, seeds, 1024, k=k2)
        one_pass(s2, X, n, push)
        q2 = method_quality(G, k2, t, s2.select(), s2.coefficients())
        s2.close()
        del G
        line["method_quality"] = {"k_eq_t": {"k": t, "t": t, **{a: round(b, 4) for a, b in q.items()}},
                                  "k_lt_t": {"k": k2, "t": t, **{a: round(b, 4) for a, b in q2.items()}},
                                  "note": "relative Frobenius errors over all n columns from A^T A in binary64"}
        log(f"  method quality {line['method_quality']}")

    # the other sketch forms; reconstructions compared with the binary32 form's
    if not args.no_compare:
        forms = ["f32"] + [f for f in ("bf16", "fp8") if f != args.sketch]
        R_ref = None
        for other in forms:
            s2 = open_stream(m, n, ell, t, other, seeds, 1024)
            ms2, prof2 = timed_passes(s2, X, n, push, max(1, min(2, args.steps)), 1, other)
            est2 = s2.error_estimate()
            R2 = sampled_reconstructions(s2, n)
            rf = sketch_roofline(prof2, f"sketch_{other}_kernel")
            entry = {"value": round(B_snap / (ms2 / 1000.0) / 1e9, 2), "ms_per_pass": round(ms2, 3),
                     "sketch_ms_per_launch": rf["ms_per_launch"], "sketch_frac": rf["frac"],
                     "rel_frobenius_error": {"nahutchpp_estimate": est2["rel"], "exact_sampled": rel_error(R2, A_smp)},
                     f"same_J_as_{args.sketch}": bool((s2.select() == J_main).all())}
            if other == "f32":
                R_ref = R2
                flops = 2.0 * ell * m * (prof2["sketch_bytes"] / max(prof2["sketch_launches"], 1)) / (4.0 * m)
                entry["sketch_fp32_mfma_frac"] = round(flops / (rf["ms_per_launch"] / 1000.0) / 1e12 /
                                                       FP32_PEAK_TFLOPS, 4)
                line["rel_frobenius_error"]["recon_vs_f32"] = rel_error(R_main, R_ref)
            else:
                entry["rel_frobenius_error"]["recon_vs_f32"] = rel_error(R2, R_ref)
            line[f"compare_{other}"] = entry
            log(f"  [{other}] {ms2:.2f} ms per pass, estimate {est2['rel']:.4e}, "
                f"exact {entry['rel_frobenius_error']['exact_sampled']:.4e}")
            s2.close()
            del R2
        del R_ref
    del D, X, R_main, A_smp
    torch.cuda.empty_cache()
    return line


# --------------------------------------------------------------------------
# the low-rank binary32 stream (FP32 matrix cores)
# --------------------------------------------------------------------------

def lowrank_bench(steps):
    import torch
    import synth
    m, n, ell, t, push = 1 << 20, 2000, 200, 100, 32
    log(f"generating the low-rank stream m={m} n={n}")
    D = synth.lowrank_torch(m, n, synth.data_seed(2), rank=200, rel_noise=1e-5, decay=10.0)
    torch.cuda.synchronize()
    X = D[:, :m]
    s = open_stream(m, n, ell, t, "f32", (1002, 2002), 0)
    ms, prof = timed_passes(s, X, n, push, steps, 1, "f32 low rank")
    rf = sketch_roofline(prof, "sketch_f32_kernel")
    flops = 2.0 * ell * m * n          # the sketch of one pass
    sk_ms = prof["sketch_ms"] / steps
    est = s.error_estimate()
    exact = rel_error(sampled_reconstructions(s, n), [X[j0:j0 + SAMPLE_WIDTH] for j0 in sample_starts(n)])
    out = {"workload": f"low-rank stream U diag(exp(-i/10)) V^T (rank 200) + 1e-5 relative noise, m={m} fp32, "
                       f"n={n}, pushes of {push}, l={ell}, k=t={t}, f32 sketch, default lookahead",
           "value": round(4.0 * m * n / (ms / 1000.0) / 1e9, 2), "unit": "GB/s", "ms_per_pass": round(ms, 3),
           "sketch_ms_per_pass": round(sk_ms, 3),
           "sketch_fp32_mfma_frac": round(flops / (sk_ms / 1000.0) / 1e12 / FP32_PEAK_TFLOPS, 4),
           "roofline_hbm": rf, "rel_frobenius_error": {"nahutchpp_estimate": est["rel"], "exact_sampled": exact}}
    s.close()
    del D, X
    torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------------------
# 64 batched image streams, n = 5000, frames generated round by round
# --------------------------------------------------------------------------

def batched_bench(n=5000, push=100, lookahead=512, tile="auto"):
    import torch
    import synth
    from paper_2405_16076_amd import StreamBatch, StreamConfig
    shapes = synth.batch_frame_shapes(64, synth.data_seed(4))
    ms_ = [h * w for h, w in shapes]
    slots = (lookahead + push) // push + 2
    log(f"64 image streams, sum m = {sum(ms_)}, n = {n}: rounds of {push} frames into a ring of {slots} rounds")
    ring = [torch.zeros((slots * push, (m + 15) // 16 * 16), dtype=torch.float32, device="cuda:0") for m in ms_]
    cfgs = [StreamConfig(m=m, ell=200, k=100, t=100, n_max=n, dtype=torch.float32, sketch="bf16",
                         omega_seed=1004 + i, select_seed=2004 + i, lookahead=lookahead, tile=tile)
            for i, m in enumerate(ms_)]
    B = StreamBatch(cfgs)
    lib_s = gen_s = 0.0
    rounds = (n + push - 1) // push
    for r in range(rounds):
        c = min(push, n - r * push)
        sl = r % slots
        if r >= slots:
            for mbr in B.members:
                assert mbr.info().release_watermark >= (r - slots + 1) * push
        t0 = time.perf_counter()
        for i, (h, w) in enumerate(shapes):
            synth.blobs_torch(h, w, c, synth.data_seed(4) + 31 * i, t_start=r * push,
                              out=ring[i][sl * push:sl * push + c])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.push([ring[i][sl * push:sl * push + c, :m] for i, m in enumerate(ms_)], borrow=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gen_s += t1 - t0
        lib_s += t2 - t1
        if r % 10 == 0:
            log(f"  [batch] round {r + 1}/{rounds}: library {lib_s:.2f} s, generation {gen_s:.2f} s")
    t1 = time.perf_counter()
    B.finalize()
    torch.cuda.synchronize()
    lib_s += time.perf_counter() - t1
    info = B.info()
    est = sorted(mbr.error_estimate()["rel"] for mbr in B.members)
    B_snap = float(sum(ms_)) * n * 4
    out = {"workload": f"64 image streams (advected Gaussian blobs, m log-uniform in [1e4, 1e6], sum m = {sum(ms_)}),"
                       f" n = {n} each, l = 200, k = t = 100, bf16 sketch, lookahead {lookahead}, rounds of {push} "
                       f"frames generated into borrowed buffers outside the timed library calls",
           "value": round(B_snap / lib_s / 1e9, 2), "unit": "GB/s", "library_s": round(lib_s, 3),
           "generation_s": round(gen_s, 3), "rounds": info["rounds"], "graph_launches": info["graph_launches"],
           "graph_instantiations": info["graph_instantiations"], "graph_updates": info["graph_updates"],
           "slab_rows": info["slab_rows"], "tile": "wide" if info["wide"] else "narrow",
           "tune_table_ms": B.tune_table(),
           "nahutchpp_rel_estimate": {"min": est[0], "median": est[len(est) // 2], "max": est[-1]}}
    B.close()
    del ring
    torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------------------
# the ignition-shaped fp8 stream, generated round by round
# --------------------------------------------------------------------------

def ignition_pass(gen, sketch, n, push, lookahead, ring, seeds, samples):
    """One pass of one form; returns (library seconds, generation seconds,
    stream handle, sampled reconstructions)."""
    import torch
    m = gen.m
    slots = ring.shape[0] // push
    s = open_stream(m, n, 400, 200, sketch, seeds, lookahead)
    lib_s = gen_s = 0.0
    rounds = (n + push - 1) // push
    for r in range(rounds):
        c = min(push, n - r * push)
        sl = r % slots
        if r >= slots and s.info().release_watermark < (r - slots + 1) * push:
            t0 = time.perf_counter()
            s.flush()
            torch.cuda.synchronize()
            lib_s += time.perf_counter() - t0
        assert r < slots or s.info().release_watermark >= (r - slots + 1) * push
        t0 = time.perf_counter()
        gen.generate(r * push, c, ring[sl * push:sl * push + c])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.push(ring[sl * push:sl * push + c, :m], borrow=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gen_s += t1 - t0
        lib_s += t2 - t1
        if r % 10 == 0:
            log(f"  [ignition {sketch}] round {r + 1}/{rounds}: library {lib_s:.2f} s, generation {gen_s:.2f} s")
    t0 = time.perf_counter()
    s.finalize()
    torch.cuda.synchronize()
    lib_s += time.perf_counter() - t0
    R = [s.reconstruct(j, 1) for j in samples]
    return lib_s, gen_s, s, R


def ignition_bench(n=10000, push=200, lookahead=400):
    import torch
    import synth
    nx, ny, nz = 165, 165, 167
    gen = synth.IgnitionStream(nx, ny, nz, n, synth.data_seed(5))
    m = gen.m
    slots = (lookahead + push) // push + 1
    ring = torch.zeros((slots * push, (m + 63) // 64 * 64), dtype=torch.float32, device="cuda:0")
    samples = [0, 1234, 4999, 7777, n - 1]
    log(f"ignition stream m={m} n={n}: rounds of {push} snapshots into a ring of {slots} rounds "
        f"({ring.numel() * 4 / 1e9:.0f} GB)")
    out = {"workload": f"ignition-shaped stream: 10 species + T on {nx}x{ny}x{nz} (m={m}) fp32, n={n}, l=400, "
                       f"k=t=200, fp8 sketch (e4m3, per-block scales) against the f32 form; rounds of {push} "
                       f"snapshots generated into borrowed buffers outside the timed library calls, "
                       f"lookahead {lookahead}"}
    B_snap = float(m) * n * 4
    recon = {}
    for sketch in ("fp8", "f32"):
        lib_s, gen_s, s, R = ignition_pass(gen, sketch, n, push, lookahead, ring, (1005, 2005), samples)
        est = s.error_estimate()
        info = s.info()
        J = s.select()
        s.close()
        recon[sketch] = (R, J)
        out[sketch] = {"value": round(B_snap / lib_s / 1e9, 2), "unit": "GB/s", "library_s": round(lib_s, 3),
                       "generation_s": round(gen_s, 3), "device_bytes": int(info.device_bytes),
                       "nahutchpp_rel_estimate": est["rel"]}
        log(f"  [ignition {sketch}] {B_snap / lib_s / 1e9:.1f} GB/s (library {lib_s:.2f} s)")
    # exact error of the sampled snapshots (regenerated) and fp8 against f32
    A = []
    buf = torch.zeros((1, ring.shape[1]), dtype=torch.float32, device="cuda:0")
    for j in samples:
        gen.generate(j, 1, buf)
        A.append(buf[:, :m].clone())
    for sketch in ("fp8", "f32"):
        out[sketch]["exact_sampled"] = rel_error(recon[sketch][0], A)
    out["fp8"]["recon_vs_f32"] = rel_error(recon["fp8"][0], recon["f32"][0])
    out["fp8"]["same_J_as_f32"] = bool((recon["fp8"][1] == recon["f32"][1]).all())
    out["sketch_reads_per_element"] = 2
    out["note"] = ("l = 400 needs two test-matrix row tiles of the sketch (at most 320 rows per workgroup), so the "
                   "sketch reads each snapshot element twice")
    del ring, A, recon
    torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------------------
# the oracle on the host
# --------------------------------------------------------------------------

def cpu_baseline(wl, seeds, operand, rows=1 << 19, cols=None):
    """The oracle timed on the host on a bounded sample of the same stream."""
    import numpy as np
    import synth
    from oracle.rid import Config, OnlineRID as OracleRID
    cols = cols or wl["t"]
    modes = synth.channel_modes(synth.data_seed(3), n_modes=wl["n_modes"], fields=wl["fields"])
    Bm = synth.channel_spatial_rows(modes, (wl["nx"], wl["ny"], wl["nz"]), 0, np.arange(rows))
    A = (Bm @ synth.channel_temporal(modes, cols)).astype(np.float32)
    cfg = Config(m=rows, ell=wl["ell"], k=wl["t"], t=wl["t"], omega_seed=seeds[0], select_seed=seeds[1],
                 operand=operand)
    o = OracleRID(cfg, n_max=cols)
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    model, blas = host_info()
    t0 = time.perf_counter()
    o.push(A)
    o.finalize()
    dt = time.perf_counter() - t0
    return {"value": A.nbytes / dt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "blas": blas,
            "sample": f"rows 0..{rows} of field u, snapshots 0..{cols} (one full update of the method, "
                      f"{operand} operands, binary64 sums) in {dt:.1f} s on {threads} BLAS threads"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sketch", default="bf16", choices=["bf16", "f32", "fp8"])
    ap.add_argument("--push", type=int, default=100, help="snapshots per push call")
    ap.add_argument("--small", action="store_true", help="a small stream (quick check)")
    ap.add_argument("--no-compare", action="store_true", help="skip the other sketch forms")
    ap.add_argument("--no-lookahead", action="store_true", help="skip the lookahead 300 and 600 passes")
    ap.add_argument("--no-quality", action="store_true", help="skip the SVD / random-subset comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched image streams")
    ap.add_argument("--no-lowrank", action="store_true", help="skip the low-rank binary32 stream")
    ap.add_argument("--no-ignition", action="store_true", help="skip the ignition-shaped fp8 stream")
    ap.add_argument("--only", choices=["batch", "lowrank", "ignition"],
                    help="run one of the extra workloads alone and print its JSON object")
    ap.add_argument("--batch-tile", default="auto", choices=["auto", "narrow", "wide"],
                    help="bf16 work split of the batched streams (auto: the tuner picks)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the stream is row-sharded across GPUs only in the design "
              f"(no multi-GPU path is built); got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_16076_amd import _lib
    _lib.lib()  # fails loudly without the HIP library
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.only == "batch":
        print(json.dumps(batched_bench(tile=args.batch_tile)), flush=True)
        return
    if args.only == "lowrank":
        print(json.dumps(lowrank_bench(max(1, min(3, args.steps)))), flush=True)
        return
    if args.only == "ignition":
        print(json.dumps(ignition_bench()), flush=True)
        return
    line = channel_bench(args)
    if not args.small:
        if not args.no_lowrank:
            line["lowrank_f32"] = lowrank_bench(max(1, min(3, args.steps)))
        if not args.no_batch:
            line["batched"] = batched_bench(tile=args.batch_tile)
        if not args.no_ignition:
            line["ignition_fp8"] = ignition_bench()
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)")
        line["cpu_baseline"] = cpu_baseline(channel_workload(args.small), (1003, 2003), args.sketch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
