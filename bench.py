#!/usr/bin/env python3
"""Benchmark: iALS++ training epochs on one MI355X.

A step is one epoch of Alg. 3 (recompute yhat, then for every block the user pass and the
item pass).  The headline line is the largest workload one GPU holds: the MSD-shaped
synthetic matrix (571,000 users x 41,000 items, 34,000,000 observations, Zipf(0.9) items),
d = 2048, float32 storage and arithmetic, alpha0 = 0.1, lambda = 0.05, with the block size
b chosen by the autotuner over {32, 64, 128, 256} from timed passes; 8 epochs replayed from
the captured epoch graph.  Inputs are resident in HBM before the timed region starts.

value = nnz*b per second = 2 |S| d / (seconds per epoch): every epoch touches each
observation once per block and side with b coordinates.

Beside it, in the same JSON line:
  * roofline: the dominant kernel of the headline epoch, timed with HIP events on the
    library's stream over the profiled epochs, against its algorithmic work;
  * epoch_roofline: the sum over the epoch's kernels of max(bytes / HBM peak, FLOP / peak)
    over the measured epoch time;
  * cpu_baseline: the FP64 oracle on this host's cores over a bounded sample of the
    headline epoch (full predictions and Gramians, a uniform sample of rows per pass);
  * ml20m_like: the ML20M-shaped matrix (136,000 x 20,000, 10M observations), d = 128,
    b = 64, float32, 16 epochs, with its own roofline and a full oracle epoch;
  * ml20m_like_d1024: the same matrix at d = 1024, b = 128: the plain float32 form against
    the bfloat16 form (bfloat16 Hessian and Gramian products) at matched loss;
  * serving: fold-in requests with continuous batching (p50/p99 latency, solves/s);
  * ranking: top-100 of every user and the holdout evaluation (Recall/NDCG).
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import copy
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "epoch sec + nnz·b/s; p99 fold-in ms vs plain FP32 iALS++ at matched loss"
SEG_LEN = 512           # the library's default segment length (rows longer are accumulated in segments)
PEAK_HBM = 8000.0       # GB/s, MI355X HBM3E
PEAK_MATRIX = {"fp32": 157.3, "bf16": 2500.0}  # TFLOP/s, MI355X dense matrix cores by operand type
PEAK_FP32_VECTOR = 157.3  # TFLOP/s, MI355X float32 vector ALU
SERVE_RATES = (1000, 5000, 20000)  # open-loop Poisson arrival rates, requests per second


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rows_work(lengths, b, seg_len=SEG_LEN):
    """Algorithmic FLOPs and bytes of one row-kernel launch, counted per observation and per row:
    the observations of rows of <= seg_len observations are accumulated there (rank-1 Hessian
    update 2 b^2, gradient and prediction-cache work 4 b; the partner's block b floats, its id,
    and the cache entry read and written); every row is solved (factorisation b^3/3, the two
    triangular solves 2 b^2) and its block, dense term and new block moved."""
    import numpy as np
    lengths = np.asarray(lengths, np.int64)
    nnz_s = int(lengths[lengths <= seg_len].sum())
    n = lengths.size
    flops = (2.0 * b * b + 4.0 * b) * nnz_s + n * (b ** 3 / 3.0 + 2.0 * b * b)
    bytes_ = nnz_s * (4.0 * b + 4 + 8) + n * 12.0 * b
    return flops, bytes_


def epoch_work(p):
    """Algorithmic work of one epoch, kernel family by kernel family: a list of
    (name, flops, bytes, matrix) with matrix True for contractions that run on the matrix cores
    (predictions 2 d FLOP and d floats + id + output per observation; per pass: the Gramian of the
    fixed side 2 N_o d b FLOP over its N_o d floats, the dense term 2 N d b over N d floats + the
    N b result, the gathered Hessian and gradient (2 b^2 + 4 b) per observation over its b floats,
    id and cache entry, the solves b^3/3 + 2 b^2 per row over the row's block read and written)."""
    import numpy as np
    out = []
    S, U, I, d, b = p.nnz, p.num_users, p.num_items, p.dim, p.block
    out.append(("predict", 2.0 * S * d, S * (4.0 * d + 8), False))
    nb = math.ceil(d / b)
    for blk in range(nb):
        bw = min(b, d - blk * b)
        for side, (N, No) in (("user", (U, I)), ("item", (I, U))):
            out.append((f"gram_{side}", 2.0 * No * d * bw, 4.0 * No * d, True))
            out.append((f"dense_{side}", 2.0 * N * d * bw, 4.0 * N * d + 4.0 * N * bw, True))
            out.append((f"hessian_{side}", S * (2.0 * bw * bw + 4.0 * bw), S * (4.0 * bw + 12), True))
            out.append((f"solve_{side}", N * (bw ** 3 / 3.0 + 2.0 * bw * bw), N * 8.0 * bw, False))
    return out


def epoch_floor(p, precision):
    """Sum over the epoch's kernels of max(bytes / HBM peak, FLOP / peak): the time of an epoch
    whose every kernel ran at its own roofline.  Hessian and Gramian products take the matrix
    peak of the precision's operand type; the dense term is float32 in both forms; the solves
    and predictions the float32 vector peak."""
    total = 0.0
    parts = {}
    for name, fl, by, matrix in epoch_work(p):
        if matrix and not name.startswith("dense"):
            peak = PEAK_MATRIX[precision]
        elif matrix:
            peak = PEAK_MATRIX["fp32"]
        else:
            peak = PEAK_FP32_VECTOR
        t = max(by / (PEAK_HBM * 1e9), fl / (peak * 1e12))
        total += t
        key = name.split("_")[0]
        parts[key] = parts.get(key, 0.0) + t
    return total, parts


def traffic_file(kernel_family, workload):
    return os.path.join(ROOT, "profiles", f"traffic_{kernel_family}_{workload}.txt")


def measured_traffic(kernel_family, workload, block, precision, seg_len=SEG_LEN):
    """HBM bytes per launch of a kernel family from the committed counter summary, or None if
    there is none for this workload, block, precision and segment length (which decides the rows
    the kernel takes), or if the kernel's source changed since the counters were taken (its hash
    is stored beside the figures)."""
    path = traffic_file(kernel_family, workload)
    if not os.path.exists(path):
        return None
    # records of key=value lines, separated by blank lines
    records, kv = [], {}
    for line in list(open(path)) + [""]:
        line = line.strip()
        if not line:
            if kv:
                records.append(kv)
            kv = {}
        elif "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k] = v
    for kv in records:
        if (kv.get("kernel"), kv.get("workload"), kv.get("block"), kv.get("precision"), kv.get("seg_len")) != (
                kernel_family, workload, str(block), precision, str(seg_len)):
            continue
        src = os.path.join(ROOT, "paper_2110_14044_amd", "csrc", kv.get("source", "sweep.hip"))
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("source_sha256"):
            return None
        return (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                float(kv["write_kib"]) * float(kv["write_scale"])) * 1024
    return None


def _open_loop(srv, reqs, arrivals, d):
    """Submit request k at its scheduled arrival time (retrying while the server answers BUSY)
    and poll continuously; latency = host time the result is seen - scheduled arrival."""
    import numpy as np
    from paper_2110_14044_amd import binding
    n = len(reqs)
    lat = np.zeros(n)
    hit_busy = np.zeros(n, bool)
    tags = np.zeros(1024, np.uint64)
    rows = np.zeros((1024, d), np.float32)
    st = np.zeros(1024, np.int32)
    i = got = 0
    h = srv.srv
    t0 = time.perf_counter()
    while got < n:
        now = time.perf_counter() - t0
        while i < n and arrivals[i] <= now:
            if binding.ials_server_submit(h, reqs[i], None, i) != binding.IALS_OK:
                hit_busy[i] = True
                break
            i += 1
        k = binding.ials_server_poll_into(h, 0, tags, rows, st)
        if k:
            t = time.perf_counter() - t0
            idx = tags[:k].astype(np.int64)
            lat[idx] = t - arrivals[idx]
            got += k
            if np.any(st[:k] != 0) or not np.all(np.isfinite(rows[:k])):
                raise RuntimeError("a fold-in result failed")
    return lat, time.perf_counter() - t0, int(hit_busy.sum())


def serving_bench(n_req, warm, rates):
    """Fold-in serving: item table 41,000 x 256 (seeded N(0, 0.1/sqrt(d))), b=64, alpha0=0.1,
    lambda=0.05, 3 sweeps per request, request lengths lognormal(3.5, 1.2) clipped to [1, 2000]
    over Zipf(0.9) items, open-loop Poisson arrivals.  Two modes on the same kernel:
    continuous batching (1024 slots, 4 streams) and the per-request path (1 slot, 1 stream:
    every request is its own launch, one at a time)."""
    import numpy as np
    import torch

    import synth
    from paper_2110_14044_amd import FoldinServer
    H = torch.from_numpy(synth.serving_table(2024)).cuda()
    ptr, items = synth.serving_requests(2025, n_req + warm)
    reqs = [np.ascontiguousarray(items[ptr[r]:ptr[r + 1]]) for r in range(n_req + warm)]
    out = {"workload": f"fold-in: H 41000 x 256 fp32 resident, b=64, 3 sweeps, lengths lognormal(3.5,1.2) "
                       f"clipped [1,2000] (mean {float(np.diff(ptr).mean()):.1f}), Zipf(0.9) items; "
                       f"{n_req} requests per rate after {warm} warm-up"}
    for mode, kw in (("batched", dict(max_slots=1024, streams=4)), ("per_request", dict(max_slots=1, streams=1))):
        srv = FoldinServer(H, 64, 0.1, 0.05, passes=3, **kw)
        res = {}
        for rate in rates:
            arr = synth.poisson_arrivals(3000 + rate, n_req + warm, float(rate))
            b0 = srv.stats()["batches"]
            lat, wall, busy = _open_loop(srv, reqs, arr, 256)
            m = lat[warm:] * 1e3
            done = arr[warm:] + lat[warm:]
            res[str(rate)] = {"p50_ms": round(float(np.percentile(m, 50)), 4),
                              "p99_ms": round(float(np.percentile(m, 99)), 4),
                              "mean_ms": round(float(m.mean()), 4),
                              "solves_per_s": round(n_req / float(done.max() - arr[warm]), 1),
                              "busy_retried": busy, "batches": srv.stats()["batches"] - b0}
            log(f"[bench] serving {mode} {rate}/s: p50 {res[str(rate)]['p50_ms']:.3f} ms "
                f"p99 {res[str(rate)]['p99_ms']:.3f} ms, {res[str(rate)]['solves_per_s']:.0f} solves/s, "
                f"{res[str(rate)]['batches']} batches, wall {wall:.1f}s")
        st = srv.stats()
        res["max_batch"] = st["max_batch"]
        srv.close()
        out[mode] = res
    return out


RANK_K = 100
RANK_METRICS = (("recall", 20), ("recall", 50), ("ndcg", 100))


def ranking_bench(W, H, reps=3):
    """Top-100 recommendation for every row of W against H (scoring on the matrix cores, then the
    selection), timed with events on the current stream over `reps` calls after one warm-up."""
    import torch
    from paper_2110_14044_amd import rank_topk
    rank_topk(W, H, RANK_K)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        rank_topk(W, H, RANK_K)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    U, d = W.shape
    I = H.shape[0]
    return {"users": U, "items": I, "d": d, "k": RANK_K, "ms": ms, "users_per_s": U / ms * 1e3,
            "score_tflops": 2.0 * U * I * d / ms / 1e9}


def holdout_eval(p, epochs, n_users=10_000):
    """Sec. 5.1's protocol on the synthetic matrix: train without n_users held-out users, fold
    them in from 80 % of their items, rank every other item and measure Recall@20, Recall@50 and
    NDCG@100 against the other 20 % (a random split: the numbers measure the pipeline, not the
    quality of a model of real data)."""
    import torch
    import synth
    from paper_2110_14044_amd import Trainer, rank_metrics, rank_topk
    split = synth.holdout_split(p, n_users)
    train = split.train
    if train.block > 64:  # the fold-in kernel takes blocks of up to 64 coordinates
        train = dataclasses.replace(train, block=64)
    tr = Trainer(train, graph=True)
    tr.epoch(epochs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Wf = tr.foldin(split.fold_ptr, split.fold_idx, passes=3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ids, _ = rank_topk(Wf, tr.H, RANK_K, split.fold_ptr, split.fold_idx)
    per, means, counts = rank_metrics(ids, split.hold_ptr, split.hold_idx, RANK_METRICS)
    t2 = time.perf_counter()
    tr.close()
    out = {"held_out_users": int(split.users.size), "train_epochs": epochs, "block": train.block,
           "foldin_s": t1 - t0,
           "rank_and_metrics_s": t2 - t1}
    for (name, k), m in zip(RANK_METRICS, means):
        out[f"{name}@{k}"] = float(m)
    return out


def block_sweep(p, blocks, epochs):
    """Epoch time and training loss against the block size b on one workload, every b from the
    same W0, H0 (sec. 5.2.1: b = 1 is iCD, b = d is iALS, the cost per epoch is U-shaped in b
    and the quality barely depends on it).  Per b: one warm-up epoch (which also captures the
    epoch graph), then `epochs` epochs replayed from the graph and timed together; the loss is
    evaluated after the last of them, outside the timed region."""
    import copy
    import torch
    from paper_2110_14044_amd import Trainer
    rows = []
    for b in blocks:
        q = copy.copy(p)
        q.block = b
        tr = Trainer(q, graph=True)
        tr.epoch(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr.epoch(epochs)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / epochs
        L = tr.loss()[0]
        tr.close()
        rows.append({"block": b, "epoch_ms": dt * 1e3, "nnz_b_per_s": 2.0 * p.nnz * p.dim / dt,
                     "loss_after": L, "epochs_trained": epochs + 1})
        log(f"[bench] b={b}: {dt * 1e3:.2f} ms per epoch, loss after {epochs + 1} epochs {L:.6e}")
    ref = rows[-1]["loss_after"]
    for r in rows:
        r["loss_rel_to_last"] = r["loss_after"] / ref - 1.0
    return rows


def kernel_table(prof, steps):
    return {name: {"ms_per_epoch": ms / steps, "launches": cnt, "avg_ms": ms / max(cnt, 1)}
            for name, (ms, cnt) in prof.items() if cnt > 0}


def train_leg(p, prec_name, steps, warmup, deal="auto", seg_len=0, graph=True, prof_steps=None, gram_split=0):
    """Warm-up epochs, then `steps` epochs timed together (replayed from the epoch graph), then
    `prof_steps` epochs launched kernel by kernel with HIP events around every kernel."""
    import torch
    from paper_2110_14044_amd import Trainer, binding
    prec = binding.IALS_PREC_BF16 if prec_name == "bf16" else binding.IALS_PREC_FP32
    prof_steps = steps if prof_steps is None else prof_steps
    tr = Trainer(p, graph=graph, precision=prec, deal=deal, seg_len=seg_len, gram_split=gram_split)
    torch.cuda.synchronize()
    st = tr.stats()
    log(f"[bench] {p.name} b={p.block} {prec_name}: index built, long rows user {st['long_rows_user']} item "
        f"{st['long_rows_item']}, segments {st['segments_user']}/{st['segments_item']}, device bytes "
        f"{st['device_bytes'] / 1e9:.2f} GB")
    for w in range(warmup):
        tr.epoch(1)
        torch.cuda.synchronize()
        log(f"[bench] warm-up epoch {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.epoch(1)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    log(f"[bench] {p.name}: timed {steps} epochs in {t_total:.4f}s ({'graph' if graph else 'eager'})")
    binding.ials_profile_enable(tr.ctx, True)
    for _ in range(prof_steps):
        tr.epoch(1)
    prof = binding.ials_profile_read(tr.ctx)
    binding.ials_profile_enable(tr.ctx, False)
    L, parts = tr.loss()
    res = {"trainer": tr, "epoch_s": t_total / steps, "steps": steps, "warmup": warmup,
           "kernels": kernel_table(prof, prof_steps), "loss_after": L, "epochs_trained": warmup + steps + prof_steps,
           "fallback_rows": tr.stats()["fallback_rows"]}
    return res


ROW_FAMILIES = ("rows_user", "rows_user_move", "rows_item")


def row_kernel_name(fam, p, prec_name):
    bf = "true" if prec_name == "bf16" else "false"
    if p.block == 1:
        return {"rows_user": "k_icd_rows<false> (first user pass)",
                "rows_user_move": "k_icd_rows<true> (user pass that moves the prediction cache)",
                "rows_item": "k_icd_rows<false> (item pass)"}[fam]
    if 64 < p.block <= 128:
        return {"rows_user": f"k_rows_w8<.,false,{bf}> (first user pass)",
                "rows_user_move": f"k_rows_w8<.,true,{bf}> (user pass that moves the prediction cache)",
                "rows_item": f"k_rows_w8<.,false,{bf}> (item pass)"}[fam]
    if p.block > 128:
        return {"rows_user": f"k_rows_big<16,false,{bf}> (first user pass)",
                "rows_user_move": f"k_rows_big<16,true,{bf}> (user pass that moves the prediction cache)",
                "rows_item": f"k_rows_big<16,false,{bf}> (item pass)"}[fam]
    nt = (p.block + 15) // 16
    return {"rows_user": f"k_sweep_rows<{nt},.,false,.,{bf}> (first user pass)",
            "rows_user_move": f"k_sweep_rows<{nt},.,true,.,{bf}> (user pass that moves the prediction cache)",
            "rows_item": f"k_sweep_rows<{nt},.,false,.,{bf}> (item pass)"}[fam]


def rooflines(p, prec_name, kern, seg_len, epoch_s):
    """The dominant row kernel against its roofline, the other kernel families' rates and the
    epoch-level fraction, all from the profiled epochs' HIP-event times."""
    import numpy as np
    lu = np.bincount(p.user, minlength=p.num_users)
    li = np.bincount(p.item, minlength=p.num_items)
    seg = seg_len or SEG_LEN
    dom = max(ROW_FAMILIES, key=lambda k: kern.get(k, {"ms_per_epoch": 0})["ms_per_epoch"])
    flops, bytes_ = rows_work(li if dom == "rows_item" else lu, p.block, seg)
    avg_s = kern[dom]["avg_ms"] / 1e3
    peak_f = PEAK_MATRIX[prec_name]
    t_f, t_b = flops / (peak_f * 1e12), bytes_ / (PEAK_HBM * 1e9)
    if t_f >= t_b:
        bound, achieved, peak, unit = "mfma", flops / avg_s / 1e12, peak_f, "TFLOP/s"
    else:
        bound, achieved, peak, unit = "hbm", bytes_ / avg_s / 1e9, PEAK_HBM, "GB/s"
    roof = {
        "kernel": row_kernel_name(dom, p, prec_name) + ": gather + MFMA Hessian + blocked LDL^T solve + update",
        "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": measured_traffic(dom, p.name, p.block, prec_name, seg),
        "peak_basis": f"{prec_name} operands on the matrix cores" if bound == "mfma" else "HBM3E",
        "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": bytes_,
        "avg_launch_ms": kern[dom]["avg_ms"], "algorithmic_TFLOPs": round(flops / avg_s / 1e12, 2),
        "algorithmic_GBps": round(bytes_ / avg_s / 1e9, 1),
    }
    # the Gramian of the updated side (the larger one, for an item pass when U > I), the dense
    # term and the gathers, from the same profiled epochs
    big_user = p.num_users >= p.num_items
    n_big = max(p.num_users, p.num_items)
    bw = p.block
    gram_fam, dense_fam = ("gram_item", "dense_user") if big_user else ("gram_user", "dense_item")
    gram_flops = 2.0 * n_big * p.dim * bw
    dense_flops = 2.0 * n_big * p.dim * bw
    pred_cols = p.dim - min(p.block, p.dim)
    pred_bytes = p.nnz * (4.0 * pred_cols + 8) + 4.0 * p.num_users * pred_cols
    seg_nnz = int(li[li > seg].sum())
    seg_bytes = seg_nnz * (4.0 * p.block + 12)

    def _rate(name, work, scale, peak, unit, what):
        if name not in kern or kern[name]["avg_ms"] <= 0:
            return None
        a = work / (kern[name]["avg_ms"] / 1e3) / scale
        return {"what": what, "achieved": round(a, 2), "peak": peak, "unit": unit, "frac": round(a / peak, 4),
                "avg_launch_ms": kern[name]["avg_ms"]}
    gram_peak = PEAK_MATRIX[prec_name]
    rates = {
        "gramian": _rate(gram_fam, gram_flops, 1e12, gram_peak, "TFLOP/s",
                         f"Gramian X^T X[:, pi] of the {n_big}-row side ({prec_name} operands) + float64 reduction"),
        "dense": _rate(dense_fam, dense_flops, 1e12, PEAK_MATRIX["fp32"], "TFLOP/s",
                       f"dense term alpha0 X G^pi + lambda X_pi of the {n_big}-row side (float32)"),
        "predict": _rate("predict", pred_bytes, 1e9, PEAK_HBM, "GB/s",
                         "prediction recompute (the cache relative to block 0: the d - b other columns), "
                         "algorithmic bytes; the L2 serves repeated partner rows"),
        "seg_item": _rate("seg_item", seg_bytes, 1e9, PEAK_HBM, "GB/s",
                          "item long-row segments, algorithmic gather bytes (partner block, id, slot, cache)"),
    }
    if rates["seg_item"] is not None:
        # the same launches against the matrix cores: 2b^2 + 4b FLOP per observation (Hessian
        # as the full rank-1 update, gradient and prediction work), and the roofline that binds
        seg_flops = seg_nnz * (2.0 * p.block * p.block + 4.0 * p.block)
        seg_s = kern["seg_item"]["avg_ms"] / 1e3
        mpeak = PEAK_MATRIX[prec_name]
        rates["seg_item"].update({
            "flop_achieved": round(seg_flops / seg_s / 1e12, 2), "flop_peak": mpeak, "flop_unit": "TFLOP/s",
            "flop_frac": round(seg_flops / seg_s / 1e12 / mpeak, 4),
            "bound": "mfma" if seg_flops / (mpeak * 1e12) > seg_bytes / (PEAK_HBM * 1e9) else "hbm"})
    floor_s, parts = epoch_floor(p, prec_name)
    eroof = {"floor_ms": round(floor_s * 1e3, 3), "epoch_ms": round(epoch_s * 1e3, 3),
             "frac": round(floor_s / epoch_s, 4),
             "floor_ms_by_part": {k: round(v * 1e3, 3) for k, v in parts.items()},
             "rule": "sum over kernels of max(algorithmic bytes / 8 TB/s, FLOP / peak): Hessian and Gramian "
                     f"at the {prec_name} matrix peak, dense term at the float32 matrix peak, solves and "
                     "predictions at the float32 vector peak"}
    return roof, rates, eroof


def cpu_baseline_full_epoch(p):
    """The FP64 oracle for one full epoch of the workload on this host."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
    log(f"[bench] cpu baseline: FP64 oracle, one epoch of {p.name} on {threads} threads")
    tc = time.perf_counter()
    oracle.epochs(csr, p.W0, p.H0, p.block, p.alpha0, p.lam, 1)
    t = time.perf_counter() - tc
    return {"value": 2.0 * p.nnz * p.dim / t, "unit": "nnz·b/s", "cores": threads, "kind": "oracle",
            "sample": f"one full epoch of {p.name} from W0, H0 (d={p.dim}, b={p.block}, including the loss): "
                      f"{t:.2f} s", "seconds": t, "epoch_s_estimate": t}


def cpu_baseline_sampled(p, frac=0.05, seed=7):
    """The FP64 oracle on a bounded sample of one epoch: the full prediction recompute, the two
    Gramians of block 0 in full, and the user and item passes of block 0 on a seeded uniform
    sample `frac` of each side's rows (rows are independent within a pass).  The epoch estimate
    is predictions + nblocks x (Gramians + passes / frac)."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
    rng = np.random.default_rng(seed)
    users = np.sort(rng.choice(p.num_users, size=max(1, int(frac * p.num_users)), replace=False)).astype(np.int32)
    items = np.sort(rng.choice(p.num_items, size=max(1, int(frac * p.num_items)), replace=False)).astype(np.int32)
    W = p.W0.astype(np.float64)
    H = p.H0.astype(np.float64)
    bw = min(p.block, p.dim)
    nb = math.ceil(p.dim / p.block)
    log(f"[bench] cpu baseline: FP64 oracle, sampled epoch of {p.name} on {threads} threads")
    t0 = time.perf_counter()
    yhat = oracle.predict(csr, W, H)
    t1 = time.perf_counter()
    GH = oracle.gramian(H, 0, bw)
    t2 = time.perf_counter()
    oracle.pass_rows(csr, "user", users, 0, bw, p.alpha0, p.lam, W, H, yhat, GH)
    t3 = time.perf_counter()
    GW = oracle.gramian(W, 0, bw)
    t4 = time.perf_counter()
    oracle.pass_rows(csr, "item", items, 0, bw, p.alpha0, p.lam, W, H, yhat, GW)
    t5 = time.perf_counter()
    fu = users.size / p.num_users
    fi = items.size / p.num_items
    est = (t1 - t0) + nb * ((t2 - t1) + (t3 - t2) / fu + (t4 - t3) + (t5 - t4) / fi)
    sample = (f"{p.name} d={p.dim} b={p.block}: full prediction recompute {t1 - t0:.2f} s, Gramians of block 0 "
              f"{t2 - t1 + t4 - t3:.2f} s, block-0 passes over {users.size} users and {items.size} items "
              f"({frac:.0%} uniform samples) {t3 - t2 + t5 - t4:.2f} s; epoch estimate = predictions + {nb} x "
              f"(Gramians + passes / sampled fraction) = {est:.1f} s")
    return {"value": 2.0 * p.nnz * p.dim / est, "unit": "nnz·b/s", "cores": threads, "kind": "oracle",
            "sample": sample, "seconds": t5 - t0, "epoch_s_estimate": est}


def matched_loss(p, epochs, deal="auto", seg_len=0, gram_split=0):
    """Plain float32 form against the bfloat16 form on the same workload at the same b.  Each form
    runs `epochs` epochs from W0, H0; L* is the float32 form's loss after the last one.  Each form
    is charged the time of its epochs up to the first whose loss is within L*(1 + 1e-3) (the same
    rule for both).  Epochs are timed one by one (synchronised, launched kernel by kernel so that no
    graph capture falls inside an epoch; one warm-up context per form loads its kernels first);
    the losses are evaluated outside the timed epochs.  Two more epochs per form are profiled
    kernel by kernel."""
    import torch
    from paper_2110_14044_amd import Trainer, binding
    out = {}
    for name, prec in (("fp32", binding.IALS_PREC_FP32), ("bf16", binding.IALS_PREC_BF16)):
        warm = Trainer(p, precision=prec, deal=deal, seg_len=seg_len, gram_split=gram_split)
        warm.epoch(1)
        warm.close()
        tr = Trainer(p, precision=prec, deal=deal, seg_len=seg_len, gram_split=gram_split)
        times, losses = [], []
        for t in range(epochs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tr.epoch(1)
            tr.synchronize()
            times.append(time.perf_counter() - t0)
            losses.append(tr.loss()[0])
        binding.ials_profile_enable(tr.ctx, True)
        tr.epoch(2)
        prof = binding.ials_profile_read(tr.ctx)
        binding.ials_profile_enable(tr.ctx, False)
        tr.close()
        out[name] = {"epoch_s": times, "loss": losses, "kernels": kernel_table(prof, 2)}
        log(f"[bench] {p.name} {name}: median epoch {sorted(times)[epochs // 2] * 1e3:.1f} ms, "
            f"final loss {losses[-1]:.8e}")
    Lstar = out["fp32"]["loss"][-1]
    thr = Lstar * (1 + 1e-3)
    res = {"epochs": epochs, "loss_fp32_final": Lstar, "threshold": thr, "rule": "first epoch with loss <= L*(1+1e-3)"}
    for name in ("fp32", "bf16"):
        ls, ts = out[name]["loss"], out[name]["epoch_s"]
        e = next((k for k, L in enumerate(ls) if L <= thr), None)
        med = sorted(ts)[epochs // 2]
        res[name] = {"median_epoch_s": med, "mean_epoch_s": sum(ts[1:]) / max(len(ts) - 1, 1),
                     "nnz_b_per_s": 2.0 * p.nnz * p.dim / med,
                     "epochs_to_threshold": None if e is None else e + 1,
                     "time_to_threshold_s": None if e is None else sum(ts[:e + 1]),
                     "loss_per_epoch": ls, "epoch_s": ts}
        roof, rates, eroof = rooflines(p, name, out[name]["kernels"], seg_len, med)
        res[name].update({"roofline": roof, "kernel_rates": rates, "epoch_roofline": eroof,
                          "kernels": out[name]["kernels"]})
    res["median_epoch_ratio_fp32_over_bf16"] = res["fp32"]["median_epoch_s"] / res["bf16"]["median_epoch_s"]
    if res["fp32"]["time_to_threshold_s"] and res["bf16"]["time_to_threshold_s"]:
        res["time_to_threshold_ratio_fp32_over_bf16"] = (res["fp32"]["time_to_threshold_s"] /
                                                          res["bf16"]["time_to_threshold_s"])
    res["loss_rel_diff_per_epoch"] = [abs(a - b) / b for a, b in zip(out["bf16"]["loss"], out["fp32"]["loss"])]
    return res


def gramian_rates(p, reps=10):
    """The Gramian of the larger table (eq. 4: X^T X, d x d, and one block slab of eq. 7) in both
    arithmetic forms, timed with HIP events on the library's stream over `reps` calls after a
    warm-up.  The full Gramian is a contraction of 2 N d^2 FLOP over N d floats (matrix-core
    bound at d = 1024); a slab is 2 N d b FLOP over the same floats (HBM bound)."""
    import torch
    from paper_2110_14044_amd import Trainer, binding
    N, d, b = p.num_users, p.dim, p.block
    out = {}
    for name, prec in (("fp32", binding.IALS_PREC_FP32), ("bf16", binding.IALS_PREC_BF16)):
        tr = Trainer(p, precision=prec)
        res = {}
        for what, blk, flops in (("full", -1, 2.0 * N * d * d), ("slab", 0, 2.0 * N * d * b)):
            cols = d if blk < 0 else b
            G = torch.empty((d, cols), dtype=torch.float32, device="cuda")
            binding.ials_gramian(tr.ctx, binding.IALS_MAT_W, blk, G)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                binding.ials_gramian(tr.ctx, binding.IALS_MAT_W, blk, G)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tf = flops / (ms * 1e-3) / 1e12
            gbs = 4.0 * N * d / (ms * 1e-3) / 1e9
            res[what] = {"ms": ms, "TFLOP/s": round(tf, 2), "matrix_peak": PEAK_MATRIX[name],
                         "frac_of_matrix_peak": round(tf / PEAK_MATRIX[name], 4),
                         "GB/s_of_X": round(gbs, 1), "frac_of_hbm": round(gbs / PEAK_HBM, 4)}
        tr.close()
        out[name] = res
        log(f"[bench] Gramian of W ({N} x {d}) {name}: full {res['full']['ms']:.3f} ms "
            f"({res['full']['TFLOP/s']} TFLOP/s), slab {res['slab']['ms']:.3f} ms")
    return out


def secondary_c2(args):
    """ML20M-shaped matrix, d = 128, b = 64, float32: 16 epochs from the epoch graph."""
    import synth
    p = synth.make_problem("ml20m_like")
    leg = train_leg(p, "fp32", 16, 2)
    roof, rates, eroof = rooflines(p, "fp32", leg["kernels"], 0, leg["epoch_s"])
    tr = leg.pop("trainer")
    ranking = None
    if args.rank == "on":
        log(f"[bench] ranking: top-{RANK_K} of every user of {p.name}")
        ranking = {"all_users": ranking_bench(tr.W, tr.H)}
    tr.close()
    if args.rank == "on":
        log("[bench] holdout evaluation: 10,000 users held out, fold-in, top-100, Recall/NDCG")
        ranking["holdout"] = holdout_eval(p, 16)
    out = {"workload": f"{p.name}: {p.num_users} users x {p.num_items} items, {p.nnz} observations (y=alpha=1), "
                       f"d={p.dim}, b={p.block}, alpha0={p.alpha0}, lambda={p.lam}, float32, 16 epochs (graph)",
           "bf16_vs_fp32": matched_loss(p, 16) if args.matched_loss_epochs > 0 else None,
           "epoch_s": leg["epoch_s"], "nnz_b_per_s": 2.0 * p.nnz * p.dim / leg["epoch_s"],
           "loss_after": leg["loss_after"], "epochs_trained": leg["epochs_trained"],
           "roofline": roof, "kernel_rates": rates, "epoch_roofline": eroof, "kernels": leg["kernels"],
           "ranking": ranking}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_full_epoch(p)
    return out


def secondary_c3(args):
    """ML20M-shaped matrix at d = 1024, b = 128: float32 against bfloat16 at matched loss."""
    import synth
    p = synth.make_problem("ml20m_like_d1024")
    res = matched_loss(p, args.matched_loss_epochs)
    res["gramian"] = gramian_rates(p)
    res["workload"] = (f"{p.name}: {p.num_users} users x {p.num_items} items, {p.nnz} observations, d={p.dim}, "
                       f"b={p.block}, alpha0={p.alpha0}, lambda={p.lam}; float32 vs bfloat16 Hessian/Gramian "
                       f"products, {args.matched_loss_epochs} epochs each")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8, help="timed epochs of the headline workload")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="msd_like", help="headline workload (synth.WORKLOADS)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch epochs kernel by kernel")
    ap.add_argument("--block", type=int, default=0, help="block size b (0: the autotuner's, or the workload's "
                                                          "with --no-autotune)")
    ap.add_argument("--no-autotune", action="store_true", help="use the workload's b instead of the autotuner's")
    ap.add_argument("--seg-len", type=int, default=0,
                    help="observations per segment of long rows (0: the library default, 512)")
    ap.add_argument("--deal", choices=("auto", "static", "queue"), default="auto", help="row dealing of the row kernels")
    ap.add_argument("--gram-split", type=int, default=0,
                    help="workgroups the Gramian slab's split-K is sized for (0: the library's 512 or the autotuner's)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (default: the autotuner's own)")
    ap.add_argument("--precision", choices=("fp32", "bf16"), default="fp32",
                    help="arithmetic of the headline epochs (bf16: bfloat16 Hessian and Gramian products)")
    ap.add_argument("--secondary", choices=("on", "off"), default="on",
                    help="the ML20M-shaped lines (d = 128 and the d = 1024 precision comparison)")
    ap.add_argument("--matched-loss-epochs", type=int, default=16,
                    help="epochs per form of the float32 vs bfloat16 comparison at d = 1024 (0 = skip)")
    ap.add_argument("--serving", choices=("on", "off", "only"), default="on",
                    help="fold-in serving measurement beside the training epochs")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-warmup", type=int, default=2000)
    ap.add_argument("--rank", choices=("on", "off", "only"), default="on",
                    help="top-100 ranking of every user after the d = 128 training, and the holdout evaluation "
                         "(only: the ranking of the initial embeddings of --workload, nothing else)")
    ap.add_argument("--block-sweep", default="",
                    help="comma-separated block sizes: report epoch time and loss per b on --workload, then exit")
    ap.add_argument("--sweep-epochs", type=int, default=4, help="timed epochs per block size of --block-sweep")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = 256 * 2 ** 20
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "dispatches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the sharding of the sweep over several "
              "GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth

    if args.serving == "only":
        print(json.dumps({"serving": serving_bench(args.serve_requests, args.serve_warmup, SERVE_RATES)}))
        return
    wl = synth.workload(args.workload)
    torch.cuda.set_device(0)
    if args.rank == "only":
        p = synth.make_problem(args.workload)
        W = torch.from_numpy(p.W0).cuda()
        H = torch.from_numpy(p.H0).cuda()
        print(json.dumps({"ranking": {"all_users": ranking_bench(W, H)}, "workload": wl.name, "dtype": "f32",
                          "data": "synthetic"}))
        return
    if args.block_sweep:
        blocks = [int(x) for x in args.block_sweep.split(",")]
        p = synth.make_problem(args.workload)
        rows = block_sweep(p, blocks, args.sweep_epochs)
        print(json.dumps({"block_sweep": rows, "workload": wl.name, "d": wl.dim, "dtype": "f32",
                          "data": "synthetic"}))
        return

    # ---- headline: the largest workload, b from the autotuner ----
    log(f"[bench] generating {wl.name}: {wl.num_users}x{wl.num_items}, {wl.nnz} obs, d={wl.dim}")
    t0 = time.time()
    p = synth.make_problem(args.workload)
    log(f"[bench] generated in {time.time() - t0:.1f}s")
    deal, seg_len, gram_split, tuned = args.deal, args.seg_len, args.gram_split, None
    if args.block:
        p.block = args.block
    elif not args.no_autotune:
        from paper_2110_14044_amd import autotune, binding
        prec = binding.IALS_PREC_BF16 if args.precision == "bf16" else binding.IALS_PREC_FP32
        t0 = time.time()
        tuned = autotune.tune(p, prec, cache_path=args.tune_cache, log=log)
        p.block, deal, seg_len, gram_split = tuned["block"], tuned["deal"], tuned["seg_len"], tuned["gram_split"]
        tuned = {k: v for k, v in tuned.items() if k != "trials"} | {
            "trials": [{k: t[k] for k in ("block", "deal", "seg_len", "gram_split", "epoch_ms")}
                       for t in tuned["trials"]],
            "tune_s": round(time.time() - t0, 1)}
        log(f"[bench] tuned: b={p.block} deal={deal} seg_len={seg_len} gram_split={gram_split} "
            f"(estimated epoch {tuned['epoch_ms']:.1f} ms)")
    leg = train_leg(p, args.precision, args.steps, args.warmup, deal=deal, seg_len=seg_len, gram_split=gram_split,
                    graph=not args.no_graph)
    leg.pop("trainer").close()
    epoch_s = leg["epoch_s"]
    value = 2.0 * p.nnz * p.dim / epoch_s
    roof, rates, eroof = rooflines(p, args.precision, leg["kernels"], seg_len, epoch_s)
    b_used = p.block
    matched = None
    if args.matched_loss_epochs > 0 and args.precision == "fp32":
        log(f"[bench] {p.name}: float32 vs bfloat16 at matched loss, {args.steps} epochs")
        matched = matched_loss(p, args.steps, deal=deal, seg_len=seg_len, gram_split=gram_split)
        for k in ("fp32", "bf16"):
            for drop in ("kernels", "kernel_rates"):
                matched[k].pop(drop, None)
    cpu = None
    if not args.no_cpu_baseline:
        nb = math.ceil(p.dim / p.block)
        cpu = cpu_baseline_full_epoch(p) if nb <= 2 and p.nnz <= 20_000_000 else cpu_baseline_sampled(p)
        log(f"[bench] cpu baseline {cpu['sample']}")
    del p

    secondary = {}
    if args.secondary == "on":
        log("[bench] ML20M-shaped d=128 line")
        secondary["ml20m_like"] = secondary_c2(args)
        if args.matched_loss_epochs > 0:
            log("[bench] ML20M-shaped d=1024: float32 vs bfloat16 at matched loss")
            secondary["ml20m_like_d1024"] = secondary_c3(args)
    serving = None
    if args.serving == "on":
        serving = serving_bench(args.serve_requests, args.serve_warmup, SERVE_RATES)

    out = {
        "metric": METRIC, "value": value, "unit": "nnz·b/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": epoch_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16" if args.precision == "bf16" else "f32", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.num_users} users x {wl.num_items} items, {wl.nnz} observations "
                               f"(y=alpha=1, Zipf({wl.zipf_s}) items), d={wl.dim}, b={b_used} "
                               f"({'autotuned over 32/64/128/256' if tuned else 'fixed'}), alpha0={wl.alpha0}, "
                               f"lambda={wl.lam}, {args.precision} arithmetic",
                   "epoch_s": epoch_s, "parallelism": "single GPU", "deal": deal, "seg_len": seg_len or SEG_LEN,
                   "gram_split": gram_split or 512,
                   "graph": not args.no_graph},
        "autotune": tuned,
        "epoch_s": epoch_s, "loss_after": leg["loss_after"], "epochs_trained": leg["epochs_trained"],
        "roofline": roof, "epoch_roofline": eroof, "kernel_rates": rates, "cpu_baseline": cpu,
        "bf16_vs_fp32": matched,
        "kernels": leg["kernels"], **secondary, "serving": serving,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
