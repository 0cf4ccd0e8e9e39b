#!/usr/bin/env python3
"""Benchmark: iALS++ training epochs on one MI355X.

A step is one epoch of Alg. 3 (recompute yhat, then for every block the user
pass and the item pass) over the ML20M-shaped synthetic matrix (136,000 users x
20,000 items, 10,000,000 observations, d=128, b=64, alpha0=0.1, lambda=0.05).
Inputs are resident in HBM before the timed region starts.

value = nnz*b per second = 2 |S| d / (seconds per epoch): every epoch touches
each observation once per block and side with b coordinates.

The timed region replays the captured epoch graph K times.  The roofline
object covers the dominant kernel, timed with HIP events on the library's
stream over K more epochs launched kernel by kernel; the CPU baseline is the
FP64 oracle timed on this host over one full epoch of the same workload.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "epoch sec + nnz·b/s; p99 fold-in ms vs plain FP32 iALS++ at matched loss"
SEG_LEN = 512           # the library's default segment length (rows longer are accumulated in segments)
PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0       # GB/s
SERVE_RATES = (1000, 5000, 20000)  # open-loop Poisson arrival rates, requests per second


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rows_work(lengths, b, trans_fraction, seg_len=SEG_LEN):
    """Algorithmic FLOPs and bytes of one row-kernel launch.  Rows of <= seg_len observations are
    accumulated there (per observation: rank-1 Hessian update 2 b^2, gradient 2 b, prediction dot
    product 2 b, plus 2 b more when the pass moves the cache to a new block); every row is solved
    (LDL^T factorisation b^3/3 + two triangular solves 2 b^2) and updated.  trans_fraction is the
    share of launches that move the cache."""
    import numpy as np
    lengths = np.asarray(lengths, np.int64)
    nnz_s = int(lengths[lengths <= seg_len].sum())
    n = lengths.size
    per_obs_flops = 2.0 * b * b + 4.0 * b + trans_fraction * 2.0 * b
    flops = per_obs_flops * nnz_s + n * (b ** 3 / 3.0 + 2.0 * b * b)
    # bytes: per observation the partner's block (4 b), its id, the cache entry, and for a moving
    # pass the partner's old block and the cache write; per row the dense term and the row's block
    per_obs_bytes = 4 * b + 4 + 4 + trans_fraction * (4 * b + 4)
    bytes_ = nnz_s * per_obs_bytes + n * (4 * b + 2 * 4 * b + trans_fraction * 4 * b)
    return flops, bytes_


def measured_traffic(kernel_family, workload, block, precision):
    """HBM bytes per launch from the committed counter summary, or None if the sweep kernels
    changed since the counters were taken (or the summary is for another kernel or workload)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k_sweep_rows_ml20m_like.txt")
    if not os.path.exists(path):
        return None
    kv = dict(line.strip().split("=", 1) for line in open(path) if "=" in line and not line.startswith("#"))
    src = os.path.join(ROOT, "paper_2110_14044_amd", "csrc", "sweep.hip")
    if (kv.get("kernel"), kv.get("workload"), kv.get("block"), kv.get("precision")) != (
            kernel_family, workload, str(block), precision):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get(
            "sweep_hip_sha256"):
        return None
    return (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) + float(kv["write_kib"]) * float(kv["write_scale"])) * 1024


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


def matched_loss(p, epochs):
    """Plain FP32 form against the bfloat16 form on the same workload at the same b: the FP32
    form runs `epochs` epochs to a final loss L*; the bfloat16 form is timed until its loss is
    within L*(1 + 1e-3).  Epochs are replayed from each context's epoch graph and timed one by
    one (synchronised, launched kernel by kernel so that no graph capture falls inside an
    epoch); the losses are evaluated outside the timed epochs."""
    import torch
    from paper_2110_14044_amd import Trainer, binding
    out = {}
    for name, prec in (("fp32", binding.IALS_PREC_FP32), ("bf16", binding.IALS_PREC_BF16)):
        warm = Trainer(p, precision=prec)  # loads this form's kernels before the timed context
        warm.epoch(1)
        warm.close()
        tr = Trainer(p, precision=prec)
        times, losses = [], []
        for t in range(epochs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tr.epoch(1)
            tr.synchronize()
            times.append(time.perf_counter() - t0)
            losses.append(tr.loss()[0])
        tr.close()
        out[name] = {"epoch_s": times, "loss": losses}
    Lstar = out["fp32"]["loss"][-1]
    bl = out["bf16"]["loss"]
    reach = next((e for e, L in enumerate(bl) if L <= Lstar * (1 + 1e-3)), None)
    t32 = sum(out["fp32"]["epoch_s"])
    res = {"epochs_fp32": epochs, "loss_fp32_final": Lstar,
           "fp32_total_s": t32, "fp32_median_epoch_s": sorted(out["fp32"]["epoch_s"])[epochs // 2],
           "bf16_median_epoch_s": sorted(out["bf16"]["epoch_s"])[epochs // 2],
           "bf16_epochs_to_match": None if reach is None else reach + 1,
           "bf16_time_to_match_s": None if reach is None else sum(out["bf16"]["epoch_s"][:reach + 1]),
           "loss_rel_diff_per_epoch": [abs(a - b) / b for a, b in zip(bl, out["fp32"]["loss"])]}
    if reach is not None:
        res["speedup_at_matched_loss"] = t32 / res["bf16_time_to_match_s"]
    return res


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ml20m_like")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch epochs kernel by kernel")
    ap.add_argument("--block", type=int, default=0, help="block size b (0: the workload's)")
    ap.add_argument("--seg-len", type=int, default=0,
                    help="observations per segment of long rows (0: the library default, 512)")
    ap.add_argument("--deal", choices=("auto", "static", "queue"), default="auto", help="row dealing of the row kernels")
    ap.add_argument("--autotune", action="store_true",
                    help="choose b, row dealing and segment length by measurement first (cached in --tune-cache)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (default: the autotuner's own)")
    ap.add_argument("--precision", choices=("fp32", "bf16"), default="fp32",
                    help="arithmetic of the timed epochs (the bf16 form: bfloat16 Hessian and Gramian products)")
    ap.add_argument("--matched-loss-epochs", type=int, default=16,
                    help="epochs of the FP32 vs BF16 matched-loss comparison (0 = skip)")
    ap.add_argument("--serving", choices=("on", "off", "only"), default="on",
                    help="fold-in serving measurement beside the training epochs")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-warmup", type=int, default=2000)
    ap.add_argument("--rank", choices=("on", "off", "only"), default="on",
                    help="top-100 ranking of every user after training, and the holdout evaluation "
                         "(only: the ranking of the initial embeddings, nothing else)")
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

    import numpy as np
    import torch

    import synth
    from paper_2110_14044_amd import Trainer, binding

    if args.serving == "only":
        print(json.dumps({"serving": serving_bench(args.serve_requests, args.serve_warmup, SERVE_RATES)}))
        return

    wl = synth.workload(args.workload)
    if args.rank == "only":
        torch.cuda.set_device(0)
        p = synth.make_problem(args.workload)
        W = torch.from_numpy(p.W0).cuda()
        H = torch.from_numpy(p.H0).cuda()
        print(json.dumps({"ranking": {"all_users": ranking_bench(W, H)}, "workload": wl.name, "dtype": "f32",
                          "data": "synthetic"}))
        return
    if args.block_sweep:
        blocks = [int(x) for x in args.block_sweep.split(",")]
        torch.cuda.set_device(0)
        p = synth.make_problem(args.workload)
        rows = block_sweep(p, blocks, args.sweep_epochs)
        print(json.dumps({"block_sweep": rows, "workload": wl.name, "d": wl.dim, "dtype": "f32",
                          "data": "synthetic"}))
        return
    log(f"[bench] generating {wl.name}: {wl.num_users}x{wl.num_items}, {wl.nnz} obs, d={wl.dim} b={wl.block}")
    t0 = time.time()
    p = synth.make_problem(args.workload)
    if args.block:
        p.block = args.block
    log(f"[bench] generated in {time.time() - t0:.1f}s; building the index on the GPU")
    torch.cuda.set_device(0)
    prec = binding.IALS_PREC_BF16 if args.precision == "bf16" else binding.IALS_PREC_FP32
    deal, seg_len, tuned = args.deal, args.seg_len, None
    if args.autotune:
        from paper_2110_14044_amd import autotune
        tuned = autotune.tune(p, prec, cache_path=args.tune_cache, log=log)
        p.block, deal, seg_len = tuned["block"], tuned["deal"], tuned["seg_len"]
        log(f"[bench] tuned: b={p.block} deal={deal} seg_len={seg_len} (estimated epoch {tuned['epoch_ms']:.1f} ms)")
    tr = Trainer(p, graph=not args.no_graph, precision=prec, deal=deal, seg_len=seg_len)
    torch.cuda.synchronize()
    st = tr.stats()
    log(f"[bench] index built: long rows user {st['long_rows_user']} item {st['long_rows_item']}, "
        f"segments {st['segments_user']}/{st['segments_item']}, device bytes {st['device_bytes'] / 1e9:.2f} GB")

    for w in range(args.warmup):
        tr.epoch(1)
        torch.cuda.synchronize()
        log(f"[bench] warmup epoch {w + 1}/{args.warmup} done")

    # timed region: K epochs replayed from the captured epoch graph (launch by launch with --no-graph)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        tr.epoch(1)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    log(f"[bench] timed {args.steps} epochs in {t_total:.4f}s ({'graph' if not args.no_graph else 'eager'})")
    # per-kernel times: the same K epochs launch by launch with HIP events around every kernel
    binding.ials_profile_enable(tr.ctx, True)
    torch.cuda.synchronize()
    t_p = time.perf_counter()
    for s in range(args.steps):
        tr.epoch(1)
    torch.cuda.synchronize()
    t_prof = time.perf_counter() - t_p
    prof = binding.ials_profile_read(tr.ctx)
    binding.ials_profile_enable(tr.ctx, False)
    log(f"[bench] profiled {args.steps} epochs in {t_prof:.4f}s")

    L, parts = tr.loss()
    epoch_s = t_total / args.steps
    nnzb = 2.0 * p.nnz * p.dim
    value = nnzb / epoch_s

    # dominant kernel: the larger of the two row kernels per launch-time share
    lu = np.bincount(p.user, minlength=p.num_users)
    li = np.bincount(p.item, minlength=p.num_items)
    kern = {}
    for name, (ms, cnt) in prof.items():
        kern[name] = {"ms_per_epoch": ms / args.steps, "launches": cnt, "avg_ms": ms / max(cnt, 1)}
    # dominant kernel: the row-kernel family with the most time per epoch
    dom = max(("rows_user", "rows_user_move", "rows_item"),
              key=lambda k: kern.get(k, {"ms_per_epoch": 0})["ms_per_epoch"])
    flops, bytes_ = rows_work(li if dom == "rows_item" else lu, p.block, 1.0 if dom.endswith("_move") else 0.0,
                              seg_len or SEG_LEN)
    avg_s = kern[dom]["avg_ms"] / 1e3
    achieved = flops / avg_s / 1e12
    if p.block > 64:
        nt = 8 if p.block <= 128 else 16
        kname = {"rows_user": f"k_rows_big<{nt},false,.> (user pass)",
                 "rows_user_move": f"k_rows_big<{nt},true,.> (user pass that moves the prediction cache)",
                 "rows_item": f"k_rows_big<{nt},false,.> (item pass)"}[dom]
    else:
        kname = {"rows_user": "k_sweep_rows<NT,.,false,.> (user pass)",
                 "rows_user_move": "k_sweep_rows<NT,.,true,.> (user pass that moves the prediction cache)",
                 "rows_item": "k_sweep_rows<NT,.,false,.> (item pass)"}[dom]
    roofline = {
        "kernel": kname + ": gather + MFMA Hessian + blocked LDL^T solve + update",
        "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_MFMA, 4), "traffic": measured_traffic(dom, wl.name, p.block, args.precision),
        "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": bytes_,
        "avg_launch_ms": kern[dom]["avg_ms"],
        "algorithmic_GBps": round(bytes_ / avg_s / 1e9, 1),
    }

    # the Gramian (GEMM on the matrix cores) and the gather kernels, from the same timed epochs
    bcols = ((p.block + 15) // 16) * 16
    gram_flops = 2.0 * p.num_users * p.dim * bcols  # W^T W[:, pi] for an item pass
    dense_flops = 2.0 * p.num_users * p.dim * bcols  # W G^pi for a user pass
    # the epoch-start cache relative to block 0 needs the d - b columns outside the block
    pred_cols = p.dim - min(p.block, p.dim)
    pred_bytes = p.nnz * (4.0 * pred_cols + 8) + 4.0 * p.num_users * pred_cols
    seg_nnz = int(li[li > (seg_len or SEG_LEN)].sum())
    seg_bytes = seg_nnz * (4.0 * p.block + 12)

    def _rate(name, work, scale, peak, unit, what):
        if name not in kern or kern[name]["avg_ms"] <= 0:
            return None
        a = work / (kern[name]["avg_ms"] / 1e3) / scale
        return {"what": what, "achieved": round(a, 2), "peak": peak, "unit": unit, "frac": round(a / peak, 4),
                "avg_launch_ms": kern[name]["avg_ms"]}
    kernel_rates = {
        "gramian_W": _rate("gram_item", gram_flops, 1e12, PEAK_FP32_MFMA, "TFLOP/s",
                           "k_gram_vec + float64 split-K reduction + Dmat: W^T W[:, pi] per item pass"),
        "dense_W": _rate("dense_user", dense_flops, 1e12, PEAK_FP32_MFMA, "TFLOP/s",
                         "k_dense_vec: alpha0 W G^pi + lambda W_pi per user pass"),
        "predict": _rate("predict", pred_bytes, 1e9, PEAK_HBM, "GB/s",
                         "prediction recompute (the cache relative to block 0: the d - b other columns), "
                         "algorithmic bytes (partner columns, id, output per observation; W once); the L2 "
                         "serves repeated partner rows, so frac can exceed what HBM sees"),
        "seg_item": _rate("seg_item", seg_bytes, 1e9, PEAK_HBM, "GB/s",
                          "item long-row segments, algorithmic gather bytes (partner block, id, slot, cache)"),
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
        nblocks = (p.dim + p.block - 1) // p.block
        if nblocks <= 2:
            log(f"[bench] cpu baseline: FP64 oracle, one epoch of {wl.name} on {threads} threads")
            tc = time.perf_counter()
            oracle.epochs(csr, p.W0, p.H0, p.block, p.alpha0, p.lam, 1)
            t_cpu = time.perf_counter() - tc
            sample = f"one full epoch of {wl.name} (from W0, H0; includes the per-epoch loss), {t_cpu:.2f} s"
            work = nnzb
        else:
            # one block of the epoch: predictions, then the user pass and the item pass of block 0
            log(f"[bench] cpu baseline: FP64 oracle, block 0 (both passes) of {wl.name} on {threads} threads")
            import numpy as np
            W = p.W0.astype(np.float64)
            H = p.H0.astype(np.float64)
            tc = time.perf_counter()
            yhat = oracle.predict(csr, W, H)
            bw = min(p.block, p.dim)
            oracle.block_pass(csr, "user", 0, bw, p.alpha0, p.lam, W, H, yhat, oracle.gramian(H, 0, bw))
            oracle.block_pass(csr, "item", 0, bw, p.alpha0, p.lam, W, H, yhat, oracle.gramian(W, 0, bw))
            t_cpu = time.perf_counter() - tc
            sample = (f"block 0 of {nblocks} of {wl.name} at b={p.block} (predictions + user pass + item pass), "
                      f"{t_cpu:.2f} s; value = 2 |S| b / that time")
            work = 2.0 * p.nnz * p.block
        log(f"[bench] oracle sample {t_cpu:.2f}s")
        cpu = {"value": work / t_cpu, "unit": "nnz·b/s", "cores": threads, "kind": "oracle", "sample": sample,
               "seconds": t_cpu}

    ranking = None
    if args.rank == "on":
        log(f"[bench] ranking: top-{RANK_K} of every user")
        ranking = {"all_users": ranking_bench(tr.W, tr.H)}
        log(f"[bench] ranking {ranking['all_users']['ms']:.2f} ms for {p.num_users} users")
    tr.close()
    if args.rank == "on":
        log("[bench] holdout evaluation: 10,000 users held out, fold-in, top-100, Recall/NDCG")
        ranking["holdout"] = holdout_eval(p, args.steps)
        log(f"[bench] holdout {ranking['holdout']}")
    matched = None
    if args.matched_loss_epochs > 0:
        log(f"[bench] matched-loss comparison: fp32 vs bf16, {args.matched_loss_epochs} epochs")
        matched = matched_loss(p, args.matched_loss_epochs)
        log(f"[bench] fp32 median epoch {matched['fp32_median_epoch_s'] * 1e3:.2f} ms, bf16 "
            f"{matched['bf16_median_epoch_s'] * 1e3:.2f} ms; bf16 reaches L* in {matched['bf16_epochs_to_match']} epochs")
    serving = None
    if args.serving == "on":
        serving = serving_bench(args.serve_requests, args.serve_warmup, SERVE_RATES)

    out = {
        "metric": METRIC, "value": value, "unit": "nnz·b/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": epoch_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16" if args.precision == "bf16" else "f32", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.num_users} users x {wl.num_items} items, {wl.nnz} observations "
                               f"(y=alpha=1), d={wl.dim}, b={p.block}, alpha0={wl.alpha0}, lambda={wl.lam}",
                   "epoch_s": epoch_s, "parallelism": "single GPU", "deal": deal, "seg_len": seg_len or SEG_LEN},
        "autotune": tuned,
        "epoch_s": epoch_s, "epoch_s_profiled_eager": t_prof / args.steps, "loss_after": L,
        "roofline": roofline, "kernel_rates": kernel_rates, "cpu_baseline": cpu, "kernels": kern, "bf16_vs_fp32": matched, "serving": serving,
        "ranking": ranking,
    }
    tr.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
