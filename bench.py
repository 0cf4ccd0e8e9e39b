#!/usr/bin/env python3
"""Benchmark: iALS++ training epochs on one MI355X.

A step is one epoch of Alg. 3 (recompute yhat, then for every block the user
pass and the item pass) over the ML20M-shaped synthetic matrix (136,000 users x
20,000 items, 10,000,000 observations, d=128, b=64, alpha0=0.1, lambda=0.05).
Inputs are resident in HBM before the timed region starts.

value = nnz*b per second = 2 |S| d / (seconds per epoch): every epoch touches
each observation once per block and side with b coordinates.

Prints ONE JSON line.  The roofline object covers the dominant kernel, timed
live with HIP events on the library's stream during the timed region; the CPU
baseline is the FP64 oracle timed on this host over one full epoch of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "epoch sec + nnz·b/s; p99 fold-in ms vs plain FP32 iALS++ at matched loss"
SEG_LEN = 1024          # rows longer than this are accumulated by the segment kernel
PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0       # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rows_work(lengths, b):
    """Algorithmic FLOPs and bytes of one row-kernel launch: rows of <= SEG_LEN observations are
    accumulated, solved, updated and patched; longer rows are only solved and updated there."""
    import numpy as np
    lengths = np.asarray(lengths, np.int64)
    short = lengths[lengths <= SEG_LEN]
    nnz_s = int(short.sum())
    n = lengths.size
    flops = 2.0 * b * b * nnz_s + 2.0 * b * nnz_s + 2.0 * b * nnz_s + n * (b ** 3 / 3.0 + 2.0 * b * b)
    # bytes: per observation gather b floats + index + yhat read, again gather + index + yhat write in the patch;
    # per row: dense term b floats read, b floats of x read and written
    bytes_ = nnz_s * (2 * (4 * b + 4) + 8) + n * (3 * 4 * b)
    return flops, bytes_


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ml20m_like")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding of the sweep is "
              "a design in DESIGN.md, not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2110_14044_amd import Trainer, binding

    wl = synth.workload(args.workload)
    log(f"[bench] generating {wl.name}: {wl.num_users}x{wl.num_items}, {wl.nnz} obs, d={wl.dim} b={wl.block}")
    t0 = time.time()
    p = synth.make_problem(args.workload)
    log(f"[bench] generated in {time.time() - t0:.1f}s; building the index on the GPU")
    torch.cuda.set_device(0)
    tr = Trainer(p)
    torch.cuda.synchronize()
    st = tr.stats()
    log(f"[bench] index built: long rows user {st['long_rows_user']} item {st['long_rows_item']}, "
        f"segments {st['segments_user']}/{st['segments_item']}, device bytes {st['device_bytes'] / 1e9:.2f} GB")

    for w in range(args.warmup):
        tr.epoch(1)
        torch.cuda.synchronize()
        log(f"[bench] warmup epoch {w + 1}/{args.warmup} done")

    binding.ials_profile_enable(tr.ctx, True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        tr.epoch(1)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof = binding.ials_profile_read(tr.ctx)
    binding.ials_profile_enable(tr.ctx, False)
    log(f"[bench] timed {args.steps} epochs in {t_total:.4f}s")

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
    dom = max(("rows_user", "rows_item"), key=lambda k: kern.get(k, {"ms_per_epoch": 0})["ms_per_epoch"])
    flops, bytes_ = rows_work(lu if dom == "rows_user" else li, p.block)
    avg_s = kern[dom]["avg_ms"] / 1e3
    achieved = flops / avg_s / 1e12
    roofline = {
        "kernel": f"k_sweep_rows ({dom.split('_')[1]} pass): gather + MFMA Hessian + Cholesky + update + yhat patch",
        "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_MFMA, 4), "traffic": None,
        "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": bytes_,
        "avg_launch_ms": kern[dom]["avg_ms"],
        "algorithmic_GBps": round(bytes_ / avg_s / 1e9, 1),
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"[bench] cpu baseline: FP64 oracle, one epoch of {wl.name} on {threads} threads")
        csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
        tc = time.perf_counter()
        oracle.epochs(csr, p.W0, p.H0, p.block, p.alpha0, p.lam, 1)
        t_cpu = time.perf_counter() - tc
        log(f"[bench] oracle epoch {t_cpu:.2f}s")
        cpu = {"value": nnzb / t_cpu, "unit": "nnz·b/s", "cores": threads, "kind": "oracle",
               "sample": f"one full epoch of {wl.name} (from W0, H0; includes the per-epoch loss), "
                         f"{t_cpu:.2f} s", "epoch_s": t_cpu}

    out = {
        "metric": METRIC, "value": value, "unit": "nnz·b/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": epoch_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.num_users} users x {wl.num_items} items, {wl.nnz} observations "
                               f"(y=alpha=1), d={wl.dim}, b={wl.block}, alpha0={wl.alpha0}, lambda={wl.lam}",
                   "epoch_s": epoch_s, "parallelism": "single GPU"},
        "epoch_s": epoch_s, "loss_after": L,
        "roofline": roofline, "cpu_baseline": cpu, "kernels": kern,
    }
    tr.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
