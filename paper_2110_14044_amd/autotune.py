"""Block-size and launch autotuner.

The paper measures the epoch time of iALS++ as a U-shaped function of the block
size b whose minimum is a hardware-dependent constant (sec. 5.2.1): a small b
re-reads the updated side's rows once per block, a large b pays b^2 per
observation for the Hessian and b^3 per row for the solve.  On the GPU the shape
of that curve also depends on which kernels serve the block (one wavefront per row
up to b = 64, one workgroup per row above) and on how rows are dealt.  The tuner
measures instead of assuming: for every candidate it builds a context over the
same observations, runs real passes and times them with the library's HIP-event
hooks, and estimates the epoch as

    predictions + (user pass + item pass) of the first block
                + (nb - 1) x (user pass that moves the prediction cache + item pass)

Then, at the best b, it tries the other row dealing, the other segment lengths
(the split-K of long rows) and the split-K of the per-pass Gramian slab (how many
workgroups its row chunks are sized for).  A different b is a different trajectory of the iteration (the blocks
are different coordinate subspaces), so results must be checked against the
oracle at the chosen b.  Results are cached in a JSON file keyed by the problem
shape, the arithmetic and the device.
"""
from __future__ import annotations

import copy
import json
import math
import os

from . import binding

CANDIDATE_B = (32, 64, 128, 256)
SEG_LENS = (256, 512, 1024, 2048)
DEFAULT_SEG_LEN = 512  # the library's segment length when ials_config.seg_len is 0
DEALS = ("static", "queue")
GRAM_SPLITS = (256, 512, 1024, 2048)
DEFAULT_GRAM_SPLIT = 512  # the library's Gramian split when ials_config.gram_split is 0


def default_cache_path() -> str:
    return os.environ.get("IALS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2110_14044_amd", "autotune.json"))


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def problem_key(p, precision: int) -> str:
    prec = "bf16" if precision == binding.IALS_PREC_BF16 else "fp32"
    return f"U{p.num_users}:I{p.num_items}:S{p.nnz}:d{p.dim}:{prec}:{_device_name()}"


def _pass_ms(tr, side: int, blk: int) -> float:
    """Time of one pass from the HIP events around its kernels."""
    binding.ials_profile_enable(tr.ctx, True)
    tr.block_sweep(side, blk)
    prof = binding.ials_profile_read(tr.ctx)
    binding.ials_profile_enable(tr.ctx, False)
    return sum(ms for ms, _ in prof.values())


def _predict_ms(tr) -> float:
    """Time of the prediction refresh that starts an epoch."""
    binding.ials_profile_enable(tr.ctx, True)
    tr.refresh_predictions()
    prof = binding.ials_profile_read(tr.ctx)
    binding.ials_profile_enable(tr.ctx, False)
    return sum(ms for ms, _ in prof.values())


def estimate_epoch_ms(problem, block: int, precision: int = binding.IALS_PREC_FP32, deal: str = "auto",
                      seg_len: int = 0, gram_split: int = 0, repeats: int = 2) -> dict:
    """Build a context for `problem` at block size `block` and estimate its epoch time from timed passes."""
    from . import Trainer
    q = copy.copy(problem)
    q.block = block
    nb = math.ceil(q.dim / block)
    tr = Trainer(q, precision=precision, deal=deal, seg_len=seg_len, gram_split=gram_split)
    try:
        # load every kernel once (the first pass of a new block moves the prediction cache)
        tr.block_sweep(0, 0)
        tr.block_sweep(1, 0)
        if nb > 1:
            tr.block_sweep(0, 1)
            tr.block_sweep(1, 1)
        tr.synchronize()
        best = None
        for _ in range(repeats):
            tr.block_sweep(1, 0)  # the cache is relative to block 0 again, as at the start of an epoch
            first_user = _pass_ms(tr, 0, 0)
            first_item = _pass_ms(tr, 1, 0)
            move_user = _pass_ms(tr, 0, 1) if nb > 1 else 0.0
            item = _pass_ms(tr, 1, 1) if nb > 1 else 0.0
            pred = _predict_ms(tr)
            est = pred + first_user + first_item + (nb - 1) * (move_user + item)
            cur = {"epoch_ms": est, "predict_ms": pred, "user_first_ms": first_user, "item_first_ms": first_item,
                   "user_move_ms": move_user, "item_ms": item}
            if best is None or cur["epoch_ms"] < best["epoch_ms"]:
                best = cur
        best.update({"block": block, "nblocks": nb, "deal": deal, "seg_len": seg_len or DEFAULT_SEG_LEN,
                     "gram_split": gram_split or DEFAULT_GRAM_SPLIT})
        return best
    finally:
        tr.close()


def tune(problem, precision: int = binding.IALS_PREC_FP32, candidates=CANDIDATE_B, cache_path: str | None = None,
         refresh: bool = False, log=None, min_gain: float = 0.01) -> dict:
    """Choose b (then row dealing, segment length and Gramian split at that b) for `problem` by
    measurement.  b takes the fastest candidate; the later settings replace the library's default
    only when they are faster by more than `min_gain` (a fraction of the estimated epoch), so that
    run-to-run timing noise does not flip the choice.

    Returns {"block", "deal", "seg_len", "gram_split", "epoch_ms", "trials": [...]} and stores it in the
    cache."""
    import torch
    cache_path = cache_path or default_cache_path()
    key = problem_key(problem, precision)
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache and not refresh and "gram_split" in cache[key]:
        return cache[key]
    say = log or (lambda *a: None)
    trials = []
    for b in candidates:
        if b > problem.dim:
            continue
        r = estimate_epoch_ms(problem, b, precision)
        trials.append(r)
        say(f"[tune] b={b}: epoch {r['epoch_ms']:.1f} ms (user {r['user_first_ms']:.2f}/{r['user_move_ms']:.2f}, "
            f"item {r['item_ms']:.2f} ms per pass, {r['nblocks']} blocks)")
        torch.cuda.empty_cache()
    best = min(trials, key=lambda r: r["epoch_ms"])
    for deal in DEALS:
        r = estimate_epoch_ms(problem, best["block"], precision, deal=deal)
        trials.append(r)
        say(f"[tune] b={best['block']} deal={deal}: epoch {r['epoch_ms']:.1f} ms")
        if r["epoch_ms"] < best["epoch_ms"] * (1.0 - min_gain):
            best = r
    for seg in SEG_LENS:
        if seg == DEFAULT_SEG_LEN:
            continue
        r = estimate_epoch_ms(problem, best["block"], precision, deal=best["deal"], seg_len=seg)
        trials.append(r)
        say(f"[tune] b={best['block']} deal={best['deal']} seg_len={seg}: epoch {r['epoch_ms']:.1f} ms")
        if r["epoch_ms"] < best["epoch_ms"] * (1.0 - min_gain):
            best = r
    for split in GRAM_SPLITS:
        if split == DEFAULT_GRAM_SPLIT:
            continue
        r = estimate_epoch_ms(problem, best["block"], precision, deal=best["deal"], seg_len=best["seg_len"],
                              gram_split=split)
        trials.append(r)
        say(f"[tune] b={best['block']} deal={best['deal']} seg_len={best['seg_len']} gram_split={split}: "
            f"epoch {r['epoch_ms']:.1f} ms")
        if r["epoch_ms"] < best["epoch_ms"] * (1.0 - min_gain):
            best = r
    out = {"block": best["block"], "deal": best["deal"], "seg_len": best["seg_len"],
           "gram_split": best["gram_split"], "epoch_ms": best["epoch_ms"],
           "key": key, "trials": trials}
    cache[key] = out
    os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)
    return out
