"""Failure paths of the training context through the C ABI: the HBM budget (create-time
temporaries included), a non-finite loss, a block Hessian that is singular up to the L2
term (float64 redo without forcing it), and a Hessian that is not SPD even in float64.
None of these makes a kernel fault or wait: the inputs are ordinary finite or NaN floats
and every kernel runs its fixed number of steps."""
import copy

import numpy as np
import pytest

import oracle
import synth
from paper_2110_14044_amd import IalsError, binding
from tests.gpu_util import gpu_trainer, host, need_gpu, oracle_setup, rel, row_rel_max, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def test_hbm_budget_bounds_create_including_temporaries():
    p = synth.small_problem(500, 3000, 400, 60_000, 64, 32, labels=True, zipf_s=0.8, std=0.1)
    tr = gpu_trainer(p)
    st = tr.stats()
    tr.close()
    held, peak = st["device_bytes"], st["peak_device_bytes"]
    say(f"budget: held {held} bytes, peak during create {peak} bytes")
    assert peak > held > 0  # the index build's temporaries come on top of what the context keeps
    tr = gpu_trainer(p, hbm_budget=peak)  # exactly enough
    assert tr.stats()["peak_device_bytes"] == peak
    tr.epoch(1)
    tr.loss()
    tr.close()
    for budget in (peak - 1, held, 1 << 20):
        with pytest.raises(IalsError, match="IALS_E_NOMEM"):
            gpu_trainer(p, hbm_budget=budget)
        say(f"budget {budget}: {binding.ials_last_error(None)}")


def test_nan_in_W_makes_the_loss_fail():
    p = synth.small_problem(501, 500, 300, 6000, 32, 16, std=0.1)
    p.W0 = p.W0.copy()
    p.W0[7, 3] = np.nan
    tr = gpu_trainer(p)
    with pytest.raises(IalsError, match="IALS_E_INVALID") as ei:
        tr.loss()
    say(f"NaN in W: {ei.value}")
    assert "not finite" in str(ei.value)
    tr.close()


@pytest.mark.parametrize("d,b", [(32, 16), (256, 128)])
def test_not_spd_in_float64_is_reported(d, b):
    # a NaN row of W makes every item's Gramian term NaN in the item pass: the NaN pivots fail
    # the float32 check, no factorisation succeeds even in float64, and the next synchronising
    # call reports it (the narrow and the wide-block kernels)
    p = synth.small_problem(502 + d, 500, 300, 6000, d, b, std=0.1)
    p.W0 = p.W0.copy()
    p.W0[11, :] = np.nan
    tr = gpu_trainer(p)
    tr.block_sweep(0, 0)
    tr.block_sweep(1, 0)
    with pytest.raises(IalsError, match="IALS_E_NOT_SPD") as ei:
        tr.loss()
    say(f"NaN row: {ei.value}")
    assert tr.stats()["fallback_rows"] >= p.num_items
    tr.close()


@pytest.mark.parametrize("d,b", [(16, 8), (128, 64), (256, 128)])
def test_near_singular_blocks_fall_back_unforced(d, b):
    """alpha0 = 0, lambda = 1e-7 and an item table of rank one: every user's block Hessian is
    lambda I + s v_pi v_pi^T, whose pivot ratio (about lambda / s) is far below the default
    threshold 1e-6, so the float64 redo takes every user with an observation.  The pass then
    matches the oracle (which solves in float64 throughout)."""
    p = synth.small_problem(503 + d, 600, 300, 6000, d, b, std=0.1)
    p.alpha0 = 0.0
    p.lam = 1e-7
    p.H0 = synth.rank_one_table(504 + d, p.num_items, d)
    tr = gpu_trainer(p)
    tr.block_sweep(0, 0)
    Wg = host(tr.W)
    st = tr.stats()
    tr.close()
    csr, _, _ = oracle_setup(p)
    W = p.W0.astype(np.float64)
    H = p.H0.astype(np.float64)
    yhat = oracle.predict(csr, W, H)
    oracle.block_pass(csr, "user", 0, b, p.alpha0, p.lam, W, H, yhat, oracle.gramian(H, 0, b))
    nonempty = int(np.count_nonzero(np.diff(csr.uptr)))
    e, er = rel(Wg, W), row_rel_max(Wg, W)
    say(f"near-singular d={d} b={b}: {st['fallback_rows']} of {nonempty} users redone in float64; "
        f"W {e:.2e}, worst row {er:.1e}")
    assert st["fallback_rows"] == nonempty
    assert e < 1e-4 and er < 1e-3


def test_set_stream_moves_the_context_and_releases_its_own_stream():
    """A graph context created on the NULL stream runs on a stream the library made; moving it
    to a caller's stream waits for the queued work and releases the library's stream; the epoch
    graph then replays on the new stream with the eager results, bit for bit.  A NULL stream is
    refused for a graph context."""
    import torch
    p = synth.small_problem(505, 2000, 150, 40_000, 64, 32, zipf_s=0.9, std=0.1, labels=True)
    ref = gpu_trainer(p)
    ref.epoch(2)
    Wr, Hr = host(ref.W), host(ref.H)
    ref.close()
    W = torch.from_numpy(p.W0.copy()).cuda()
    H = torch.from_numpy(p.H0.copy()).cuda()
    cfg = binding.make_config(p.num_users, p.num_items, p.dim, p.block, p.alpha0, p.lam,
                              flags=binding.IALS_FLAG_GRAPH)
    keep = [np.ascontiguousarray(x) for x in (p.user, p.item, p.y, p.alpha)]
    coo = binding.make_coo(*keep, binding.IALS_MEM_HOST)
    torch.cuda.synchronize()
    ctx = binding.ials_create(cfg, coo, W, H, None)
    try:
        binding.ials_epoch(ctx, 1)
        with pytest.raises(IalsError, match="IALS_E_INVALID"):
            binding.ials_set_stream(ctx, None)
        s = torch.cuda.Stream()
        binding.ials_set_stream(ctx, s)
        binding.ials_epoch(ctx, 1)
        s.synchronize()
        assert np.array_equal(host(W), Wr) and np.array_equal(host(H), Hr)
        binding.ials_loss(ctx)
    finally:
        binding.ials_destroy(ctx)
