"""Fold-in of new users (ials_foldin) and the continuous-batching fold-in server,
through the C ABI, against the FP64 oracle on the same seeded inputs.

Tolerance: the fold-in rows within 1e-4 relative (Frobenius over all rows) of
the float64 oracle, as for the embeddings after one epoch; the float64 redo
within 1e-6 (its inputs G and H are float32 on both sides, G rounded from a
float64 sum on the GPU).  A server result must equal the same request served
alone bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import bruteforce as bf
from tests.gpu_util import gpu_trainer, host, need_gpu, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _rows_rel(W, ref):
    """Largest per-row relative error over rows with a non-negligible reference."""
    num = np.linalg.norm(np.asarray(W, np.float64) - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    ok = den > 1e-3 * den.max()
    return float((num[ok] / den[ok]).max()) if ok.any() else 0.0


def test_foldin_on_trained_context_matches_oracle():
    p = synth.small_problem(90, 600, 400, 8000, 32, 16, std=0.1)
    say("foldin trained context d=32 b=16")
    tr = gpu_trainer(p)
    tr.epoch(1)
    ptr, items = synth.serving_requests(91, 40, num_items=p.num_items, hi=300)
    W = host(tr.foldin(ptr, items, passes=3))
    H = host(tr.H)
    ref = oracle.foldin(H, p.block, p.alpha0, p.lam, ptr, items, 3)
    e, er = rel(W, ref), _rows_rel(W, ref)
    say(f"foldin vs oracle: {e:.2e} (worst row {er:.2e})")
    assert e < 1e-4 and er < 1e-3
    st = tr.stats()
    assert st["foldin_requests"] == 40 and st["foldin_float64"] == 0
    # a second call after more training uses the new H (the Gramian is re-formed)
    tr.epoch(1)
    W2 = host(tr.foldin(ptr, items, passes=3))
    ref2 = oracle.foldin(host(tr.H), p.block, p.alpha0, p.lam, ptr, items, 3)
    assert rel(W2, ref2) < 1e-4
    tr.close()


@pytest.mark.parametrize("d,b", [(16, 8), (20, 8), (40, 16), (48, 48), (64, 64), (128, 64), (256, 64), (1024, 64)])
def test_foldin_block_shapes(d, b):
    """Ragged last blocks (20/8, 40/16), padded blocks, d/b from 1 to 16 blocks; (1024, 64)
    keeps the factors in the request scratch instead of LDS."""
    p = synth.small_problem(100 + d + b, 300, 500, 3000, d, b, std=0.1)
    say(f"foldin d={d} b={b}")
    tr = gpu_trainer(p)
    ptr, items = synth.serving_requests(d + b, 24, num_items=p.num_items, hi=400)
    rng = np.random.default_rng(d)
    y = rng.uniform(0.0, 2.0, size=items.size).astype(np.float32)
    W = host(tr.foldin(ptr, items, y, passes=3))
    ref = oracle.foldin(p.H0, p.block, p.alpha0, p.lam, ptr, items, 3, y)
    e = rel(W, ref)
    say(f"d={d} b={b}: {e:.2e} (worst row {_rows_rel(W, ref):.2e})")
    assert e < 1e-4
    tr.close()


def test_foldin_empty_requests_and_zero_passes():
    p = synth.small_problem(110, 300, 200, 2000, 32, 16, std=0.1)
    tr = gpu_trainer(p)
    ptr = np.array([0, 0, 5, 5, 12, 12], np.int64)  # empty requests between non-empty ones
    items = np.arange(12, dtype=np.int32) * 7 % p.num_items
    W = host(tr.foldin(ptr, items, passes=3))
    ref = oracle.foldin(p.H0, p.block, p.alpha0, p.lam, ptr, items, 3)
    assert np.all(W[[0, 2, 4]] == 0.0)
    assert rel(W, ref) < 1e-4
    W0 = host(tr.foldin(ptr, items, passes=0))
    assert np.all(W0 == 0.0)
    tr.close()


def test_foldin_b_equals_d_one_pass_is_exact_solve():
    """With b = d one sweep is the closed form of eq. 3 (a library solve, independent of the oracle)."""
    p = synth.small_problem(120, 300, 250, 2500, 32, 32, std=0.1)
    tr = gpu_trainer(p)
    rng = np.random.default_rng(5)
    ptr, items = synth.serving_requests(121, 16, num_items=p.num_items, hi=200)
    y = rng.uniform(0.0, 2.0, size=items.size).astype(np.float32)
    W = host(tr.foldin(ptr, items, y, passes=1))
    exact = np.stack([bf.foldin_exact(p.H0, items[ptr[r]:ptr[r + 1]], y[ptr[r]:ptr[r + 1]], p.alpha0, p.lam)
                      for r in range(ptr.size - 1)])
    assert rel(W, exact) < 1e-4
    tr.close()


def test_foldin_forced_float64_redo():
    p = synth.small_problem(130, 400, 300, 4000, 64, 32, std=0.1)
    tr = gpu_trainer(p, chol_fallback_ratio=1.0)
    ptr, items = synth.serving_requests(131, 20, num_items=p.num_items, hi=250)
    W = host(tr.foldin(ptr, items, passes=3))
    ref = oracle.foldin(p.H0, p.block, p.alpha0, p.lam, ptr, items, 3)
    e = rel(W, ref)
    say(f"float64 redo vs oracle: {e:.2e}")
    assert e < 1e-6
    assert tr.stats()["foldin_float64"] == 20
    tr.close()


def test_foldin_rejects_bad_ids_and_offsets():
    from paper_2110_14044_amd import IalsError
    p = synth.small_problem(140, 100, 80, 800, 16, 8)
    tr = gpu_trainer(p)
    with pytest.raises(IalsError, match="IALS_E_INVALID"):
        tr.foldin(np.array([0, 3], np.int64), np.array([1, 80, 2], np.int32))
    with pytest.raises(IalsError, match="IALS_E_INVALID"):
        tr.foldin(np.array([0, 3, 2], np.int64), np.array([1, 2, 3], np.int32))
    W = host(tr.foldin(np.array([0, 3], np.int64), np.array([1, 2, 3], np.int32)))  # still usable
    assert np.all(np.isfinite(W))
    tr.close()


def _serve_all(srv, reqs, d, y=None):
    """Submit every request (retrying on BUSY) and collect the rows by tag."""
    out, i = {}, 0
    while len(out) < len(reqs):
        while i < len(reqs):
            ok = srv.submit(reqs[i], None if y is None else y[i], tag=i)
            if not ok:
                break
            i += 1
        tags, rows, st = srv.poll(256, 2000)
        for t, r, s in zip(tags, rows, st):
            out[int(t)] = (r.copy(), int(s))
    return out


def test_server_matches_oracle_and_alone_vs_mix():
    import torch
    from paper_2110_14044_amd import FoldinServer
    H = synth.serving_table(7)
    ptr, items = synth.serving_requests(8, 300)
    reqs = [items[ptr[r]:ptr[r + 1]] for r in range(ptr.size - 1)]
    say(f"server: 300 requests, {items.size} items, longest {max(len(q) for q in reqs)}")
    srv = FoldinServer(torch.from_numpy(H).cuda(), 64, 0.1, 0.05, passes=3, max_slots=1024)
    mix = _serve_all(srv, reqs, 256)
    st = srv.stats()
    say(f"mix: {st['batches']} batches, largest {st['max_batch']}")
    assert st["max_batch"] > 1
    # alone: one request at a time, each its own batch
    for r in range(0, 300, 10):
        assert srv.submit(reqs[r], None, tag=10_000 + r)
        got = []
        while not got:
            tags, rows, _ = srv.poll(4, 100_000)
            got = list(zip(tags, rows))
        assert int(got[0][0]) == 10_000 + r
        assert np.array_equal(got[0][1], mix[r][0]), r
    srv.close()
    W = np.stack([mix[r][0] for r in range(300)])
    assert all(mix[r][1] == 0 for r in range(300))
    ref = oracle.foldin(H, 64, 0.1, 0.05, ptr, items, 3)
    e = rel(W, ref)
    say(f"server vs oracle: {e:.2e} (worst row {_rows_rel(W, ref):.2e})")
    assert e < 1e-4


def test_server_labels_and_float64_redo():
    import torch
    from paper_2110_14044_amd import FoldinServer
    H = synth.serving_table(9, 3000, 64)
    ptr, items = synth.serving_requests(10, 40, num_items=3000, hi=500)
    rng = np.random.default_rng(3)
    y_all = rng.uniform(0.0, 2.0, size=items.size).astype(np.float32)
    reqs = [items[ptr[r]:ptr[r + 1]] for r in range(40)]
    ys = [y_all[ptr[r]:ptr[r + 1]] for r in range(40)]
    ref = oracle.foldin(H, 32, 0.1, 0.05, ptr, items, 3, y_all)
    for tau, tol, code in ((0.0, 1e-4, 0), (1.0, 1e-6, 1)):
        srv = FoldinServer(torch.from_numpy(H).cuda(), 32, 0.1, 0.05, passes=3, chol_fallback_ratio=tau)
        out = _serve_all(srv, reqs, 64, ys)
        st = srv.stats()
        srv.close()
        W = np.stack([out[r][0] for r in range(40)])
        assert all(out[r][1] == code for r in range(40))
        e = rel(W, ref)
        say(f"labels tau={tau}: {e:.2e}")
        assert e < tol
        assert st["float64_requests"] == (40 if code else 0)


def test_server_admission_by_slots_and_memory():
    import torch
    from paper_2110_14044_amd import FoldinServer, IalsError
    H = torch.from_numpy(synth.serving_table(11, 5000, 256)).cuda()
    rng = np.random.default_rng(12)
    # slots: 4 admitted at once; the rest are answered BUSY until results are polled
    srv = FoldinServer(H, 64, 0.1, 0.05, max_slots=4, hbm_budget=1 << 20)
    req = rng.integers(0, 5000, size=50).astype(np.int32)
    ok = [srv.submit(req, None, tag=t) for t in range(10)]
    assert sum(ok) == 4 and ok[:4] == [True] * 4
    got = 0
    while got < 4:
        tags, _, _ = srv.poll(8, 100_000)
        got += len(tags)
    assert srv.submit(req, None, tag=99)
    assert srv.stats()["rejected_busy"] == 6
    # a request larger than the whole arena is invalid, not busy
    with pytest.raises(IalsError, match="IALS_E_INVALID"):
        srv.submit(np.zeros(80_000, np.int32), None, tag=1)
    with pytest.raises(IalsError, match="IALS_E_INVALID"):
        srv.submit(np.array([5000], np.int32), None, tag=1)
    srv.close()
    # memory: 1 MiB holds four requests of 15,000 items (about 0.24 MB of state each), not five
    srv = FoldinServer(H, 64, 0.1, 0.05, max_slots=100, hbm_budget=1 << 20)
    big = rng.integers(0, 5000, size=15_000).astype(np.int32)
    ok = [srv.submit(big, None, tag=t) for t in range(5)]
    st = srv.stats()
    assert 1 <= sum(ok) < 5 and st["rejected_busy"] == 5 - sum(ok)
    assert st["bytes_peak"] <= st["arena_bytes"]
    n = 0
    while n < sum(ok):
        tags, rows, _ = srv.poll(8, 200_000)
        n += len(tags)
        assert np.all(np.isfinite(rows))
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()
