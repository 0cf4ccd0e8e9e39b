"""Top-k recommendation and ranking metrics (ials_rank_topk, ials_rank_metrics) through the C ABI,
against the float64 oracle (oracle/rank.py) on the same seeded inputs.

Scores are float32 matrix-core dot products, so ranks can differ from the float64 ranking only
between items whose scores lie within the rounding bound of each other.  With
tol(u, i) = 2 d 2^-24 sum_f |w_uf h_if| (twice the bound of a float32 dot product of length d):
  * every returned score is within tol of the float64 score of the returned item;
  * every returned item is eligible, appears once, and its float64 score is at least the
    oracle's k-th score minus 2 max tol; every oracle item scoring more than the k-th plus
    2 max tol is returned; lists are ordered by returned score, then id;
  * inputs with exact ties (identical item rows, all-zero scores) are compared id for id.
Metrics (integer hits and float64 sums) must equal the oracle's on the same lists to 1e-12.
"""
import numpy as np
import pytest

import synth
from oracle import rank as orank
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _csr(lists):
    ptr = np.zeros(len(lists) + 1, np.int64)
    ptr[1:] = np.cumsum([len(x) for x in lists])
    idx = np.array([i for x in lists for i in x], np.int32)
    return ptr, idx


def _run(W, H, k, excl=None, buf=0):
    import torch
    from paper_2110_14044_amd import rank_topk
    ep, ei = (None, None) if excl is None else _csr(excl)
    Wt = torch.from_numpy(np.ascontiguousarray(W, np.float32)).cuda()
    Ht = torch.from_numpy(np.ascontiguousarray(H, np.float32)).cuda()
    ids, sc = rank_topk(Wt, Ht, k, ep, ei, score_buffer_bytes=buf)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), sc.cpu().numpy()


def _check(W, H, k, ids, sc, excl=None, users=None):
    W = np.asarray(W, np.float64)
    H = np.asarray(H, np.float64)
    d = W.shape[1]
    I = H.shape[0]
    users = range(W.shape[0]) if users is None else users
    for u in users:
        s64 = H @ W[u]
        tol = 2 * d * 2.0 ** -24 * (np.abs(H) @ np.abs(W[u]))
        ex = set() if excl is None else set(excl[u])
        elig = np.array([i for i in range(I) if i not in ex], np.int64)
        n = min(k, elig.size)
        got = ids[u, :n]
        assert np.all(ids[u, n:] == -1) and np.all(np.isneginf(sc[u, n:]))
        assert np.all((got >= 0) & (got < I)) and len(set(got.tolist())) == n
        assert not set(got.tolist()) & ex
        assert np.all(np.abs(sc[u, :n] - s64[got]) <= tol[got])
        # ordered by returned score, then id
        for r in range(n - 1):
            assert sc[u, r] > sc[u, r + 1] or (sc[u, r] == sc[u, r + 1] and got[r] < got[r + 1])
        if n == 0:
            continue
        order = elig[np.lexsort((elig, -s64[elig]))]
        kth = s64[order[n - 1]]
        slack = 2 * tol[elig].max()
        assert np.all(s64[got] >= kth - slack)
        must = set(order[s64[order] > kth + slack].tolist())
        assert must <= set(got.tolist())


@pytest.mark.parametrize("U,I,d,k,nex", [(300, 1000, 16, 20, 0), (130, 777, 40, 1, 5), (257, 2050, 128, 100, 30),
                                         (70, 5000, 64, 512, 0), (64, 129, 12, 50, 3)])
def test_topk_matches_oracle(U, I, d, k, nex):
    rng = np.random.default_rng(U + I + d + k)
    W = (rng.standard_normal((U, d)) / np.sqrt(d)).astype(np.float32)
    H = rng.standard_normal((I, d)).astype(np.float32)
    excl = [sorted(rng.choice(I, size=rng.integers(0, nex + 1), replace=False).tolist()) for _ in range(U)] if nex else None
    say(f"rank topk U={U} I={I} d={d} k={k} excl={nex}")
    ids, sc = _run(W, H, k, excl)
    _check(W, H, k, ids, sc, excl)


def test_topk_batches_and_exact_ties():
    # 3 distinct item rows repeated: every score is one of 3 values per user, with hundreds of
    # bitwise-equal scores at the k-th place; a 64 KiB score buffer forces many user batches
    rng = np.random.default_rng(7)
    U, I, d, k = 200, 2001, 32, 50
    base = rng.standard_normal((3, d)).astype(np.float32)
    H = base[rng.integers(0, 3, size=I)]
    W = rng.standard_normal((U, d)).astype(np.float32)
    excl = [sorted(rng.choice(I, size=10, replace=False).tolist()) for _ in range(U)]
    say("rank topk ties, small buffer")
    ids, sc = _run(W, H, k, excl, buf=64 * 1024)
    ref, _ = orank.topk(W.astype(np.float64), H.astype(np.float64), k, *_csr(excl))
    assert np.array_equal(ids, ref)
    ids2, sc2 = _run(W, H, k, excl)
    assert np.array_equal(ids2, ids) and np.array_equal(sc2, sc)


def test_topk_all_equal_scores_take_smallest_ids():
    # all scores 0 (-0 and +0 alike): more equal keys than the candidate buffer holds
    U, I, d, k = 9, 3000, 8, 300
    W = np.random.default_rng(3).standard_normal((U, d)).astype(np.float32)
    H = np.zeros((I, d), np.float32)
    excl = [list(range(u, 40 * u, 7)) for u in range(U)]
    say("rank topk all ties")
    ids, sc = _run(W, H, k, excl)
    ref, _ = orank.topk(W, H, k, *_csr(excl))
    assert np.array_equal(ids, ref) and np.all(sc == 0)


def test_topk_short_and_empty():
    import torch
    from paper_2110_14044_amd import rank_topk
    rng = np.random.default_rng(11)
    W = rng.standard_normal((5, 8)).astype(np.float32)
    H = rng.standard_normal((6, 8)).astype(np.float32)
    excl = [[0, 1], [], [5], [0, 1, 2, 3, 4, 5], [2]]
    say("rank topk short lists")
    ids, sc = _run(W, H, 8, excl)
    _check(W, H, 8, ids, sc, excl)
    assert np.all(ids[3] == -1)
    # no items at all, and no users
    ids, sc = _run(W, np.zeros((0, 8), np.float32), 3)
    assert np.all(ids == -1) and np.all(np.isneginf(sc))
    e_ids, e_sc = rank_topk(torch.zeros((0, 8), device="cuda"), torch.from_numpy(H).cuda(), 4)
    assert e_ids.shape == (0, 4)


def test_topk_rejects_bad_arguments():
    import torch
    from paper_2110_14044_amd import binding, rank_topk
    W = torch.zeros((4, 6), device="cuda")  # d not a multiple of 4
    with pytest.raises(binding.IalsError):
        rank_topk(W, torch.zeros((5, 6), device="cuda"), 3)
    with pytest.raises(binding.IalsError):
        rank_topk(torch.zeros((4, 8), device="cuda"), torch.zeros((5, 8), device="cuda"), 513)


def test_metrics_match_oracle():
    import torch
    from paper_2110_14044_amd import rank_metrics
    rng = np.random.default_rng(21)
    U, I, K = 1000, 500, 100
    ids = np.stack([rng.permutation(I)[:K] for _ in range(U)]).astype(np.int32)
    ids[::7, 60:] = -1  # short lists
    hold = [sorted(rng.choice(I, size=rng.integers(0, 40), replace=False).tolist()) for _ in range(U)]
    hp, hi = _csr(hold)
    ms = [("recall", 20), ("recall", 50), ("ndcg", 100), ("ndcg", 1)]
    say("rank metrics")
    per, means, counts = rank_metrics(torch.from_numpy(ids).cuda(), hp, hi, ms)
    per = per.cpu().numpy()
    ref = orank.metrics(ids, hp, hi, ms)
    assert np.array_equal(np.isnan(per), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.max(np.abs(per[ok] - ref[ok])) <= 1e-12
    assert np.array_equal(counts, ok.sum(axis=0))
    assert np.allclose(means, np.nanmean(ref, axis=0), rtol=0, atol=1e-12)


def test_holdout_evaluation_pipeline():
    # train without the held-out users, fold them in from 80 % of their items, rank everything
    # else, and measure against the other 20 %: the GPU pipeline against the oracle's ranking and
    # metrics of the same folded-in rows
    import torch
    from paper_2110_14044_amd import Trainer, rank_metrics, rank_topk
    p = synth.small_problem(95, 2000, 600, 40_000, 32, 16, std=0.1)
    split = synth.holdout_split(p, 150)
    say("rank holdout pipeline")
    tr = Trainer(split.train)
    tr.epoch(3)
    Wf = tr.foldin(split.fold_ptr, split.fold_idx, passes=3)
    H = tr.H.clone()
    tr.close()
    ids, sc = rank_topk(Wf, H, 50, split.fold_ptr, split.fold_idx)
    ms = [("recall", 20), ("recall", 50), ("ndcg", 50)]
    per, means, counts = rank_metrics(ids, split.hold_ptr, split.hold_idx, ms)
    torch.cuda.synchronize()
    ids_h, sc_h = ids.cpu().numpy(), sc.cpu().numpy()
    Wh, Hh = Wf.cpu().numpy(), H.cpu().numpy()
    excl = [split.fold_idx[split.fold_ptr[j]:split.fold_ptr[j + 1]].tolist() for j in range(split.users.size)]
    _check(Wh, Hh, 50, ids_h, sc_h, excl)
    ref = orank.metrics(ids_h, split.hold_ptr, split.hold_idx, ms)
    assert np.max(np.abs(per.cpu().numpy() - ref)) <= 1e-12
    ref_ids, _ = orank.topk(Wh, Hh, 50, split.fold_ptr, split.fold_idx)
    ref_e2e = np.nanmean(orank.metrics(ref_ids, split.hold_ptr, split.hold_idx, ms), axis=0)
    assert np.allclose(means, ref_e2e, rtol=0, atol=0.02)
    assert np.all(counts == split.users.size)


def test_topk_full_size_sampled():
    # the ML20M shape: 20,000 items x d = 128; 20,000 users scored in two batches of the default
    # 1 GiB score buffer (13,421 rows, then 6,579); 66 sampled users checked against the oracle
    rng = np.random.default_rng(2021)
    U, I, d, k = 20_000, 20_000, 128, 100
    W = (rng.standard_normal((U, d)) * 0.1).astype(np.float32)
    H = (rng.standard_normal((I, d)) * 0.1).astype(np.float32)
    lens = np.clip(rng.lognormal(3.681, 1.116, size=U).astype(np.int64), 1, 2000)
    excl = [np.unique(rng.integers(0, I, size=n)).tolist() for n in lens]
    say("rank topk full size 20000 x 20000 d=128 k=100")
    ids, sc = _run(W, H, k, excl)
    users = sorted(rng.choice(U, size=64, replace=False).tolist() + [0, U - 1])
    _check(W, H, k, ids, sc, excl, users=users)
