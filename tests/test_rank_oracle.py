"""Pins of the top-k and ranking-metric oracle (oracle/rank.py) against what the definitions fix.

Each test ties the oracle to something other than itself: a hand-worked example
(tests/golden/rank_metrics_example.txt), Python's built-in sort, heapq.nlargest, closed forms of
a perfect and of a fully missed ranking, and invariants of the metrics.
"""
import heapq
import math
import os

import numpy as np
import pytest

from oracle import rank

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rank_metrics_example.txt")


def _csr(lists):
    ptr = np.zeros(len(lists) + 1, np.int64)
    ptr[1:] = np.cumsum([len(x) for x in lists])
    idx = np.array([i for x in lists for i in x], np.int32)
    return ptr, idx


def _golden():
    g = {"H": [], "excl": {}, "hold": {}, "top": {}, "metric": []}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "k":
            g["k"] = int(f[1])
        elif f[0] == "H":
            g["H"].append([float(x) for x in f[1:]])
        elif f[0] in ("excl", "hold", "top"):
            g[f[0]][int(f[1])] = [int(x) for x in f[2:]]
        elif f[0] == "metric":
            g["metric"].append((f[1], int(f[2]), int(f[3]), float(f[4])))
    return g


def test_golden_example():
    g = _golden()
    H = np.array(g["H"])
    U = H.shape[1]
    W = np.eye(U)
    ep, ei = _csr([g["excl"].get(u, []) for u in range(U)])
    hp, hi = _csr([g["hold"].get(u, []) for u in range(U)])
    ids, sc = rank.topk(W, H, g["k"], ep, ei)
    for u in range(U):
        assert list(ids[u]) == g["top"][u]
        assert np.array_equal(sc[u], H[ids[u], u])
    for name, k, u, val in g["metric"]:
        m = rank.metrics(ids, hp, hi, [(name, k)])[u, 0]
        if math.isnan(val):
            assert math.isnan(m)
        else:
            assert m == pytest.approx(val, abs=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_topk_matches_python_sort(seed):
    rng = np.random.default_rng(seed)
    U, I, d, k = 7, 40, 5, 9
    W = rng.standard_normal((U, d))
    H = rng.standard_normal((I, d))
    # a few exact ties: duplicated item rows
    H[5] = H[17]
    H[30] = H[17]
    excl = [sorted(rng.choice(I, size=rng.integers(0, 6), replace=False).tolist()) for _ in range(U)]
    ep, ei = _csr(excl)
    ids, sc = rank.topk(W, H, k, ep, ei)
    for u in range(U):
        s = [(sum(W[u, f] * H[i, f] for f in range(d)), i) for i in range(I) if i not in excl[u]]
        s.sort(key=lambda t: (-t[0], t[1]))
        assert list(ids[u]) == [i for _, i in s[:k]]
        # the same scores as heapq's selection of the k largest
        best = heapq.nlargest(k, [t[0] for t in s])
        assert np.allclose(sc[u], best, rtol=0, atol=1e-12)
        assert not set(ids[u].tolist()) & set(excl[u])


def test_short_lists_are_padded():
    W = np.ones((2, 3))
    H = np.arange(12, dtype=float).reshape(4, 3)
    ep, ei = _csr([[0, 1], []])
    ids, sc = rank.topk(W, H, 6, ep, ei)
    assert list(ids[0]) == [3, 2, -1, -1, -1, -1]
    assert list(ids[1]) == [3, 2, 1, 0, -1, -1]
    assert np.all(np.isneginf(sc[0, 2:])) and np.all(np.isneginf(sc[1, 4:]))


def test_metric_closed_forms():
    # a perfect ranking (the held-out items first) scores 1; a list missing every held-out item scores 0
    ids = np.array([[4, 7, 1, 0, 2], [0, 1, 2, 3, 5]], np.int32)
    hp, hi = _csr([[7, 4, 1], [6, 8]])
    m = rank.metrics(ids, hp, hi, [("recall", 3), ("ndcg", 3), ("recall", 5), ("ndcg", 5), ("ndcg", 2)])
    assert np.allclose(m[0], 1.0, rtol=0, atol=1e-15)
    assert np.all(m[1] == 0.0)
    # recall@k divides by min(k, |T|): one hit of a two-item holdout within k = 1 is 1
    m = rank.metrics(np.array([[3, 9]], np.int32), *_csr([[3, 5]]), [("recall", 1), ("recall", 2)])
    assert m[0, 0] == 1.0 and m[0, 1] == 0.5


def test_metric_invariants():
    rng = np.random.default_rng(5)
    U, I, K = 30, 200, 20
    ids = np.stack([rng.permutation(I)[:K] for _ in range(U)]).astype(np.int32)
    hold = [sorted(rng.choice(I, size=rng.integers(0, 15), replace=False).tolist()) for _ in range(U)]
    hp, hi = _csr(hold)
    ks = [("recall", 5), ("recall", 20), ("ndcg", 10), ("ndcg", 20)]
    m = rank.metrics(ids, hp, hi, ks)
    ok = ~np.isnan(m)
    assert np.all((m[ok] >= 0) & (m[ok] <= 1))
    assert np.all(np.isnan(m[[u for u in range(U) if not hold[u]]]))
    # relabelling the items changes nothing
    perm = rng.permutation(I)
    m2 = rank.metrics(perm[ids].astype(np.int32), hp, perm[hi].astype(np.int32), ks)
    assert np.allclose(m, m2, equal_nan=True, rtol=0, atol=1e-15)
    # the hit count recall@k * min(k, |T|) grows with k, and a hit moved to an earlier rank raises NDCG
    sz = np.array([len(h) for h in hold])
    r = ok[:, 0]
    assert np.all(m[r, 0] * np.minimum(5, sz[r]) <= m[r, 1] * np.minimum(20, sz[r]) + 1e-12)
    ids2 = np.array([[1, 2, 3, 4]], np.int32)
    hp1, hi1 = _csr([[3]])
    a = rank.metrics(ids2, hp1, hi1, [("ndcg", 4)])[0, 0]
    b = rank.metrics(np.array([[3, 1, 2, 4]], np.int32), hp1, hi1, [("ndcg", 4)])[0, 0]
    assert b == 1.0 and a < b
