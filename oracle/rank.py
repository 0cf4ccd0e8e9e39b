"""FP64 CPU oracle for top-k recommendation and its ranking metrics -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark may import this module; the GPU library
never calls it and shares no code with it.

What it computes (plain numpy, float64, no blocking or reordering beyond the definitions):
  scores        the scoring function of matrix factorisation, yhat(u, i) = <w_u, h_i>
                (sec. 2, eq. 1), for every user of W against every item of H
  topk          the items recommended to each user (sec. 2: items are ranked by yhat):
                the k largest scores among the items not excluded for that user, ordered
                by score (descending), equal scores by item id (ascending); fewer than k
                eligible items leave the tail as id -1, score -inf
  metrics       Recall@k and NDCG@k of a ranked list against the held-out items of each
                user (sec. 5.1 names them; the definitions are those of the holdout protocol
                the paper follows): with T_u the held-out set and rel_r = [item at rank r in
                T_u] (r = 1, 2, ...),
                  Recall@k = sum_{r<=k} rel_r / min(k, |T_u|)
                  NDCG@k   = sum_{r<=k} rel_r / log2(r + 1)  /  sum_{r<=min(k,|T_u|)} 1 / log2(r + 1)
                users with an empty T_u have no value (NaN) and are left out of the means.

Pins (tests/test_rank_oracle.py): hand-worked examples (tests/golden/rank_metrics_example.txt),
the ranking against Python's own sort on small random cases, ties ordered by id, exclusions
never returned, the closed forms of a perfect and of a fully missed ranking, and the metric
invariants (range, relabelling of items).
"""
from __future__ import annotations

import math

import numpy as np


def scores(W: np.ndarray, H: np.ndarray) -> np.ndarray:
    """yhat(u, i) = <w_u, h_i> for all u, i (eq. 1), in float64."""
    return np.asarray(W, np.float64) @ np.asarray(H, np.float64).T


def topk(W, H, k: int, excl_ptr=None, excl_idx=None):
    """Top-k items per user by eq. 1 with the excluded items (CSR per user) removed.

    Returns (ids int32 [U, k], scores float64 [U, k])."""
    S = scores(W, H)
    U, I = S.shape
    ids = np.full((U, k), -1, np.int32)
    sc = np.full((U, k), -np.inf)
    for u in range(U):
        eligible = np.ones(I, bool)
        if excl_ptr is not None:
            eligible[np.asarray(excl_idx[excl_ptr[u]:excl_ptr[u + 1]], np.int64)] = False
        items = np.nonzero(eligible)[0]
        # score descending, then item id ascending
        order = np.lexsort((items, -S[u, items]))
        take = items[order[:k]]
        ids[u, :len(take)] = take
        sc[u, :len(take)] = S[u, take]
    return ids, sc


def metrics(ids: np.ndarray, hold_ptr, hold_idx, ks) -> np.ndarray:
    """Per-user Recall@k and NDCG@k of ranked lists `ids` [U, K] (id -1: no item).

    `ks` is a sequence of (name, k) with name 'recall' or 'ndcg'; returns float64 [U, len(ks)]
    with NaN for users without held-out items."""
    U = ids.shape[0]
    out = np.full((U, len(ks)), np.nan)
    for u in range(U):
        T = set(int(x) for x in hold_idx[hold_ptr[u]:hold_ptr[u + 1]])
        if not T:
            continue
        for c, (name, k) in enumerate(ks):
            rel = [1.0 if int(x) in T else 0.0 for x in ids[u, :k]]
            if name == "recall":
                out[u, c] = sum(rel) / min(k, len(T))
            elif name == "ndcg":
                dcg = sum(r / math.log2(pos + 2) for pos, r in enumerate(rel))
                idcg = sum(1.0 / math.log2(pos + 2) for pos in range(min(k, len(T))))
                out[u, c] = dcg / idcg
            else:
                raise ValueError(name)
    return out
