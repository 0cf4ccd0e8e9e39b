"""Seeded synthetic inputs for iALS++ (implicit-feedback matrix factorisation).

This module only draws random numbers: observation sets S (user, item[, y, alpha]),
initial embeddings W0/H0 and serving request streams.  It holds none of the
method's arithmetic, so both the FP64 oracle and the GPU library can consume
the same inputs without sharing any code of the method.

Workload shapes follow the two benchmarks of the paper's evaluation (Table 2:
an ML20M-shaped matrix of 136k users x 20k items with 10M observations, and an
MSD-shaped matrix of 571k x 41k with 34M observations).  The real datasets are
not used; these generators stand in for them.

Recipe (all draws from numpy PCG64 with a fixed seed per workload):
  * user history lengths n_u ~ lognormal(mu, sigma), clipped to [lo, hi], then
    rescaled so that sum(n_u) equals the stated |S| exactly (bisection on a
    scale factor, floor, then largest-remainder top-up; deterministic);
  * per user, n_u distinct items drawn with P(rank r) proportional to r^-s
    (Zipf), without replacement (sequential draws, duplicates rejected);
  * popularity ranks are mapped to item ids by a seeded random permutation, so
    popularity is not correlated with the id;
  * the COO order is shuffled (the library has to sort it);
  * W0, H0 ~ N(0, (0.1/sqrt(d))^2), drawn in float32 (sec. 5.1.1 initial std 0.1,
    read as a standard deviation scaled by 1/sqrt(d)).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "workload", "user_lengths", "sample_histories",
    "make_observations", "init_embeddings", "Problem", "make_problem",
    "random_labels", "serving_requests", "serving_table", "poisson_arrivals",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    num_users: int
    num_items: int
    nnz: int
    len_mu: float
    len_sigma: float
    len_lo: int
    len_hi: int
    zipf_s: float
    dim: int
    block: int
    alpha0: float
    lam: float
    epochs: int
    seed: int


# Named by shape.  mu/sigma for the two large shapes are chosen so that the
# mean history length and the expected maximum over all users match the stated
# mean and cap (ML20M-like: mean 74, cap 5,000; MSD-like: mean 60, cap 20,000).
WORKLOADS = {
    "tiny": Workload("tiny", 2_000, 1_000, 50_000, 2.8, 0.8, 1, 200, 1.0,
                     16, 8, 0.1, 0.1, 4, 20211027),
    "ml20m_like": Workload("ml20m_like", 136_000, 20_000, 10_000_000, 3.681, 1.116, 1, 5_000, 1.0,
                           128, 64, 0.1, 0.05, 16, 20211028),
    "ml20m_like_d1024": Workload("ml20m_like_d1024", 136_000, 20_000, 10_000_000, 3.681, 1.116, 1, 5_000,
                                 1.0, 1024, 128, 0.1, 0.05, 16, 20211028),
    "msd_like": Workload("msd_like", 571_000, 41_000, 34_000_000, 2.981, 1.492, 1, 20_000, 0.9,
                         2048, 64, 0.1, 0.05, 8, 20211029),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def user_lengths(rng: np.random.Generator, n_users: int, nnz: int, mu: float, sigma: float,
                 lo: int, hi: int) -> np.ndarray:
    """History lengths: lognormal draws clipped to [lo, hi], rescaled to sum to nnz exactly."""
    if not (n_users * lo <= nnz <= n_users * hi):
        raise ValueError("nnz not reachable with the given clip range")
    raw = rng.lognormal(mu, sigma, size=n_users)

    def total(scale: float) -> int:
        return int(np.clip(np.floor(raw * scale), lo, hi).sum())

    a, b = 0.0, 1.0
    while total(b) <= nnz:
        b *= 2.0
        if b > 1e12:
            break
    for _ in range(200):
        m = 0.5 * (a + b)
        if total(m) <= nnz:
            a = m
        else:
            b = m
    n = np.clip(np.floor(raw * a), lo, hi).astype(np.int64)
    deficit = nnz - int(n.sum())
    if deficit > 0:
        frac = raw * a - np.floor(raw * a)
        order = np.lexsort((np.arange(n_users), -frac))  # largest remainder first, ties by index
        eligible = order[n[order] < hi]
        if eligible.size < deficit:
            raise RuntimeError("cannot distribute history lengths")
        n[eligible[:deficit]] += 1
    assert int(n.sum()) == nnz
    return n


def sample_histories(rng: np.random.Generator, lengths: np.ndarray, n_items: int,
                     s: float) -> tuple[np.ndarray, np.ndarray]:
    """For each user u draw lengths[u] distinct popularity ranks (0-based) with
    P(r) proportional to (r+1)^-s; repeated draws are rejected.  Returns (user, rank)
    arrays in user-major, draw order."""
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.size and lengths.max() > n_items:
        raise ValueError("history longer than the catalogue")
    p = np.arange(1, n_items + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    n_users = lengths.size
    need = lengths.copy()
    acc_keys = np.empty(0, dtype=np.int64)  # sorted keys user*n_items+rank accepted so far
    out_u, out_r = [], []
    factor = 1.3
    while True:
        users = np.nonzero(need > 0)[0]
        if users.size == 0:
            break
        draws = np.ceil(need[users] * factor).astype(np.int64) + 4
        u = np.repeat(users, draws)
        r = np.searchsorted(cdf, rng.random(u.size), side="right")
        r = np.minimum(r, n_items - 1)
        key = u * n_items + r
        # reject pairs drawn in an earlier round
        if acc_keys.size:
            pos = np.searchsorted(acc_keys, key)
            pos = np.minimum(pos, acc_keys.size - 1)
            fresh = acc_keys[pos] != key
            u, r, key = u[fresh], r[fresh], key[fresh]
        # keep the first occurrence of each pair, in draw order
        _, first = np.unique(key, return_index=True)
        first.sort()
        u, r, key = u[first], r[first], key[first]
        # per user, keep at most need[u] of the survivors (the earliest ones)
        start = np.searchsorted(u, u, side="left")  # u is non-decreasing
        rank_in_user = np.arange(u.size) - start
        keep = rank_in_user < need[u]
        u, r, key = u[keep], r[keep], key[keep]
        need -= np.bincount(u, minlength=n_users)
        out_u.append(u)
        out_r.append(r)
        acc_keys = np.union1d(acc_keys, key)
        factor = min(factor * 1.5, 16.0)
    uu = np.concatenate(out_u) if out_u else np.empty(0, np.int64)
    rr = np.concatenate(out_r) if out_r else np.empty(0, np.int64)
    order = np.argsort(uu, kind="stable")
    return uu[order], rr[order]


def make_observations(wl: Workload, rng: Optional[np.random.Generator] = None):
    """COO observation set of a workload, in a shuffled order: (user int32, item int32)."""
    rng = rng if rng is not None else np.random.Generator(np.random.PCG64(wl.seed))
    n = user_lengths(rng, wl.num_users, wl.nnz, wl.len_mu, wl.len_sigma, wl.len_lo, wl.len_hi)
    u, r = sample_histories(rng, n, wl.num_items, wl.zipf_s)
    rank_to_item = rng.permutation(wl.num_items)
    item = rank_to_item[r]
    shuffle = rng.permutation(u.size)
    return u[shuffle].astype(np.int32), item[shuffle].astype(np.int32)


def init_embeddings(rng: np.random.Generator, rows: int, dim: int, std: Optional[float] = None) -> np.ndarray:
    std = (0.1 / math.sqrt(dim)) if std is None else std
    x = rng.standard_normal((rows, dim), dtype=np.float32)
    return (x * np.float32(std)).astype(np.float32)


@dataclasses.dataclass
class Problem:
    num_users: int
    num_items: int
    dim: int
    block: int
    alpha0: float
    lam: float
    user: np.ndarray            # int32[nnz]
    item: np.ndarray            # int32[nnz]
    y: Optional[np.ndarray]     # float32[nnz] or None (all ones)
    alpha: Optional[np.ndarray]  # float32[nnz] or None (all ones)
    W0: np.ndarray              # float32[U, d]
    H0: np.ndarray              # float32[I, d]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.user.size)


def make_problem(name: str, dim: Optional[int] = None, block: Optional[int] = None) -> Problem:
    wl = WORKLOADS[name]
    rng = np.random.Generator(np.random.PCG64(wl.seed))
    u, i = make_observations(wl, rng)
    d = wl.dim if dim is None else dim
    b = wl.block if block is None else block
    W0 = init_embeddings(rng, wl.num_users, d)
    H0 = init_embeddings(rng, wl.num_items, d)
    return Problem(wl.num_users, wl.num_items, d, b, wl.alpha0, wl.lam, u, i, None, None, W0, H0, name)


def random_labels(rng: np.random.Generator, nnz: int):
    """General observations (sec. 2: labels y in R, weights alpha > 0): y ~ U(0, 2), alpha ~ U(0.5, 3)."""
    y = rng.uniform(0.0, 2.0, size=nnz).astype(np.float32)
    a = rng.uniform(0.5, 3.0, size=nnz).astype(np.float32)
    return y, a


def small_problem(seed: int, num_users: int, num_items: int, nnz: int, dim: int, block: int,
                  alpha0: float = 0.1, lam: float = 0.1, labels: bool = False,
                  zipf_s: float = 1.0, std: float = 0.3) -> Problem:
    """A tiny random problem: distinct (u, i) pairs, optionally with random y and alpha."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if nnz > num_users * num_items:
        raise ValueError("too many observations")
    hi = min(num_items, max(1, 4 * nnz // max(num_users, 1) + 1))
    hi = max(hi, -(-nnz // num_users))
    lo = 1 if nnz >= num_users else 0
    if lo == 0:
        n = np.zeros(num_users, np.int64)
        n[rng.choice(num_users, size=nnz, replace=False)] = 1
    else:
        n = user_lengths(rng, num_users, nnz, 0.0, 0.8, lo, hi)
    u, r = sample_histories(rng, n, num_items, zipf_s)
    item = rng.permutation(num_items)[r]
    shuffle = rng.permutation(u.size)
    u = u[shuffle].astype(np.int32)
    item = item[shuffle].astype(np.int32)
    y = a = None
    if labels:
        y, a = random_labels(rng, u.size)
    W0 = init_embeddings(rng, num_users, dim, std)
    H0 = init_embeddings(rng, num_items, dim, std)
    return Problem(num_users, num_items, dim, block, alpha0, lam, u, item, y, a, W0, H0,
                   f"small{seed}")


def rank_one_table(seed: int, rows: int, dim: int, lo: float = 1.0, hi: float = 2.0) -> np.ndarray:
    """Rows c_r v on one seeded direction v (|v| = 1, c_r ~ U(lo, hi)), float32: a table whose
    Gramian has rank one, for problems whose block Hessians are singular up to the L2 term."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(dim)
    v /= np.linalg.norm(v)
    c = rng.uniform(lo, hi, size=rows)
    return (c[:, None] * v[None, :]).astype(np.float32)


def serving_requests(seed: int, n_requests: int, num_items: int = 41_000, mu: float = 3.5,
                     sigma: float = 1.2, lo: int = 1, hi: int = 2_000, zipf_s: float = 0.9):
    """Fold-in request histories: lengths lognormal(mu, sigma) clipped to [lo, hi] (no
    rescaling), distinct Zipf(s) items.  Returns (ptr int64[n+1], items int32[total])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.clip(np.round(rng.lognormal(mu, sigma, size=n_requests)), lo, hi).astype(np.int64)
    u, r = sample_histories(rng, n, num_items, zipf_s)
    item = rng.permutation(num_items)[r].astype(np.int32)
    ptr = np.zeros(n_requests + 1, np.int64)
    ptr[1:] = np.cumsum(n)
    return ptr, item


def serving_table(seed: int, num_items: int = 41_000, dim: int = 256) -> np.ndarray:
    """The fixed item table of the serving workload: N(0, 0.1/sqrt(d)) float32."""
    return init_embeddings(np.random.Generator(np.random.PCG64(seed)), num_items, dim)


def poisson_arrivals(seed: int, n: int, rate_per_s: float) -> np.ndarray:
    """Open-loop arrival times (seconds) of a Poisson process."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


@dataclasses.dataclass
class HoldoutSplit:
    """Users held out of training: their observations are split into a fold-in part (given at
    evaluation time, excluded from their recommendations) and a held-out part (the items the
    ranking metrics look for).  Lists are CSR over the held-out users, item ids ascending."""
    train: Problem
    users: np.ndarray        # int32[n] ids of the held-out users (in the original numbering)
    fold_ptr: np.ndarray     # int64[n+1]
    fold_idx: np.ndarray     # int32
    hold_ptr: np.ndarray     # int64[n+1]
    hold_idx: np.ndarray     # int32


def holdout_split(p: Problem, n_users: int, frac: float = 0.2, seed: int = 20211101,
                  min_len: int = 5) -> HoldoutSplit:
    """The shape of the holdout protocol of sec. 5.1 on a synthetic matrix: n_users users with at
    least min_len observations are drawn at random; each keeps a random 1 - frac of its items
    for fold-in and frac (at least one) are held out; the training problem keeps every other
    user's observations (the held-out users' rows are empty there)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = np.bincount(p.user, minlength=p.num_users)
    cand = np.nonzero(lens >= min_len)[0]
    users = np.sort(rng.choice(cand, size=min(n_users, cand.size), replace=False)).astype(np.int32)
    is_held = np.zeros(p.num_users, bool)
    is_held[users] = True
    keep = ~is_held[p.user]
    train = dataclasses.replace(
        p, user=p.user[keep], item=p.item[keep],
        y=None if p.y is None else p.y[keep], alpha=None if p.alpha is None else p.alpha[keep],
        name=p.name + "_train")
    order = np.argsort(p.user, kind="stable")
    ptr = np.zeros(p.num_users + 1, np.int64)
    ptr[1:] = np.cumsum(lens)
    fold, hold = [], []
    for u in users:
        its = p.item[order[ptr[u]:ptr[u + 1]]]
        its = its[rng.permutation(its.size)]
        nh = max(1, int(round(frac * its.size)))
        hold.append(np.sort(its[:nh]))
        fold.append(np.sort(its[nh:]))

    def csr(lists):
        q = np.zeros(len(lists) + 1, np.int64)
        q[1:] = np.cumsum([x.size for x in lists])
        return q, (np.concatenate(lists) if lists else np.zeros(0)).astype(np.int32)

    fp, fi = csr(fold)
    hp, hi = csr(hold)
    return HoldoutSplit(train, users, fp, fi, hp, hi)
