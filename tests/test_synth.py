"""The seeded input generators: determinism and the realised statistics of the recipe."""
import numpy as np

import synth


def test_tiny_workload_is_deterministic_and_exact():
    a = synth.make_problem("tiny")
    b = synth.make_problem("tiny")
    assert np.array_equal(a.user, b.user) and np.array_equal(a.item, b.item)
    assert np.array_equal(a.W0, b.W0) and np.array_equal(a.H0, b.H0)
    assert a.nnz == 50_000
    n = np.bincount(a.user, minlength=a.num_users)
    assert n.min() >= 1 and n.max() <= 200
    key = a.user.astype(np.int64) * a.num_items + a.item
    assert np.unique(key).size == a.nnz  # distinct (u, i) pairs
    assert a.W0.dtype == np.float32 and a.W0.shape == (2_000, 16)
    assert abs(a.W0.std() - 0.1 / 4) < 0.002


def test_user_lengths_rescaled_to_exact_total():
    rng = np.random.default_rng(0)
    n = synth.user_lengths(rng, 1000, 60_000, 3.0, 1.0, 1, 500)
    assert n.sum() == 60_000 and n.min() >= 1 and n.max() <= 500


def test_zipf_head_is_most_popular():
    rng = np.random.default_rng(1)
    lengths = np.full(2000, 20)
    u, r = synth.sample_histories(rng, lengths, 500, 1.0)
    counts = np.bincount(r, minlength=500)
    assert counts[0] == counts.max()
    assert counts[:10].sum() > counts[-100:].sum()
    assert np.unique(u.astype(np.int64) * 500 + r).size == u.size


def test_serving_requests_shape():
    ptr, items = synth.serving_requests(3, 200, num_items=1000, hi=300)
    n = np.diff(ptr)
    assert n.min() >= 1 and n.max() <= 300 and ptr[-1] == items.size
    for r in range(200):
        seg = items[ptr[r]:ptr[r + 1]]
        assert np.unique(seg).size == seg.size
    t = synth.poisson_arrivals(4, 1000, 500.0)
    assert np.all(np.diff(t) > 0) and 1.5 < t[-1] < 2.5


def test_holdout_split_partitions_the_held_out_users():
    p = synth.small_problem(3, 500, 300, 8000, 16, 8)
    s = synth.holdout_split(p, 50)
    assert s.users.size == 50 and np.all(np.diff(s.users) > 0)
    assert s.train.nnz + s.fold_ptr[-1] + s.hold_ptr[-1] == p.nnz
    assert not np.isin(s.train.user, s.users).any()
    for j, u in enumerate(s.users):
        own = np.sort(p.item[p.user == u])
        f = s.fold_idx[s.fold_ptr[j]:s.fold_ptr[j + 1]]
        h = s.hold_idx[s.hold_ptr[j]:s.hold_ptr[j + 1]]
        assert h.size >= 1 and np.all(np.diff(f) > 0) and np.all(np.diff(h) > 0)
        assert np.array_equal(np.sort(np.concatenate([f, h])), own)
        assert h.size == max(1, round(0.2 * own.size))
