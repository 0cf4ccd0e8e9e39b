"""ials_rank_topk_noalloc (the top-k entry point that allocates nothing: its score buffer is a
fixed device array) against ials_rank_topk on the same inputs, through the C ABI: two calls in
a row, the second with a smaller input; ids and scores bit for bit (the same kernels compute
every score with the same arithmetic whatever the batch), and a request whose single row of
scores exceeds the fixed buffer is refused before any device work."""
import numpy as np
import pytest

from paper_2110_14044_amd import IalsError, binding

pytestmark = pytest.mark.gpu


def _inputs(seed, U, I, d, with_excl):
    import torch
    rng = np.random.default_rng(seed)
    W = torch.from_numpy(rng.standard_normal((U, d)).astype(np.float32)).cuda()
    H = torch.from_numpy(rng.standard_normal((I, d)).astype(np.float32)).cuda()
    ep = ei = None
    if with_excl:
        n = rng.integers(0, 40, size=U)
        ptr = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
        idx = np.concatenate([np.sort(rng.choice(I, size=m, replace=False)) for m in n]).astype(np.int32)
        ep = torch.from_numpy(ptr).cuda()
        ei = torch.from_numpy(idx if idx.size else np.zeros(1, np.int32)).cuda()
    return W, H, ep, ei


def _both(W, H, ep, ei, k):
    import torch
    U, d = W.shape
    I = H.shape[0]
    st = torch.cuda.current_stream()
    ids_a = torch.full((U, k), -7, dtype=torch.int32, device="cuda")
    sc_a = torch.zeros((U, k), dtype=torch.float32, device="cuda")
    ids_b = torch.full((U, k), -9, dtype=torch.int32, device="cuda")
    sc_b = torch.ones((U, k), dtype=torch.float32, device="cuda")
    binding.ials_rank_topk(W, U, H, I, d, ep, ei, k, ids_a, sc_a, 0, st)
    binding.ials_rank_topk_noalloc(W, U, H, I, d, ep, ei, k, ids_b, sc_b, st)
    torch.cuda.synchronize()
    return ids_a.cpu().numpy(), sc_a.cpu().numpy(), ids_b.cpu().numpy(), sc_b.cpu().numpy()


def test_noalloc_topk_matches_the_allocating_entry_point_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # first call: 20,000 items (80 KB of scores per user), 3,000 users: 4 batches of the
    # 64 MiB scratch; exclusions; second call smaller, without exclusions (the scratch keeps
    # the first call's scores, which the second must not see)
    for seed, U, I, d, k, excl in ((1, 3000, 20_000, 64, 100, True), (2, 257, 777, 16, 10, False)):
        W, H, ep, ei = _inputs(seed, U, I, d, excl)
        ia, sa, ib, sb = _both(W, H, ep, ei, k)
        print(f"no-alloc top-k U={U} I={I} d={d} k={k}: ids equal {np.array_equal(ia, ib)}, "
              f"scores equal {np.array_equal(sa, sb)}", flush=True)
        assert np.array_equal(ia, ib)
        assert np.array_equal(sa, sb)
        assert (ia >= 0).all() and (ia < I).all()


def test_noalloc_topk_rejects_rows_beyond_the_scratch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    W = torch.zeros((4, 16), dtype=torch.float32, device="cuda")
    H = torch.zeros((4, 16), dtype=torch.float32, device="cuda")
    ids = torch.zeros((4, 8), dtype=torch.int32, device="cuda")
    with pytest.raises(IalsError, match="IALS_E_INVALID") as ei:
        # 20M items need 80 MB of scores per user, more than the 64 MiB scratch (refused
        # before any access to H)
        binding.ials_rank_topk_noalloc(W, 4, H, 20_000_000, 16, None, None, 8, ids, None, None)
    assert "scratch" in str(ei.value)
