"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one oracle function to something other than itself: a library
routine (numpy lexsort, einsum, matmul), the all-pairs brute-force loss of eq. 2,
scipy minimisation of that loss over one block, central finite differences,
the closed form of eq. 3 (Alg. 1 is iALS++ with b = d), the scalar update of
eq. 5-6 (Alg. 2 is iALS++ with b = 1) and monotonicity of block coordinate descent.
"""
import numpy as np
import pytest
from scipy import optimize

import oracle
import synth
from tests import bruteforce as bf


def _problem(seed, U, I, nnz, d, b, labels, **kw):
    return synth.small_problem(seed, U, I, nnz, d, b, labels=labels, **kw)


def _setup(p):
    csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
    y, a = bf.coo_labels(p)
    ys = None if p.y is None else oracle.to_slot_order(csr, p.y)
    as_ = None if p.alpha is None else oracle.to_slot_order(csr, p.alpha)
    return csr, y, a, ys, as_


# ---------------------------------------------------------------- index (a1)

def test_csr_matches_lexsort(oracle_lib):
    p = synth.make_problem("tiny")
    csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
    o = np.lexsort((p.item, p.user))
    assert np.array_equal(csr.ucol, p.item[o])
    assert np.array_equal(csr.usrc, o)
    assert np.array_equal(csr.uptr, np.concatenate([[0], np.cumsum(np.bincount(p.user, minlength=p.num_users))]))
    oi = np.lexsort((p.user, p.item))
    assert np.array_equal(csr.icol, p.user[oi])
    assert np.array_equal(csr.iptr, np.concatenate([[0], np.cumsum(np.bincount(p.item, minlength=p.num_items))]))
    # perm is a bijection item-slot -> user-slot holding the same observation
    assert np.array_equal(np.sort(csr.perm), np.arange(p.nnz))
    assert np.array_equal(csr.usrc[csr.perm], oi)
    assert csr.uptr[-1] == p.nnz and csr.iptr[-1] == p.nnz


def test_csr_rejects_bad_input(oracle_lib):
    with pytest.raises(ValueError):
        oracle.build_csr(3, 3, np.array([0, 1, 0], np.int32), np.array([1, 2, 1], np.int32))  # duplicate
    with pytest.raises(ValueError):
        oracle.build_csr(3, 3, np.array([0, 3], np.int32), np.array([1, 2], np.int32))  # user id out of range
    with pytest.raises(ValueError):
        oracle.build_csr(3, 3, np.array([0, 1], np.int32), np.array([-1, 2], np.int32))


def test_csr_empty(oracle_lib):
    csr = oracle.build_csr(4, 3, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert np.array_equal(csr.uptr, np.zeros(5, np.int64))
    assert np.array_equal(csr.iptr, np.zeros(4, np.int64))
    assert csr.perm.size == 0


# ---------------------------------------------------------------- eq. 1, 4, 7, 2

def test_predict_and_gramian_match_library(oracle_lib):
    p = _problem(1, 40, 30, 300, 12, 5, labels=False)
    csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
    W, H = p.W0.astype(np.float64), p.H0.astype(np.float64)
    users_sorted = np.repeat(np.arange(p.num_users), np.diff(csr.uptr))
    ref = np.einsum("kf,kf->k", W[users_sorted], H[csr.ucol])
    assert np.allclose(oracle.predict(csr, W, H), ref, rtol=1e-13, atol=1e-15)
    for p0, bw in [(0, 12), (0, 5), (5, 5), (10, 2)]:
        G = oracle.gramian(H, p0, bw)
        assert np.allclose(G, H.T @ H[:, p0:p0 + bw], rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("labels", [False, True])
def test_loss_equals_allpairs_sum(oracle_lib, labels):
    p = _problem(2, 30, 25, 200, 6, 3, labels=labels)
    csr, y, a, ys, as_ = _setup(p)
    ref = bf.loss_allpairs(p.user, p.item, y, a, p.W0, p.H0, p.alpha0, p.lam)
    got = oracle.loss(csr, p.W0, p.H0, p.alpha0, p.lam, ys, as_)
    assert abs(got - ref) <= 1e-12 * abs(ref)


# ---------------------------------------------------------------- one block step (sec. 4)

def _central_grad(f, z, h=1e-3):
    """Central differences; exact up to rounding for the quadratic loss of eq. 2 in one block."""
    g = np.zeros_like(z)
    for j in range(z.size):
        e = np.zeros_like(z)
        e[j] = h
        g[j] = (f(z + e) - f(z - e)) / (2 * h)
    return g


def _minimise(f, z0):
    res = optimize.minimize(f, z0, jac=lambda z: _central_grad(f, z), method="BFGS",
                            options={"gtol": 1e-12})
    return res.x


def _block_minimiser_check(p, p0, bw):
    csr, y, a, ys, as_ = _setup(p)
    W = p.W0.astype(np.float64).copy()
    H = p.H0.astype(np.float64).copy()
    yhat = oracle.predict(csr, W, H)
    Wold = W.copy()
    assert oracle.block_pass(csr, "user", p0, bw, p.alpha0, p.lam, W, H, yhat,
                             oracle.gramian(H, p0, bw), ys, as_) == 0
    L = lambda W_, H_: bf.loss_allpairs(p.user, p.item, y, a, W_, H_, p.alpha0, p.lam)
    for u in range(p.num_users):
        def f(z, u=u):
            Wt = Wold.copy()
            Wt[u, p0:p0 + bw] = z
            return L(Wt, H)
        x = _minimise(f, Wold[u, p0:p0 + bw])
        assert np.allclose(W[u, p0:p0 + bw], x, atol=1e-7), (u, W[u, p0:p0 + bw], x)
    # item side against the updated W
    Hold = H.copy()
    assert oracle.block_pass(csr, "item", p0, bw, p.alpha0, p.lam, W, H, yhat,
                             oracle.gramian(W, p0, bw), ys, as_) == 0
    for i in range(p.num_items):
        def g(z, i=i):
            Ht = Hold.copy()
            Ht[i, p0:p0 + bw] = z
            return L(W, Ht)
        x = _minimise(g, Hold[i, p0:p0 + bw])
        assert np.allclose(H[i, p0:p0 + bw], x, atol=1e-7), (i, H[i, p0:p0 + bw], x)
    # the cached predictions stay equal to fresh ones (delta update of sec. 3.3 / Alg. 3)
    assert np.allclose(yhat, oracle.predict(csr, W, H), atol=1e-12)


@pytest.mark.parametrize("b", [1, 2, 4])
@pytest.mark.parametrize("labels", [False, True])
def test_block_step_is_scipy_minimiser_5x4(oracle_lib, b, labels):
    p = _problem(10 + b, 5, 4, 10, 4, b, labels=labels)
    for p0 in range(0, 4, b):
        _block_minimiser_check(p, p0, b)


def test_block_step_ragged_last_block_and_empty_rows(oracle_lib):
    # d = 6, b = 4: blocks [0,4) and [4,6); 8 users but 5 observations -> empty rows
    p = _problem(21, 8, 4, 5, 6, 4, labels=True)
    assert np.bincount(p.user, minlength=8).min() == 0
    _block_minimiser_check(p, 0, 4)
    _block_minimiser_check(p, 4, 2)


def test_block_gradient_vanishes_after_step(oracle_lib):
    p = _problem(3, 12, 9, 40, 6, 3, labels=True)
    csr, y, a, ys, as_ = _setup(p)
    W = p.W0.astype(np.float64).copy()
    H = p.H0.astype(np.float64).copy()
    yhat = oracle.predict(csr, W, H)
    p0, bw = 3, 3
    oracle.block_pass(csr, "user", p0, bw, p.alpha0, p.lam, W, H, yhat, oracle.gramian(H, p0, bw), ys, as_)
    h = 1e-4
    for u in range(p.num_users):
        for q in range(p0, p0 + bw):
            Wp, Wm = W.copy(), W.copy()
            Wp[u, q] += h
            Wm[u, q] -= h
            grad = (bf.loss_allpairs(p.user, p.item, y, a, Wp, H, p.alpha0, p.lam)
                    - bf.loss_allpairs(p.user, p.item, y, a, Wm, H, p.alpha0, p.lam)) / (2 * h)
            assert abs(grad) < 1e-8, (u, q, grad)


def test_loss_never_increases_over_passes(oracle_lib):
    p = _problem(4, 60, 40, 500, 8, 3, labels=True)
    csr, y, a, ys, as_ = _setup(p)
    W = p.W0.astype(np.float64).copy()
    H = p.H0.astype(np.float64).copy()
    Lprev = oracle.loss(csr, W, H, p.alpha0, p.lam, ys, as_)
    for t in range(3):
        yhat = oracle.predict(csr, W, H)
        for p0 in range(0, 8, 3):
            bw = min(3, 8 - p0)
            for side in ("user", "item"):
                G = oracle.gramian(H if side == "user" else W, p0, bw)
                oracle.block_pass(csr, side, p0, bw, p.alpha0, p.lam, W, H, yhat, G, ys, as_)
                L = oracle.loss(csr, W, H, p.alpha0, p.lam, ys, as_)
                assert L <= Lprev * (1 + 1e-12), (t, p0, side, L, Lprev)
                Lprev = L


# ---------------------------------------------------------------- special cases b = d and b = 1

@pytest.mark.parametrize("labels", [False, True])
def test_full_block_equals_ials_alg1(oracle_lib, labels):
    p = _problem(5, 50, 30, 400, 6, 6, labels=labels)
    csr, y, a, ys, as_ = _setup(p)
    W, H, _, _ = oracle.epochs(csr, p.W0, p.H0, 6, p.alpha0, p.lam, 1, ys, as_)
    Wr, Hr = bf.ials_epoch(p.user, p.item, y, a, p.W0.astype(np.float64), p.H0.astype(np.float64),
                           p.alpha0, p.lam)
    assert np.linalg.norm(W - Wr) <= 1e-10 * np.linalg.norm(Wr)
    assert np.linalg.norm(H - Hr) <= 1e-10 * np.linalg.norm(Hr)


@pytest.mark.parametrize("labels", [False, True])
def test_unit_block_equals_icd_alg2(oracle_lib, labels):
    p = _problem(6, 30, 20, 150, 4, 1, labels=labels)
    csr, y, a, ys, as_ = _setup(p)
    W, H, _, _ = oracle.epochs(csr, p.W0, p.H0, 1, p.alpha0, p.lam, 2, ys, as_)
    Wr, Hr = bf.icd_epochs(p.user, p.item, y, a, p.W0, p.H0, p.alpha0, p.lam, 2)
    assert np.linalg.norm(W - Wr) <= 1e-10 * np.linalg.norm(Wr)
    assert np.linalg.norm(H - Hr) <= 1e-10 * np.linalg.norm(Hr)


def test_epochs_loss_matches_allpairs_and_decreases(oracle_lib):
    p = synth.make_problem("tiny")
    csr, y, a, ys, as_ = _setup(p)
    W, H, yhat, losses = oracle.epochs(csr, p.W0, p.H0, p.block, p.alpha0, p.lam, 2)
    assert np.all(np.diff(losses) < 0)
    ref = bf.loss_allpairs(p.user, p.item, y, a, W, H, p.alpha0, p.lam)
    assert abs(losses[-1] - ref) <= 1e-11 * ref
    assert np.allclose(yhat, oracle.predict(csr, W, H), atol=1e-12)


# ---------------------------------------------------------------- fold-in

def test_foldin_limits(oracle_lib):
    rng = np.random.default_rng(7)
    I, d = 60, 8
    H = rng.normal(0, 0.3, size=(I, d))
    ptr = np.array([0, 5, 5, 17, 18], np.int64)  # includes an empty history
    items = np.concatenate([rng.choice(I, 5, replace=False), rng.choice(I, 12, replace=False),
                            rng.choice(I, 1)]).astype(np.int32)
    y = rng.uniform(0.5, 1.5, size=items.size)
    alpha0, lam = 0.1, 0.05
    exact = np.stack([bf.foldin_exact(H, items[ptr[r]:ptr[r + 1]], y[ptr[r]:ptr[r + 1]], alpha0, lam)
                      for r in range(4)])
    # b = d and one sweep: exactly eq. 3
    w1 = oracle.foldin(H, d, alpha0, lam, ptr, items, 1, y)
    assert np.allclose(w1, exact, rtol=1e-10, atol=1e-12)
    # b < d: block coordinate descent on a strongly convex quadratic converges to eq. 3,
    # and the row objective never increases from one sweep to the next
    def obj(w, r):
        hs = H[items[ptr[r]:ptr[r + 1]]]
        return np.sum((hs @ w - y[ptr[r]:ptr[r + 1]]) ** 2) + alpha0 * w @ (H.T @ H) @ w + lam * w @ w
    prev = [obj(np.zeros(d), r) for r in range(4)]
    for passes in (1, 2, 3, 5):
        w = oracle.foldin(H, 3, alpha0, lam, ptr, items, passes, y)
        cur = [obj(w[r], r) for r in range(4)]
        assert all(c <= pv * (1 + 1e-12) + 1e-15 for c, pv in zip(cur, prev))
        prev = cur
    w = oracle.foldin(H, 3, alpha0, lam, ptr, items, 400, y)
    assert np.allclose(w, exact, rtol=1e-8, atol=1e-10)


def test_pass_rows_equals_the_full_pass_on_those_rows(oracle_lib):
    """Rows are independent within a pass (sec. 3.2): the sampled-rows pass gives each listed row
    exactly the full pass's block step and leaves every other row alone."""
    import synth
    p = synth.small_problem(17, 60, 40, 700, 12, 5, labels=True, alpha0=0.2, lam=0.07)
    csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
    ys, as_ = oracle.to_slot_order(csr, p.y), oracle.to_slot_order(csr, p.alpha)
    rng = np.random.default_rng(3)
    for side, n in (("user", p.num_users), ("item", p.num_items)):
        W, H = p.W0.astype(np.float64), p.H0.astype(np.float64)
        yhat = oracle.predict(csr, W, H)
        G = oracle.gramian(H if side == "user" else W, 5, 5)
        Wf, Hf, yf = W.copy(), H.copy(), yhat.copy()
        oracle.block_pass(csr, side, 5, 5, p.alpha0, p.lam, Wf, Hf, yf, G, ys, as_)
        rows = rng.choice(n, size=n // 3, replace=False)
        Ws, Hs, ysamp = W.copy(), H.copy(), yhat.copy()
        oracle.pass_rows(csr, side, rows, 5, 5, p.alpha0, p.lam, Ws, Hs, ysamp, G, ys, as_)
        full, samp, orig = (Wf, Ws, W) if side == "user" else (Hf, Hs, H)
        assert np.array_equal(samp[rows], full[rows])
        rest = np.setdiff1d(np.arange(n), rows)
        assert np.array_equal(samp[rest], orig[rest])


# ---------------------------------------------------------------- the epoch schedule (Alg. 3)

def _scipy_epochs(p, n_epochs):
    """Alg. 3's schedule written out with every block step taken by scipy: for each epoch, for
    each block of the partition (contiguous, ascending, the last one shorter), every user's
    block minimises the brute-force loss of eq. 2 with everything else fixed, then every item's
    block does, against the users just updated.  Rows of one side are independent given the
    other side (sec. 3.2), so they are minimised one by one from the state at the start of the
    side's pass.  Returns the iterates and the brute-force loss after each epoch."""
    y, a = bf.coo_labels(p)
    W = p.W0.astype(np.float64).copy()
    H = p.H0.astype(np.float64).copy()
    L = lambda W_, H_: bf.loss_allpairs(p.user, p.item, y, a, W_, H_, p.alpha0, p.lam)
    d, b = p.dim, p.block
    losses = []
    for _ in range(n_epochs):
        for p0 in range(0, d, b):
            bw = min(b, d - p0)
            Wstart = W.copy()
            for u in range(p.num_users):
                def f(z, u=u):
                    Wt = Wstart.copy()
                    Wt[u, p0:p0 + bw] = z
                    return L(Wt, H)
                W[u, p0:p0 + bw] = _minimise(f, Wstart[u, p0:p0 + bw])
            Hstart = H.copy()
            for i in range(p.num_items):
                def g(z, i=i):
                    Ht = Hstart.copy()
                    Ht[i, p0:p0 + bw] = z
                    return L(W, Ht)
                H[i, p0:p0 + bw] = _minimise(g, Hstart[i, p0:p0 + bw])
        losses.append(L(W, H))
    return W, H, np.array(losses)


@pytest.mark.parametrize("d,b,epochs", [(6, 4, 1), (7, 3, 2)])
def test_epoch_schedule_with_ragged_block_equals_scipy_block_minimisation(oracle_lib, d, b, epochs):
    """oracle.epochs for b not dividing d (one ragged block; with d = 7, b = 3 three blocks,
    the last of width 1) against the schedule of Alg. 3 carried out by scipy block minimisers
    of the brute-force loss: a wrong block order, a stale Gramian, a wrong width of the
    ragged block or a skipped pass would move the iterates (each planted in a copy of the
    oracle fails this test)."""
    p = _problem(40 + d, 5, 4, 12, d, b, labels=True)
    csr, y, a, ys, as_ = _setup(p)
    W, H, _, losses = oracle.epochs(csr, p.W0, p.H0, b, p.alpha0, p.lam, epochs, ys, as_)
    Wr, Hr, Lr = _scipy_epochs(p, epochs)
    assert np.allclose(W, Wr, atol=1e-7), np.abs(W - Wr).max()
    assert np.allclose(H, Hr, atol=1e-7), np.abs(H - Hr).max()
    assert np.allclose(losses, Lr, rtol=1e-12)
