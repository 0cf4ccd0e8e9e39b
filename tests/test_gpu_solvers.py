"""The two ends of the block size (sec. 3 and 5.2.1): b = 1 runs scalar coordinate descent
(Alg. 2, iCD) and b = d solves every row against its dense normal equations (Alg. 1, iALS),
each through its own passes, against the oracle's b = 1 and b = d epochs (which are pinned to
independent transcriptions of Alg. 2 and of eq. 3 on the CPU).  Same bars as the block sweep:
float32 embeddings within 1e-4 (Frobenius), every row within 1e-3, the loss within 1e-6 after
one epoch."""
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2110_14044_amd import binding
from tests.gpu_util import gpu_trainer, host, need_gpu, oracle_setup, rel, row_rel_max, say
from tests.test_gpu_parity import _epoch_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _solver(p, **kw):
    tr = gpu_trainer(p, **kw)
    s = tr.stats()["solver"]
    tr.close()
    return s


@pytest.mark.parametrize("d", [1, 8, 33, 128, 300])
def test_icd_epochs(d):
    p = synth.small_problem(700 + d, 500, 300, 6000, d, 1, labels=True, std=0.1)
    assert _solver(p) == binding.IALS_SOLVER_ICD
    _epoch_check(p, 2, 1e-4, 1e-6)


def test_icd_long_rows_in_segments_and_graph():
    # most item rows exceed one segment of 256: their sums come from segment partials
    p = synth.small_problem(710, 3000, 120, 60_000, 24, 1, labels=True, zipf_s=0.8, std=0.1)
    st = _epoch_check(p, 1, 1e-4, 1e-6, seg_len=256)
    assert st["segments_item"] > 0
    st = _epoch_check(p, 2, 1e-4, 1e-6, graph=True)
    assert st["fallback_rows"] == 0


@pytest.mark.parametrize("d", [16, 48, 64, 128, 256])
def test_ials_epochs(d):
    p = synth.small_problem(720 + d, 500, 300, 8000, d, d, labels=True, std=0.1)
    assert _solver(p) == binding.IALS_SOLVER_IALS
    _epoch_check(p, 2, 1e-4, 1e-6)


def test_ials_long_rows_and_forced_float64():
    p = synth.small_problem(730, 3000, 400, 120_000, 64, 64, labels=True, zipf_s=0.8, std=0.1)
    st = _epoch_check(p, 1, 1e-4, 1e-6, seg_len=256)
    assert st["segments_item"] > 0
    st = _epoch_check(p, 1, 1e-4, 1e-6, chol_fallback_ratio=1.0)
    assert st["fallback_rows"] == p.num_users + p.num_items


def test_ials_single_pass_equals_eq3():
    """One user pass at b = d is eq. 3 for every user (numpy.linalg.solve on the dense normal
    equations, independent of the oracle)."""
    p = synth.small_problem(740, 400, 250, 5000, 32, 32, labels=True, std=0.1)
    tr = gpu_trainer(p)
    tr.block_sweep(0, 0)
    Wg = host(tr.W)
    tr.close()
    csr, ys, as_ = oracle_setup(p)
    H = p.H0.astype(np.float64)
    A0 = p.alpha0 * H.T @ H + p.lam * np.eye(p.dim)
    W = np.zeros((p.num_users, p.dim))
    for u in range(p.num_users):
        lo, hi = csr.uptr[u], csr.uptr[u + 1]
        Hu = H[csr.ucol[lo:hi]]
        a = as_[lo:hi].astype(np.float64)
        y = ys[lo:hi].astype(np.float64)
        W[u] = np.linalg.solve(A0 + (Hu * a[:, None]).T @ Hu, Hu.T @ (a * y))
    e, er = rel(Wg, W), row_rel_max(Wg, W)
    say(f"b = d user pass vs eq. 3: {e:.2e}, worst row {er:.1e}")
    assert e < 1e-4 and er < 1e-3


def test_icd_ml20m_like_full_size_epoch():
    """ML20M-shaped workload at b = 1 (d = 128): one epoch of coordinate descent (256 passes) in
    the benchmark's launch configuration (the epoch graph) against the oracle's b = 1 epoch."""
    p = synth.make_problem("ml20m_like")
    p.block = 1
    tr = gpu_trainer(p, graph=True)
    tr.epoch(1)
    L, _ = tr.loss()
    Wg, Hg = host(tr.W), host(tr.H)
    tr.close()
    csr, _, _ = oracle_setup(p)
    t = time.time()
    W, H, _, losses = oracle.epochs(csr, p.W0, p.H0, 1, p.alpha0, p.lam, 1)
    ew, eh, el = rel(Wg, W), rel(Hg, H), abs(L - losses[0]) / losses[0]
    rw, rh = row_rel_max(Wg, W), row_rel_max(Hg, H)
    say(f"ml20m_like b=1 epoch 1: W {ew:.2e} H {eh:.2e} loss {el:.2e}; worst row W {rw:.1e} H {rh:.1e} "
        f"(oracle {time.time() - t:.1f}s)")
    assert ew < 1e-4 and eh < 1e-4 and el < 1e-6 and rw < 1e-3 and rh < 1e-3
