"""Full-size workloads too large for a float64 pass, checked on sampled rows.

Rows are independent within a pass (sec. 3.2), so the oracle can recompute any
row's block step alone (oracle.pass_rows) from the state the GPU pass started
from.  One user pass and one item pass of block 0 run on the GPU in the launch
configuration the benchmark uses; 2,000 users and 400 items are recomputed (the
longest rows, which go through the segment kernels, plus a uniform sample).  The
item rows are recomputed from the GPU's own state after its user pass.
Tolerance: 1e-4 relative (Frobenius over the sampled rows), as for whole
matrices; each sampled row within 1e-3.
"""
import time

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import gpu_trainer, host, need_gpu, oracle_setup, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _sample(lengths, n_long, n_rand, seed):
    rng = np.random.default_rng(seed)
    order = np.argsort(-lengths, kind="stable")
    rows = set(order[:n_long].tolist())
    rows.update(rng.choice(lengths.size, size=n_rand, replace=False).tolist())
    return np.array(sorted(rows), np.int32)


def _row_errors(got, ref):
    num = np.linalg.norm(got.astype(np.float64) - ref, axis=1)
    den = np.maximum(np.linalg.norm(ref, axis=1), 1e-30)
    return rel(got, ref), float((num / den).max())


@pytest.mark.parametrize("workload,block", [("msd_like", 64), ("ml20m_like_d1024", 128)])
def test_full_size_block_passes_on_sampled_rows(workload, block):
    t0 = time.time()
    p = synth.make_problem(workload)
    p.block = block
    say(f"{workload}: generated in {time.time() - t0:.0f}s")
    tr = gpu_trainer(p)
    csr, _, _ = oracle_setup(p)
    W0 = p.W0.astype(np.float64)
    H0 = p.H0.astype(np.float64)
    yhat = oracle.predict(csr, W0, H0)
    say(f"{workload}: oracle predictions done at {time.time() - t0:.0f}s")
    G = oracle.gramian(H0, 0, block)
    tr.block_sweep(0, 0)
    Wg = host(tr.W)
    users = _sample(np.diff(csr.uptr), 200, 1800, 1)
    W = W0.copy()
    oracle.pass_rows(csr, "user", users, 0, block, p.alpha0, p.lam, W, H0, yhat, G)
    e, emax = _row_errors(Wg[users], W[users])
    say(f"{workload} b={block}: user pass, {users.size} sampled users: {e:.2e} (worst row {emax:.1e}) "
        f"at {time.time() - t0:.0f}s")
    assert e < 1e-4 and emax < 1e-3
    del W, W0
    # the item pass from the GPU's state after its user pass
    yh = tr.predictions().astype(np.float64)
    Wg64 = Wg.astype(np.float64)
    G2 = oracle.gramian(Wg64, 0, block)
    Hg0 = host(tr.H).astype(np.float64)
    tr.block_sweep(1, 0)
    Hg = host(tr.H)
    tr.close()
    items = _sample(np.diff(csr.iptr), 100, 300, 2)
    H = Hg0.copy()
    oracle.pass_rows(csr, "item", items, 0, block, p.alpha0, p.lam, Wg64, H, yh, G2)
    e, emax = _row_errors(Hg[items], H[items])
    say(f"{workload} b={block}: item pass, {items.size} sampled items: {e:.2e} (worst row {emax:.1e}) "
        f"at {time.time() - t0:.0f}s")
    assert e < 1e-4 and emax < 1e-3
