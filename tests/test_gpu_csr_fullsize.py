"""The observation index at full size, bit for bit: user-major CSR, item-major CSR and perm
against numpy's lexsort (independent of the oracle and of the GPU radix sort).  The sort keys
are row * ncols + col: 32 bits on the ML20M-shaped matrix (4 radix passes of 8 bits) and 35 bits
on the MSD-shaped one (5 passes)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import gpu_trainer, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("workload", ["ml20m_like", "msd_like"])
def test_index_bit_exact_at_full_size(workload):
    p = synth.make_problem(workload)
    p.dim = p.block = 16  # the index does not depend on d; small tables keep the test light
    p.W0 = p.W0[:, :16].copy()
    p.H0 = p.H0[:, :16].copy()
    tr = gpu_trainer(p)
    uptr, ucol, _ = tr.csr(0)
    iptr, icol, perm = tr.csr(1)
    tr.close()
    say(f"{workload}: keys of {int(p.num_users * p.num_items - 1).bit_length()} bits, {p.nnz} observations")
    ou = np.lexsort((p.item, p.user))           # user-major: by user, then item
    oi = np.lexsort((p.user, p.item))           # item-major: by item, then user
    assert np.array_equal(uptr, np.concatenate([[0], np.cumsum(np.bincount(p.user, minlength=p.num_users))]))
    assert np.array_equal(ucol, p.item[ou])
    assert np.array_equal(iptr, np.concatenate([[0], np.cumsum(np.bincount(p.item, minlength=p.num_items))]))
    assert np.array_equal(icol, p.user[oi])
    pos = np.empty(p.nnz, np.int64)
    pos[ou] = np.arange(p.nnz)                  # user-major slot of every observation
    assert np.array_equal(perm, pos[oi])
