"""The ML20M-shaped matrix at d = 1024, b = 128 (the wide-block kernels) against the float64
oracle's own trajectory, epoch by epoch, in both arithmetic forms.

A float64 epoch takes minutes at this size, so the oracle's trajectory was written once by
tests/golden/make_d1024_trajectory.py (seeded inputs and the oracle only): the eq. 2 loss after
each of the first epochs and, after each epoch, the rows of W and H of a fixed sample of users
and items (the longest rows, whose Hessians are summed over segments, and a uniform sample).
The GPU runs the same epochs from the same start and the errors are printed per epoch.

Bars: float32 -- the loss within 1e-6 of the oracle's after epoch 1 and within 1e-5 after
the later ones, the sampled rows within 1e-4 (Frobenius) and every sampled row within 1e-3
after epoch 1; bfloat16 (Hessian and Gramian products on bfloat16 operands) -- the loss within
1e-3 every epoch and the sampled rows within 3e-2 after epoch 1."""
import os

import numpy as np
import pytest

import synth
from paper_2110_14044_amd import binding
from tests.gpu_util import gpu_trainer, host, need_gpu, rel, row_rel_max, say

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "ml20m_like_d1024_oracle_trajectory.npz")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def case():
    g = dict(np.load(GOLDEN))
    p = synth.make_problem(str(g["workload"]))
    assert p.dim == int(g["dim"]) and p.block == int(g["block"])
    return p, g


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_d1024_epochs_against_the_oracle_trajectory(case, prec):
    p, g = case
    users, items = g["users"], g["items"]
    E = g["loss"].size
    tr = gpu_trainer(p, precision=binding.IALS_PREC_BF16 if prec == "bf16" else binding.IALS_PREC_FP32,
                     graph=True)
    L0 = tr.loss()[0]
    el0 = abs(L0 - float(g["loss0"])) / float(g["loss0"])
    rows = []
    for e in range(E):
        tr.epoch(1)
        L = tr.loss()[0]
        Wg = host(tr.W)[users]
        Hg = host(tr.H)[items]
        ew, eh = rel(Wg, g["W_rows"][e]), rel(Hg, g["H_rows"][e])
        rw, rh = row_rel_max(Wg, g["W_rows"][e]), row_rel_max(Hg, g["H_rows"][e])
        el = abs(L - g["loss"][e]) / g["loss"][e]
        rows.append((ew, eh, rw, rh, el))
        say(f"d1024 {prec} epoch {e + 1}: sampled W {ew:.2e} H {eh:.2e} (worst row {rw:.1e} / {rh:.1e}), "
            f"loss {el:.2e}")
    st = tr.stats()
    tr.close()
    say(f"d1024 {prec}: start loss {el0:.1e}, float64 redo on {st['fallback_rows']} rows")
    assert el0 < 1e-10
    ew, eh, rw, rh, el = rows[0]
    if prec == "fp32":
        assert ew < 1e-4 and eh < 1e-4 and rw < 1e-3 and rh < 1e-3 and el < 1e-6
        assert max(r[4] for r in rows) < 1e-5
    else:
        assert ew < 3e-2 and eh < 3e-2 and max(r[4] for r in rows) < 1e-3
