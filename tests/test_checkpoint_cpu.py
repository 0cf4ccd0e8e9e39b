"""Checkpoint format and the resume property of the method, on the CPU.

At an epoch boundary the state of Alg. 3 is W, H, the epoch count and the configuration: the
predictions are recomputed at the start of every epoch and the Gramians in every pass.  The
oracle therefore continues from a saved (W, H) exactly as if it had not stopped, and the
checkpoint file must hold those tables bit for bit and refuse other data or settings.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2110_14044_amd import checkpoint
from tests.gpu_util import oracle_setup

CFG = dict(num_users=0, num_items=0, dim=0, block=0, alpha0=0.1, lam=0.1, precision=0, chol_fallback_ratio=0.0,
           deal="auto", seg_len=0, gram_split=0)


def _cfg(p, **kw):
    c = dict(CFG, num_users=p.num_users, num_items=p.num_items, dim=p.dim, block=p.block, alpha0=float(p.alpha0),
             lam=float(p.lam))
    c.update(kw)
    return c


@pytest.mark.parametrize("d,b", [(8, 3), (12, 12), (6, 1)])
def test_oracle_resumes_exactly_at_an_epoch_boundary(d, b):
    p = synth.small_problem(300 + d + b, 40, 30, 400, d, b, labels=True)
    csr, ys, as_ = oracle_setup(p)
    W4, H4, _, L4 = oracle.epochs(csr, p.W0, p.H0, b, p.alpha0, p.lam, 4, ys, as_)
    W2, H2, _, L2 = oracle.epochs(csr, p.W0, p.H0, b, p.alpha0, p.lam, 2, ys, as_)
    Wr, Hr, _, Lr = oracle.epochs(csr, W2, H2, b, p.alpha0, p.lam, 2, ys, as_)
    assert np.array_equal(W4, Wr) and np.array_equal(H4, Hr)
    assert np.array_equal(L4[:2], L2) and np.array_equal(L4[2:], Lr)


def test_round_trip_is_bitwise(tmp_path):
    p = synth.small_problem(310, 50, 20, 300, 16, 8, labels=True)
    rng = np.random.default_rng(0)
    W = rng.standard_normal((p.num_users, p.dim)).astype(np.float32)
    H = rng.standard_normal((p.num_items, p.dim)).astype(np.float32)
    W[3, 5] = np.float32(1e-40)  # a subnormal survives too
    path = str(tmp_path / "ck.npz")
    fp = checkpoint.data_fingerprint(p)
    checkpoint.save(path, W, H, 7, _cfg(p), fp)
    W2, H2, meta = checkpoint.load(path, _cfg(p), fp)
    assert W2.tobytes() == W.tobytes() and H2.tobytes() == H.tobytes()
    assert meta["epochs_done"] == 7 and meta["data_sha256"] == fp


def test_refuses_other_data_settings_and_shapes(tmp_path):
    p = synth.small_problem(320, 50, 20, 300, 16, 8, labels=True)
    path = str(tmp_path / "ck.npz")
    checkpoint.save(path, p.W0, p.H0, 2, _cfg(p), checkpoint.data_fingerprint(p))
    with pytest.raises(ValueError, match="block"):
        checkpoint.load(path, _cfg(p, block=4))
    with pytest.raises(ValueError, match="precision"):
        checkpoint.load(path, _cfg(p, precision=1))
    q = synth.small_problem(321, 50, 20, 300, 16, 8, labels=True)
    assert checkpoint.data_fingerprint(q) != checkpoint.data_fingerprint(p)
    with pytest.raises(ValueError, match="different observations"):
        checkpoint.load(path, _cfg(p), checkpoint.data_fingerprint(q))
    bad = str(tmp_path / "bad.npz")
    checkpoint.save(bad, p.W0[:-1], p.H0, 2, _cfg(p), checkpoint.data_fingerprint(p))
    with pytest.raises(ValueError, match="shapes"):
        checkpoint.load(bad)
    np.savez(str(tmp_path / "other.npz"), x=np.zeros(3))
    with pytest.raises(ValueError, match="not a checkpoint"):
        checkpoint.load(str(tmp_path / "other.npz"))


def test_kernel_record():
    read = {"rows_user": (3.0, 3), "predict": (0.5, 1), "gram_item": (0.0, 0)}
    assert checkpoint.kernel_record(read) == {"rows_user": {"ms": 3.0, "launches": 3},
                                              "predict": {"ms": 0.5, "launches": 1}}
