"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def row_rel_max(a, b):
    """Worst per-row relative error max_r |a_r - b_r| / |b_r| (2-norms over each row): a few wrong
    rows among many can hide under the Frobenius ratio, never under this one.  Rows whose
    reference is (nearly) zero -- rows without observations end at 0 up to rounding -- are
    measured against 1e-3 of the root-mean-square row norm instead."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if a.size == 0:
        return 0.0
    num = np.linalg.norm(a - b, axis=1)
    nb = np.linalg.norm(b, axis=1)
    floor = max(1e-3 * float(np.sqrt(np.mean(nb * nb))), 1e-30)
    return float((num / np.maximum(nb, floor)).max())


def gpu_trainer(p, **kw):
    from paper_2110_14044_amd import Trainer
    return Trainer(p, **kw)


def oracle_setup(p):
    import oracle
    csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
    ys = None if p.y is None else oracle.to_slot_order(csr, p.y)
    as_ = None if p.alpha is None else oracle.to_slot_order(csr, p.alpha)
    return csr, ys, as_


def host(t):
    return t.detach().cpu().numpy()
