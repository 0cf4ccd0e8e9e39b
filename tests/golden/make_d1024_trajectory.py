"""Write the float64 oracle's trajectory on the ML20M-shaped matrix at d = 1024, b = 128.

The oracle (Alg. 3 in float64) needs minutes per epoch at this size, too long for a
test, so this script stores what the GPU tests compare against: the eq. 2 loss after
each of the first EPOCHS epochs and, after each epoch, the rows of W and H of a fixed
sample of users and items (the longest rows, whose Hessians are summed over segments,
and a seeded uniform sample).  It calls only the seeded input generator and the
oracle.  Run from the repository root:

    python tests/golden/make_d1024_trajectory.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

WORKLOAD = "ml20m_like_d1024"
EPOCHS = 3
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ml20m_like_d1024_oracle_trajectory.npz")


def sample_rows(lengths, n_long, n_rand, seed):
    rng = np.random.default_rng(seed)
    order = np.argsort(-lengths, kind="stable")
    rows = set(order[:n_long].tolist())
    rest = np.setdiff1d(np.arange(lengths.size), order[:n_long])
    rows.update(rng.choice(rest, size=n_rand, replace=False).tolist())
    return np.array(sorted(rows), np.int32)


def main():
    t0 = time.time()
    p = synth.make_problem(WORKLOAD)
    csr = oracle.build_csr(p.num_users, p.num_items, p.user, p.item)
    users = sample_rows(np.diff(csr.uptr), 24, 24, 11)
    items = sample_rows(np.diff(csr.iptr), 12, 12, 12)
    W, H = p.W0, p.H0
    Wr, Hr, losses = [], [], []
    for e in range(EPOCHS):
        W, H, _, L = oracle.epochs(csr, W, H, p.block, p.alpha0, p.lam, 1)
        Wr.append(W[users].copy())
        Hr.append(H[items].copy())
        losses.append(float(L[0]))
        print(f"epoch {e + 1}: loss {L[0]:.12e} at {time.time() - t0:.0f}s", flush=True)
    L0 = oracle.loss(csr, p.W0, p.H0, p.alpha0, p.lam)
    tmp = OUT + ".tmp.npz"
    np.savez_compressed(tmp, workload=np.array(WORKLOAD), dim=p.dim, block=p.block, alpha0=p.alpha0, lam=p.lam,
                        users=users, items=items, W_rows=np.stack(Wr), H_rows=np.stack(Hr),
                        loss=np.array(losses), loss0=L0)
    os.replace(tmp, OUT)
    print(f"wrote {OUT} in {time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
