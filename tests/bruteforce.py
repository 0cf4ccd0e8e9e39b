"""Brute-force checkers used to pin the oracle (independent of oracle/ and of the GPU library).

Everything here is written from the definitions in the paper, by brute force:
the loss of eq. 2 summed over every (u, i) pair, the closed-form iALS update of
eq. 3 solved with numpy.linalg.solve, and the scalar coordinate update of
eq. 5-6 (iCD, Alg. 2).  They are tiny-size tools, not fast code.
"""
from __future__ import annotations

import numpy as np


def coo_labels(p):
    n = p.user.size
    y = np.ones(n) if p.y is None else p.y.astype(np.float64)
    a = np.ones(n) if p.alpha is None else p.alpha.astype(np.float64)
    return y, a


def loss_allpairs(user, item, y, a, W, H, alpha0, lam):
    """eq. 2 term by term: observed term, alpha0 times the sum over all U x I pairs of
    yhat^2, and lambda times the squared Frobenius norms."""
    W = np.asarray(W, np.float64)
    H = np.asarray(H, np.float64)
    Y = W @ H.T  # every pair's prediction (eq. 1)
    obs = np.sum(a * (Y[user, item] - y) ** 2)
    allp = np.sum(Y * Y)
    reg = np.sum(W * W) + np.sum(H * H)
    return obs + alpha0 * allp + lam * reg


def ials_side_exact(rows, cols, y, a, X_other, n_rows, alpha0, lam):
    """eq. 3 for every row of one side: x_r = (sum a h h^T + alpha0 G + lam I)^-1 sum a y h."""
    d = X_other.shape[1]
    G = X_other.T @ X_other
    out = np.zeros((n_rows, d))
    for r in range(n_rows):
        m = rows == r
        Hs = X_other[cols[m]]
        A = (Hs.T * a[m]) @ Hs + alpha0 * G + lam * np.eye(d)
        rhs = Hs.T @ (a[m] * y[m])
        out[r] = np.linalg.solve(A, rhs)
    return out


def ials_epoch(user, item, y, a, W, H, alpha0, lam):
    """Alg. 1: users from eq. 3 against H, then items against the new W."""
    W = ials_side_exact(user, item, y, a, H, W.shape[0], alpha0, lam)
    H = ials_side_exact(item, user, y, a, W, H.shape[0], alpha0, lam)
    return W, H


def icd_epochs(user, item, y, a, W, H, alpha0, lam, T):
    """Alg. 2 with scheme (ii): dimension outer; users then items inside; scalar eq. 5-6."""
    W = np.array(W, np.float64)
    H = np.array(H, np.float64)
    U, d = W.shape
    I = H.shape[0]
    by_user = [np.nonzero(user == u)[0] for u in range(U)]
    by_item = [np.nonzero(item == i)[0] for i in range(I)]
    for _ in range(T):
        yhat = np.einsum("kf,kf->k", W[user], H[item])
        for f in range(d):
            gI = H.T @ H[:, f]
            for u in range(U):
                ks = by_user[u]
                hf = H[item[ks], f]
                num = np.sum(a[ks] * (yhat[ks] - y[ks]) * hf) + alpha0 * W[u] @ gI + lam * W[u, f]
                den = np.sum(a[ks] * hf * hf) + alpha0 * gI[f] + lam
                delta = num / den
                W[u, f] -= delta
                yhat[ks] -= delta * hf
            gU = W.T @ W[:, f]
            for i in range(I):
                ks = by_item[i]
                wf = W[user[ks], f]
                num = np.sum(a[ks] * (yhat[ks] - y[ks]) * wf) + alpha0 * H[i] @ gU + lam * H[i, f]
                den = np.sum(a[ks] * wf * wf) + alpha0 * gU[f] + lam
                delta = num / den
                H[i, f] -= delta
                yhat[ks] -= delta * wf
    return W, H


def foldin_exact(H, items, y, alpha0, lam):
    """eq. 3 for one new row against a fixed item table (weights 1)."""
    H = np.asarray(H, np.float64)
    d = H.shape[1]
    Hs = H[items]
    A = Hs.T @ Hs + alpha0 * (H.T @ H) + lam * np.eye(d)
    return np.linalg.solve(A, Hs.T @ y)
