"""Checkpoints at an epoch boundary and per-epoch metrics records.

Every epoch starts by recomputing the predictions from W and H, and every pass recomputes its
Gramian slab from the current tables (Alg. 3), so the whole training state at an epoch boundary
is W, H, the number of epochs done and the configuration.  A checkpoint stores exactly that,
with a fingerprint of the observations, so that a resumed run on the same data and device
repeats the uninterrupted run bit for bit (the kernels are deterministic).

The file is a plain ``.npz`` (no pickled objects): W and H as float32 arrays and the metadata
as one JSON string.
"""
from __future__ import annotations

import hashlib
import json
from typing import Optional

import numpy as np

FORMAT = "ials-checkpoint-1"
# configuration fields a resumed run must share with the saved one
CONFIG_KEYS = ("num_users", "num_items", "dim", "block", "alpha0", "lam", "precision", "chol_fallback_ratio",
               "deal", "seg_len", "gram_split")


def data_fingerprint(problem) -> str:
    """sha256 over the observation arrays (ids, labels and weights) in their given order."""
    h = hashlib.sha256()
    for name in ("user", "item", "y", "alpha"):
        a = getattr(problem, name)
        h.update(name.encode())
        if a is None:
            h.update(b"none")
        else:
            a = np.ascontiguousarray(a)
            h.update(str(a.dtype).encode() + str(a.shape).encode())
            h.update(a.tobytes())
    return h.hexdigest()


def save(path: str, W: np.ndarray, H: np.ndarray, epochs_done: int, config: dict, fingerprint: str) -> None:
    meta = {"format": FORMAT, "epochs_done": int(epochs_done), "config": {k: config[k] for k in CONFIG_KEYS},
            "data_sha256": fingerprint}
    with open(path, "wb") as f:
        np.savez(f, W=np.ascontiguousarray(W, np.float32), H=np.ascontiguousarray(H, np.float32),
                 meta=np.array(json.dumps(meta, sort_keys=True)))


def load(path: str, config: Optional[dict] = None, fingerprint: Optional[str] = None):
    """(W, H, meta) from a checkpoint; raises ValueError when the file is not a checkpoint, when
    its configuration differs from `config` in any of CONFIG_KEYS, when its data fingerprint
    differs from `fingerprint`, or when W and H do not have the configured shapes."""
    with np.load(path, allow_pickle=False) as z:
        if not {"W", "H", "meta"} <= set(z.files):
            raise ValueError(f"{path}: not a checkpoint (arrays {sorted(z.files)})")
        W, H = z["W"], z["H"]
        meta = json.loads(str(z["meta"]))
    if meta.get("format") != FORMAT:
        raise ValueError(f"{path}: unknown checkpoint format {meta.get('format')!r}")
    saved = meta["config"]
    if config is not None:
        diff = [k for k in CONFIG_KEYS if saved.get(k) != config.get(k)]
        if diff:
            raise ValueError("checkpoint configuration differs in " + ", ".join(
                f"{k} (saved {saved.get(k)!r}, now {config.get(k)!r})" for k in diff))
    if fingerprint is not None and meta["data_sha256"] != fingerprint:
        raise ValueError("checkpoint was written for different observations")
    if W.dtype != np.float32 or H.dtype != np.float32 or W.shape != (saved["num_users"], saved["dim"]) \
            or H.shape != (saved["num_items"], saved["dim"]):
        raise ValueError(f"checkpoint tables have shapes {W.shape}, {H.shape} and types {W.dtype}, {H.dtype}")
    return W, H, meta


def kernel_record(read: dict) -> dict:
    """Per-kernel-family milliseconds and launches from one profile read (ials_profile_read
    returns the totals since the previous read)."""
    return {name: {"ms": round(ms, 4), "launches": cnt} for name, (ms, cnt) in read.items() if cnt > 0}
