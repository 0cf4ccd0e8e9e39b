"""iALS++ block-coordinate sweep on AMD Instinct MI355X (gfx950).

The work runs in libials.so (hand-written HIP kernels behind a C ABI, declared
in include/ials.h).  ``binding`` is the ctypes layer with the C names;
``Trainer`` is a small convenience wrapper that owns W and H as torch device
tensors.
"""
from __future__ import annotations

from . import binding
from .binding import IalsError

__all__ = ["binding", "IalsError", "Trainer", "FoldinServer"]


class Trainer:
    """Owns device copies of W, H (torch tensors) and one libials context."""

    def __init__(self, problem, precision: int = binding.IALS_PREC_FP32, chol_fallback_ratio: float = 0.0,
                 stream=None, device: str = "cuda", hbm_budget: int = 0, graph: bool = False, deal: str = "auto",
                 seg_len: int = 0, W0=None, H0=None, gram_split: int = 0):
        import numpy as np
        import torch

        binding.load()
        self.problem = problem
        self.config = {"num_users": problem.num_users, "num_items": problem.num_items, "dim": problem.dim,
                       "block": problem.block, "alpha0": float(problem.alpha0), "lam": float(problem.lam),
                       "precision": int(precision), "chol_fallback_ratio": float(chol_fallback_ratio),
                       "deal": deal, "seg_len": int(seg_len), "gram_split": int(gram_split)}
        self.epochs_done = 0
        self.W = torch.from_numpy(np.ascontiguousarray(problem.W0 if W0 is None else W0)).to(device)
        self.H = torch.from_numpy(np.ascontiguousarray(problem.H0 if H0 is None else H0)).to(device)
        if stream is None:
            stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()
        self.stream = stream
        flags = (binding.IALS_FLAG_GRAPH if graph else 0) | {"auto": 0, "queue": binding.IALS_FLAG_DEAL_QUEUE,
                                                             "static": binding.IALS_FLAG_DEAL_STATIC}[deal]
        cfg = binding.make_config(problem.num_users, problem.num_items, problem.dim, problem.block,
                                  problem.alpha0, problem.lam, precision, chol_fallback_ratio, hbm_budget, flags,
                                  seg_len, gram_split)
        u = np.ascontiguousarray(problem.user, np.int32)
        i = np.ascontiguousarray(problem.item, np.int32)
        y = None if problem.y is None else np.ascontiguousarray(problem.y, np.float32)
        a = None if problem.alpha is None else np.ascontiguousarray(problem.alpha, np.float32)
        coo = binding.make_coo(u, i, y, a, binding.IALS_MEM_HOST)
        self._keep = (u, i, y, a)
        torch.cuda.synchronize()
        self.ctx = binding.ials_create(cfg, coo, self.W, self.H, self.stream)

    def epoch(self, n: int = 1):
        binding.ials_epoch(self.ctx, n)
        self.epochs_done += n

    def save_checkpoint(self, path: str):
        """W, H, the epochs done and the configuration at this epoch boundary (see checkpoint)."""
        from . import checkpoint
        self.synchronize()
        checkpoint.save(path, self.W.cpu().numpy(), self.H.cpu().numpy(), self.epochs_done, self.config,
                        checkpoint.data_fingerprint(self.problem))

    @classmethod
    def resume(cls, path: str, problem, precision: int = binding.IALS_PREC_FP32, chol_fallback_ratio: float = 0.0,
               deal: str = "auto", seg_len: int = 0, gram_split: int = 0, **kw):
        """A trainer that continues the run saved in `path` on the same observations and configuration
        (checked: ValueError otherwise); on the same device it repeats the uninterrupted run bit for bit."""
        from . import checkpoint
        config = {"num_users": problem.num_users, "num_items": problem.num_items, "dim": problem.dim,
                  "block": problem.block, "alpha0": float(problem.alpha0), "lam": float(problem.lam),
                  "precision": int(precision), "chol_fallback_ratio": float(chol_fallback_ratio), "deal": deal,
                  "seg_len": int(seg_len), "gram_split": int(gram_split)}
        W, H, meta = checkpoint.load(path, config, checkpoint.data_fingerprint(problem))
        tr = cls(problem, precision=precision, chol_fallback_ratio=chol_fallback_ratio, deal=deal, seg_len=seg_len,
                 gram_split=gram_split, W0=W, H0=H, **kw)
        tr.epochs_done = meta["epochs_done"]
        return tr

    def fit(self, epochs: int, metrics_path: str | None = None, profile: bool = False, extra=None,
            checkpoint_path: str | None = None, checkpoint_every: int = 0, with_loss: bool = True):
        """Run `epochs` epochs one at a time; after each, append one JSON record to `metrics_path`
        (if given) and return the records: epoch index, loss (float64, eq. 2; skipped without
        with_loss, as it recomputes every prediction), epoch_s (HIP events
        on the context's stream), nnz*b/s (2 |S| d per epoch), the rows redone in float64 during the
        epoch, per-kernel-family milliseconds and launches when `profile`, and whatever
        extra(trainer, epoch) returns.  With checkpoint_path and checkpoint_every = k, a checkpoint
        is written after every k-th epoch."""
        import json
        import torch
        from . import checkpoint
        records = []
        if profile:
            binding.ials_profile_enable(self.ctx, True)
        fb0 = self.stats()["fallback_rows"]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(epochs):
            e0.record(self.stream)
            self.epoch(1)
            e1.record(self.stream)
            e1.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3
            kern = checkpoint.kernel_record(binding.ials_profile_read(self.ctx)) if profile else None
            st = self.stats()
            rec = {"epoch": self.epochs_done, "epoch_s": sec,
                   "nnz_b_per_s": 2.0 * self.problem.nnz * self.problem.dim / sec,
                   "fallback_rows": st["fallback_rows"] - fb0}
            fb0 = st["fallback_rows"]
            if with_loss:
                L, parts = self.loss()
                rec["loss"], rec["loss_parts"] = L, list(parts)
            if profile:
                rec["kernels"] = kern
                binding.ials_profile_read(self.ctx)  # drop the loss evaluation's launches
            if extra is not None:
                rec.update(extra(self, self.epochs_done))
            records.append(rec)
            if metrics_path:
                with open(metrics_path, "a") as f:
                    f.write(json.dumps(rec) + "\n")
            if checkpoint_path and checkpoint_every and self.epochs_done % checkpoint_every == 0:
                self.save_checkpoint(checkpoint_path)
        if profile:
            binding.ials_profile_enable(self.ctx, False)
        return records

    def synchronize(self):
        self.stream.synchronize()

    def block_sweep(self, side: int, block: int):
        binding.ials_block_sweep(self.ctx, side, block)

    def refresh_predictions(self):
        binding.ials_refresh_predictions(self.ctx)

    def loss(self):
        return binding.ials_loss(self.ctx)

    def gramian(self, which: int, block: int = -1):
        import torch
        d, b = self.problem.dim, self.problem.block
        cols = d if block < 0 else min(b, d - block * b)
        out = torch.empty((d, cols), dtype=torch.float32, device=self.W.device)
        binding.ials_gramian(self.ctx, which, block, out)
        return out

    def predictions(self):
        return binding.ials_get_predictions(self.ctx, self.problem.nnz)

    def csr(self, side: int):
        nrows = self.problem.num_users if side == binding.IALS_SIDE_USER else self.problem.num_items
        return binding.ials_get_csr(self.ctx, side, nrows, self.problem.nnz)

    def stats(self):
        return binding.ials_get_stats(self.ctx)

    def foldin(self, req_ptr, items, y=None, passes: int = 3):
        """Fold in new users against the current H: req_ptr (host int64 offsets), items and
        y host arrays or device tensors; returns a (n_req, d) float32 device tensor."""
        import numpy as np
        import torch
        dev = self.W.device
        it = items if isinstance(items, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(items, np.int32))
        it = it.to(dev)
        yv = None
        if y is not None:
            yv = y if isinstance(y, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(y, np.float32))
            yv = yv.to(dev)
        req_ptr = np.ascontiguousarray(req_ptr, np.int64)
        out = torch.empty((req_ptr.size - 1, self.problem.dim), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        binding.ials_foldin(self.ctx, req_ptr, it, yv, passes, out)
        return out

    def close(self):
        if getattr(self, "ctx", None):
            binding.ials_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FoldinServer:
    """Continuous-batching fold-in server around a device item table H (torch tensor, kept alive here)."""

    def __init__(self, H, block: int, alpha0: float, lam: float, passes: int = 3, max_slots: int = 1024,
                 streams: int = 4, hbm_budget: int = 0, chol_fallback_ratio: float = 0.0):
        import torch
        binding.load()
        self.H = H.contiguous()
        self.d = int(self.H.shape[1])
        cfg = binding.make_server_config(int(self.H.shape[0]), self.d, block, alpha0, lam, passes, max_slots,
                                         streams, hbm_budget, chol_fallback_ratio)
        torch.cuda.synchronize()
        self.srv = binding.ials_server_create(cfg, self.H)

    def submit(self, items, y=None, tag: int = 0) -> bool:
        """True if admitted, False if the server answered IALS_E_BUSY."""
        return binding.ials_server_submit(self.srv, items, y, tag) == binding.IALS_OK

    def poll(self, max_n: int = 256, wait_us: int = 0):
        return binding.ials_server_poll(self.srv, max_n, wait_us, self.d)

    def stats(self):
        return binding.ials_server_stats_get(self.srv)

    def close(self):
        if getattr(self, "srv", None):
            binding.ials_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rank_topk(W, H, k: int, excl_ptr=None, excl_idx=None, score_buffer_bytes: int = 0):
    """Top-k items per row of W by <w_u, h_i> (eq. 1) with the excluded items (CSR per row of W,
    ids ascending or not) removed.  W, H: float32 device tensors (d a multiple of 4);
    excl_ptr / excl_idx: int64 / int32 host arrays or device tensors.  Returns (ids int32 [U, k],
    scores float32 [U, k]) device tensors on the current stream."""
    import numpy as np
    import torch
    dev = W.device
    U, d = W.shape
    I = H.shape[0]

    def dev_arr(a, dt):
        if a is None:
            return None
        t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a, dt))
        return t.to(dev).contiguous()
    ep = dev_arr(excl_ptr, np.int64)
    ei = dev_arr(excl_idx, np.int32)
    if ei is not None and ei.numel() == 0:
        ei = torch.zeros(1, dtype=torch.int32, device=dev)
    ids = torch.empty((U, k), dtype=torch.int32, device=dev)
    sc = torch.empty((U, k), dtype=torch.float32, device=dev)
    binding.ials_rank_topk(W.contiguous(), U, H.contiguous(), I, d, ep, ei, k, ids, sc, score_buffer_bytes,
                           torch.cuda.current_stream())
    return ids, sc


def rank_metrics(ids, hold_ptr, hold_idx, metrics):
    """Recall@k / NDCG@k of ranked lists ids (int32 device tensor [U, K]) against held-out items
    (CSR, ids ascending per row).  metrics: sequence of ('recall' | 'ndcg', k).  Returns
    (per_user float64 device tensor [U, m], means float64 [m], counts int64 [m])."""
    import numpy as np
    import torch
    dev = ids.device
    U, K = ids.shape
    hp = torch.from_numpy(np.ascontiguousarray(hold_ptr, np.int64)).to(dev)
    hi = torch.from_numpy(np.ascontiguousarray(hold_idx, np.int32)).to(dev)
    if hi.numel() == 0:
        hi = torch.zeros(1, dtype=torch.int32, device=dev)
    kinds = [binding.RANK_RECALL if n == "recall" else binding.RANK_NDCG for n, _ in metrics]
    ks = [k for _, k in metrics]
    per = torch.empty((U, len(ks)), dtype=torch.float64, device=dev)
    sums, counts = binding.ials_rank_metrics(ids, U, K, hp, hi, kinds, ks, per, torch.cuda.current_stream())
    means = np.where(counts > 0, sums / np.maximum(counts, 1), np.nan)
    return per, means, counts
