"""Learned warm start of the batched CAVI path.

A dataset's per-gene summary features (``cavi_features``: moments and rank-bin means, or
moments and nearest-rank quantiles) go through an MLP
(``CaviMLP``: 18G -> 256 -> 256 -> 256 -> K(2G+1), GELU, BF16 matrix-core
products with FP32 master weights) whose output row is turned into the
starting variational state of every dataset of a batch
(``CaviBatch.set_state_warm``).  The MLP is trained on the GPU on generated
datasets whose generating parameters give the targets
(``cavi_warm_targets``): mean squared error, AdamW, every step in
``libcavi.so``.  This module only sequences those calls.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import synth
from .cavi import FEATURES_PER_GENE, CaviMLP, cavi_features, cavi_warm_targets


class WarmStart:
    """MLP for datasets of ``G`` genes and ``K`` subpopulations."""

    def __init__(self, G: int = 48, K: int = 8, hidden: int = 256, n_hidden: int = 3, max_batch: int = 1024,
                 seed: int = 0, features: str = "bins"):
        if features not in ("bins", "quantiles"):
            raise ValueError(f"features must be 'bins' or 'quantiles', not {features!r}")
        self.features = features
        self.G, self.K = int(G), int(K)
        self.in_dim = FEATURES_PER_GENE * self.G
        self.out_dim = self.K * (2 * self.G + 1)
        self.mlp = CaviMLP(self.in_dim, hidden, n_hidden, self.out_dim, max_batch, seed)
        self.max_batch = int(max_batch)

    # ------------------------------------------------------------------ training
    def train(self, n_datasets: int, batch: int = 1024, lr: float = 1e-3, warmup: int = 50,
              weight_decay: float = 1e-4, data_seed: int = 4, n_lo: int = 500, n_hi: int = 50_000,
              recipe: synth.Recipe | None = None, log_every: int = 0, log=print):
        """One pass over ``n_datasets`` generated datasets (dataset indices 0 .. n_datasets-1 of
        ``data_seed``), ``batch`` per AdamW step; learning rate: linear warm-up then cosine decay
        to lr/20.  Returns the per-step losses."""
        import torch

        rec = recipe or synth.Recipe(K=self.K, G=self.G, dir_alpha=1.0)
        batch = min(int(batch), self.max_batch)
        steps = max(1, n_datasets // batch)
        losses = np.zeros(steps)
        t0 = time.perf_counter()
        for s in range(steps):
            off = s * batch
            Ns, _ = synth.batch_shapes(data_seed, batch, n_lo, n_hi, self.K, self.K, offset=off)
            Ks = np.full(batch, self.K, dtype=np.int32)
            x, row_off, _, pi, mu, tau, _ = synth.make_batch_gpu(data_seed, Ns, Ks, rec, ds_offset=off)
            feat = cavi_features(x, row_off.to(x.device), kind=self.features)
            tgt = cavi_warm_targets(pi, mu, tau)
            del x
            want = log_every and (s % log_every == 0 or s == steps - 1)
            losses[s] = self.mlp.loss_grad(feat, tgt, want_loss=True)
            if s < warmup:
                cur = lr * (s + 1) / warmup
            else:
                frac = (s - warmup) / max(1, steps - warmup)
                cur = lr / 20 + (lr - lr / 20) * 0.5 * (1 + math.cos(math.pi * frac))
            self.mlp.adamw(cur, 0.9, 0.999, 1e-8, weight_decay)
            if want:
                torch.cuda.synchronize()
                log(f"step {s + 1}/{steps}: loss {losses[s]:.5f}  lr {cur:.2e}  {time.perf_counter() - t0:.1f} s")
        return losses

    # ------------------------------------------------------------------ inference
    def predict(self, x, row_off_dev):
        """MLP output rows (B x K(2G+1), device) for concatenated rows ``x`` cut at ``row_off_dev``."""
        B = row_off_dev.numel() - 1
        feat = cavi_features(x, row_off_dev, kind=self.features)
        outs = [self.mlp.forward(feat[i:i + self.max_batch].contiguous()) for i in range(0, B, self.max_batch)]
        import torch

        return outs[0] if len(outs) == 1 else torch.cat(outs, 0)

    def warm_start(self, batch, x, row_off_dev):
        """Set every dataset of ``batch`` (a ``CaviBatch`` over ``x``) from the MLP."""
        if int(batch.K.min()) != self.K or int(batch.K.max()) != self.K:
            raise ValueError(f"the warm start is for K={self.K} datasets")
        batch.set_state_warm(self.predict(x, row_off_dev))

    # ------------------------------------------------------------------ parameters
    def save(self, path: str):
        np.save(path, self.mlp.get_params())

    def load(self, path: str):
        self.mlp.set_params(np.load(path, allow_pickle=False))

    def close(self):
        self.mlp.close()

