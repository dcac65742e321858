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



class RefineStart:
    """Learned refinement of the standard initialisation.

    The standard initialisation (k-means++ seeds, hard nearest-seed responsibilities, one
    conjugate update) is kept, and an MLP (K(2G+1) + G -> hidden x n_hidden (GELU) ->
    K(2G+1)) maps that state, as a row of the warm-start layout (``CaviBatch.get_rows``) with the
    prior centre, to the move from it to the state that plain CAVI converges to from it.  The
    starting state is the initial row plus the predicted move (``cavi_rows_axpy``, then
    ``CaviBatch.set_state_warm``).  An untrained or useless network leaves the initial state in
    place up to its output, and the subpopulation slots are those of the initialisation, so the
    refined start stays in plain CAVI's basin unless the move crosses into another.  Training
    targets come from running plain CAVI to convergence on generated datasets, all on the GPU.
    """

    def __init__(self, G: int = 48, K: int = 8, hidden: int = 256, n_hidden: int = 3, max_batch: int = 1024,
                 seed: int = 0):
        self.G, self.K = int(G), int(K)
        self.out_dim = self.K * (2 * self.G + 1)
        self.in_dim = self.out_dim + self.G
        self.mlp = CaviMLP(self.in_dim, hidden, n_hidden, self.out_dim, max_batch, seed)
        self.max_batch = int(max_batch)

    def train(self, n_datasets: int, batch: int = 1024, lr: float = 1e-3, warmup: int = 20,
              weight_decay: float = 1e-4, data_seed: int = 4, n_lo: int = 500, n_hi: int = 50_000,
              recipe: synth.Recipe | None = None, max_sweeps: int = 2000, log_every: int = 0, log=print):
        """One pass over ``n_datasets`` generated datasets, ``batch`` per AdamW step (learning rate:
        linear warm-up, then cosine decay to lr/20).  Returns the per-step losses."""
        import torch

        from .cavi import CaviBatch, cavi_rows_axpy

        rec = recipe or synth.Recipe(K=self.K, G=self.G, dir_alpha=1.0)
        batch = min(int(batch), self.max_batch)
        steps = max(1, n_datasets // batch)
        losses = np.zeros(steps)
        t0 = time.perf_counter()
        for s in range(steps):
            off = s * batch
            Ns, _ = synth.batch_shapes(data_seed, batch, n_lo, n_hi, self.K, self.K, offset=off)
            Ks = np.full(batch, self.K, dtype=np.int32)
            x, _, _, _, _, _, _ = synth.make_batch_gpu(data_seed, Ns, Ks, rec, ds_offset=off)
            bt = CaviBatch(x, Ns, Ks)
            bt.init_standard(1_000_003 * data_seed + off)
            feat = bt.get_rows(with_centre=True)
            bt.run(max_sweeps, 1e-6)
            tgt = bt.get_rows()
            cavi_rows_axpy(feat, tgt, -1.0, cols=self.out_dim)  # converged - initial
            bt.close()
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
                log(f"step {s + 1}/{steps}: loss {losses[s]:.6f}  lr {cur:.2e}  {time.perf_counter() - t0:.1f} s")
        return losses

    def warm_start(self, batch, seed: int, step: float = 1.0):
        """Standard initialisation of every dataset of ``batch`` (seed as in init_standard), then
        ``step`` times the learned move."""
        import torch

        from .cavi import cavi_rows_axpy

        if int(batch.K.min()) != self.K or int(batch.K.max()) != self.K:
            raise ValueError(f"the refinement is for K={self.K} datasets")
        batch.init_standard(seed)
        feat = batch.get_rows(with_centre=True)
        outs = [self.mlp.forward(feat[i:i + self.max_batch].contiguous()) for i in range(0, batch.B, self.max_batch)]
        out = outs[0] if len(outs) == 1 else torch.cat(outs, 0)
        cavi_rows_axpy(out, feat, float(step), cols=self.out_dim)  # initial rows + step x move
        torch.cuda.current_stream().synchronize()
        batch.set_state_warm(feat, ld=self.in_dim)

    def save(self, path: str):
        np.save(path, self.mlp.get_params())

    def load(self, path: str):
        self.mlp.set_params(np.load(path, allow_pickle=False))

    def close(self):
        self.mlp.close()
