"""torch.autograd binding of the embedding-bag forward/backward through the block-I/O path.

The tables live in the store, not in torch: the forward pools rows read through the HBM
cache, and the backward applies SGD directly to the cached rows (which become dirty lines
written back on eviction or flush) instead of returning a gradient tensor.  A one-element
`anchor` parameter makes autograd call the backward.  Given the next step's batch, the
backward also prefetches its lines (the asynchronous mode of Sec. 4.3 for a training
step), so the next forward finds them in the cache.
"""
from __future__ import annotations

import torch

from . import agile


class EmbeddingBagFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, anchor, ctx, tb, idx, off, B, lr, mode, nxt):
        out = torch.empty((B * tb.num_tables, tb.dim), dtype=torch.float32, device=idx.device)
        ctx.embbag_forward(tb, idx, off, B, 0, out, mode=mode)
        fctx.ctx, fctx.tb, fctx.B, fctx.lr, fctx.nxt = ctx, tb, B, lr, nxt
        fctx.save_for_backward(idx, off)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        idx, off = fctx.saved_tensors
        if fctx.nxt is None:
            fctx.ctx.embbag_backward_sgd(fctx.tb, idx, off, fctx.B, grad_out.contiguous(), fctx.lr)
        else:
            nidx, noff, nB = fctx.nxt
            fctx.ctx.embbag_backward_sgd_prefetch(fctx.tb, idx, off, fctx.B, grad_out.contiguous(),
                                                  fctx.lr, nidx, noff, nB)
        return (None,) * 9


class EmbeddingBag(torch.nn.Module):
    """Sum-pooled embedding bags over `num_tables` tables kept in an agile store."""

    def __init__(self, ctx: agile.Context, rows: int, dim: int, num_tables: int, lr: float,
                 base_offset: int = 0, mode: int = agile.MODE_ASYNC):
        super().__init__()
        self.ctx = ctx
        self.tb = ctx.tables(rows, dim, num_tables, base_offset)
        self.lr = lr
        self.mode = mode
        self.anchor = torch.nn.Parameter(torch.zeros(1, device="cuda"))

    def forward(self, idx: torch.Tensor, off: torch.Tensor, B: int, next_batch=None) -> torch.Tensor:
        """next_batch: (idx, off, B) of the next step, prefetched during this backward."""
        return EmbeddingBagFunction.apply(self.anchor, self.ctx, self.tb, idx, off, B, self.lr,
                                          self.mode, next_batch)
