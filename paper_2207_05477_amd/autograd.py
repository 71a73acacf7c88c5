"""torch.autograd wrappers around the block entry points.

A block is the activation-checkpoint boundary (paper, Section "Recompute"):
its forward keeps only the block input (m, z); its backward calls
evoformer_block_bwd, which recomputes the block forward on the GPU before
running the backward kernels.  A stack of blocks therefore stores one (m, z)
pair per block.
"""
from __future__ import annotations

import torch

from . import binding


class EvoformerBlockFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, z, flat_buffer, cfg, flat, msa_mask, pair_mask, dtype):
        assert flat_buffer is flat.buffer
        m_out, z_out = binding.evoformer_block_fwd(cfg, flat, m.contiguous(), z.contiguous(), msa_mask,
                                                   pair_mask, dtype=dtype)
        ctx.save_for_backward(m, z)
        ctx.cfg, ctx.flat, ctx.masks, ctx.dtype = cfg, flat, (msa_mask, pair_mask), dtype
        return m_out, z_out

    @staticmethod
    def backward(ctx, dm_out, dz_out):
        m, z = ctx.saved_tensors
        if dm_out is None:
            dm_out = torch.zeros_like(m)
        if dz_out is None:
            dz_out = torch.zeros_like(z)
        dm, dz, dflat = binding.evoformer_block_bwd(ctx.cfg, ctx.flat, m.contiguous(), z.contiguous(),
                                                    ctx.masks[0], ctx.masks[1], dm_out.contiguous(),
                                                    dz_out.contiguous(), dtype=ctx.dtype)
        return dm, dz, dflat, None, None, None, None, None


def evoformer_block(cfg, flat, m, z, msa_mask=None, pair_mask=None, dtype=None):
    return EvoformerBlockFn.apply(m, z, flat.buffer, cfg, flat, msa_mask, pair_mask, dtype)


class EvoformerStack(torch.nn.Module):
    """A stack of Evoformer blocks with independent parameters, each block's
    parameters fused into one FP32 buffer (one nn.Parameter per block)."""

    def __init__(self, cfg, block_params: list, device):
        super().__init__()
        self.cfg = cfg
        self.flats = [binding.FlatParams(p, device) for p in block_params]
        self.buffers_ = torch.nn.ParameterList()
        for f in self.flats:
            f.buffer = torch.nn.Parameter(f.buffer)
            self.buffers_.append(f.buffer)

    def forward(self, m, z, msa_mask=None, pair_mask=None, dtype=None):
        for f in self.flats:
            m, z = evoformer_block(self.cfg, f, m, z, msa_mask, pair_mask, dtype)
        return m, z

    def param_grads(self) -> list:
        """Per-block {subop: {name: grad view}} of the fused gradient buffers."""
        return [f.views(f.buffer.grad) for f in self.flats]
