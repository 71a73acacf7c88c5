"""torch.autograd wrappers around the block entry points.

A block is the activation-checkpoint boundary (paper, Section "Recompute"):
its forward keeps only the block input (m, z); its backward calls
evoformer_block_bwd, which recomputes the block forward on the GPU before
running the backward kernels.  A stack of blocks therefore stores one (m, z)
pair per block.  With checkpoint=False a block keeps its whole state instead
(evoformer_block_fwd_save / evoformer_block_bwd_saved): no recomputation, at
the memory cost of the block's intermediates.
"""
from __future__ import annotations

import torch

from . import binding


class EvoformerBlockFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, z, flat_buffer, cfg, flat, msa_mask, pair_mask, dtype, dropout=None, checkpoint=True):
        assert flat_buffer is flat.buffer
        m, z = m.contiguous(), z.contiguous()
        if checkpoint:
            m_out, z_out = binding.evoformer_block_fwd(cfg, flat, m, z, msa_mask, pair_mask, dtype=dtype,
                                                       dropout=dropout)
            ctx.state = None
        else:
            m_out, z_out, ctx.state = binding.evoformer_block_fwd_save(cfg, flat, m, z, msa_mask, pair_mask,
                                                                       dtype=dtype, dropout=dropout)
        ctx.save_for_backward(m, z)
        ctx.cfg, ctx.flat, ctx.masks, ctx.dtype, ctx.dropout = cfg, flat, (msa_mask, pair_mask), dtype, dropout
        return m_out, z_out

    @staticmethod
    def backward(ctx, dm_out, dz_out):
        m, z = ctx.saved_tensors
        if dm_out is None:
            dm_out = torch.zeros_like(m)
        if dz_out is None:
            dz_out = torch.zeros_like(z)
        if ctx.state is None:
            dm, dz, dflat = binding.evoformer_block_bwd(ctx.cfg, ctx.flat, m, z, ctx.masks[0], ctx.masks[1],
                                                        dm_out.contiguous(), dz_out.contiguous(), dtype=ctx.dtype,
                                                        dropout=ctx.dropout)
        else:
            dm, dz, dflat = binding.evoformer_block_bwd_saved(ctx.cfg, ctx.flat, m, z, ctx.masks[0], ctx.masks[1],
                                                              ctx.state, dm_out.contiguous(), dz_out.contiguous(),
                                                              dtype=ctx.dtype, dropout=ctx.dropout)
            ctx.state = None
        return dm, dz, dflat, None, None, None, None, None, None, None


def evoformer_block(cfg, flat, m, z, msa_mask=None, pair_mask=None, dtype=None, dropout=None, checkpoint=True):
    """dropout: None or (seed, offset) of the dropout generator (training); checkpoint=False keeps
    the block's state for the backward instead of recomputing the forward."""
    return EvoformerBlockFn.apply(m, z, flat.buffer, cfg, flat, msa_mask, pair_mask, dtype, dropout, checkpoint)


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

    def forward(self, m, z, msa_mask=None, pair_mask=None, dtype=None, dropout=None, checkpoint=True):
        """dropout: None or (seed, offset); block l draws its masks at offset + l."""
        for i, f in enumerate(self.flats):
            dr = None if dropout is None else (dropout[0], dropout[1] + i)
            m, z = evoformer_block(self.cfg, f, m, z, msa_mask, pair_mask, dtype, dr, checkpoint)
        return m, z

    def param_grads(self) -> list:
        """Per-block {subop: {name: grad view}} of the fused gradient buffers."""
        return [f.views(f.buffer.grad) for f in self.flats]


class TemplatePairBlockFn(torch.autograd.Function):
    """One template's pair features through one template pair stack block."""

    @staticmethod
    def forward(ctx, t, flat_buffer, cfg, flat, pair_mask, dtype, dropout, template_index):
        assert flat_buffer is flat.buffer
        t_out = binding.template_pair_block_fwd(cfg, flat, t.contiguous(), pair_mask, dtype=dtype,
                                                dropout=dropout, template_index=template_index)
        ctx.save_for_backward(t)
        ctx.args = (cfg, flat, pair_mask, dtype, dropout, template_index)
        return t_out

    @staticmethod
    def backward(ctx, dt_out):
        (t,) = ctx.saved_tensors
        cfg, flat, pair_mask, dtype, dropout, template_index = ctx.args
        dt, dflat = binding.template_pair_block_bwd(cfg, flat, t.contiguous(), pair_mask, dt_out.contiguous(),
                                                    dtype=dtype, dropout=dropout, template_index=template_index)
        return dt, dflat, None, None, None, None, None, None


class TemplatePairStack(torch.nn.Module):
    """The template pair stack: every template t[n] [R, R, c_t] through the same
    blocks (one fused FP32 parameter buffer per block); template n enters the
    dropout counter, block l draws at offset + l."""

    def __init__(self, cfg, block_params: list, device):
        super().__init__()
        self.cfg = cfg
        self.flats = [binding.FlatParams(p, device, subops=binding.TEMPLATE_SUBOPS) for p in block_params]
        self.buffers_ = torch.nn.ParameterList()
        for f in self.flats:
            f.buffer = torch.nn.Parameter(f.buffer)
            self.buffers_.append(f.buffer)

    def forward(self, t, pair_mask=None, dtype=None, dropout=None):
        outs = []
        for n in range(t.shape[0]):
            x = t[n]
            pm = None if pair_mask is None else pair_mask[n]
            for i, f in enumerate(self.flats):
                dr = None if dropout is None else (dropout[0], dropout[1] + i)
                x = TemplatePairBlockFn.apply(x, f.buffer, self.cfg, f, pm, dtype, dr, n)
            outs.append(x)
        return torch.stack(outs)

    def param_grads(self) -> list:
        return [f.views(f.buffer.grad) for f in self.flats]
