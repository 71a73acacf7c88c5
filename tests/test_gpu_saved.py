"""The block without its checkpoint (evoformer_block_fwd_save /
evoformer_block_bwd_saved): the forward keeps the block's state and the
backward consumes it instead of recomputing the forward (paper, Section
"Recompute": recomputation only trades compute for memory).  Both run the
same kernels in the same order as the checkpointed pair, so outputs and
gradients must agree bit for bit with evoformer_block_fwd / evoformer_block_bwd,
whose parity against the FP64 oracle the block tests establish.  The backward
reads the state without changing it: two backward calls over one saved state
agree too."""
import os

import pytest
import torch

from synth import get, make_inputs

from gpu_util import device_view, say, to_dev
from test_gpu_block import SMALL

pytestmark = pytest.mark.gpu

torch.set_num_threads(min(32, os.cpu_count() or 8))

DROP = (1234567890123, 7)


SMALL_EXTRA = SMALL.replace(name="small_extra", extra_msa=True, msa_heads=4, msa_head_dim=8)


@pytest.mark.parametrize("cfg,dtype,variant", [
    (SMALL, "f32", ""),
    (SMALL, "bf16", "opm_first+dropout"),
    (SMALL_EXTRA, "f32", "dropout"),
    (get("C1"), "f32", ""),
    (get("C1"), "bf16", "dropout"),
    (get("C3"), "bf16", ""),
], ids=["small_f32", "small_bf16_opm_first_dropout", "small_extra_f32_dropout", "c1_f32", "c1_bf16_dropout",
        "c3_bf16"])
def test_saved_block_equals_checkpointed(cfg, dtype, variant):
    from paper_2207_05477_amd import binding as B
    cfg = cfg.replace(n_blocks=1, opm_first="opm_first" in variant)
    dropout = DROP if "dropout" in variant else None
    inp = device_view(make_inputs(cfg, seed=11, perturb=True), dtype)
    flat = B.FlatParams(inp["params"][0], "cuda")
    m, z = to_dev(inp["m"], dtype), to_dev(inp["z"], dtype)
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    dmo, dzo = to_dev(inp["dm_out"], dtype), to_dev(inp["dz_out"], dtype)
    say(f"saved block {cfg.name} dtype={dtype} variant={variant or 'plain'}: "
        f"{B.evoformer_block_saved_bytes(cfg, dtype, dropout) / 2**20:.1f} MiB of state")
    f_ck = B.evoformer_block_fwd(cfg, flat, m, z, mm, pm, dtype=dtype, dropout=dropout)
    r_ck = B.evoformer_block_bwd(cfg, flat, m, z, mm, pm, dmo, dzo, dtype=dtype, dropout=dropout)
    mo, zo, saved = B.evoformer_block_fwd_save(cfg, flat, m, z, mm, pm, dtype=dtype, dropout=dropout)
    r1 = B.evoformer_block_bwd_saved(cfg, flat, m, z, mm, pm, saved, dmo, dzo, dtype=dtype, dropout=dropout)
    r2 = B.evoformer_block_bwd_saved(cfg, flat, m, z, mm, pm, saved, dmo, dzo, dtype=dtype, dropout=dropout)
    torch.cuda.synchronize()
    names = ["m_out", "z_out", "dm", "dz", "dparams"]
    for name, a, b in zip(names, f_ck + r_ck, (mo, zo) + r1):
        assert torch.equal(a, b), f"{name}: saved-state path differs from the checkpointed path"
    for name, a, b in zip(names[2:], r1, r2):
        assert torch.equal(a, b), f"{name}: second backward over the same saved state differs"


def test_saved_stack_autograd_equals_checkpointed():
    from paper_2207_05477_amd.autograd import EvoformerStack
    cfg = SMALL.replace(n_blocks=2)
    dtype = "bf16"
    inp = device_view(make_inputs(cfg, seed=5, perturb=True), dtype)
    stack = EvoformerStack(cfg, inp["params"], "cuda")
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    dmo, dzo = to_dev(inp["dm_out"], dtype), to_dev(inp["dz_out"], dtype)
    res = []
    for ck in (True, False):
        for p in stack.parameters():
            p.grad = None
        m = to_dev(inp["m"], dtype).requires_grad_(True)
        z = to_dev(inp["z"], dtype).requires_grad_(True)
        mo, zo = stack(m, z, mm, pm, dtype=dtype, dropout=DROP, checkpoint=ck)
        torch.autograd.backward([mo, zo], [dmo, dzo])
        torch.cuda.synchronize()
        res.append([mo.detach(), zo.detach(), m.grad, z.grad] + [p.grad.clone() for p in stack.parameters()])
    for i, (a, b) in enumerate(zip(*res)):
        assert torch.equal(a, b), f"tensor {i}: checkpoint=False differs from checkpoint=True"
