"""Checkpointed stacks through torch.autograd (EvoformerBlockFn): each block
keeps only its input and recomputes its forward in the backward (paper,
Section "Recompute").  Compared with the oracle's stack, and checkpointed
gradients compared with a direct per-block backward chain on the GPU."""
import pytest
import torch

from oracle import evoformer as O
from synth import EvoConfig, get, make_inputs

from gpu_util import TOL, bf16_weight_view, check, check_update, margin_view, say, to_dev
from test_gpu_block import check_block_grads

pytestmark = pytest.mark.gpu

STACK = EvoConfig("stack3", n_seq=12, n_res=40, c_m=32, c_z=16, msa_heads=2, msa_head_dim=16,
                  tri_heads=2, tri_head_dim=8, tri_mul_hidden=16, opm_hidden=8, n_blocks=3,
                  mask_mode="residue10")


def _boundary(dtype):
    # a BF16 stack hands BF16 tensors between blocks; the oracle stores them alike
    return "bf16" if dtype == "bf16" else None


def _stack_run(cfg, dtype, seed, perturb=True):
    from paper_2207_05477_amd.autograd import EvoformerStack
    inp = margin_view(make_inputs(cfg, seed=seed, perturb=perturb), cfg, dtype, _boundary(dtype))
    model = EvoformerStack(cfg, inp["params"], "cuda")
    m = to_dev(inp["m"], dtype).requires_grad_(True)
    z = to_dev(inp["z"], dtype).requires_grad_(True)
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    mo, zo = model(m, z, mm, pm, dtype=dtype)
    loss = (mo.float() * to_dev(inp["dm_out"], dtype).float()).sum() + \
        (zo.float() * to_dev(inp["dz_out"], dtype).float()).sum()
    loss.backward()
    torch.cuda.synchronize()
    return inp, model, mo, zo, m.grad, z.grad


def _per_block_param_grads(cfg, inp, model, dtype, quant=False):
    """Parameter gradients of each block of a BF16 stack against the oracle's
    block evaluated at the same block input and upstream gradient as the GPU
    block (both as stored in BF16 between blocks).  Through a stack the error
    of the gradient reaching a block compounds with the blocks above it; this
    gates each block's own arithmetic at the tolerance, while the stack's
    outputs and input gradients are gated end to end."""
    from paper_2207_05477_amd import binding as B
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    acts = [(to_dev(inp["m"], dtype), to_dev(inp["z"], dtype))]
    with torch.no_grad():
        for f in model.flats:
            acts.append(B.evoformer_block_fwd(cfg, f, acts[-1][0], acts[-1][1], mm, pm, dtype=dtype))
    gm, gz = to_dev(inp["dm_out"], dtype), to_dev(inp["dz_out"], dtype)
    one = cfg.replace(n_blocks=1)
    for i in reversed(range(len(model.flats))):
        up = (gm.double().cpu(), gz.double().cpu())
        gm, gz, gp = B.evoformer_block_bwd(cfg, model.flats[i], acts[i][0], acts[i][1], mm, pm, gm, gz, dtype=dtype)
        torch.cuda.synchronize()
        # the checkpointed (autograd) gradients are this chain's, bit for bit
        assert torch.equal(gp, model.flats[i].buffer.grad), f"block {i} parameter gradient"
        blk = dict(inp)
        blk.update(params=[inp["params"][i]], m=acts[i][0].double().cpu(), z=acts[i][1].double().cpu(),
                   dm_out=up[0], dz_out=up[1])
        say(f"  oracle block {i}")
        _, _, g = O.stack_fwd_bwd(blk, one)
        gq = O.stack_fwd_bwd(bf16_weight_view(blk), one)[2]["params"][0] if quant else None
        check_block_grads(f"block{i}.", model.flats[i].views(gp), g["params"][0], TOL[dtype], gref_q=gq)


def _stack_vs_oracle(cfg, dtype, seed, perturb=True, quant=False):
    inp, model, mo, zo, dm, dz = _stack_run(cfg, dtype, seed=seed, perturb=perturb)
    say("  oracle")
    mo_ref, zo_ref, g = O.stack_fwd_bwd(inp, cfg, boundary=_boundary(dtype))
    tol = TOL[dtype]
    check_update("m update", mo, inp["m"], mo_ref - inp["m"], dtype)
    check_update("z update", zo, inp["z"], zo_ref - inp["z"], dtype)
    check("dm", dm, g["m"], tol)
    check("dz", dz, g["z"], tol)
    if dtype == "bf16":
        _per_block_param_grads(cfg, inp, model, dtype, quant)
        return
    for b, views in enumerate(model.param_grads()):
        check_block_grads(f"block{b}.", views, g["params"][b], tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_stack_autograd_vs_oracle(dtype):
    say(f"stack autograd {dtype}")
    # small fan-ins (16-32 channels): BF16 gradients gated with the weight quantization's own effect
    _stack_vs_oracle(STACK, dtype, 21, quant=dtype == "bf16")


@pytest.mark.timeout(900)
def test_stack_c2_bf16_four_blocks():
    # the headline BF16 form: 4 checkpointed blocks at N_seq=128, N_res=256, 10 % residue masks
    from synth import get
    say("stack C2 (4 blocks, bf16)")
    _stack_vs_oracle(get("C2"), "bf16", 32, perturb=False)


def test_checkpointed_grads_equal_direct_chain():
    # autograd over the checkpointed stack == explicit backward chain of the blocks
    from paper_2207_05477_amd import binding as B
    cfg = STACK
    inp, model, mo, zo, dm, dz = _stack_run(cfg, "f32", seed=22)
    flats = model.flats
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    acts = [(to_dev(inp["m"]), to_dev(inp["z"]))]
    with torch.no_grad():
        for f in flats:
            acts.append(B.evoformer_block_fwd(cfg, f, acts[-1][0], acts[-1][1], mm, pm))
    gm, gz = to_dev(inp["dm_out"]), to_dev(inp["dz_out"])
    grads = [None] * len(flats)
    for i in reversed(range(len(flats))):
        gm, gz, grads[i] = B.evoformer_block_bwd(cfg, flats[i], acts[i][0], acts[i][1], mm, pm, gm, gz)
    torch.cuda.synchronize()
    assert torch.equal(gm, dm) and torch.equal(gz, dz)
    for i, f in enumerate(flats):
        assert torch.equal(grads[i], f.buffer.grad)


@pytest.mark.timeout(600)
def test_stack_c4a_bf16_eight_blocks_checkpointed_equals_direct_chain():
    # the fine-tuning crop: 8 checkpointed blocks at N_seq = 512, N_res = 384 in BF16
    # through torch.autograd, against an explicit per-block backward chain (bit for bit)
    from paper_2207_05477_amd import binding as B
    from paper_2207_05477_amd.autograd import EvoformerStack
    cfg = get("C4a")
    say(f"stack {cfg.name}")
    inp = make_inputs(cfg, seed=32)
    model = EvoformerStack(cfg, inp["params"], "cuda")
    del inp["params"]
    dt = "bf16"
    m0, z0 = to_dev(inp["m"], dt), to_dev(inp["z"], dt)
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    dmo, dzo = to_dev(inp["dm_out"], dt), to_dev(inp["dz_out"], dt)
    m = m0.clone().requires_grad_(True)
    z = z0.clone().requires_grad_(True)
    mo, zo = model(m, z, mm, pm, dtype=dt)
    torch.autograd.backward([mo, zo], [dmo, dzo])
    torch.cuda.synchronize()
    say("  autograd done")
    assert torch.isfinite(m.grad.float()).all() and torch.isfinite(z.grad.float()).all()
    acts = [(m0, z0)]
    with torch.no_grad():
        for f in model.flats:
            acts.append(B.evoformer_block_fwd(cfg, f, acts[-1][0], acts[-1][1], mm, pm, dtype=dt))
    assert torch.equal(acts[-1][0], mo) and torch.equal(acts[-1][1], zo)
    gm, gz = dmo, dzo
    for i in reversed(range(len(model.flats))):
        gm, gz, gp = B.evoformer_block_bwd(cfg, model.flats[i], acts[i][0], acts[i][1], mm, pm, gm, gz,
                                           dtype=dt)
        assert torch.equal(gp, model.flats[i].buffer.grad), f"block {i} parameter gradient"
        acts[i + 1] = None
    torch.cuda.synchronize()
    assert torch.equal(gm, m.grad) and torch.equal(gz, z.grad)
