"""Checkpointed stacks through torch.autograd (EvoformerBlockFn): each block
keeps only its input and recomputes its forward in the backward (paper,
Section "Recompute").  Compared with the oracle's stack, and checkpointed
gradients compared with a direct per-block backward chain on the GPU."""
import pytest
import torch

from oracle import evoformer as O
from synth import EvoConfig, make_inputs, round_inputs

from gpu_util import TOL, check, say, to_dev

pytestmark = pytest.mark.gpu

STACK = EvoConfig("stack3", n_seq=12, n_res=40, c_m=32, c_z=16, msa_heads=2, msa_head_dim=16,
                  tri_heads=2, tri_head_dim=8, tri_mul_hidden=16, opm_hidden=8, n_blocks=3,
                  mask_mode="residue10")


def _stack_run(cfg, dtype, seed):
    from paper_2207_05477_amd.autograd import EvoformerStack
    inp = round_inputs(make_inputs(cfg, seed=seed, perturb=True), dtype)
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


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_stack_autograd_vs_oracle(dtype):
    say(f"stack autograd {dtype}")
    cfg = STACK
    inp, model, mo, zo, dm, dz = _stack_run(cfg, dtype, seed=21)
    dec = "bf16" if dtype == "bf16" else None
    mo_ref, zo_ref, g = O.stack_fwd_bwd(inp, cfg, relu_decision=dec)
    tol = TOL[dtype]
    check("m update", mo.double().cpu() - inp["m"], mo_ref - inp["m"], tol)
    check("z update", zo.double().cpu() - inp["z"], zo_ref - inp["z"], tol)
    check("dm", dm, g["m"], tol)
    check("dz", dz, g["z"], tol)
    for b, views in enumerate(model.param_grads()):
        for sub, ps in g["params"][b].items():
            for name, ref in ps.items():
                floor = ps["ln_z_g"].norm().item() if name == "ln_z_b" else 0.0
                check(f"block{b}.{sub}.{name}", views[sub][name], ref, tol, floor=floor)


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
