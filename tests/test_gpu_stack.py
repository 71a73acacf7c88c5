"""Checkpointed stacks through torch.autograd (EvoformerBlockFn): each block
keeps only its input and recomputes its forward in the backward (paper,
Section "Recompute").  Compared with the oracle's stack, and checkpointed
gradients compared with a direct per-block backward chain on the GPU."""
import pytest
import torch

from oracle import evoformer as O
from synth import EvoConfig, make_inputs

from gpu_util import device_view, KINK_TOL, TOL, check, kink_free, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

STACK = EvoConfig("stack3", n_seq=12, n_res=40, c_m=32, c_z=16, msa_heads=2, msa_head_dim=16,
                  tri_heads=2, tri_head_dim=8, tri_mul_hidden=16, opm_hidden=8, n_blocks=3,
                  mask_mode="residue10")


def _stack_run(cfg, dtype, seed, kinks=False, perturb=True):
    from paper_2207_05477_amd.autograd import EvoformerStack
    inp = device_view(make_inputs(cfg, seed=seed, perturb=perturb), dtype)
    if not kinks:
        inp = kink_free(inp)
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


def _stack_vs_oracle(cfg, dtype, seed, kinks, perturb=True):
    inp, model, mo, zo, dm, dz = _stack_run(cfg, dtype, seed=seed, kinks=kinks, perturb=perturb)
    dec = "bf16" if dtype == "bf16" else None
    say("  oracle")
    # the BF16 stack hands BF16 tensors between blocks; the oracle stores them alike
    mo_ref, zo_ref, g = O.stack_fwd_bwd(inp, cfg, relu_decision=dec, boundary="bf16" if dtype == "bf16" else None)
    tol = TOL[dtype]
    check("m update", mo.double().cpu() - inp["m"], mo_ref - inp["m"], tol)
    check("z update", zo.double().cpu() - inp["z"], zo_ref - inp["z"], tol)
    gtol = KINK_TOL[dtype] if kinks else tol
    check("dm", dm, g["m"], gtol)
    check("dz", dz, g["z"], gtol)
    for b, views in enumerate(model.param_grads()):
        for sub, ps in g["params"][b].items():
            if dtype == "f32":
                for name, ref in ps.items():
                    floor = ps["ln_z_g"].norm().item() if name == "ln_z_b" else 0.0
                    check(f"block{b}.{sub}.{name}", views[sub][name], ref, gtol, floor=floor)
                continue
            # BF16 stacks: the gradient w.r.t. each sub-operation's parameter
            # vector (all its tensors together) is gated; per-tensor errors are
            # reported.  The pair-bias LayerNorm offset of row attention has a
            # zero gradient by an identity and keeps its own floor-relative gate.
            got, ref = [], []
            for name, r in ps.items():
                if name == "ln_z_b":
                    check(f"block{b}.{sub}.{name}", views[sub][name], r, gtol, floor=ps["ln_z_g"].norm().item())
                    continue
                say(f"    block{b}.{sub}.{name}: {rel_err(views[sub][name], r):.3e}")
                got.append(views[sub][name].detach().double().cpu().reshape(-1))
                ref.append(r.reshape(-1))
            check(f"block{b}.{sub} (all parameters)", torch.cat(got), torch.cat(ref), gtol)


@pytest.mark.parametrize("kinks", [False, True], ids=["kink_free", "full_params"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_stack_autograd_vs_oracle(dtype, kinks):
    say(f"stack autograd {dtype} kinks={kinks}")
    _stack_vs_oracle(STACK, dtype, 21, kinks)


def test_stack_c2_bf16_four_blocks():
    # the headline BF16 form: 4 checkpointed blocks at N_seq=128, N_res=256, 10 % residue masks
    from synth import get
    say("stack C2 (4 blocks, bf16)")
    _stack_vs_oracle(get("C2"), "bf16", 32, kinks=False, perturb=False)


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
