"""GPU parity of the whole Evoformer block against the FP64 oracle: forward
residual updates, input gradients and every parameter gradient, each tensor
gated on its own (normwise and max-norm relative error), at small ragged
shapes and at the paper's crop shapes (initial training N_seq=128, N_res=256;
extra MSA N_extra=1024; fine-tuning N_seq=512, N_res=384).

Gradient tests use margin-constructed inputs (oracle.with_relu_margins): the
transitions keep their drawn W_1 and the oracle re-chooses b_1 so that every
ReLU decision is clear at the tested precision.  Forward-only tests use the
workload's own parameters."""
import os

import pytest
import torch

from oracle import evoformer as O
from synth import EvoConfig, get, make_inputs

from gpu_util import TOL, bf16_weight_view, check, check_quant, check_update, device_view, margin_view, say, to_dev

pytestmark = pytest.mark.gpu

SMALL = EvoConfig("small", n_seq=12, n_res=40, c_m=32, c_z=16, msa_heads=2, msa_head_dim=16,
                  tri_heads=2, tri_head_dim=8, tri_mul_hidden=16, opm_hidden=8, mask_mode="random")

torch.set_num_threads(min(32, os.cpu_count() or 8))


def check_block_grads(tag, views, gref, tol, report=None, gref_q=None):
    """Every parameter gradient of one block, tensor by tensor (with gref_q, the
    oracle's gradients under BF16-rounded matrix weights: see check_quant)."""
    for sub, ps in gref.items():
        for name, ref in ps.items():
            # zero by an identity (the pair-bias gradient sums to zero over
            # keys): bounded by the magnitude of the matching gamma gradient
            floor = ps["ln_z_g"].norm().item() if name == "ln_z_b" else 0.0
            efloor = ps["ln_z_g"].abs().max().item() if name == "ln_z_b" else 0.0
            if gref_q is None:
                check(f"{tag}{sub}.{name}", views[sub][name], ref, tol, report, floor=floor, efloor=efloor)
            else:
                check_quant(f"{tag}{sub}.{name}", views[sub][name], ref, gref_q[sub][name], tol, report,
                            floor=floor, efloor=efloor)


def _run(cfg, dtype, seed=32, backward=True, perturb=False, mask_mode=None, report=None, margins=True,
         quant=False):
    from paper_2207_05477_amd import binding as B
    inp = make_inputs(cfg, seed=seed, perturb=perturb, mask_mode=mask_mode)
    inp = margin_view(inp, cfg, dtype) if margins else device_view(inp, dtype)
    tol = TOL[dtype]
    say(f"block {cfg.name} dtype={dtype} bwd={backward}: oracle")
    if backward:
        mo_ref, zo_ref, g = O.stack_fwd_bwd(inp, cfg)
    else:
        mo_ref, zo_ref = O.stack_fwd(inp, cfg)
    say("  gpu")
    flat = B.FlatParams(inp["params"][0], "cuda")
    m, z = to_dev(inp["m"], dtype), to_dev(inp["z"], dtype)
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    mo, zo = B.evoformer_block_fwd(cfg, flat, m, z, mm, pm, dtype=dtype)
    torch.cuda.synchronize()
    check_update("m update", mo, inp["m"], mo_ref - inp["m"], dtype, report)
    check_update("z update", zo, inp["z"], zo_ref - inp["z"], dtype, report)
    if not backward:
        return
    del mo, zo
    dm, dz, dflat = B.evoformer_block_bwd(cfg, flat, m, z, mm, pm, to_dev(inp["dm_out"], dtype),
                                          to_dev(inp["dz_out"], dtype), dtype=dtype)
    torch.cuda.synchronize()
    if quant:   # small fan-ins: the BF16 weight quantization's own effect (see check_quant)
        say("  oracle with BF16-rounded matrix weights")
        _, _, gq = O.stack_fwd_bwd(bf16_weight_view(inp), cfg)
        check_quant("dm", dm, g["m"], gq["m"], tol, report)
        check_quant("dz", dz, g["z"], gq["z"], tol, report)
        check_block_grads("", flat.views(dflat), g["params"][0], tol, report, gq["params"][0])
        return
    check("dm", dm, g["m"], tol, report)
    check("dz", dz, g["z"], tol, report)
    check_block_grads("", flat.views(dflat), g["params"][0], tol, report)


def _worst(report):
    mx = report.pop("_max", {})
    say("  worst normwise:", max(report.items(), key=lambda kv: kv[1]))
    if mx:
        say("  worst max-norm:", max(mx.items(), key=lambda kv: kv[1]))


def test_block_c0_forward_f32():
    _run(get("C0"), "f32", backward=False, margins=False)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_block_small_fwd_bwd(dtype):
    _run(SMALL, dtype, seed=5, perturb=True, quant=dtype == "bf16")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_extra_msa_block_small_fwd_bwd(dtype):
    cfg = SMALL.replace(name="small_extra", extra_msa=True, msa_heads=4, msa_head_dim=8,
                        msa_input="onehot23")
    _run(cfg, dtype, seed=6, perturb=True, quant=dtype == "bf16")


def test_block_c1_fwd_bwd_f32():
    report = {}
    _run(get("C1"), "f32", report=report)
    _worst(report)


def test_block_c1_forward_f32_workload_params():
    # the headline workload's own parameters (transition b_1 = 0)
    _run(get("C1"), "f32", backward=False, margins=False)


def test_block_c1_shape_bf16_residue_masks():
    report = {}
    _run(get("C2").replace(n_blocks=1), "bf16", report=report)
    _worst(report)


@pytest.mark.timeout(900)
def test_extra_msa_block_c3_bf16_fwd_bwd():
    # the extra-MSA block at its full shape (N_extra = 1024, c_e = 64, 8 x 8 heads)
    report = {}
    _run(get("C3"), "bf16", report=report)
    _worst(report)


@pytest.mark.timeout(1200)
def test_block_c4a_shape_bf16_fwd_bwd():
    # one block at the fine-tuning crop (N_seq = 512, N_res = 384)
    report = {}
    _run(get("C4a").replace(n_blocks=1), "bf16", report=report)
    _worst(report)


@pytest.mark.parametrize("cfg,dtype", [(SMALL, "f32"), (get("C1"), "bf16")], ids=["small_f32", "c1_bf16"])
def test_block_is_deterministic(cfg, dtype):
    from paper_2207_05477_amd import binding as B
    inp = device_view(make_inputs(cfg.replace(n_blocks=1), seed=3, perturb=True), dtype)
    flat = B.FlatParams(inp["params"][0], "cuda")
    m, z = to_dev(inp["m"], dtype), to_dev(inp["z"], dtype)
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    dmo, dzo = to_dev(inp["dm_out"], dtype), to_dev(inp["dz_out"], dtype)
    f1 = B.evoformer_block_fwd(cfg, flat, m, z, mm, pm, dtype=dtype)
    f2 = B.evoformer_block_fwd(cfg, flat, m, z, mm, pm, dtype=dtype)
    r1 = B.evoformer_block_bwd(cfg, flat, m, z, mm, pm, dmo, dzo, dtype=dtype)
    r2 = B.evoformer_block_bwd(cfg, flat, m, z, mm, pm, dmo, dzo, dtype=dtype)
    torch.cuda.synchronize()
    for a, b in zip(f1 + r1, f2 + r2):
        assert torch.equal(a, b)
