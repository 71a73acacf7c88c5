"""The extra-MSA stack at the fine-tuning crop (paper, model-settings table:
N_extra_seq = 5120, N_res = 384; c_e = 64, 8 x 8 heads), the case whose
attention logits the paper's Subbatch section sizes at 11.25 GiB: the kernels
never store them.

* The global column attention alone, forward and backward, against the FP64
  oracle at the full shape (every output and gradient tensor), with a random
  MSA mask that also masks one residue column completely.
* The whole extra-MSA block forward against the FP64 oracle at the full shape
  (the oracle's row attention evaluated in chunks of MSA rows, which are
  independent), and its backward run twice: finite and bitwise repeatable.
"""
import os

import pytest
import torch

from oracle import evoformer as O
from synth import get, make_inputs

from gpu_util import TOL, check, check_update, device_view, oracle_grads, params_dev, say, to_dev

pytestmark = pytest.mark.gpu

torch.set_num_threads(min(32, os.cpu_count() or 8))


@pytest.mark.timeout(900)
def test_global_col_attn_finetune_shape_bf16():
    from paper_2207_05477_amd import binding as B, _abi as A
    cfg = get("C5")
    dtype = "bf16"
    say(f"global column attention S={cfg.n_seq} R={cfg.n_res} c={cfg.c_m}")
    inp = device_view(make_inputs(cfg, seed=32, perturb=True, mask_mode="random"), dtype)
    H, D = cfg.msa_heads, cfg.msa_head_dim
    p = inp["params"][0]["col_attn"]
    M = inp["msa_mask"]
    desc = B.attn_desc(A.EVO_ATTN_COL_GLOBAL, dtype, cfg.n_seq, cfg.n_res, cfg.c_m, H, D,
                       global_eps=cfg.global_eps)
    pd = params_dev(p)
    w = B.weight_struct("col_attn", pd)
    x, mask = to_dev(inp["m"], dtype), M.float().cuda()
    out, saved = B.evo_attn_fwd(desc, w, x, None, mask)
    dpar = {k: torch.zeros_like(v) for k, v in pd.items()}
    dx = B.evo_attn_bwd(desc, w, x, None, mask, saved, to_dev(inp["dm_out"], dtype),
                        B.weight_struct("col_attn", dpar))
    torch.cuda.synchronize()
    out, dx = out.cpu(), dx.cpu()
    del saved
    say("  oracle")
    upd, g = oracle_grads(lambda m, p: O.col_global_attn(m, M, p, H, D, cfg.ln_eps, cfg.global_eps),
                          {"m": inp["m"], "p": p}, inp["dm_out"])
    tol = TOL[dtype]
    check_update("gcol fwd", out, inp["m"], upd, dtype)
    check("gcol dx", dx, inp["dm_out"] + g["m"], tol)
    for k in dpar:
        check(f"gcol d{k}", dpar[k], g["p"][k], tol)


def _extra_block_oracle_fwd(inp, cfg, rows_per_chunk=256):
    """The oracle's extra-MSA block (oracle.block's order) with its row attention
    evaluated in chunks of MSA rows (each row attends over residues on its own)."""
    p = inp["params"][0]
    eps = cfg.ln_eps
    m, z = inp["m"], inp["z"]
    mm, pm = inp["msa_mask"], inp["pair_mask"]
    with torch.no_grad():
        upd = torch.cat([O.row_attn(m[s:s + rows_per_chunk], z, mm[s:s + rows_per_chunk], p["row_attn"],
                                    cfg.msa_heads, cfg.msa_head_dim, eps)
                         for s in range(0, cfg.n_seq, rows_per_chunk)])
        m = m + upd
        del upd
        m = m + O.col_global_attn(m, mm, p["col_attn"], cfg.msa_heads, cfg.msa_head_dim, eps, cfg.global_eps)
        m = m + O.transition(m, p["msa_trans"], eps)
        z = z + O.outer_product_mean(m, mm, p["opm"], eps, cfg.opm_eps)
        z = z + O.tri_mul_out(z, pm, p["tri_mul_out"], eps)
        z = z + O.tri_mul_in(z, pm, p["tri_mul_in"], eps)
        z = z + O.tri_att_start(z, pm, p["tri_att_start"], cfg.tri_heads, cfg.tri_head_dim, eps)
        z = z + O.tri_att_end(z, pm, p["tri_att_end"], cfg.tri_heads, cfg.tri_head_dim, eps)
        z = z + O.transition(z, p["pair_trans"], eps)
    return m, z


@pytest.mark.timeout(1100)
def test_extra_msa_block_finetune_shape_bf16():
    from paper_2207_05477_amd import binding as B
    cfg = get("C5")
    dtype = "bf16"
    say(f"extra-MSA block {cfg.name}: S={cfg.n_seq} R={cfg.n_res}")
    inp = device_view(make_inputs(cfg, seed=32), dtype)
    flat = B.FlatParams(inp["params"][0], "cuda")
    m, z = to_dev(inp["m"], dtype), to_dev(inp["z"], dtype)
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    mo, zo = B.evoformer_block_fwd(cfg, flat, m, z, mm, pm, dtype=dtype)
    dmo, dzo = to_dev(inp["dm_out"], dtype), to_dev(inp["dz_out"], dtype)
    r1 = B.evoformer_block_bwd(cfg, flat, m, z, mm, pm, dmo, dzo, dtype=dtype)
    torch.cuda.synchronize()
    r1 = tuple(t.cpu() for t in r1)
    r2 = B.evoformer_block_bwd(cfg, flat, m, z, mm, pm, dmo, dzo, dtype=dtype)
    torch.cuda.synchronize()
    for a, b in zip(r1, r2):
        assert torch.isfinite(a.float()).all()
        assert torch.equal(a, b.cpu()), "block backward not bitwise repeatable"
    del r2
    mo, zo = mo.cpu(), zo.cpu()
    say("  oracle forward")
    mo_ref, zo_ref = _extra_block_oracle_fwd(inp, cfg)
    check_update("m update", mo, inp["m"], mo_ref - inp["m"], dtype)
    check_update("z update", zo, inp["z"], zo_ref - inp["z"], dtype)
