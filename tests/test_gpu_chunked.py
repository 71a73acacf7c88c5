"""Query-chunked forward (long chains): chunked results equal unchunked ones.

The paper's Subbatch splits a batch-like axis whose computation is
independent (Section "Subbatch VS DAP"), so chunking must not change the
result.  Checked per op against the oracle at a small shape, per op and per
block chunked vs unchunked on the GPU (same per-row arithmetic, so equal to the
last bit), for the whole block at the long-chain shape N_res = 1024 with
128-row chunks, and per op at that shape against the oracle on sampled output
rows (the first, a middle and the last row of the chunk grid, where whole and
ragged query blocks and the chunk seams meet).
"""
import pytest
import torch

from oracle import evoformer as O
from synth import EvoConfig, get, make_inputs

from gpu_util import device_view, TOL, check, check_update, params_dev, say, to_dev

pytestmark = pytest.mark.gpu

CCFG = EvoConfig("chunk", n_seq=8, n_res=64, c_m=32, c_z=16, msa_heads=2, msa_head_dim=16,
                 tri_heads=2, tri_head_dim=16, tri_mul_hidden=16, opm_hidden=8, mask_mode="random")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("op", ["tri_att_start", "tri_att_end", "tri_mul_out", "tri_mul_in", "opm"])
def test_chunked_op_equals_unchunked_and_oracle(dtype, op):
    from paper_2207_05477_amd import binding as B, _abi as A
    say(f"chunked {op} {dtype}")
    cfg = CCFG
    inp = device_view(make_inputs(cfg, seed=11, perturb=True), dtype)
    p = inp["params"][0][op]
    pd = params_dev(p)
    w = B.weight_struct(op, pd)
    z, P = to_dev(inp["z"], dtype), inp["pair_mask"].float().cuda()
    outs = []
    for chunk in (0, 16):
        if op.startswith("tri_att"):
            kind = A.EVO_ATTN_TRI_START if op.endswith("start") else A.EVO_ATTN_TRI_END
            d = B.attn_desc(kind, dtype, cfg.n_res, cfg.n_res, cfg.c_z, cfg.tri_heads, cfg.tri_head_dim,
                            chunk=chunk)
            out, _ = B.evo_attn_fwd(d, w, z, None, P, keep_saved=False)
        elif op.startswith("tri_mul"):
            dirn = A.EVO_TRI_OUT if op.endswith("out") else A.EVO_TRI_IN
            d = B.trimul_desc(dtype, dirn, cfg.n_res, cfg.c_z, cfg.tri_mul_hidden, chunk=chunk)
            out, _ = B.tri_mul_fwd(d, w, z, P, keep_saved=False)
        else:
            m, M = to_dev(inp["m"], dtype), inp["msa_mask"].float().cuda()
            d = B.opm_desc(dtype, cfg.n_seq, cfg.n_res, cfg.c_m, cfg.opm_hidden, cfg.c_z, chunk=chunk)
            out, _ = B.opm_fwd(d, w, m, M, z, keep_saved=False)
        outs.append(out.clone())
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]), f"{op}: chunked forward differs from unchunked"
    if op == "tri_att_start":
        ref = O.tri_att_start(inp["z"], inp["pair_mask"], p, cfg.tri_heads, cfg.tri_head_dim)
    elif op == "tri_att_end":
        ref = O.tri_att_end(inp["z"], inp["pair_mask"], p, cfg.tri_heads, cfg.tri_head_dim)
    elif op == "tri_mul_out":
        ref = O.tri_mul_out(inp["z"], inp["pair_mask"], p)
    elif op == "tri_mul_in":
        ref = O.tri_mul_in(inp["z"], inp["pair_mask"], p)
    else:
        ref = O.outer_product_mean(inp["m"], inp["msa_mask"], p, 1e-5, cfg.opm_eps)
    check_update(f"{op} chunked fwd", outs[1], inp["z"], ref.detach(), dtype)


def _block_chunk_pair(cfg, dtype, seed):
    from paper_2207_05477_amd import binding as B
    inp = device_view(make_inputs(cfg, seed=seed), dtype)
    flat = B.FlatParams(inp["params"][0], "cuda")
    m, z = to_dev(inp["m"], dtype), to_dev(inp["z"], dtype)
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    m0, z0 = B.evoformer_block_fwd(cfg, flat, m, z, mm, pm, dtype=dtype, chunk=0)
    m1, z1 = B.evoformer_block_fwd(cfg, flat, m, z, mm, pm, dtype=dtype, chunk=cfg.chunk or 16)
    torch.cuda.synchronize()
    return (m0, z0), (m1, z1), inp


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_chunked_block_equals_unchunked_small(dtype):
    say(f"chunked block small {dtype}")
    (m0, z0), (m1, z1), inp = _block_chunk_pair(CCFG.replace(chunk=16), dtype, seed=12)
    assert torch.equal(m0, m1)
    assert torch.equal(z0, z1)
    mo_ref, zo_ref = O.stack_fwd(inp, CCFG)
    check_update("z update", z1, inp["z"], zo_ref - inp["z"], dtype)


def test_chunked_block_long_chain_bf16():
    # N_res = 1024, forward only, 128-row chunks (the long-chain inference case)
    cfg = get("C4b")
    say(f"chunked block {cfg.name}")
    (m0, z0), (m1, z1), _ = _block_chunk_pair(cfg, "bf16", seed=32)
    assert torch.isfinite(z1.float()).all()
    assert torch.equal(m0, m1)
    assert torch.equal(z0, z1)


# rows of the long chain checked against the oracle: first and last row, the
# two rows on either side of a chunk seam, and one inside a chunk
C4B_ROWS = [0, 127, 128, 511, 1023]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("op", ["tri_att_start", "tri_att_end", "tri_mul_out", "tri_mul_in", "opm"])
def test_chunked_op_long_chain_sampled_rows_vs_oracle(op):
    from paper_2207_05477_amd import binding as B, _abi as A
    cfg = get("C4b")
    dtype = "bf16"
    say(f"long chain {op}: N_res={cfg.n_res}, chunk {cfg.chunk}")
    inp = device_view(make_inputs(cfg, seed=32, with_grads=False), dtype)
    p = inp["params"][0][op]
    w = B.weight_struct(op, params_dev(p))
    z = to_dev(inp["z"], dtype)
    P = inp["pair_mask"].float().cuda()
    R = cfg.n_res
    if op.startswith("tri_att"):
        kind = A.EVO_ATTN_TRI_START if op.endswith("start") else A.EVO_ATTN_TRI_END
        d = B.attn_desc(kind, dtype, R, R, cfg.c_z, cfg.tri_heads, cfg.tri_head_dim, chunk=cfg.chunk)
        out, _ = B.evo_attn_fwd(d, w, z, None, P, keep_saved=False)
    elif op.startswith("tri_mul"):
        dirn = A.EVO_TRI_OUT if op.endswith("out") else A.EVO_TRI_IN
        d = B.trimul_desc(dtype, dirn, R, cfg.c_z, cfg.tri_mul_hidden, chunk=cfg.chunk)
        out, _ = B.tri_mul_fwd(d, w, z, P, keep_saved=False)
    else:
        m, M = to_dev(inp["m"], dtype), inp["msa_mask"].float().cuda()
        d = B.opm_desc(dtype, cfg.n_seq, R, cfg.c_m, cfg.opm_hidden, cfg.c_z, opm_eps=cfg.opm_eps,
                       chunk=cfg.chunk)
        out, _ = B.opm_fwd(d, w, m, M, z, keep_saved=False)
    torch.cuda.synchronize()
    rows = torch.tensor(C4B_ROWS)
    say("  oracle rows", C4B_ROWS)
    if op == "tri_att_end":
        got, x = out[:, rows], inp["z"][:, rows]
        ref = O.tri_att_end_cols(inp["z"], inp["pair_mask"], p, cfg.tri_heads, cfg.tri_head_dim, rows)
    else:
        got, x = out[rows], inp["z"][rows]
        if op == "tri_att_start":
            ref = O.tri_att_start_rows(inp["z"], inp["pair_mask"], p, cfg.tri_heads, cfg.tri_head_dim, rows)
        elif op.startswith("tri_mul"):
            ref = O.tri_mul_rows(inp["z"], inp["pair_mask"], p, op[-3:].strip("_"), rows)
        else:
            ref = O.outer_product_mean_rows(inp["m"], inp["msa_mask"], p, rows, 1e-5, cfg.opm_eps)
    check_update(f"{op} sampled rows", got, x, ref, dtype)
