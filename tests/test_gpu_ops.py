"""GPU parity of every sub-operation entry point against the FP64 oracle.

Forward: the residual update out - x.  Backward: d_x (including the identity
path), cross-input gradients and every parameter gradient.  Shapes are ragged
(N_res = 40 is not a multiple of any tile) and masks are random with a fully
masked MSA column and pair row, so the uniform-weight reading of fully masked
softmax rows is exercised.  Tolerance: normwise relative 1e-4 (FP32), 2e-2 (BF16), and the max-norm
relative error of each tensor (gpu_util.ETOL).  BF16 runs get the same FP32
parameters as the oracle.
"""
import pytest
import torch

from oracle import evoformer as O
from synth import EvoConfig, make_inputs

from gpu_util import MARGIN, TOL, check, check_update, device_view, oracle_grads, params_dev, say, to_dev

pytestmark = pytest.mark.gpu

OPCFG = EvoConfig("op", n_seq=12, n_res=40, c_m=32, c_z=16, msa_heads=2, msa_head_dim=16,
                  tri_heads=2, tri_head_dim=8, tri_mul_hidden=16, opm_hidden=8,
                  mask_mode="random")


def _setup(dtype, cfg=OPCFG, seed=7):
    from paper_2207_05477_amd import binding as B  # noqa: F401
    inp = make_inputs(cfg, seed=seed, perturb=True)
    return device_view(inp, dtype)


def _zeros_like(p):
    return {k: torch.zeros_like(v) for k, v in p.items()}


def _check_param_grads(tag, dpar, gref, tol):
    for k in dpar:
        check(f"{tag} d{k}", dpar[k], gref[k], tol)


# N_res = 64: whole 64-wide tiles, so the attention kernels stage the pair
# bias with vector loads (keys contiguous in the forward and dQ kernels,
# queries contiguous in the dK/dV kernel); N_res = 40 takes the general path.
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("hd,n_res", [(8, 40), (16, 40), (32, 40), (64, 40), (32, 64)])
def test_row_attn(dtype, hd, n_res):
    from paper_2207_05477_amd import binding as B, _abi as A
    cfg = OPCFG.replace(msa_head_dim=hd, msa_heads=2 if hd < 64 else 1, n_res=n_res)
    say(f"row_attn dtype={dtype} hd={hd} n_res={n_res}")
    inp = _setup(dtype, cfg)
    tol = TOL[dtype]
    H, D = cfg.msa_heads, cfg.msa_head_dim
    p = inp["params"][0]["row_attn"]
    M = inp["msa_mask"]
    upd, g = oracle_grads(lambda m, z, p: O.row_attn(m, z, M, p, H, D),
                          {"m": inp["m"], "z": inp["z"], "p": p}, inp["dm_out"])
    desc = B.attn_desc(A.EVO_ATTN_ROW, dtype, cfg.n_seq, cfg.n_res, cfg.c_m, H, D, c_pair=cfg.c_z)
    pd = params_dev(p)
    w = B.weight_struct("row_attn", pd)
    x, pair, mask = to_dev(inp["m"], dtype), to_dev(inp["z"], dtype), M.float().cuda()
    out, saved = B.evo_attn_fwd(desc, w, x, pair, mask)
    torch.cuda.synchronize()
    check_update("row fwd", out, inp["m"], upd, dtype)
    dpar = _zeros_like(pd)
    dpair = torch.zeros_like(pair)
    dx = B.evo_attn_bwd(desc, w, x, pair, mask, saved, to_dev(inp["dm_out"], dtype),
                        B.weight_struct("row_attn", dpar), d_pair=dpair)
    torch.cuda.synchronize()
    check("row dx", dx, inp["dm_out"] + g["m"], tol)
    check("row dpair", dpair, g["z"], tol)
    # The pair-bias LayerNorm shift gradient is zero by an identity (the bias
    # gradient sums to zero over keys): bound it by its sibling's magnitude.
    zb = dpar.pop("ln_z_b")
    check("row dln_z_b", zb, g["p"]["ln_z_b"], tol, floor=g["p"]["ln_z_g"].norm().item(),
          efloor=g["p"]["ln_z_g"].abs().max().item())
    _check_param_grads("row", dpar, g["p"], tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_col_attn(dtype):
    from paper_2207_05477_amd import binding as B, _abi as A
    say(f"col_attn dtype={dtype}")
    inp = _setup(dtype)
    tol = TOL[dtype]
    cfg = OPCFG
    H, D = cfg.msa_heads, cfg.msa_head_dim
    p = inp["params"][0]["col_attn"]
    M = inp["msa_mask"]
    upd, g = oracle_grads(lambda m, p: O.col_attn(m, M, p, H, D), {"m": inp["m"], "p": p}, inp["dm_out"])
    desc = B.attn_desc(A.EVO_ATTN_COL, dtype, cfg.n_seq, cfg.n_res, cfg.c_m, H, D)
    pd = params_dev(p)
    w = B.weight_struct("col_attn", pd)
    x, mask = to_dev(inp["m"], dtype), M.float().cuda()
    out, saved = B.evo_attn_fwd(desc, w, x, None, mask)
    torch.cuda.synchronize()
    check_update("col fwd", out, inp["m"], upd, dtype)
    dpar = _zeros_like(pd)
    dx = B.evo_attn_bwd(desc, w, x, None, mask, saved, to_dev(inp["dm_out"], dtype),
                        B.weight_struct("col_attn", dpar))
    torch.cuda.synchronize()
    check("col dx", dx, inp["dm_out"] + g["m"], tol)
    _check_param_grads("col", dpar, g["p"], tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_col_global_attn(dtype):
    from paper_2207_05477_amd import binding as B, _abi as A
    say(f"col_global_attn dtype={dtype}")
    cfg = OPCFG.replace(extra_msa=True, msa_heads=4, msa_head_dim=8)
    inp = _setup(dtype, cfg)
    tol = TOL[dtype]
    H, D = cfg.msa_heads, cfg.msa_head_dim
    p = inp["params"][0]["col_attn"]
    M = inp["msa_mask"]
    upd, g = oracle_grads(lambda m, p: O.col_global_attn(m, M, p, H, D, 1e-5, cfg.global_eps),
                          {"m": inp["m"], "p": p}, inp["dm_out"])
    desc = B.attn_desc(A.EVO_ATTN_COL_GLOBAL, dtype, cfg.n_seq, cfg.n_res, cfg.c_m, H, D,
                       global_eps=cfg.global_eps)
    pd = params_dev(p)
    w = B.weight_struct("col_attn", pd)
    x, mask = to_dev(inp["m"], dtype), M.float().cuda()
    out, saved = B.evo_attn_fwd(desc, w, x, None, mask)
    torch.cuda.synchronize()
    check_update("gcol fwd", out, inp["m"], upd, dtype)
    dpar = _zeros_like(pd)
    dx = B.evo_attn_bwd(desc, w, x, None, mask, saved, to_dev(inp["dm_out"], dtype),
                        B.weight_struct("col_attn", dpar))
    torch.cuda.synchronize()
    check("gcol dx", dx, inp["dm_out"] + g["m"], tol)
    _check_param_grads("gcol", dpar, g["p"], tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["start", "end"])
@pytest.mark.parametrize("n_res", [40, 64])
def test_tri_attn(dtype, kind, n_res):
    from paper_2207_05477_amd import binding as B, _abi as A
    say(f"tri_attn_{kind} dtype={dtype} n_res={n_res}")
    cfg = OPCFG.replace(n_res=n_res)
    inp = _setup(dtype, cfg)
    tol = TOL[dtype]
    H, D = cfg.tri_heads, cfg.tri_head_dim
    sub = "tri_att_start" if kind == "start" else "tri_att_end"
    fn = O.tri_att_start if kind == "start" else O.tri_att_end
    p = inp["params"][0][sub]
    P = inp["pair_mask"]
    upd, g = oracle_grads(lambda z, p: fn(z, P, p, H, D), {"z": inp["z"], "p": p}, inp["dz_out"])
    k = A.EVO_ATTN_TRI_START if kind == "start" else A.EVO_ATTN_TRI_END
    desc = B.attn_desc(k, dtype, cfg.n_res, cfg.n_res, cfg.c_z, H, D)
    pd = params_dev(p)
    w = B.weight_struct(sub, pd)
    x, mask = to_dev(inp["z"], dtype), P.float().cuda()
    out, saved = B.evo_attn_fwd(desc, w, x, None, mask)
    torch.cuda.synchronize()
    check_update(f"{sub} fwd", out, inp["z"], upd, dtype)
    dpar = _zeros_like(pd)
    dx = B.evo_attn_bwd(desc, w, x, None, mask, saved, to_dev(inp["dz_out"], dtype),
                        B.weight_struct(sub, dpar))
    torch.cuda.synchronize()
    check(f"{sub} dx", dx, inp["dz_out"] + g["z"], tol)
    _check_param_grads(sub, dpar, g["p"], tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("direction", ["out", "in"])
def test_tri_mul(dtype, direction):
    from paper_2207_05477_amd import binding as B, _abi as A
    say(f"tri_mul_{direction} dtype={dtype}")
    inp = _setup(dtype)
    tol = TOL[dtype]
    cfg = OPCFG
    sub = f"tri_mul_{direction}"
    fn = O.tri_mul_out if direction == "out" else O.tri_mul_in
    p = inp["params"][0][sub]
    P = inp["pair_mask"]
    upd, g = oracle_grads(lambda z, p: fn(z, P, p), {"z": inp["z"], "p": p}, inp["dz_out"])
    desc = B.trimul_desc(dtype, A.EVO_TRI_OUT if direction == "out" else A.EVO_TRI_IN, cfg.n_res,
                         cfg.c_z, cfg.tri_mul_hidden)
    pd = params_dev(p)
    w = B.weight_struct(sub, pd)
    x, mask = to_dev(inp["z"], dtype), P.float().cuda()
    out, saved = B.tri_mul_fwd(desc, w, x, mask)
    torch.cuda.synchronize()
    check_update(f"{sub} fwd", out, inp["z"], upd, dtype)
    dpar = _zeros_like(pd)
    dz = B.tri_mul_bwd(desc, w, x, mask, saved, to_dev(inp["dz_out"], dtype), B.weight_struct(sub, dpar))
    torch.cuda.synchronize()
    check(f"{sub} dz", dz, inp["dz_out"] + g["z"], tol)
    _check_param_grads(sub, dpar, g["p"], tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_opm(dtype):
    from paper_2207_05477_amd import binding as B
    say(f"opm dtype={dtype}")
    inp = _setup(dtype)
    tol = TOL[dtype]
    cfg = OPCFG
    p = inp["params"][0]["opm"]
    M = inp["msa_mask"]
    upd, g = oracle_grads(lambda m, p: O.outer_product_mean(m, M, p, 1e-5, cfg.opm_eps),
                          {"m": inp["m"], "p": p}, inp["dz_out"])
    desc = B.opm_desc(dtype, cfg.n_seq, cfg.n_res, cfg.c_m, cfg.opm_hidden, cfg.c_z, opm_eps=cfg.opm_eps)
    pd = params_dev(p)
    w = B.weight_struct("opm", pd)
    m, z, mask = to_dev(inp["m"], dtype), to_dev(inp["z"], dtype), M.float().cuda()
    zo, saved = B.opm_fwd(desc, w, m, mask, z)
    torch.cuda.synchronize()
    check("opm fwd", zo.double().cpu() - inp["z"], upd, tol)
    dpar = _zeros_like(pd)
    dm = torch.zeros_like(m)
    B.opm_bwd(desc, w, m, mask, saved, to_dev(inp["dz_out"], dtype), dm, B.weight_struct("opm", dpar))
    torch.cuda.synchronize()
    check("opm dm", dm, g["m"], tol)
    _check_param_grads("opm", dpar, g["p"], tol)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("which", ["msa", "pair"])
def test_transition(dtype, which):
    say(f"transition_{which} dtype={dtype}")
    _transition_case(dtype, which, OPCFG)


def _profiled_kernels(fn):
    """Names of the kernels the library launches inside fn() (its launch profiler)."""
    import ctypes
    from paper_2207_05477_amd import _abi as A
    lib = A.load()

    class Stat(ctypes.Structure):
        _fields_ = [("name", ctypes.c_char * 120), ("launches", ctypes.c_int64),
                    ("total_ms", ctypes.c_double), ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]
    lib.evo_profile_begin.restype = None
    lib.evo_profile_end.argtypes = [ctypes.POINTER(Stat), ctypes.c_int32]
    lib.evo_profile_end.restype = ctypes.c_int32
    torch.cuda.synchronize()
    lib.evo_profile_begin()
    try:
        fn()
    finally:
        recs = (Stat * 1024)()
        n = lib.evo_profile_end(recs, 1024)
    assert n >= 0, lib.evo_last_error().decode()
    return [r.name.decode() for r in recs[:n]]


def test_transition_generic_gemm():
    """Rows x channels past 2 GiB (FP32, 1048581 rows of 512, ragged): the plain
    GEMM kernel addresses its operands through 32-bit buffer offsets and rejects
    them, so the general two-level kernel runs the transition's GEMMs.  The
    transition is row-wise, so its forward and input gradient are checked
    against the oracle on sampled rows (first, last, middle)."""
    from paper_2207_05477_amd import binding as B
    dtype = "f32"
    cfg = OPCFG.replace(c_m=512)
    say("transition_generic_gemm dtype=f32 rows=1048581 c=512")
    inp = _setup(dtype, cfg)
    C = 512
    rows = (1 << 31) // (C * 4) + 5
    gen = torch.Generator().manual_seed(11)
    x32 = torch.randn(rows, C, generator=gen)
    up32 = torch.randn(rows, C, generator=gen)
    idx = torch.tensor([0, 1, 777777, rows // 2, rows - 2, rows - 1])
    x64, up = x32[idx].double(), up32[idx].double()
    p = dict(inp["params"][0]["msa_trans"])
    probe = {"choose": MARGIN[dtype]}
    with torch.no_grad():
        O.transition(x64, p, 1e-5, probe)
    p["b_1"] = p["b_1"].to(torch.float32).to(torch.float64)
    upd, g = oracle_grads(lambda x, p: O.transition(x, p, 1e-5), {"x": x64, "p": p}, up)
    desc = B.trans_desc(dtype, rows, C, cfg.transition_factor)
    pd = params_dev(p)
    w = B.weight_struct("msa_trans", pd)
    x = x32.cuda()
    res = {}

    def run():
        res["out"], saved = B.evo_transition_fwd(desc, w, x)
        dpar = _zeros_like(pd)
        res["dx"] = B.evo_transition_bwd(desc, w, x, saved, up32.cuda(), B.weight_struct("msa_trans", dpar))
        torch.cuda.synchronize()
    names = _profiled_kernels(run)
    assert any(n.startswith("gemm_kernel<") for n in names), names
    di = idx.cuda()
    check_update("msa_trans fwd (sampled rows)", res["out"][di], x64, upd, dtype)
    check("msa_trans dx (sampled rows)", res["dx"][di], up + g["x"], TOL[dtype])


def _transition_case(dtype, which, cfg):
    from paper_2207_05477_amd import binding as B
    inp = _setup(dtype, cfg)
    tol = TOL[dtype]
    sub = "msa_trans" if which == "msa" else "pair_trans"
    x64 = inp["m"] if which == "msa" else inp["z"]
    up = inp["dm_out"] if which == "msa" else inp["dz_out"]
    # b_1 re-chosen by the oracle so that every ReLU pre-activation clears zero
    # by MARGIN[dtype] (W_1 as drawn): the ReLU decisions are then the same at
    # any precision whose pre-activation error is below the margin
    p = dict(inp["params"][0][sub])
    probe = {"choose": MARGIN[dtype]}
    with torch.no_grad():
        O.transition(x64, p, 1e-5, probe)
    p["b_1"] = p["b_1"].to(torch.float32).to(torch.float64)
    probe = {}
    with torch.no_grad():
        O.transition(x64, p, 1e-5, probe)
    assert probe["min_abs"][0] >= 0.99 * MARGIN[dtype]
    upd, g = oracle_grads(lambda x, p: O.transition(x, p, 1e-5), {"x": x64, "p": p}, up)
    C = x64.shape[-1]
    rows = x64.numel() // C
    desc = B.trans_desc(dtype, rows, C, cfg.transition_factor)
    pd = params_dev(p)
    w = B.weight_struct(sub, pd)
    x = to_dev(x64, dtype)
    out, saved = B.evo_transition_fwd(desc, w, x)
    torch.cuda.synchronize()
    check_update(f"{sub} fwd", out, x64, upd, dtype)
    dpar = _zeros_like(pd)
    dx = B.evo_transition_bwd(desc, w, x, saved, to_dev(up, dtype), B.weight_struct(sub, dpar))
    torch.cuda.synchronize()
    check(f"{sub} dx", dx, up + g["x"], tol)
    _check_param_grads(sub, dpar, g["p"], tol)
