"""Pins of the FP64 oracle against things other than itself.

* brute-force pure-Python loops (tests/brute.py) on tiny inputs, every op and
  the whole block, with masks that include fully masked rows and columns;
* library routines (F.layer_norm, matmul) where an op reduces to one;
* invariants fixed by the mathematics: transposition identities between the
  starting/ending-node and outgoing/incoming ops, permutation equivariance,
  LayerNorm shift-equivariance of the whole block, softmax normalisation and
  mask semantics, closed forms (outer product mean with one MSA row);
* central finite differences (gradcheck) for the oracle's gradients;
* the paper's worked memory example (tests/golden/).
"""
import json
import math
import os

import pytest
import torch
import torch.nn.functional as F

import brute
from oracle import evoformer as O
from oracle import sizes
from synth import EvoConfig, make_inputs

F64 = torch.float64

TINY = EvoConfig("tiny", n_seq=3, n_res=4, c_m=6, c_z=5, msa_heads=2, msa_head_dim=3,
                 tri_heads=2, tri_head_dim=2, tri_mul_hidden=3, opm_hidden=2,
                 transition_factor=2, mask_mode="random")
TINY_X = TINY.replace(name="tiny_extra", extra_msa=True)


def _inp(cfg=TINY, seed=5, mask_mode="random"):
    return make_inputs(cfg, seed=seed, perturb=True, mask_mode=mask_mode)


def _pl(p):
    return {k: brute.t2l(v) for k, v in p.items()}


def _close(a, b, tol=1e-10):
    a = torch.as_tensor(a, dtype=F64)
    b = torch.as_tensor(b, dtype=F64)
    assert a.shape == b.shape, (a.shape, b.shape)
    err = (a - b).abs().max().item()
    scale = max(1.0, b.abs().max().item())
    assert err <= tol * scale, f"max abs err {err} (scale {scale})"


# ---------------------------------------------------------------- LayerNorm

def test_layer_norm_matches_library_and_invariants():
    g = torch.Generator().manual_seed(1)
    x = torch.randn(7, 11, dtype=F64, generator=g) * 3 + 2
    gam = torch.randn(11, dtype=F64, generator=g)
    bet = torch.randn(11, dtype=F64, generator=g)
    ref = F.layer_norm(x, (11,), gam, bet, eps=1e-5)
    _close(O.layer_norm(x, gam, bet, 1e-5), ref, 1e-12)
    y = O.layer_norm(x, torch.ones(11, dtype=F64), torch.zeros(11, dtype=F64), 0.0)
    _close(y.mean(-1), torch.zeros(7), 1e-12)
    _close(y.var(-1, unbiased=False), torch.ones(7), 1e-12)


# ---------------------------------------------------------------- softmax / masks

def test_masked_softmax_semantics():
    g = torch.Generator().manual_seed(2)
    logits = torch.randn(5, 6, dtype=F64, generator=g) * 10
    keep = (torch.rand(5, 6, generator=g) > 0.4).to(F64)
    keep[0] = 0.0                       # fully masked row
    keep[1] = 1.0
    keep[1, 2] = 0.0
    a = O.masked_softmax(logits, keep)
    _close(a.sum(-1), torch.ones(5), 1e-14)
    _close(a[0], torch.full((6,), 1 / 6, dtype=F64), 1e-14)   # uniform when fully masked
    for r in range(1, 5):
        if keep[r].sum() > 0:
            assert torch.all(a[r][keep[r] == 0] == 0.0)       # exactly zero weight
    for r in range(5):
        _close(a[r], brute.softmax_masked(logits[r].tolist(), keep[r].tolist()), 1e-14)


def test_masked_softmax_gradient_rows_sum_to_zero_and_masked_zero():
    g = torch.Generator().manual_seed(3)
    logits = torch.randn(4, 7, dtype=F64, generator=g).requires_grad_(True)
    keep = (torch.rand(4, 7, generator=g) > 0.3).to(F64)
    keep[2] = 0.0
    up = torch.randn(4, 7, dtype=F64, generator=g)
    (O.masked_softmax(logits, keep) * up).sum().backward()
    d = logits.grad
    _close(d.sum(-1), torch.zeros(4), 1e-13)       # sum_k dS_k = 0 (pair-bias grad rows)
    assert torch.all(d[keep == 0] == 0.0)          # no gradient through masked logits


# ---------------------------------------------------------------- brute force, per op

def test_row_attn_vs_brute():
    inp = _inp()
    p = inp["params"][0]["row_attn"]
    got = O.row_attn(inp["m"], inp["z"], inp["msa_mask"], p, TINY.msa_heads, TINY.msa_head_dim)
    ref = brute.row_attn(brute.t2l(inp["m"]), brute.t2l(inp["z"]), brute.t2l(inp["msa_mask"]),
                         _pl(p), TINY.msa_heads, TINY.msa_head_dim)
    _close(got, ref)


def test_col_attn_vs_brute():
    inp = _inp()
    p = inp["params"][0]["col_attn"]
    got = O.col_attn(inp["m"], inp["msa_mask"], p, TINY.msa_heads, TINY.msa_head_dim)
    ref = brute.col_attn(brute.t2l(inp["m"]), brute.t2l(inp["msa_mask"]), _pl(p),
                         TINY.msa_heads, TINY.msa_head_dim)
    _close(got, ref)


def test_col_global_attn_vs_brute():
    inp = _inp(TINY_X)
    p = inp["params"][0]["col_attn"]
    got = O.col_global_attn(inp["m"], inp["msa_mask"], p, TINY.msa_heads, TINY.msa_head_dim)
    ref = brute.col_global_attn(brute.t2l(inp["m"]), brute.t2l(inp["msa_mask"]), _pl(p),
                                TINY.msa_heads, TINY.msa_head_dim)
    _close(got, ref)


@pytest.mark.parametrize("sub", ["msa_trans", "pair_trans"])
def test_transition_vs_brute(sub):
    inp = _inp()
    x = inp["m"] if sub == "msa_trans" else inp["z"]
    p = inp["params"][0][sub]
    _close(O.transition(x, p), brute.transition(brute.t2l(x), _pl(p)))


def test_opm_vs_brute():
    inp = _inp()
    p = inp["params"][0]["opm"]
    got = O.outer_product_mean(inp["m"], inp["msa_mask"], p)
    ref = brute.outer_product_mean(brute.t2l(inp["m"]), brute.t2l(inp["msa_mask"]), _pl(p))
    _close(got, ref)


@pytest.mark.parametrize("sub", ["tri_mul_out", "tri_mul_in"])
def test_tri_mul_vs_brute(sub):
    inp = _inp()
    p = inp["params"][0][sub]
    fn = O.tri_mul_out if sub == "tri_mul_out" else O.tri_mul_in
    bf = brute.tri_mul_out if sub == "tri_mul_out" else brute.tri_mul_in
    _close(fn(inp["z"], inp["pair_mask"], p), bf(brute.t2l(inp["z"]), brute.t2l(inp["pair_mask"]), _pl(p)))


@pytest.mark.parametrize("sub", ["tri_att_start", "tri_att_end"])
def test_tri_att_vs_brute(sub):
    inp = _inp()
    p = inp["params"][0][sub]
    fn = O.tri_att_start if sub == "tri_att_start" else O.tri_att_end
    bf = brute.tri_att_start if sub == "tri_att_start" else brute.tri_att_end
    got = fn(inp["z"], inp["pair_mask"], p, TINY.tri_heads, TINY.tri_head_dim)
    ref = bf(brute.t2l(inp["z"]), brute.t2l(inp["pair_mask"]), _pl(p), TINY.tri_heads, TINY.tri_head_dim)
    _close(got, ref)


@pytest.mark.parametrize("cfg", [TINY, TINY_X], ids=["evoformer", "extra_msa"])
def test_block_vs_brute(cfg):
    inp = _inp(cfg)
    p = inp["params"][0]
    m, z = O.block(inp["m"], inp["z"], inp["msa_mask"], inp["pair_mask"], p, cfg)
    pl = {s: _pl(p[s]) for s in p}
    bm, bz = brute.block(brute.t2l(inp["m"]), brute.t2l(inp["z"]), brute.t2l(inp["msa_mask"]),
                         brute.t2l(inp["pair_mask"]), pl, cfg)
    _close(m, bm)
    _close(z, bz)


# ---------------------------------------------------------------- invariants

def test_col_attn_is_row_attn_without_bias_on_transposed_msa():
    inp = _inp()
    pc = inp["params"][0]["col_attn"]
    pr = dict(pc)
    pr["ln_z_g"] = torch.ones(TINY.c_z, dtype=F64)
    pr["ln_z_b"] = torch.zeros(TINY.c_z, dtype=F64)
    pr["w_bias"] = torch.zeros(TINY.c_z, TINY.msa_heads, dtype=F64)
    mT = inp["m"].transpose(0, 1).contiguous()
    zT = torch.zeros(TINY.n_seq, TINY.n_seq, TINY.c_z, dtype=F64)
    row = O.row_attn(mT, zT, inp["msa_mask"].t(), pr, TINY.msa_heads, TINY.msa_head_dim)
    col = O.col_attn(inp["m"], inp["msa_mask"], pc, TINY.msa_heads, TINY.msa_head_dim)
    _close(col, row.transpose(0, 1), 1e-12)


def test_tri_att_end_is_transposed_start():
    inp = _inp()
    p = inp["params"][0]["tri_att_start"]
    z, P = inp["z"], inp["pair_mask"]
    end = O.tri_att_end(z, P, p, TINY.tri_heads, TINY.tri_head_dim)
    start_T = O.tri_att_start(z.transpose(0, 1), P.t(), p, TINY.tri_heads, TINY.tri_head_dim)
    _close(end, start_T.transpose(0, 1), 1e-12)


def test_tri_mul_in_is_transposed_out_with_swapped_operands():
    inp = _inp()
    p = inp["params"][0]["tri_mul_in"]
    swapped = dict(p)
    for x, y in (("w_ap", "w_bp"), ("b_ap", "b_bp"), ("w_ag", "w_bg"), ("b_ag", "b_bg")):
        swapped[x], swapped[y] = p[y], p[x]
    z, P = inp["z"], inp["pair_mask"]
    tin = O.tri_mul_in(z, P, p)
    tout_T = O.tri_mul_out(z.transpose(0, 1), P.t(), swapped)
    _close(tin, tout_T.transpose(0, 1), 1e-12)


def test_tri_mul_contraction_is_per_channel_matmul():
    # x_ij = sum_k a_ik b_jk is, channel by channel, the matrix product A_c B_c^T
    g = torch.Generator().manual_seed(4)
    a = torch.randn(5, 5, 3, dtype=F64, generator=g)
    b = torch.randn(5, 5, 3, dtype=F64, generator=g)
    x_out = torch.einsum("ikc,jkc->ijc", a, b)
    x_in = torch.einsum("kic,kjc->ijc", a, b)
    for c in range(3):
        _close(x_out[..., c], a[..., c] @ b[..., c].t(), 1e-13)
        _close(x_in[..., c], a[..., c].t() @ b[..., c], 1e-13)


def test_row_attn_equivariant_to_msa_row_and_residue_permutation():
    inp = _inp(TINY.replace(n_seq=4, n_res=5))
    p = inp["params"][0]["row_attn"]
    m, z, M = inp["m"], inp["z"], inp["msa_mask"]
    H, c = TINY.msa_heads, TINY.msa_head_dim
    base = O.row_attn(m, z, M, p, H, c)
    ps = torch.tensor([2, 0, 3, 1])
    _close(O.row_attn(m[ps], z, M[ps], p, H, c), base[ps], 1e-12)
    pr = torch.tensor([4, 2, 0, 1, 3])
    got = O.row_attn(m[:, pr], z[pr][:, pr], M[:, pr], p, H, c)
    _close(got, base[:, pr], 1e-12)


def test_tri_att_start_equivariant_to_residue_permutation():
    inp = _inp(TINY.replace(n_res=5))
    p = inp["params"][0]["tri_att_start"]
    z, P = inp["z"], inp["pair_mask"]
    pr = torch.tensor([3, 0, 4, 2, 1])
    base = O.tri_att_start(z, P, p, TINY.tri_heads, TINY.tri_head_dim)
    got = O.tri_att_start(z[pr][:, pr], P[pr][:, pr], p, TINY.tri_heads, TINY.tri_head_dim)
    _close(got, base[pr][:, pr], 1e-12)


def test_masked_keys_do_not_influence_output():
    # Perturbing m at (s=0, j=3) moves key/value 3 of MSA row 0, which is masked
    # there, and query (0, 3) itself; every other query of row 0 is unchanged.
    inp = _inp()
    pr = inp["params"][0]["row_attn"]
    m, zz, M = inp["m"].clone(), inp["z"], inp["msa_mask"].clone()
    M[0] = 1.0
    M[0, 3] = 0.0
    out = O.row_attn(m, zz, M, pr, TINY.msa_heads, TINY.msa_head_dim)
    m2 = m.clone()
    m2[0, 3] += torch.linspace(-2.0, 3.0, TINY.c_m, dtype=F64) ** 2
    out2 = O.row_attn(m2, zz, M, pr, TINY.msa_heads, TINY.msa_head_dim)
    _close(out2[0, [0, 1, 2]], out[0, [0, 1, 2]], 1e-12)
    assert (out2[0, 3] - out[0, 3]).abs().max() > 1e-3


def test_opm_single_row_is_one_outer_product():
    cfg = TINY.replace(n_seq=1, opm_eps=0.0)
    inp = make_inputs(cfg, seed=9, perturb=True, mask_mode="full")
    p = inp["params"][0]["opm"]
    m = inp["m"]
    got = O.outer_product_mean(m, inp["msa_mask"], p, opm_eps=0.0)
    y = F.layer_norm(m[0], (cfg.c_m,), p["ln_g"], p["ln_b"], eps=1e-5)
    a = y @ p["w_a"] + p["b_a"]
    b = y @ p["w_b"] + p["b_b"]
    R, ch = cfg.n_res, cfg.opm_hidden
    for i in range(R):
        for j in range(R):
            flat = torch.outer(a[i], b[j]).reshape(ch * ch)
            _close(got[i, j], flat @ p["w_o"] + p["b_o"], 1e-12)


def test_opm_is_matmul_of_projections():
    inp = _inp(mask_mode="full")
    p = inp["params"][0]["opm"]
    S, R, ch = TINY.n_seq, TINY.n_res, TINY.opm_hidden
    y = F.layer_norm(inp["m"], (TINY.c_m,), p["ln_g"], p["ln_b"], eps=1e-5)
    a = (y @ p["w_a"] + p["b_a"]).reshape(S, R * ch)
    b = (y @ p["w_b"] + p["b_b"]).reshape(S, R * ch)
    outer = (a.t() @ b).reshape(R, ch, R, ch).permute(0, 2, 1, 3).reshape(R, R, ch * ch)
    ref = outer / (1e-3 + S) @ p["w_o"] + p["b_o"]
    _close(O.outer_product_mean(inp["m"], inp["msa_mask"], p), ref, 1e-12)


@pytest.mark.parametrize("cfg", [TINY, TINY_X], ids=["evoformer", "extra_msa"])
def test_block_layernorm_shift_equivariance(cfg):
    # Every update reads only LayerNormed inputs, so adding a per-position
    # constant to all channels of m or z passes straight through the block.
    inp = _inp(cfg)
    p = inp["params"][0]
    g = torch.Generator().manual_seed(11)
    dm = torch.randn(cfg.n_seq, cfg.n_res, 1, dtype=F64, generator=g) * 3
    dz = torch.randn(cfg.n_res, cfg.n_res, 1, dtype=F64, generator=g) * 3
    m0, z0 = O.block(inp["m"], inp["z"], inp["msa_mask"], inp["pair_mask"], p, cfg)
    m1, z1 = O.block(inp["m"] + dm, inp["z"] + dz, inp["msa_mask"], inp["pair_mask"], p, cfg)
    _close(m1, m0 + dm, 1e-10)
    _close(z1, z0 + dz, 1e-10)


# ---------------------------------------------------------------- gradients

def _gc(fn, *args):
    assert torch.autograd.gradcheck(fn, args, eps=1e-6, atol=1e-7, rtol=1e-5)


def test_gradcheck_ops():
    inp = _inp()
    P = inp["params"][0]
    M, Pm = inp["msa_mask"], inp["pair_mask"]
    m = inp["m"].clone().requires_grad_(True)
    z = inp["z"].clone().requires_grad_(True)
    H, c, Ht, ct = TINY.msa_heads, TINY.msa_head_dim, TINY.tri_heads, TINY.tri_head_dim
    wq = P["row_attn"]["w_q"].clone().requires_grad_(True)

    def row(m_, z_, wq_):
        p = dict(P["row_attn"]); p["w_q"] = wq_
        return O.row_attn(m_, z_, M, p, H, c)
    _gc(row, m, z, wq)
    _gc(lambda m_: O.col_attn(m_, M, P["col_attn"], H, c), m)
    _gc(lambda m_: O.transition(m_, P["msa_trans"]), m)
    wo = P["opm"]["w_o"].clone().requires_grad_(True)

    def opm(m_, wo_):
        p = dict(P["opm"]); p["w_o"] = wo_
        return O.outer_product_mean(m_, M, p)
    _gc(opm, m, wo)
    _gc(lambda z_: O.tri_mul_out(z_, Pm, P["tri_mul_out"]), z)
    _gc(lambda z_: O.tri_mul_in(z_, Pm, P["tri_mul_in"]), z)
    wb = P["tri_att_start"]["w_bias"].clone().requires_grad_(True)

    def tas(z_, wb_):
        p = dict(P["tri_att_start"]); p["w_bias"] = wb_
        return O.tri_att_start(z_, Pm, p, Ht, ct)
    _gc(tas, z, wb)
    _gc(lambda z_: O.tri_att_end(z_, Pm, P["tri_att_end"], Ht, ct), z)


def test_gradcheck_global_attn_and_block():
    inp = _inp(TINY_X)
    p = inp["params"][0]
    m = inp["m"].clone().requires_grad_(True)
    z = inp["z"].clone().requires_grad_(True)
    _gc(lambda m_: O.col_global_attn(m_, inp["msa_mask"], p["col_attn"], 2, 3), m)
    inp2 = _inp(TINY)
    m2 = inp2["m"].clone().requires_grad_(True)
    z2 = inp2["z"].clone().requires_grad_(True)
    _gc(lambda a, b: O.block(a, b, inp2["msa_mask"], inp2["pair_mask"], inp2["params"][0], TINY), m2, z2)
    assert z.shape[0] == TINY.n_res


def test_stack_fwd_bwd_grads_match_gradcheck_direction():
    # directional derivative of the stack loss vs a central difference
    cfg = TINY.replace(n_blocks=2)
    inp = make_inputs(cfg, seed=13, perturb=True)
    m_out, z_out, grads = O.stack_fwd_bwd(inp, cfg)
    g = torch.Generator().manual_seed(14)
    vm = torch.randn(inp["m"].shape, dtype=F64, generator=g)
    vz = torch.randn(inp["z"].shape, dtype=F64, generator=g)
    h = 1e-5

    def loss(dm_, dz_):
        x = dict(inp); x["m"] = inp["m"] + dm_; x["z"] = inp["z"] + dz_
        mo, zo = O.stack_fwd(x, cfg)
        return (mo * inp["dm_out"]).sum() + (zo * inp["dz_out"]).sum()
    fd = (loss(h * vm, h * vz) - loss(-h * vm, -h * vz)) / (2 * h)
    an = (grads["m"] * vm).sum() + (grads["z"] * vz).sum()
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_stack_bf16_boundary_one_block_is_plain():
    # a single block has no internal boundary: the storage reading changes nothing
    cfg = TINY.replace(n_blocks=1)
    inp = make_inputs(cfg, seed=15, perturb=True)
    a = O.stack_fwd_bwd(inp, cfg)
    b = O.stack_fwd_bwd(inp, cfg, boundary="bf16")
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert torch.equal(a[2]["m"], b[2]["m"]) and torch.equal(a[2]["z"], b[2]["z"])


def test_stack_bf16_boundary_rounds_between_blocks():
    # two blocks: the second block sees the BF16-stored output of the first, and
    # the first block's backward sees the BF16-stored gradient of the second
    cfg = TINY.replace(n_blocks=2)
    inp = make_inputs(cfg, seed=16, perturb=True)
    mo, zo, g = O.stack_fwd_bwd(inp, cfg, boundary="bf16")
    mm, pm = inp["msa_mask"], inp["pair_mask"]
    rnd = lambda t: t.detach().to(torch.bfloat16).to(F64)
    with torch.no_grad():
        m1, z1 = O.block(inp["m"], inp["z"], mm, pm, inp["params"][0], cfg)
        m2, z2 = O.block(rnd(m1), rnd(z1), mm, pm, inp["params"][1], cfg)
    assert torch.equal(mo, m2) and torch.equal(zo, z2)
    assert not torch.equal(rnd(m1), m1)            # the rounding is not a no-op here
    # block 1's input gradient, rounded, drives block 0's backward
    m1r, z1r = rnd(m1).requires_grad_(True), rnd(z1).requires_grad_(True)
    a, b = O.block(m1r, z1r, mm, pm, inp["params"][1], cfg)
    ((a * inp["dm_out"]).sum() + (b * inp["dz_out"]).sum()).backward()
    m0 = inp["m"].clone().requires_grad_(True)
    z0 = inp["z"].clone().requires_grad_(True)
    a, b = O.block(m0, z0, mm, pm, inp["params"][0], cfg)
    ((a * rnd(m1r.grad)).sum() + (b * rnd(z1r.grad)).sum()).backward()
    assert torch.allclose(g["m"], m0.grad, rtol=1e-12, atol=1e-12)
    assert torch.allclose(g["z"], z0.grad, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- paper's worked example

def test_golden_logits_memory_example():
    path = os.path.join(os.path.dirname(__file__), "golden", "logits_memory.json")
    with open(path) as f:
        cases = json.load(f)["cases"]
    for cse in cases:
        if cse["kind"] == "logits":
            got = sizes.logits_bytes(cse["n_seq"], cse["n_head"], cse["n_res"], cse["elem_bytes"],
                                     cse.get("chunk", 0))
        else:
            got = sizes.activation_bytes(cse["rows"], cse["cols"], cse["elem_bytes"], cse.get("chunk", 0))
        exp = cse["bytes"] if "bytes" in cse else cse["gib"] * 2 ** 30
        assert math.isclose(got, exp, rel_tol=1e-12), (cse, got)


# ---------------------------------------------------------------- margin-constructed inputs

def test_relu_margin_bias_clears_zero_and_follows_targets():
    g = torch.Generator().manual_seed(3)
    pre = torch.randn(400, 10, dtype=F64, generator=g)
    for margin in (1e-3, 0.05):
        b = O.relu_margin_bias(pre, margin)
        x = pre + b
        assert x.abs().min().item() >= margin * (1 - 1e-12)
        frac = (x > 0).to(F64).mean(0)
        for u in range(10):
            t = O.MARGIN_TARGETS[u % len(O.MARGIN_TARGETS)]
            if t in (0.0, 1.0):
                assert frac[u].item() == t            # always-off / always-on units
        # a unit aiming at 0.5 ends on a feasible gap, so its decisions are mixed
        # whenever one exists (400 normal samples have gaps of 2e-3 near the tails)
        assert 0.0 < frac[2].item() < 1.0 or margin == 0.05


def test_relu_margin_bias_brute_force_small():
    # brute force over every threshold between sorted values
    pre = torch.tensor([[0.0, 1.0], [0.5, 1.02], [2.0, 3.0], [2.1, 5.0]], dtype=F64)
    b = O.relu_margin_bias(pre, 0.2)
    # unit 0 aims at 0.0 (always off): threshold above 2.1 by the margin
    assert math.isclose(b[0].item(), -(2.1 + 0.2), rel_tol=1e-12)
    # unit 1 aims at 1.0 (always on): threshold below 1.0 by the margin
    assert math.isclose(b[1].item(), -(1.0 - 0.2), rel_tol=1e-12)
    pre3 = torch.tensor([[0.0] * 3, [0.1] * 3, [1.0] * 3, [1.1] * 3], dtype=F64)
    b3 = O.relu_margin_bias(pre3, 0.2)
    # unit 2 aims at 0.5: the only interior gap >= 0.4 is (0.1, 1.0), midpoint 0.55
    assert math.isclose(b3[2].item(), -0.55, rel_tol=1e-12)


@pytest.mark.parametrize("boundary", [None, "bf16"])
def test_with_relu_margins_changes_only_b1_and_holds_margin(boundary):
    cfg = TINY.replace(n_blocks=2, n_seq=5, n_res=6)
    inp = make_inputs(cfg, seed=9, perturb=True)
    out = O.with_relu_margins(inp, cfg, 0.05, boundary)
    assert O.relu_margin(out, cfg, boundary) >= 0.05 * (1 - 1e-9)
    for bi, (pa, pb) in enumerate(zip(inp["params"], out["params"])):
        for sub in pa:
            for k in pa[sub]:
                same = torch.equal(pa[sub][k], pb[sub][k])
                assert same == (not (sub in ("msa_trans", "pair_trans") and k == "b_1")), (bi, sub, k)
    # the oracle's gradients on the constructed inputs agree with a central
    # difference taken with steps that stay inside the margin
    m_out, z_out, grads = O.stack_fwd_bwd(out, cfg, boundary=None)
    g = torch.Generator().manual_seed(2)
    vm = torch.randn(inp["m"].shape, dtype=F64, generator=g)
    h = 1e-6

    def loss(dm_):
        x = dict(out); x["m"] = out["m"] + dm_
        mo, zo = O.stack_fwd(x, cfg)
        return (mo * out["dm_out"]).sum() + (zo * out["dz_out"]).sum()
    fd = (loss(h * vm) - loss(-h * vm)) / (2 * h)
    an = (grads["m"] * vm).sum()
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


# ---------------------------------------------------------------- selected rows

def test_row_restricted_pair_ops_equal_full_ops():
    cfg = TINY.replace(n_res=7, c_z=6, n_seq=4)
    inp = make_inputs(cfg, seed=17, perturb=True)
    z, P, M, m = inp["z"], inp["pair_mask"], inp["msa_mask"], inp["m"]
    blk = inp["params"][0]
    rows = [0, 3, 6]
    H, c = cfg.tri_heads, cfg.tri_head_dim
    _close(O.tri_att_start_rows(z, P, blk["tri_att_start"], H, c, rows),
           O.tri_att_start(z, P, blk["tri_att_start"], H, c)[rows], 1e-12)
    _close(O.tri_att_end_cols(z, P, blk["tri_att_end"], H, c, rows),
           O.tri_att_end(z, P, blk["tri_att_end"], H, c)[:, rows], 1e-12)
    _close(O.tri_mul_rows(z, P, blk["tri_mul_out"], "out", rows), O.tri_mul_out(z, P, blk["tri_mul_out"])[rows], 1e-12)
    _close(O.tri_mul_rows(z, P, blk["tri_mul_in"], "in", rows), O.tri_mul_in(z, P, blk["tri_mul_in"])[rows], 1e-12)
    _close(O.outer_product_mean_rows(m, M, blk["opm"], rows), O.outer_product_mean(m, M, blk["opm"])[rows], 1e-12)


# ---------------------------------------------------------------- dropout generator

def test_philox_known_answer_vectors():
    from oracle import philox
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")
    with open(path) as f:
        cases = json.load(f)["cases"]
    for cse in cases:
        ctr = [int(x, 16) for x in cse["ctr"]]
        key = [int(x, 16) for x in cse["key"]]
        got = philox.philox4x32_10([ctr], key)[0].tolist()
        assert got == [int(x, 16) for x in cse["out"]], cse


def test_dropout_mask_rate_and_scale():
    from oracle import philox
    m = philox.dropout_mask(seed=123, offset=7, subop=4, n_idx=256, channels=128, rate=0.25)
    vals = set(m.ravel().tolist())
    assert vals <= {0.0, 1.0 / (1.0 - float(torch.tensor(0.25, dtype=torch.float32)))}
    frac = (m == 0).mean()
    assert abs(frac - 0.25) < 0.01                    # 32768 draws: 4 sigma ~ 0.01
    assert philox.dropout_mask(123, 7, 4, 4, 4, 0.0).min() == 1.0
    # counters differ by sub-op and offset: the masks differ
    a = philox.dropout_mask(1, 0, 0, 16, 16, 0.5)
    assert not (a == philox.dropout_mask(1, 0, 1, 16, 16, 0.5)).all()
    assert not (a == philox.dropout_mask(1, 1, 0, 16, 16, 0.5)).all()



# ---------------------------------------------------------------- block variants

def _dropout_masks(cfg, seed, offset, R, template=0):
    """The dropout multipliers of each sub-operation, drawn straight from the generator."""
    from oracle import philox
    rates = {"row_attn": cfg.drop_row_attn, "tri_mul_out": cfg.drop_tri_mul, "tri_mul_in": cfg.drop_tri_mul,
             "tri_att_start": cfg.drop_tri_att, "tri_att_end": cfg.drop_tri_att}
    chans = {"row_attn": cfg.c_m}
    return {s: philox.dropout_mask(seed, offset, O.SUBOP_ID[s] | (template << 8), R, chans.get(s, cfg.c_z),
                                   r).tolist()
            for s, r in rates.items()}


@pytest.mark.parametrize("opm_first", [False, True], ids=["af2_order", "opm_first"])
@pytest.mark.parametrize("dropout", [False, True], ids=["no_dropout", "dropout"])
def test_block_variants_vs_brute(opm_first, dropout):
    cfg = TINY.replace(opm_first=opm_first, drop_row_attn=0.3, drop_tri_mul=0.4, drop_tri_att=0.5)
    inp = _inp(cfg)
    p = inp["params"][0]
    dr = (77, 5) if dropout else None
    m, z = O.block(inp["m"], inp["z"], inp["msa_mask"], inp["pair_mask"], p, cfg, dropout=dr)
    pl = {s: _pl(p[s]) for s in p}
    masks = _dropout_masks(cfg, 77, 5, cfg.n_res) if dropout else None
    if dropout:   # the masks really drop something at these rates
        assert any(v == 0.0 for row in masks["tri_att_end"] for v in row)
    bm, bz = brute.block(brute.t2l(inp["m"]), brute.t2l(inp["z"]), brute.t2l(inp["msa_mask"]),
                         brute.t2l(inp["pair_mask"]), pl, cfg, masks)
    _close(m, bm)
    _close(z, bz)


def test_opm_first_makes_the_branches_independent():
    # OPM first: the pair stack's output does not depend on the MSA stack's
    # parameters, and the MSA stack's output does not depend on the pair stack's
    # (in the AlphaFold2 order the pair stack reads the updated MSA)
    inp = _inp(TINY)
    p = inp["params"][0]
    p2 = {s: dict(v) for s, v in p.items()}
    p2["msa_trans"]["w_2"] = p2["msa_trans"]["w_2"] * 3.0
    p3 = {s: dict(v) for s, v in p.items()}
    p3["tri_mul_out"]["w_o"] = p3["tri_mul_out"]["w_o"] * 3.0
    args = (inp["m"], inp["z"], inp["msa_mask"], inp["pair_mask"])
    for first in (True, False):
        cfg = TINY.replace(opm_first=first)
        m1, z1 = O.block(*args, p, cfg)
        m2, z2 = O.block(*args, p2, cfg)
        m3, z3 = O.block(*args, p3, cfg)
        assert torch.equal(m1, m3)                     # MSA output never reads the pair stack
        assert torch.equal(z1, z2) == first            # pair output ignores the MSA stack only when OPM is first


def test_dropout_rate_zero_is_identity_and_masks_are_shared_along_their_axis():
    cfg = TINY.replace(drop_row_attn=0.0, drop_tri_mul=0.0, drop_tri_att=0.0)
    inp = _inp(cfg)
    p = inp["params"][0]
    args = (inp["m"], inp["z"], inp["msa_mask"], inp["pair_mask"], p)
    a = O.block(*args, cfg)
    b = O.block(*args, cfg, dropout=(3, 4))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # row-wise: one multiplier per (j, c) for every i; column-wise: per (i, c) for every j
    x = torch.ones(5, 6, 7, dtype=F64)
    r = O.drop(x, (9, 1), "tri_mul_out", "row", 0.5)
    assert torch.equal(r, r[:1].expand_as(r))
    c = O.drop(x, (9, 1), "tri_att_end", "col", 0.5)
    assert torch.equal(c, c[:, :1].expand_as(c))


def test_template_block_vs_brute_and_gradcheck():
    from synth import make_template_inputs
    cfg = TINY.replace(n_templ=2, c_z=4, tri_heads=2, tri_head_dim=2, tri_mul_hidden=3, transition_factor=2)
    inp = make_template_inputs(cfg, seed=8, perturb=True)
    p = inp["params"][0]
    pl = {s: _pl(p[s]) for s in p}
    for n in range(cfg.n_templ):
        for dr in (None, (5, 2)):
            got = O.template_pair_block(inp["t"][n], inp["pair_mask"][n], p, cfg, dropout=dr, template=n)
            masks = None
            if dr is not None:
                masks = _dropout_masks(cfg, 5, 2, cfg.n_res, template=n)
                masks.pop("row_attn")
            ref = brute.template_block(brute.t2l(inp["t"][n]), brute.t2l(inp["pair_mask"][n]), pl, cfg, masks)
            _close(got, ref)
    t = inp["t"][0].clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: O.template_pair_block(x, inp["pair_mask"][0], p, cfg, dropout=(5, 2)),
                                    (t,), eps=1e-6, atol=1e-6)
    # the stack helper: same outputs as the block applied per template
    out, g = O.template_stack_fwd_bwd(inp, cfg, dropout=(5, 2))
    for n in range(cfg.n_templ):
        ref = O.template_pair_block(inp["t"][n], inp["pair_mask"][n], p, cfg, dropout=(5, 2), template=n)
        _close(out[n], ref.detach(), 1e-12)


def test_template_stack_forward_and_relu_margins():
    # the block-by-block template forward equals the per-template chain, and the
    # margin construction clears the margin on every template at once
    from synth import make_template_inputs
    cfg = TINY.replace(n_templ=3, n_blocks=2, c_z=4, tri_heads=2, tri_head_dim=2, tri_mul_hidden=3,
                       transition_factor=2)
    inp = make_template_inputs(cfg, seed=9, perturb=True)
    out, _ = O.template_stack_fwd_bwd(inp, cfg, dropout=(3, 1), want_param_grads=False)
    _close(O.template_stack_fwd(inp, cfg, dropout=(3, 1)), out, 1e-12)
    m = O.with_template_relu_margins(inp, cfg, 0.05, dropout=(3, 1))
    probe = {}
    O.template_stack_fwd(m, cfg, dropout=(3, 1), probe=probe)
    assert min(probe["min_abs"]) >= 0.05 * (1 - 1e-9)
    assert len(probe["min_abs"]) == cfg.n_blocks * cfg.n_templ
    # only the transitions' b_1 change
    for b0, b1 in zip(inp["params"], m["params"]):
        for s in b0:
            for k in b0[s]:
                if not (s == "pair_trans" and k == "b_1"):
                    assert torch.equal(b0[s][k], b1[s][k])


def test_relu_margins_with_dropout():
    cfg = TINY.replace(n_blocks=2)
    inp = make_inputs(cfg, seed=10, perturb=True)
    m = O.with_relu_margins(inp, cfg, 0.05, dropout=(4, 7))
    assert O.relu_margin(m, cfg, dropout=(4, 7)) >= 0.05 * (1 - 1e-9)
