"""The oracle's pins are sensitive: plausible mistakes planted in copies of
oracle functions (on the CPU) are caught by the brute-force loops or by the
invariants.  Each mutant below must disagree with its pin."""
import math

import torch

import brute
from oracle import evoformer as O
from synth import make_inputs
from test_oracle import TINY, _pl

F64 = torch.float64


def _inp():
    return make_inputs(TINY, seed=5, perturb=True, mask_mode="random")


def _differs(a, b):
    a = torch.as_tensor(a, dtype=F64)
    b = torch.as_tensor(b, dtype=F64)
    return (a - b).abs().max().item() > 1e-6


def test_mutant_tri_mul_in_with_outgoing_contraction_is_caught():
    inp = _inp()
    p = inp["params"][0]["tri_mul_in"]
    mutant = O.tri_mul_out(inp["z"], inp["pair_mask"], p)      # wrong contraction indices
    ref = brute.tri_mul_in(brute.t2l(inp["z"]), brute.t2l(inp["pair_mask"]), _pl(p))
    assert _differs(mutant, ref)


def test_mutant_tri_att_end_untransposed_bias_is_caught():
    inp = _inp()
    p = inp["params"][0]["tri_att_end"]
    z, P = inp["z"], inp["pair_mask"]
    R, H, c = TINY.n_res, TINY.tri_heads, TINY.tri_head_dim
    y = O.layer_norm(z, p["ln_g"], p["ln_b"], 1e-5)
    q = (y @ p["w_q"]).reshape(R, R, H, c)
    k = (y @ p["w_k"]).reshape(R, R, H, c)
    v = (y @ p["w_v"]).reshape(R, R, H, c)
    bias = (y @ p["w_bias"]).permute(2, 0, 1)
    logits = torch.einsum("ijhc,kjhc->jhik", q, k) / math.sqrt(c) + bias[None]   # b_ik, not b_ki
    a = O.masked_softmax(logits, P.t()[:, None, None, :])
    o = torch.einsum("jhik,kjhc->ijhc", a, v)
    g = torch.sigmoid(y @ p["w_g"] + p["b_g"]).reshape(R, R, H, c)
    mutant = (g * o).reshape(R, R, H * c) @ p["w_o"] + p["b_o"]
    ref = brute.tri_att_end(brute.t2l(z), brute.t2l(P), _pl(p), H, c)
    assert _differs(mutant, ref)


def test_mutant_opm_bias_divided_by_count_is_caught():
    inp = _inp()
    p = dict(inp["params"][0]["opm"])
    p["b_o"] = p["b_o"] + 0.5
    S = TINY.n_seq
    good = O.outer_product_mean(inp["m"], inp["msa_mask"], p)
    norm = inp["msa_mask"].t() @ inp["msa_mask"]
    mutant = good - p["b_o"] + p["b_o"] / (1e-3 + norm[..., None])            # bias inside the mean
    ref = brute.outer_product_mean(brute.t2l(inp["m"]), brute.t2l(inp["msa_mask"]), _pl(p))
    assert _differs(mutant, ref) and not _differs(good, ref)
    assert S == TINY.n_seq


def test_mutant_additive_mask_is_caught_on_fully_masked_rows():
    # an additive -1e9 penalty instead of replacement changes fully masked rows
    logits = torch.tensor([[3.0, -2.0, 0.5]], dtype=F64)
    keep = torch.zeros(1, 3, dtype=F64)
    mutant = torch.softmax(logits + 1e9 * (keep - 1), -1)
    ref = brute.softmax_masked(logits[0].tolist(), keep[0].tolist())
    assert _differs(mutant[0], ref)


def test_mutant_unbiased_layernorm_variance_is_caught():
    x = torch.randn(3, 5, dtype=F64, generator=torch.Generator().manual_seed(0))
    g = torch.ones(5, dtype=F64)
    b = torch.zeros(5, dtype=F64)
    mu = x.mean(-1, keepdim=True)
    mutant = (x - mu) / torch.sqrt(x.var(-1, keepdim=True, unbiased=True) + 1e-5)
    ref = [brute.ln_vec(r, g.tolist(), b.tolist(), 1e-5) for r in x.tolist()]
    assert _differs(mutant, ref)


def test_mutant_scaled_pair_bias_is_caught():
    inp = _inp()
    p = dict(inp["params"][0]["row_attn"])
    scaled = dict(p)
    scaled["w_bias"] = p["w_bias"] / math.sqrt(TINY.msa_head_dim)              # bias scaled like q.k
    mutant = O.row_attn(inp["m"], inp["z"], inp["msa_mask"], scaled, TINY.msa_heads, TINY.msa_head_dim)
    ref = brute.row_attn(brute.t2l(inp["m"]), brute.t2l(inp["z"]), brute.t2l(inp["msa_mask"]),
                         _pl(p), TINY.msa_heads, TINY.msa_head_dim)
    assert _differs(mutant, ref)
