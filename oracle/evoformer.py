"""FP64 CPU oracle of one Evoformer block, forward (and backward via autograd).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never calls it.  It
shares no code with the HIP path.

It is the plain mathematical definition, written with einsum / matmul on
float64 CPU tensors, with no blocking, fusion or reordering.  Gradients are
those of this definition (torch autograd), pinned against central finite
differences by the oracle tests.

The paper (HelixFold, arXiv 2207.05477) names the operators but defers their
equations to AlphaFold2 (Section "Challenges": the AlphaFold2 architecture;
Section "Hyperparameter setting": the AlphaFold2 settings are followed
strictly).  What the paper itself fixes:

* tensor shapes: MSA [N_seq, N_res, C_m], pair [N_res, N_res, C_z] (Section
  "Dynamic Axial Parallelism");
* the attention family: row-wise and column-wise gated self-attention with an
  optional gate before the output and a pair-derived bias added to the logits
  ("nonbatched_bias") (Section "Fused Gated Self-Attention" and the caption of
  the gated-attention figure; Section "Memory Read/Write In-place");
* the two tracks of a block: the MSA stack, the outer product mean as the only
  MSA-to-pair link, and the pair stack (Section "Branch Parallelism").

The readings taken where the paper is silent:

* LayerNorm: biased variance, eps = 1e-5, one affine per LayerNorm.
* Attention logits scale 1/sqrt(head_dim), applied to q.k only (not the bias).
* Masks replace the logits of masked keys by the constant MASK_LOGIT before
  the softmax (not an additive penalty): a partially masked row gives masked
  keys exactly zero weight, a fully masked row gives uniform weights, and no
  gradient flows through a masked logit.  Queries are never masked.
* Outer product mean: Linear_o(sum_s a_si (x) b_sj / (eps + n_ij)), the output
  bias not divided, eps a runtime argument (default 1e-3).
* Incoming triangle multiplication: x_ij = sum_k a_ki * b_kj.
* Dropout is the identity.
* The ReLU of the transitions decides on the exact pre-activation.  Its
  derivative jumps at zero, so a gradient is only precision-independent where
  no pre-activation lies within rounding of zero.  For gradient parity the
  tests therefore build inputs whose ReLU decisions are clear:
  with_relu_margins() re-chooses each transition's b_1, on this oracle's own
  forward, so that every pre-activation is at least a given margin away from
  zero, and asserts the margin it reached (test-input construction; the
  definition itself is unchanged).
* Block order: row attention, column attention, MSA transition, outer product
  mean, outgoing and incoming triangle multiplication, triangle attention
  around the starting and the ending node, pair transition.
* A stack whose activations are stored in BFloat16 (Section "BFloat16": the
  intermediate activations are BF16, the parameters FP32) hands BF16 tensors
  from block to block: with boundary="bf16" the stack rounds each block's
  output before the next block and each inter-block gradient before the
  block below, and computes every block exactly on those values.  The
  stack's own inputs, outputs and returned gradients are not rounded here.
"""
from __future__ import annotations

import math

import torch

F64 = torch.float64
MASK_LOGIT = -1e30


def layer_norm(x, g, b, eps):
    """LayerNorm over the channel (last) axis with biased variance."""
    mu = x.mean(-1, keepdim=True)
    var = ((x - mu) ** 2).mean(-1, keepdim=True)
    return (x - mu) / torch.sqrt(var + eps) * g + b


def masked_softmax(logits, keep):
    """Softmax over the last axis; logits where ``keep == 0`` are replaced by
    MASK_LOGIT first (mask reading above)."""
    s = torch.where(keep > 0, logits, torch.full_like(logits, MASK_LOGIT))
    return torch.softmax(s, dim=-1)


def row_attn(m, z, msa_mask, p, heads, head_dim, eps=1e-5):
    """MSA row-wise gated self-attention with pair bias (the gated-attention
    figure; "nonbatched_bias" of Section "Memory Read/Write In-place").

    o^h_si = g^h_si * sum_j softmax_j(q^h_si . k^h_sj / sqrt(c) + b^h_ij) v^h_sj,
    keys masked by msa_mask[s, j]; returns the update Linear_o(concat_h o)."""
    S, R, _ = m.shape
    H, c = heads, head_dim
    y = layer_norm(m, p["ln_g"], p["ln_b"], eps)
    yz = layer_norm(z, p["ln_z_g"], p["ln_z_b"], eps)
    q = (y @ p["w_q"]).reshape(S, R, H, c)
    k = (y @ p["w_k"]).reshape(S, R, H, c)
    v = (y @ p["w_v"]).reshape(S, R, H, c)
    bias = (yz @ p["w_bias"]).permute(2, 0, 1)                    # [H, i, j]
    logits = torch.einsum("sihc,sjhc->shij", q, k) / math.sqrt(c) + bias[None]
    a = masked_softmax(logits, msa_mask[:, None, None, :])
    o = torch.einsum("shij,sjhc->sihc", a, v)
    g = torch.sigmoid(y @ p["w_g"] + p["b_g"]).reshape(S, R, H, c)
    return (g * o).reshape(S, R, H * c) @ p["w_o"] + p["b_o"]


def col_attn(m, msa_mask, p, heads, head_dim, eps=1e-5):
    """MSA column-wise gated self-attention (no pair bias): for each residue i
    the MSA rows attend to each other; keys masked by msa_mask[t, i]."""
    S, R, _ = m.shape
    H, c = heads, head_dim
    y = layer_norm(m, p["ln_g"], p["ln_b"], eps)
    q = (y @ p["w_q"]).reshape(S, R, H, c)
    k = (y @ p["w_k"]).reshape(S, R, H, c)
    v = (y @ p["w_v"]).reshape(S, R, H, c)
    logits = torch.einsum("sihc,tihc->ihst", q, k) / math.sqrt(c)
    a = masked_softmax(logits, msa_mask.t()[:, None, None, :])
    o = torch.einsum("ihst,tihc->sihc", a, v)
    g = torch.sigmoid(y @ p["w_g"] + p["b_g"]).reshape(S, R, H, c)
    return (g * o).reshape(S, R, H * c) @ p["w_o"] + p["b_o"]


def col_global_attn(m, msa_mask, p, heads, head_dim, eps=1e-5, global_eps=1e-10):
    """Column global attention of the extra-MSA stack: one masked-mean query
    per residue column and head, single-head keys and values shared by all
    heads, per-row gate."""
    S, R, _ = m.shape
    H, c = heads, head_dim
    y = layer_norm(m, p["ln_g"], p["ln_b"], eps)
    q = (y @ p["w_q"]).reshape(S, R, H, c)
    k = y @ p["w_k"]                                              # [S, R, c]
    v = y @ p["w_v"]
    qbar = torch.einsum("si,sihc->ihc", msa_mask, q) / (msa_mask.sum(0)[:, None, None] + global_eps)
    logits = torch.einsum("ihc,tic->iht", qbar, k) / math.sqrt(c)
    a = masked_softmax(logits, msa_mask.t()[:, None, :])
    o = torch.einsum("iht,tic->ihc", a, v)                        # [R, H, c]
    g = torch.sigmoid(y @ p["w_g"] + p["b_g"]).reshape(S, R, H, c)
    return (g * o[None]).reshape(S, R, H * c) @ p["w_o"] + p["b_o"]


def _bf16(t):
    return t.detach().to(torch.bfloat16).to(F64)


def transition(x, p, eps=1e-5, probe=None):
    """Two-layer MLP with ReLU on the LayerNormed input:
    Linear_2(ReLU(Linear_1(LayerNorm(x)))).

    ``probe`` (test-input construction only, see with_relu_margins): a dict;
    with probe["choose"] = margin, b_1 is first replaced (in ``p``) by
    relu_margin_bias of this call's pre-activations; every call appends
    min |pre-activation| to probe["min_abs"]."""
    y = layer_norm(x, p["ln_g"], p["ln_b"], eps)
    if probe is not None and probe.get("choose") is not None:
        with torch.no_grad():
            u = p["w_1"].shape[1]
            p["b_1"] = relu_margin_bias((y @ p["w_1"]).reshape(-1, u), probe["choose"])
    pre = y @ p["w_1"] + p["b_1"]
    if probe is not None:
        probe.setdefault("min_abs", []).append(pre.detach().abs().min().item())
    return torch.relu(pre) @ p["w_2"] + p["b_2"]


# Active fractions the hidden units of a margin-constructed transition aim at,
# cycled over the units: always off, always on, and mixed decisions.
MARGIN_TARGETS = (0.0, 1.0, 0.5, 0.1, 0.9)


def relu_margin_bias(pre, margin):
    """Bias b[u] for the hidden units of one transition such that every
    pre[r, u] + b[u] is at least ``margin`` away from zero.

    pre: [rows, units] pre-activations without the bias.  The unit's threshold
    -b[u] is below all of its values (always on), above all of them (always
    off), or the midpoint of two consecutive sorted values at least 2 * margin
    apart (on for the rows above it); of these, the one whose active fraction
    is closest to MARGIN_TARGETS[u % 5] is taken."""
    n, units = pre.shape
    v, _ = torch.sort(pre.detach(), dim=0)
    ok = torch.ones(n + 1, units, dtype=torch.bool)
    ok[1:n] = (v[1:] - v[:-1]) >= 2 * margin
    frac = (n - torch.arange(n + 1, dtype=F64)) / n            # rows above threshold k
    tgt = torch.tensor(MARGIN_TARGETS, dtype=F64)[torch.arange(units) % len(MARGIN_TARGETS)]
    score = (frac[:, None] - tgt[None, :]).abs()
    score[~ok] = math.inf
    k = score.argmin(0)
    below = torch.where(k == 0, v[0] - 2 * margin, v[(k - 1).clamp(min=0), torch.arange(units)])
    above = torch.where(k == n, v[n - 1] + 2 * margin, v[k.clamp(max=n - 1), torch.arange(units)])
    return -(below + above) / 2


def outer_product_mean(m, msa_mask, p, eps=1e-5, opm_eps=1e-3):
    """Outer product mean, the only MSA-to-pair communication of a block
    (Section "Branch Parallelism").  O_ij = sum_s a_si (x) b_sj flattened as
    p*c + q, divided by eps + n_ij with n_ij = sum_s M_si M_sj, then Linear_o."""
    S, R, _ = m.shape
    y = layer_norm(m, p["ln_g"], p["ln_b"], eps)
    a = msa_mask[..., None] * (y @ p["w_a"] + p["b_a"])
    b = msa_mask[..., None] * (y @ p["w_b"] + p["b_b"])
    c = a.shape[-1]
    outer = torch.einsum("sip,sjq->ijpq", a, b).reshape(R, R, c * c)
    norm = msa_mask.t() @ msa_mask                                # n_ij
    return (outer / (opm_eps + norm[..., None])) @ p["w_o"] + p["b_o"]


def _tri_mul_proj(z, pair_mask, p, eps):
    y = layer_norm(z, p["ln_g"], p["ln_b"], eps)
    a = pair_mask[..., None] * torch.sigmoid(y @ p["w_ag"] + p["b_ag"]) * (y @ p["w_ap"] + p["b_ap"])
    b = pair_mask[..., None] * torch.sigmoid(y @ p["w_bg"] + p["b_bg"]) * (y @ p["w_bp"] + p["b_bp"])
    g = torch.sigmoid(y @ p["w_g"] + p["b_g"])
    return a, b, g


def tri_mul_out(z, pair_mask, p, eps=1e-5):
    """Triangle multiplicative update with outgoing edges: x_ij = sum_k a_ik b_jk."""
    a, b, g = _tri_mul_proj(z, pair_mask, p, eps)
    x = torch.einsum("ikc,jkc->ijc", a, b)
    return g * (layer_norm(x, p["ln_out_g"], p["ln_out_b"], eps) @ p["w_o"] + p["b_o"])


def tri_mul_in(z, pair_mask, p, eps=1e-5):
    """Triangle multiplicative update with incoming edges: x_ij = sum_k a_ki b_kj."""
    a, b, g = _tri_mul_proj(z, pair_mask, p, eps)
    x = torch.einsum("kic,kjc->ijc", a, b)
    return g * (layer_norm(x, p["ln_out_g"], p["ln_out_b"], eps) @ p["w_o"] + p["b_o"])


def tri_att_start(z, pair_mask, p, heads, head_dim, eps=1e-5):
    """Triangle attention around the starting node:
    o_ij = g_ij * sum_k softmax_k(q_ij . k_ik / sqrt(c) + b_jk) v_ik, keys masked by P_ik."""
    R = z.shape[0]
    H, c = heads, head_dim
    y = layer_norm(z, p["ln_g"], p["ln_b"], eps)
    q = (y @ p["w_q"]).reshape(R, R, H, c)
    k = (y @ p["w_k"]).reshape(R, R, H, c)
    v = (y @ p["w_v"]).reshape(R, R, H, c)
    bias = (y @ p["w_bias"]).permute(2, 0, 1)                      # [H, j, k]
    logits = torch.einsum("ijhc,ikhc->ihjk", q, k) / math.sqrt(c) + bias[None]
    a = masked_softmax(logits, pair_mask[:, None, None, :])
    o = torch.einsum("ihjk,ikhc->ijhc", a, v)
    g = torch.sigmoid(y @ p["w_g"] + p["b_g"]).reshape(R, R, H, c)
    return (g * o).reshape(R, R, H * c) @ p["w_o"] + p["b_o"]


def tri_att_end(z, pair_mask, p, heads, head_dim, eps=1e-5):
    """Triangle attention around the ending node:
    o_ij = g_ij * sum_k softmax_k(q_ij . k_kj / sqrt(c) + b_ki) v_kj, keys masked by P_kj."""
    R = z.shape[0]
    H, c = heads, head_dim
    y = layer_norm(z, p["ln_g"], p["ln_b"], eps)
    q = (y @ p["w_q"]).reshape(R, R, H, c)
    k = (y @ p["w_k"]).reshape(R, R, H, c)
    v = (y @ p["w_v"]).reshape(R, R, H, c)
    bias = (y @ p["w_bias"]).permute(2, 0, 1)                      # [H, k, i]
    logits = torch.einsum("ijhc,kjhc->jhik", q, k) / math.sqrt(c) + bias.transpose(1, 2)[None]
    a = masked_softmax(logits, pair_mask.t()[:, None, None, :])
    o = torch.einsum("jhik,kjhc->ijhc", a, v)
    g = torch.sigmoid(y @ p["w_g"] + p["b_g"]).reshape(R, R, H, c)
    return (g * o).reshape(R, R, H * c) @ p["w_o"] + p["b_o"]


# Sub-operation numbers of a block (the dropout generator's counter word 1).
SUBOP_ID = {"row_attn": 0, "col_attn": 1, "msa_trans": 2, "opm": 3, "tri_mul_out": 4, "tri_mul_in": 5,
            "tri_att_start": 6, "tri_att_end": 7, "pair_trans": 8}


def drop(x, dropout, sub, orient, rate, template=0):
    """Shared dropout of a residual update x [A, B, C] (AlphaFold2's dropout,
    which the paper keeps by following its settings): one multiplier per
    (B, C) shared along axis 0 ("row"), or per (A, C) shared along axis 1
    ("col"), 0 or 1 / (1 - rate), drawn by oracle.philox from the counter
    (element, sub-operation | template << 8, offset).  dropout: None (off) or
    (seed, offset)."""
    if dropout is None or rate == 0.0:
        return x
    from . import philox
    seed, offset = dropout
    n_idx = x.shape[1] if orient == "row" else x.shape[0]
    word = SUBOP_ID[sub] | (template << 8)
    mask = torch.from_numpy(philox.dropout_mask(seed, offset, word, n_idx, x.shape[-1], rate))
    return x * (mask[None] if orient == "row" else mask[:, None])


def block(m, z, msa_mask, pair_mask, p, cfg, probe=None, dropout=None):
    """One Evoformer block (the extra-MSA block when cfg.extra_msa): residual
    MSA stack, outer product mean, residual pair stack.  cfg.opm_first puts the
    outer product mean first (z <- z + OPM(m) on the block's input m): the MSA
    stack and the pair stack then depend only on (m, z + OPM(m)), the two
    independent branches Branch Parallelism runs on two devices (Section
    "Branch Parallelism").  dropout: None or (seed, offset), see drop()."""
    eps = cfg.ln_eps
    if cfg.opm_first:
        z = z + outer_product_mean(m, msa_mask, p["opm"], eps, cfg.opm_eps)
    m = m + drop(row_attn(m, z, msa_mask, p["row_attn"], cfg.msa_heads, cfg.msa_head_dim, eps),
                 dropout, "row_attn", "row", cfg.drop_row_attn)
    if cfg.extra_msa:
        m = m + col_global_attn(m, msa_mask, p["col_attn"], cfg.msa_heads, cfg.msa_head_dim,
                                eps, cfg.global_eps)
    else:
        m = m + col_attn(m, msa_mask, p["col_attn"], cfg.msa_heads, cfg.msa_head_dim, eps)
    m = m + transition(m, p["msa_trans"], eps, probe)
    if not cfg.opm_first:
        z = z + outer_product_mean(m, msa_mask, p["opm"], eps, cfg.opm_eps)
    z = z + drop(tri_mul_out(z, pair_mask, p["tri_mul_out"], eps), dropout, "tri_mul_out", "row",
                 cfg.drop_tri_mul)
    z = z + drop(tri_mul_in(z, pair_mask, p["tri_mul_in"], eps), dropout, "tri_mul_in", "row",
                 cfg.drop_tri_mul)
    z = z + drop(tri_att_start(z, pair_mask, p["tri_att_start"], cfg.tri_heads, cfg.tri_head_dim, eps),
                 dropout, "tri_att_start", "row", cfg.drop_tri_att)
    z = z + drop(tri_att_end(z, pair_mask, p["tri_att_end"], cfg.tri_heads, cfg.tri_head_dim, eps),
                 dropout, "tri_att_end", "col", cfg.drop_tri_att)
    z = z + transition(z, p["pair_trans"], eps, probe)
    return m, z


def template_pair_block(t, pair_mask, p, cfg, probe=None, dropout=None, template=0):
    """One block of the template pair stack (AlphaFold2's TemplatePairStack,
    which the paper's initial-training forward includes as TemplateEmbedding):
    the pair-stack operators on one template's pair features t [R, R, c_t],
    in the order triangle attention around the starting node, around the
    ending node, outgoing and incoming triangle multiplication, transition."""
    eps = cfg.ln_eps
    H, c = cfg.tri_heads, cfg.tri_head_dim
    t = t + drop(tri_att_start(t, pair_mask, p["tri_att_start"], H, c, eps), dropout, "tri_att_start", "row",
                 cfg.drop_tri_att, template)
    t = t + drop(tri_att_end(t, pair_mask, p["tri_att_end"], H, c, eps), dropout, "tri_att_end", "col",
                 cfg.drop_tri_att, template)
    t = t + drop(tri_mul_out(t, pair_mask, p["tri_mul_out"], eps), dropout, "tri_mul_out", "row",
                 cfg.drop_tri_mul, template)
    t = t + drop(tri_mul_in(t, pair_mask, p["tri_mul_in"], eps), dropout, "tri_mul_in", "row",
                 cfg.drop_tri_mul, template)
    return t + transition(t, p["pair_trans"], eps, probe)


def _store(t, boundary):
    """A tensor handed between blocks, in the stack's storage precision."""
    if boundary is None:
        return t
    if boundary == "bf16":
        return _bf16(t)
    raise ValueError(boundary)


def _block_dropout(dropout, i):
    """Block i of a stack draws its dropout masks at offset + i."""
    return None if dropout is None else (dropout[0], dropout[1] + i)


def stack(m, z, msa_mask, pair_mask, blocks, cfg, boundary=None, probe=None, dropout=None):
    """Blocks applied in sequence with independent parameters."""
    for i, p in enumerate(blocks):
        if i > 0:
            m, z = _store(m, boundary), _store(z, boundary)
        m, z = block(m, z, msa_mask, pair_mask, p, cfg, probe, _block_dropout(dropout, i))
    return m, z


def _leaf(t):
    return t.detach().clone().to(F64).requires_grad_(True)


def stack_fwd_bwd(inp, cfg, want_param_grads=True, boundary=None, dropout=None):
    """Forward and backward of the stack on float64 copies of ``inp``.

    Returns (m_out, z_out, grads) with grads = {"m", "z", "params"} where
    grads["params"] mirrors inp["params"]; the loss is
    <m_out, dm_out> + <z_out, dz_out>.  The chain rule is applied block by
    block (each block's forward is re-run under autograd during the backward),
    which keeps the memory of one block; the values are those of the plain
    definition.  `boundary`: storage precision between blocks (see the module
    docstring)."""
    msa_mask = inp["msa_mask"].to(F64)
    pair_mask = inp["pair_mask"].to(F64)
    acts = [(inp["m"].detach().to(F64), inp["z"].detach().to(F64))]
    with torch.no_grad():
        for i, p in enumerate(inp["params"]):
            mi, zi = acts[-1]
            if i > 0:
                mi, zi = _store(mi, boundary), _store(zi, boundary)
                acts[-1] = (mi, zi)
            acts.append(block(mi, zi, msa_mask, pair_mask, p, cfg, None, _block_dropout(dropout, i)))
    dm = inp["dm_out"].to(F64)
    dz = inp["dz_out"].to(F64)
    pgrads = [None] * len(inp["params"])
    for i in reversed(range(len(inp["params"]))):
        m = _leaf(acts[i][0])
        z = _leaf(acts[i][1])
        blk = inp["params"][i]
        leaves = {s: {k: (_leaf(v) if want_param_grads else v.detach().to(F64))
                      for k, v in blk[s].items()} for s in blk}
        mo, zo = block(m, z, msa_mask, pair_mask, leaves, cfg, None, _block_dropout(dropout, i))
        ((mo * dm).sum() + (zo * dz).sum()).backward()
        dm, dz = m.grad, z.grad
        if i > 0:
            dm, dz = _store(dm, boundary), _store(dz, boundary)
        if want_param_grads:
            pgrads[i] = {s: {k: v.grad for k, v in leaves[s].items()} for s in leaves}
    grads = {"m": dm, "z": dz}
    if want_param_grads:
        grads["params"] = pgrads
    return acts[-1][0], acts[-1][1], grads


def stack_fwd(inp, cfg, boundary=None, probe=None, dropout=None):
    with torch.no_grad():
        return stack(inp["m"].to(F64), inp["z"].to(F64), inp["msa_mask"].to(F64),
                     inp["pair_mask"].to(F64), inp["params"], cfg, boundary, probe, dropout)


def template_stack_fwd_bwd(inp, cfg, dropout=None, want_param_grads=True):
    """Forward and backward of the template pair stack on float64 copies of
    ``inp`` (synth.make_template_inputs): every template t[n] goes through the
    same blocks (template index n in the dropout counter); the loss is
    <t_out, dt_out>.  Returns (t_out, grads) with grads = {"t", "params"}."""
    t = inp["t"].detach().to(F64).requires_grad_(True)
    P = inp["pair_mask"].to(F64)
    leaves = [{s: {k: (v.detach().clone().to(F64).requires_grad_(want_param_grads))
                   for k, v in blk[s].items()} for s in blk} for blk in inp["params"]]
    outs = []
    for n in range(t.shape[0]):
        x = t[n]
        for i, p in enumerate(leaves):
            x = template_pair_block(x, P[n], p, cfg, None, _block_dropout(dropout, i), n)
        outs.append(x)
    out = torch.stack(outs)
    (out * inp["dt_out"].to(F64)).sum().backward()
    grads = {"t": t.grad}
    if want_param_grads:
        grads["params"] = [{s: {k: v.grad for k, v in blk[s].items()} for s in blk} for blk in leaves]
    return out.detach(), grads


def relu_margin(inp, cfg, boundary=None, dropout=None):
    """Smallest |pre-activation| over every transition of the stack's forward."""
    probe = {}
    stack_fwd(inp, cfg, boundary, probe, dropout)
    return min(probe["min_abs"])


def with_relu_margins(inp, cfg, margin, boundary=None, dropout=None):
    """A copy of ``inp`` whose transitions' b_1 are re-chosen (relu_margin_bias)
    on this oracle's forward of the stack, transition by transition in forward
    order, so that every ReLU pre-activation is at least ``margin`` from zero:
    gradients are then unambiguous at any precision whose pre-activation error
    stays below the margin.  Asserts the margin on a fresh forward."""
    out = dict(inp)
    out["params"] = [{s: {k: v.clone() for k, v in blk[s].items()} for s in blk} for blk in inp["params"]]
    stack_fwd(out, cfg, boundary, {"choose": margin}, dropout)
    got = relu_margin(out, cfg, boundary, dropout)
    assert got >= margin * (1 - 1e-9), f"ReLU margin {got} < {margin}"
    return out


def template_stack_fwd(inp, cfg, dropout=None, probe=None):
    """Forward of the template pair stack (every template through the same
    blocks), block by block.  probe (test-input construction): as in
    transition(); with probe["choose"], each block's pair-transition b_1 is
    chosen on the pre-activations of all templates together, so one b_1 clears
    the margin for every template."""
    P = inp["pair_mask"].to(F64)
    xs = [inp["t"][n].detach().to(F64) for n in range(inp["t"].shape[0])]
    eps = cfg.ln_eps
    H, c = cfg.tri_heads, cfg.tri_head_dim
    with torch.no_grad():
        for i, p in enumerate(inp["params"]):
            dr = _block_dropout(dropout, i)
            for n in range(len(xs)):
                x = xs[n]
                x = x + drop(tri_att_start(x, P[n], p["tri_att_start"], H, c, eps), dr, "tri_att_start", "row",
                             cfg.drop_tri_att, n)
                x = x + drop(tri_att_end(x, P[n], p["tri_att_end"], H, c, eps), dr, "tri_att_end", "col",
                             cfg.drop_tri_att, n)
                x = x + drop(tri_mul_out(x, P[n], p["tri_mul_out"], eps), dr, "tri_mul_out", "row",
                             cfg.drop_tri_mul, n)
                x = x + drop(tri_mul_in(x, P[n], p["tri_mul_in"], eps), dr, "tri_mul_in", "row",
                             cfg.drop_tri_mul, n)
                xs[n] = x
            pt = p["pair_trans"]
            if probe is not None and probe.get("choose") is not None:
                u = pt["w_1"].shape[1]
                pre = torch.cat([(layer_norm(x, pt["ln_g"], pt["ln_b"], eps) @ pt["w_1"]).reshape(-1, u)
                                 for x in xs])
                pt["b_1"] = relu_margin_bias(pre, probe["choose"])
            sub = None if probe is None else {}
            xs = [x + transition(x, pt, eps, sub) for x in xs]
            if probe is not None:
                probe.setdefault("min_abs", []).extend(sub["min_abs"])
    return torch.stack(xs)


def with_template_relu_margins(inp, cfg, margin, dropout=None):
    """with_relu_margins for the template pair stack: a copy of ``inp`` whose
    pair transitions' b_1 clear ``margin`` on every template; asserts it."""
    out = dict(inp)
    out["params"] = [{s: {k: v.clone() for k, v in blk[s].items()} for s in blk} for blk in inp["params"]]
    template_stack_fwd(out, cfg, dropout, {"choose": margin})
    probe = {}
    template_stack_fwd(out, cfg, dropout, probe)
    got = min(probe["min_abs"])
    assert got >= margin * (1 - 1e-9), f"ReLU margin {got} < {margin}"
    return out


# ---------------------------------------------------------------- selected output rows
# The pair-stack operators evaluated for a few output rows only, from the full
# input: the same definitions as above with the query (or output) row index
# restricted to ``rows``.  They let a long chain (N_res = 1024, whose full
# triangle-attention logits would take tens of GB in float64) be checked on
# sampled rows.  Each returns the update for those rows, [len(rows), R, C]
# (columns [R, len(cols), C] for the ending-node attention).

def tri_att_start_rows(z, pair_mask, p, heads, head_dim, rows, eps=1e-5):
    """Rows i in ``rows`` of tri_att_start: o_ij = g_ij * sum_k softmax_k(q_ij . k_ik /
    sqrt(c) + b_jk) v_ik; the bias b_jk needs LayerNorm(z) at every (j, k)."""
    R = z.shape[0]
    H, c = heads, head_dim
    rows = torch.as_tensor(rows)
    y = layer_norm(z, p["ln_g"], p["ln_b"], eps)
    bias = (y @ p["w_bias"]).permute(2, 0, 1)                      # [H, j, k]
    yr = y[rows]                                                   # [n, R, C]
    n = yr.shape[0]
    q = (yr @ p["w_q"]).reshape(n, R, H, c)
    k = (yr @ p["w_k"]).reshape(n, R, H, c)
    v = (yr @ p["w_v"]).reshape(n, R, H, c)
    logits = torch.einsum("ijhc,ikhc->ihjk", q, k) / math.sqrt(c) + bias[None]
    a = masked_softmax(logits, pair_mask[rows][:, None, None, :])
    o = torch.einsum("ihjk,ikhc->ijhc", a, v)
    g = torch.sigmoid(yr @ p["w_g"] + p["b_g"]).reshape(n, R, H, c)
    return (g * o).reshape(n, R, H * c) @ p["w_o"] + p["b_o"]


def tri_att_end_cols(z, pair_mask, p, heads, head_dim, cols, eps=1e-5):
    """Columns j in ``cols`` of tri_att_end: o_ij = g_ij * sum_k softmax_k(q_ij . k_kj /
    sqrt(c) + b_ki) v_kj, keys masked by P_kj; returns [R, len(cols), C]."""
    R = z.shape[0]
    H, c = heads, head_dim
    cols = torch.as_tensor(cols)
    y = layer_norm(z, p["ln_g"], p["ln_b"], eps)
    bias = (y @ p["w_bias"]).permute(2, 0, 1)                      # [H, k, i]
    yc = y[:, cols]                                                # [R, n, C]
    n = yc.shape[1]
    q = (yc @ p["w_q"]).reshape(R, n, H, c)
    k = (yc @ p["w_k"]).reshape(R, n, H, c)
    v = (yc @ p["w_v"]).reshape(R, n, H, c)
    logits = torch.einsum("ijhc,kjhc->jhik", q, k) / math.sqrt(c) + bias.transpose(1, 2)[None]
    a = masked_softmax(logits, pair_mask[:, cols].t()[:, None, None, :])
    o = torch.einsum("jhik,kjhc->ijhc", a, v)
    g = torch.sigmoid(yc @ p["w_g"] + p["b_g"]).reshape(R, n, H, c)
    return (g * o).reshape(R, n, H * c) @ p["w_o"] + p["b_o"]


def tri_mul_rows(z, pair_mask, p, direction, rows, eps=1e-5):
    """Rows i in ``rows`` of tri_mul_out (x_ij = sum_k a_ik b_jk) or tri_mul_in
    (x_ij = sum_k a_ki b_kj), then g * Linear_o(LayerNorm_out(x))."""
    rows = torch.as_tensor(rows)
    a, b, g = _tri_mul_proj(z, pair_mask, p, eps)
    if direction == "out":
        x = torch.einsum("ikc,jkc->ijc", a[rows], b)
    else:
        x = torch.einsum("kic,kjc->ijc", a[:, rows], b)
    return g[rows] * (layer_norm(x, p["ln_out_g"], p["ln_out_b"], eps) @ p["w_o"] + p["b_o"])


def outer_product_mean_rows(m, msa_mask, p, rows, eps=1e-5, opm_eps=1e-3):
    """Rows i in ``rows`` of outer_product_mean: O_ij = sum_s a_si (x) b_sj / (eps + n_ij)."""
    rows = torch.as_tensor(rows)
    R = m.shape[1]
    y = layer_norm(m, p["ln_g"], p["ln_b"], eps)
    a = msa_mask[..., None] * (y @ p["w_a"] + p["b_a"])
    b = msa_mask[..., None] * (y @ p["w_b"] + p["b_b"])
    c = a.shape[-1]
    outer = torch.einsum("sip,sjq->ijpq", a[:, rows], b).reshape(len(rows), R, c * c)
    norm = msa_mask[:, rows].t() @ msa_mask
    return (outer / (opm_eps + norm[..., None])) @ p["w_o"] + p["b_o"]
