"""Brute-force pure-Python loop versions of every Evoformer sub-operation.

Independent of ``oracle/``: scalar loops over explicit indices with ``math``
functions, written from the operator definitions (AlphaFold2's, which the paper
follows; readings listed in the oracle's module docstring).  Only for tiny
shapes.  Every function takes and returns nested Python lists.
"""
from __future__ import annotations

import math

MASK_LOGIT = -1e30


def t2l(t):
    return t.detach().double().tolist()


def ln_vec(x, g, b, eps):
    n = len(x)
    mean = sum(x) / n
    var = sum((v - mean) * (v - mean) for v in x) / n
    inv = 1.0 / math.sqrt(var + eps)
    return [(x[c] - mean) * inv * g[c] + b[c] for c in range(n)]


def lin(x, W, bias=None):
    n_out = len(W[0])
    out = []
    for o in range(n_out):
        acc = 0.0
        for i in range(len(x)):
            acc += x[i] * W[i][o]
        if bias is not None:
            acc += bias[o]
        out.append(acc)
    return out


def sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def softmax_masked(vals, keep):
    s = [vals[k] if keep[k] > 0 else MASK_LOGIT for k in range(len(vals))]
    mx = max(s)
    e = [math.exp(v - mx) for v in s]
    tot = sum(e)
    return [v / tot for v in e]


def _zeros(*shape):
    if len(shape) == 1:
        return [0.0] * shape[0]
    return [_zeros(*shape[1:]) for _ in range(shape[0])]


def _gated_attend(qs, ks, vs, gs, biases, keep, H, c):
    """One query position: qs[h][d], keys ks[k][h][d], vs[k][h][d], gate gs[h][d],
    biases[h][k], key mask keep[k] -> gated context flattened [h*c + d]."""
    out = []
    nk = len(ks)
    for h in range(H):
        logits = []
        for kk in range(nk):
            dot = 0.0
            for d in range(c):
                dot += qs[h][d] * ks[kk][h][d]
            logits.append(dot / math.sqrt(c) + (biases[h][kk] if biases is not None else 0.0))
        a = softmax_masked(logits, keep)
        for d in range(c):
            acc = 0.0
            for kk in range(nk):
                acc += a[kk] * vs[kk][h][d]
            out.append(gs[h][d] * acc)
    return out


def _heads(vec, H, c):
    return [[vec[h * c + d] for d in range(c)] for h in range(H)]


def row_attn(m, z, M, p, H, c, eps=1e-5):
    S, R = len(m), len(m[0])
    y = [[ln_vec(m[s][i], p["ln_g"], p["ln_b"], eps) for i in range(R)] for s in range(S)]
    yz = [[ln_vec(z[i][j], p["ln_z_g"], p["ln_z_b"], eps) for j in range(R)] for i in range(R)]
    bias = [[lin(yz[i][j], p["w_bias"]) for j in range(R)] for i in range(R)]   # [i][j][h]
    out = _zeros(S, R, len(p["b_o"]))
    for s in range(S):
        q = [_heads(lin(y[s][i], p["w_q"]), H, c) for i in range(R)]
        k = [_heads(lin(y[s][j], p["w_k"]), H, c) for j in range(R)]
        v = [_heads(lin(y[s][j], p["w_v"]), H, c) for j in range(R)]
        for i in range(R):
            g = _heads([sigmoid(t) for t in lin(y[s][i], p["w_g"], p["b_g"])], H, c)
            b_i = [[bias[i][j][h] for j in range(R)] for h in range(H)]
            o = _gated_attend(q[i], k, v, g, b_i, M[s], H, c)
            out[s][i] = lin(o, p["w_o"], p["b_o"])
    return out


def col_attn(m, M, p, H, c, eps=1e-5):
    S, R = len(m), len(m[0])
    y = [[ln_vec(m[s][i], p["ln_g"], p["ln_b"], eps) for i in range(R)] for s in range(S)]
    out = _zeros(S, R, len(p["b_o"]))
    for i in range(R):
        q = [_heads(lin(y[s][i], p["w_q"]), H, c) for s in range(S)]
        k = [_heads(lin(y[t][i], p["w_k"]), H, c) for t in range(S)]
        v = [_heads(lin(y[t][i], p["w_v"]), H, c) for t in range(S)]
        keep = [M[t][i] for t in range(S)]
        for s in range(S):
            g = _heads([sigmoid(t) for t in lin(y[s][i], p["w_g"], p["b_g"])], H, c)
            o = _gated_attend(q[s], k, v, g, None, keep, H, c)
            out[s][i] = lin(o, p["w_o"], p["b_o"])
    return out


def col_global_attn(m, M, p, H, c, eps=1e-5, geps=1e-10):
    S, R = len(m), len(m[0])
    y = [[ln_vec(m[s][i], p["ln_g"], p["ln_b"], eps) for i in range(R)] for s in range(S)]
    out = _zeros(S, R, len(p["b_o"]))
    for i in range(R):
        qs = [_heads(lin(y[s][i], p["w_q"]), H, c) for s in range(S)]
        ks = [lin(y[t][i], p["w_k"]) for t in range(S)]
        vs = [lin(y[t][i], p["w_v"]) for t in range(S)]
        msum = sum(M[s][i] for s in range(S))
        ctx = []
        for h in range(H):
            qbar = [sum(M[s][i] * qs[s][h][d] for s in range(S)) / (msum + geps) for d in range(c)]
            logits = [sum(qbar[d] * ks[t][d] for d in range(c)) / math.sqrt(c) for t in range(S)]
            a = softmax_masked(logits, [M[t][i] for t in range(S)])
            ctx.append([sum(a[t] * vs[t][d] for t in range(S)) for d in range(c)])
        for s in range(S):
            g = _heads([sigmoid(t) for t in lin(y[s][i], p["w_g"], p["b_g"])], H, c)
            o = [g[h][d] * ctx[h][d] for h in range(H) for d in range(c)]
            out[s][i] = lin(o, p["w_o"], p["b_o"])
    return out


def transition(x, p, eps=1e-5):
    """x is [A][B][C]; applied per position."""
    out = []
    for row in x:
        orow = []
        for vec in row:
            y = ln_vec(vec, p["ln_g"], p["ln_b"], eps)
            h = [max(0.0, t) for t in lin(y, p["w_1"], p["b_1"])]
            orow.append(lin(h, p["w_2"], p["b_2"]))
        out.append(orow)
    return out


def outer_product_mean(m, M, p, eps=1e-5, opm_eps=1e-3):
    S, R = len(m), len(m[0])
    a = [[None] * R for _ in range(S)]
    b = [[None] * R for _ in range(S)]
    for s in range(S):
        for i in range(R):
            y = ln_vec(m[s][i], p["ln_g"], p["ln_b"], eps)
            a[s][i] = [M[s][i] * t for t in lin(y, p["w_a"], p["b_a"])]
            b[s][i] = [M[s][i] * t for t in lin(y, p["w_b"], p["b_b"])]
    ch = len(a[0][0])
    out = _zeros(R, R, len(p["b_o"]))
    for i in range(R):
        for j in range(R):
            n = sum(M[s][i] * M[s][j] for s in range(S))
            flat = []
            for pp in range(ch):
                for qq in range(ch):
                    flat.append(sum(a[s][i][pp] * b[s][j][qq] for s in range(S)) / (opm_eps + n))
            out[i][j] = lin(flat, p["w_o"], p["b_o"])
    return out


def _tri_mul(z, P, p, outgoing, eps=1e-5):
    R = len(z)
    a = [[None] * R for _ in range(R)]
    b = [[None] * R for _ in range(R)]
    g = [[None] * R for _ in range(R)]
    for i in range(R):
        for j in range(R):
            y = ln_vec(z[i][j], p["ln_g"], p["ln_b"], eps)
            ag = lin(y, p["w_ag"], p["b_ag"]); ap = lin(y, p["w_ap"], p["b_ap"])
            bg = lin(y, p["w_bg"], p["b_bg"]); bp = lin(y, p["w_bp"], p["b_bp"])
            a[i][j] = [P[i][j] * sigmoid(ag[c]) * ap[c] for c in range(len(ap))]
            b[i][j] = [P[i][j] * sigmoid(bg[c]) * bp[c] for c in range(len(bp))]
            g[i][j] = [sigmoid(t) for t in lin(y, p["w_g"], p["b_g"])]
    ch = len(a[0][0])
    out = _zeros(R, R, len(p["b_o"]))
    for i in range(R):
        for j in range(R):
            x = []
            for c in range(ch):
                if outgoing:
                    x.append(sum(a[i][k][c] * b[j][k][c] for k in range(R)))
                else:
                    x.append(sum(a[k][i][c] * b[k][j][c] for k in range(R)))
            u = lin(ln_vec(x, p["ln_out_g"], p["ln_out_b"], eps), p["w_o"], p["b_o"])
            out[i][j] = [g[i][j][c] * u[c] for c in range(len(u))]
    return out


def tri_mul_out(z, P, p, eps=1e-5):
    return _tri_mul(z, P, p, True, eps)


def tri_mul_in(z, P, p, eps=1e-5):
    return _tri_mul(z, P, p, False, eps)


def _tri_att(z, P, p, H, c, starting, eps=1e-5):
    R = len(z)
    y = [[ln_vec(z[i][j], p["ln_g"], p["ln_b"], eps) for j in range(R)] for i in range(R)]
    q = [[_heads(lin(y[i][j], p["w_q"]), H, c) for j in range(R)] for i in range(R)]
    k = [[_heads(lin(y[i][j], p["w_k"]), H, c) for j in range(R)] for i in range(R)]
    v = [[_heads(lin(y[i][j], p["w_v"]), H, c) for j in range(R)] for i in range(R)]
    bias = [[lin(y[i][j], p["w_bias"]) for j in range(R)] for i in range(R)]    # [a][b][h]
    out = _zeros(R, R, len(p["b_o"]))
    for i in range(R):
        for j in range(R):
            g = _heads([sigmoid(t) for t in lin(y[i][j], p["w_g"], p["b_g"])], H, c)
            if starting:      # keys (i, k), bias b_jk, mask P_ik
                ks = [k[i][kk] for kk in range(R)]
                vs = [v[i][kk] for kk in range(R)]
                bs = [[bias[j][kk][h] for kk in range(R)] for h in range(H)]
                keep = [P[i][kk] for kk in range(R)]
            else:             # keys (k, j), bias b_ki, mask P_kj
                ks = [k[kk][j] for kk in range(R)]
                vs = [v[kk][j] for kk in range(R)]
                bs = [[bias[kk][i][h] for kk in range(R)] for h in range(H)]
                keep = [P[kk][j] for kk in range(R)]
            o = _gated_attend(q[i][j], ks, vs, g, bs, keep, H, c)
            out[i][j] = lin(o, p["w_o"], p["b_o"])
    return out


def tri_att_start(z, P, p, H, c, eps=1e-5):
    return _tri_att(z, P, p, H, c, True, eps)


def tri_att_end(z, P, p, H, c, eps=1e-5):
    return _tri_att(z, P, p, H, c, False, eps)


def _add(x, u):
    if isinstance(x, list):
        return [_add(a, b) for a, b in zip(x, u)]
    return x + u


def _masked(u, mask, orient):
    """u[a][b][c] times mask[b][c] ("row": shared along a) or mask[a][c] ("col")."""
    if mask is None:
        return u
    return [[[u[a][b][c] * (mask[b][c] if orient == "row" else mask[a][c]) for c in range(len(u[a][b]))]
             for b in range(len(u[a]))] for a in range(len(u))]


def block(m, z, M, P, p, cfg, masks=None):
    """masks: None or {sub-operation: [index][channel] multipliers} (dropout)."""
    eps = cfg.ln_eps
    mk = masks or {}
    if cfg.opm_first:
        z = _add(z, outer_product_mean(m, M, p["opm"], eps, cfg.opm_eps))
    m = _add(m, _masked(row_attn(m, z, M, p["row_attn"], cfg.msa_heads, cfg.msa_head_dim, eps),
                        mk.get("row_attn"), "row"))
    if cfg.extra_msa:
        m = _add(m, col_global_attn(m, M, p["col_attn"], cfg.msa_heads, cfg.msa_head_dim,
                                    eps, cfg.global_eps))
    else:
        m = _add(m, col_attn(m, M, p["col_attn"], cfg.msa_heads, cfg.msa_head_dim, eps))
    m = _add(m, transition(m, p["msa_trans"], eps))
    if not cfg.opm_first:
        z = _add(z, outer_product_mean(m, M, p["opm"], eps, cfg.opm_eps))
    z = _add(z, _masked(tri_mul_out(z, P, p["tri_mul_out"], eps), mk.get("tri_mul_out"), "row"))
    z = _add(z, _masked(tri_mul_in(z, P, p["tri_mul_in"], eps), mk.get("tri_mul_in"), "row"))
    z = _add(z, _masked(tri_att_start(z, P, p["tri_att_start"], cfg.tri_heads, cfg.tri_head_dim, eps),
                        mk.get("tri_att_start"), "row"))
    z = _add(z, _masked(tri_att_end(z, P, p["tri_att_end"], cfg.tri_heads, cfg.tri_head_dim, eps),
                        mk.get("tri_att_end"), "col"))
    z = _add(z, transition(z, p["pair_trans"], eps))
    return m, z


def template_block(t, P, p, cfg, masks=None):
    eps = cfg.ln_eps
    mk = masks or {}
    H, c = cfg.tri_heads, cfg.tri_head_dim
    t = _add(t, _masked(tri_att_start(t, P, p["tri_att_start"], H, c, eps), mk.get("tri_att_start"), "row"))
    t = _add(t, _masked(tri_att_end(t, P, p["tri_att_end"], H, c, eps), mk.get("tri_att_end"), "col"))
    t = _add(t, _masked(tri_mul_out(t, P, p["tri_mul_out"], eps), mk.get("tri_mul_out"), "row"))
    t = _add(t, _masked(tri_mul_in(t, P, p["tri_mul_in"], eps), mk.get("tri_mul_in"), "row"))
    return _add(t, transition(t, p["pair_trans"], eps))
