"""Seeded synthetic inputs for the Evoformer block (random numbers only).

Everything is drawn in float64 from one CPU ``torch.Generator`` seeded with 32,
the fixed random seed of the paper's performance methodology (Section
"Hyperparameter setting").  Draw order, fixed so that every consumer sees the
same values:

1. for each block, for each sub-operation in block order, its parameters in
   ``configs.param_spec`` order (constants draw nothing unless ``perturb``);
2. the MSA representation m;
3. the pair representation z;
4. the masks;
5. the upstream gradients dm_out, dz_out.

The module holds no arithmetic of the method: initial values, masks and casts
to the storage precision only.  Both the oracle's tests and the GPU path's
tests and benchmark take their inputs from here.
"""
from __future__ import annotations

import math

import torch

from .configs import EvoConfig, SUBOPS, TEMPLATE_SUBOPS, param_spec

SEED = 32
F64 = torch.float64


def _draw_param(gen, shape, init, perturb):
    if init == "w":
        fan_in = shape[0]
        return torch.randn(shape, generator=gen, dtype=F64) / math.sqrt(fan_in)
    base = {"gate_b": 1.0, "out_b": 0.0, "b": 0.0, "ln_g": 1.0, "ln_b": 0.0}[init]
    if perturb:
        return base + 0.1 * torch.randn(shape, generator=gen, dtype=F64)
    return torch.full(shape, base, dtype=F64)


def make_params(cfg: EvoConfig, gen: torch.Generator, perturb: bool = False):
    """Parameters of ``cfg.n_blocks`` blocks: list of {subop: {name: float64 tensor}}."""
    blocks = []
    spec = param_spec(cfg)
    for _ in range(cfg.n_blocks):
        p = {s: {} for s in SUBOPS}
        for sub, name, shape, init in spec:
            p[sub][name] = _draw_param(gen, shape, init, perturb)
        blocks.append(p)
    return blocks


def make_template_params(cfg: EvoConfig, gen: torch.Generator, perturb: bool = False):
    """Parameters of ``cfg.n_blocks`` template pair stack blocks (the pair-stack
    sub-operations' tables of param_spec, in TEMPLATE_SUBOPS order)."""
    spec = [e for e in param_spec(cfg) if e[0] in TEMPLATE_SUBOPS]
    blocks = []
    for _ in range(cfg.n_blocks):
        p = {s: {} for s in TEMPLATE_SUBOPS}
        for sub in TEMPLATE_SUBOPS:
            for s_, name, shape, init in spec:
                if s_ == sub:
                    p[sub][name] = _draw_param(gen, shape, init, perturb)
        blocks.append(p)
    return blocks


def make_template_inputs(cfg: EvoConfig, seed: int = SEED, perturb: bool = False, with_grads: bool = True):
    """Template pair stack inputs: parameters, t [n_templ, R, R, c_t] ~ N(0, 1),
    pair masks [n_templ, R, R] (all ones, or ``cfg.mask_mode`` "random" per
    template), upstream gradient dt_out ~ N(0, 1)."""
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    params = make_template_params(cfg, gen, perturb)
    T, R, C = cfg.n_templ, cfg.n_res, cfg.c_z
    t = torch.randn(T, R, R, C, generator=gen, dtype=F64)
    masks = torch.stack([make_masks(cfg, gen)[1] for _ in range(T)])
    out = {"params": params, "t": t, "pair_mask": masks}
    if with_grads:
        out["dt_out"] = torch.randn(t.shape, generator=gen, dtype=F64)
    return out


def make_masks(cfg: EvoConfig, gen: torch.Generator, mode: str | None = None):
    """MSA mask [S, R] and pair mask [R, R] as float64 0/1 arrays."""
    S, R = cfg.n_seq, cfg.n_res
    mode = cfg.mask_mode if mode is None else mode
    msa = torch.ones(S, R, dtype=F64)
    pair = torch.ones(R, R, dtype=F64)
    if mode == "full":
        pass
    elif mode == "rows_tail":
        # the last few residues zeroed in a few distinct MSA rows
        rows = torch.randperm(S, generator=gen)[: min(cfg.n_masked_rows, S)]
        msa[rows, R - cfg.n_masked_tail:] = 0.0
    elif mode == "residue10":
        # 10 % of residue positions masked in every MSA row and in the pair mask
        n = int(round(0.1 * R))
        idx = torch.randperm(R, generator=gen)[:n]
        r = torch.ones(R, dtype=F64)
        r[idx] = 0.0
        msa = r[None, :].expand(S, R).clone()
        pair = torch.outer(r, r)
    elif mode == "random":
        # independent 30 % masking plus one fully masked MSA column and pair row
        msa = (torch.rand(S, R, generator=gen, dtype=F64) > 0.3).to(F64)
        pair = (torch.rand(R, R, generator=gen, dtype=F64) > 0.3).to(F64)
        msa[:, R // 2] = 0.0
        pair[R // 3, :] = 0.0
    else:
        raise ValueError(f"unknown mask mode {mode!r}")
    return msa, pair


def make_msa(cfg: EvoConfig, gen: torch.Generator):
    S, R, C = cfg.n_seq, cfg.n_res, cfg.c_m
    if cfg.msa_input == "onehot23":
        # one-hot tokens from 23 classes times an N(0, 1/23) embedding table
        tok = torch.randint(0, 23, (S, R), generator=gen)
        table = torch.randn(23, C, generator=gen, dtype=F64) / math.sqrt(23.0)
        return table[tok]
    return torch.randn(S, R, C, generator=gen, dtype=F64)


def make_inputs(cfg: EvoConfig, seed: int = SEED, perturb: bool = False,
                mask_mode: str | None = None, with_grads: bool = True):
    """All float64 inputs of one run of ``cfg`` (see the module docstring for order)."""
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    params = make_params(cfg, gen, perturb)
    m = make_msa(cfg, gen)
    z = torch.randn(cfg.n_res, cfg.n_res, cfg.c_z, generator=gen, dtype=F64)
    msa_mask, pair_mask = make_masks(cfg, gen, mask_mode)
    out = {"params": params, "m": m, "z": z, "msa_mask": msa_mask, "pair_mask": pair_mask}
    if with_grads:
        out["dm_out"] = torch.randn(m.shape, generator=gen, dtype=F64)
        out["dz_out"] = torch.randn(z.shape, generator=gen, dtype=F64)
    return out


def to_storage(x: torch.Tensor, dtype: str) -> torch.Tensor:
    """Round float64 values to the storage precision ("f32" or "bf16", round to
    nearest even) and widen back to float64."""
    if dtype == "f32":
        return x.to(torch.float32).to(F64)
    if dtype == "bf16":
        return x.to(torch.bfloat16).to(F64)
    raise ValueError(dtype)


def round_inputs(inp: dict, dtype: str, params_dtype: str = "f32") -> dict:
    """The same inputs as the device receives them: activations and upstream
    gradients rounded to ``dtype``, parameters to ``params_dtype``; masks exact."""
    out = dict(inp)
    out["params"] = [{s: {k: to_storage(v, params_dtype) for k, v in blk[s].items()}
                      for s in blk} for blk in inp["params"]]
    for k in ("m", "z", "dm_out", "dz_out", "t", "dt_out"):
        if k in inp:
            out[k] = to_storage(inp[k], dtype)
    return out
