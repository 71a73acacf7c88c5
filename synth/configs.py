"""Workload presets for one Evoformer block (shapes only, no arithmetic).

The shapes follow the paper's problem statement for Dynamic Axial Parallelism
(Section "Hybrid Parallelism Computing": MSA representation [B, N_seq, N_res, C_m]
and pair representation [B, N_res, N_res, C_z], B = 1 per device, Section
"Hyperparameter setting") and the crop sizes of the model-settings table
(initial training N_res=256, N_seq=128, N_extra_seq=1024; fine-tuning N_res=384,
N_seq=512, N_extra_seq=5120).  Head counts and hidden sizes are the AlphaFold2
values the paper says it follows; the per-layer timing table (FastFold vs
PPFold) fixes head=8, N_seq=128, N_res=256, C_m=256, C_z=128.

This module is shared by the oracle tests and by the GPU path's tests and
benchmark: it holds dimensions and names only.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass


@dataclass(frozen=True)
class EvoConfig:
    name: str
    n_seq: int            # S: MSA rows (N_seq, or N_extra_seq for the extra-MSA block)
    n_res: int            # R: residues
    c_m: int              # MSA channels (c_e for the extra-MSA block)
    c_z: int              # pair channels
    msa_heads: int        # row / column attention heads
    msa_head_dim: int
    tri_heads: int        # triangle attention heads
    tri_head_dim: int
    tri_mul_hidden: int   # triangle multiplicative update hidden channels
    opm_hidden: int       # outer-product-mean hidden channels
    transition_factor: int = 4
    extra_msa: bool = False   # column attention is the global (mean-query) variant
    n_blocks: int = 1
    dtype: str = "f32"        # activation storage: "f32" or "bf16"
    backward: bool = True
    chunk: int = 0            # query-row chunk for the pair-stack ops (0 = none)
    mask_mode: str = "full"   # "full", "rows_tail" or "residue10"
    msa_input: str = "normal"  # "normal" or "onehot23"
    ln_eps: float = 1e-5
    opm_eps: float = 1e-3
    global_eps: float = 1e-10
    opm_first: bool = False   # outer product mean before the MSA stack (branch-independent order)
    # dropout rates, applied only when a run passes a (seed, offset) pair
    drop_row_attn: float = 0.15
    drop_tri_mul: float = 0.25
    drop_tri_att: float = 0.25
    n_templ: int = 4          # templates (template pair stack only)

    def replace(self, **kw) -> "EvoConfig":
        return dataclasses.replace(self, **kw)

    @property
    def n_masked_rows(self) -> int:
        return 4

    @property
    def n_masked_tail(self) -> int:
        return 3


# Tiny FP32 forward case: small enough for brute-force checks, large enough to
# span several kernel tiles with a ragged tail on the residue axis.
C0 = EvoConfig("c0_tiny_f32", n_seq=16, n_res=32, c_m=64, c_z=32, msa_heads=4,
               msa_head_dim=16, tri_heads=2, tri_head_dim=16, tri_mul_hidden=32,
               opm_hidden=8, dtype="f32", backward=False, mask_mode="rows_tail")

# Initial-training crop, one block forward + backward in FP32.
C1 = EvoConfig("c1_initial_f32", n_seq=128, n_res=256, c_m=256, c_z=128, msa_heads=8,
               msa_head_dim=32, tri_heads=4, tri_head_dim=32, tri_mul_hidden=128,
               opm_hidden=32, dtype="f32")

# Same block shapes in BF16 storage, a checkpointed stack of 4 blocks, 10 % residue masks.
C2 = C1.replace(name="c2_initial_bf16_stack4", dtype="bf16", n_blocks=4,
                mask_mode="residue10")

# Extra-MSA block: N_extra=1024, c_e=64, 8x8 row and global column attention.
C3 = EvoConfig("c3_extra_msa_bf16", n_seq=1024, n_res=256, c_m=64, c_z=128, msa_heads=8,
               msa_head_dim=8, tri_heads=4, tri_head_dim=32, tri_mul_hidden=128,
               opm_hidden=32, extra_msa=True, dtype="bf16", msa_input="onehot23")

# Fine-tune crop: 8 checkpointed blocks forward + backward.
C4A = C1.replace(name="c4a_finetune_bf16_stack8", n_seq=512, n_res=384, dtype="bf16",
                 n_blocks=8)

# Long-chain inference: forward only, pair-stack ops in 128-residue query chunks.
C4B = C1.replace(name="c4b_long_bf16_fwd_chunked", n_seq=128, n_res=1024, dtype="bf16",
                 backward=False, chunk=128)

# Extra-MSA block at the fine-tuning crop: N_extra = 5120, N_res = 384.
C5 = C3.replace(name="c5_extra_msa_finetune_bf16", n_seq=5120, n_res=384)

# Template pair stack block at the initial-training crop: 4 templates, c_t = 64,
# triangle attention 4 x 16, triangle-multiplication hidden 64, transition x2.
TEMPLATE = EvoConfig("template_pair_bf16", n_seq=1, n_res=256, c_m=8, c_z=64, msa_heads=1,
                     msa_head_dim=8, tri_heads=4, tri_head_dim=16, tri_mul_hidden=64, opm_hidden=8,
                     transition_factor=2, dtype="bf16", n_templ=4)

PRESETS = {c.name: c for c in (C0, C1, C2, C3, C4A, C4B, C5, TEMPLATE)}
ALIASES = {"C0": C0, "C1": C1, "C2": C2, "C3": C3, "C4a": C4A, "C4b": C4B, "C5": C5, "T": TEMPLATE}


def get(name: str) -> EvoConfig:
    if name in ALIASES:
        return ALIASES[name]
    return PRESETS[name]


# Sub-operations of one block, in the order the block applies them.
SUBOPS = ("row_attn", "col_attn", "msa_trans", "opm", "tri_mul_out", "tri_mul_in",
          "tri_att_start", "tri_att_end", "pair_trans")
# Sub-operations of one template pair stack block, in order.
TEMPLATE_SUBOPS = ("tri_att_start", "tri_att_end", "tri_mul_out", "tri_mul_in", "pair_trans")


def param_spec(cfg: EvoConfig):
    """Ordered parameter table of one block: (subop, name, shape, init).

    Linear weights are stored [fan_in, fan_out] (y = x W + b).  ``init`` is one of
    "w" (N(0, 1/fan_in)), "gate_b" (1), "out_b" (0), "b" (0), "ln_g" (1), "ln_b" (0).
    """
    cm, cz = cfg.c_m, cfg.c_z
    hm, dm = cfg.msa_heads, cfg.msa_head_dim
    ht, dt = cfg.tri_heads, cfg.tri_head_dim
    ch, co = cfg.tri_mul_hidden, cfg.opm_hidden
    tf = cfg.transition_factor
    spec = []

    def add(sub, name, shape, init):
        spec.append((sub, name, tuple(shape), init))

    # MSA row attention with pair bias
    s = "row_attn"
    add(s, "ln_g", [cm], "ln_g"); add(s, "ln_b", [cm], "ln_b")
    add(s, "ln_z_g", [cz], "ln_g"); add(s, "ln_z_b", [cz], "ln_b")
    add(s, "w_q", [cm, hm * dm], "w"); add(s, "w_k", [cm, hm * dm], "w")
    add(s, "w_v", [cm, hm * dm], "w"); add(s, "w_bias", [cz, hm], "w")
    add(s, "w_g", [cm, hm * dm], "w"); add(s, "b_g", [hm * dm], "gate_b")
    add(s, "w_o", [hm * dm, cm], "w"); add(s, "b_o", [cm], "out_b")
    # MSA column attention (global variant in the extra-MSA block)
    s = "col_attn"
    add(s, "ln_g", [cm], "ln_g"); add(s, "ln_b", [cm], "ln_b")
    add(s, "w_q", [cm, hm * dm], "w")
    if cfg.extra_msa:
        add(s, "w_k", [cm, dm], "w"); add(s, "w_v", [cm, dm], "w")
    else:
        add(s, "w_k", [cm, hm * dm], "w"); add(s, "w_v", [cm, hm * dm], "w")
    add(s, "w_g", [cm, hm * dm], "w"); add(s, "b_g", [hm * dm], "gate_b")
    add(s, "w_o", [hm * dm, cm], "w"); add(s, "b_o", [cm], "out_b")
    # MSA transition
    s = "msa_trans"
    add(s, "ln_g", [cm], "ln_g"); add(s, "ln_b", [cm], "ln_b")
    add(s, "w_1", [cm, tf * cm], "w"); add(s, "b_1", [tf * cm], "b")
    add(s, "w_2", [tf * cm, cm], "w"); add(s, "b_2", [cm], "out_b")
    # Outer product mean
    s = "opm"
    add(s, "ln_g", [cm], "ln_g"); add(s, "ln_b", [cm], "ln_b")
    add(s, "w_a", [cm, co], "w"); add(s, "b_a", [co], "b")
    add(s, "w_b", [cm, co], "w"); add(s, "b_b", [co], "b")
    add(s, "w_o", [co * co, cz], "w"); add(s, "b_o", [cz], "out_b")
    # Triangle multiplicative updates
    for s in ("tri_mul_out", "tri_mul_in"):
        add(s, "ln_g", [cz], "ln_g"); add(s, "ln_b", [cz], "ln_b")
        add(s, "w_ap", [cz, ch], "w"); add(s, "b_ap", [ch], "b")
        add(s, "w_ag", [cz, ch], "w"); add(s, "b_ag", [ch], "gate_b")
        add(s, "w_bp", [cz, ch], "w"); add(s, "b_bp", [ch], "b")
        add(s, "w_bg", [cz, ch], "w"); add(s, "b_bg", [ch], "gate_b")
        add(s, "w_g", [cz, cz], "w"); add(s, "b_g", [cz], "gate_b")
        add(s, "ln_out_g", [ch], "ln_g"); add(s, "ln_out_b", [ch], "ln_b")
        add(s, "w_o", [ch, cz], "w"); add(s, "b_o", [cz], "out_b")
    # Triangle attention around the starting and the ending node
    for s in ("tri_att_start", "tri_att_end"):
        add(s, "ln_g", [cz], "ln_g"); add(s, "ln_b", [cz], "ln_b")
        add(s, "w_q", [cz, ht * dt], "w"); add(s, "w_k", [cz, ht * dt], "w")
        add(s, "w_v", [cz, ht * dt], "w"); add(s, "w_bias", [cz, ht], "w")
        add(s, "w_g", [cz, ht * dt], "w"); add(s, "b_g", [ht * dt], "gate_b")
        add(s, "w_o", [ht * dt, cz], "w"); add(s, "b_o", [cz], "out_b")
    # Pair transition
    s = "pair_trans"
    add(s, "ln_g", [cz], "ln_g"); add(s, "ln_b", [cz], "ln_b")
    add(s, "w_1", [cz, tf * cz], "w"); add(s, "b_1", [tf * cz], "b")
    add(s, "w_2", [tf * cz, cz], "w"); add(s, "b_2", [cz], "out_b")
    return spec
