"""ctypes mirror of include/evo.h and the loader of libevo.so.

The library is required: importing the binding without a built libevo.so
raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libevo.so")

EVO_OK, EVO_EINVAL, EVO_ESHAPE, EVO_EWORKSPACE, EVO_EHIP, EVO_EUNSUPPORTED = range(6)
STATUS_NAMES = {0: "EVO_OK", 1: "EVO_EINVAL", 2: "EVO_ESHAPE", 3: "EVO_EWORKSPACE", 4: "EVO_EHIP",
                5: "EVO_EUNSUPPORTED"}
EVO_F32, EVO_BF16 = 0, 1
EVO_PHASE_FWD, EVO_PHASE_BWD = 0, 1
EVO_ATTN_ROW, EVO_ATTN_COL, EVO_ATTN_COL_GLOBAL, EVO_ATTN_TRI_START, EVO_ATTN_TRI_END = range(5)
EVO_TRI_OUT, EVO_TRI_IN = 0, 1


class AttnDesc(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("dtype", c_int32), ("n_outer", c_int64), ("n_inner", c_int64),
                ("c_in", c_int64), ("c_pair", c_int64), ("heads", c_int32), ("head_dim", c_int32),
                ("ln_eps", c_float), ("global_eps", c_float), ("chunk", c_int64)]


class AttnW(ctypes.Structure):
    _fields_ = [(n, c_void_p) for n in ("ln_g", "ln_b", "ln_z_g", "ln_z_b", "w_q", "w_k", "w_v",
                                        "w_bias", "w_g", "b_g", "w_o", "b_o")]


class TransDesc(ctypes.Structure):
    _fields_ = [("dtype", c_int32), ("rows", c_int64), ("c", c_int64), ("factor", c_int64),
                ("ln_eps", c_float)]


class TransW(ctypes.Structure):
    _fields_ = [(n, c_void_p) for n in ("ln_g", "ln_b", "w_1", "b_1", "w_2", "b_2")]


class OpmDesc(ctypes.Structure):
    _fields_ = [("dtype", c_int32), ("n_seq", c_int64), ("n_res", c_int64), ("c_m", c_int64),
                ("c_hidden", c_int64), ("c_z", c_int64), ("ln_eps", c_float), ("opm_eps", c_float),
                ("chunk", c_int64)]


class OpmW(ctypes.Structure):
    _fields_ = [(n, c_void_p) for n in ("ln_g", "ln_b", "w_a", "b_a", "w_b", "b_b", "w_o", "b_o")]


class TrimulDesc(ctypes.Structure):
    _fields_ = [("dtype", c_int32), ("dir", c_int32), ("n_res", c_int64), ("c_z", c_int64),
                ("c_hidden", c_int64), ("ln_eps", c_float), ("chunk", c_int64)]


class TrimulW(ctypes.Structure):
    _fields_ = [(n, c_void_p) for n in ("ln_g", "ln_b", "w_ap", "b_ap", "w_ag", "b_ag", "w_bp", "b_bp",
                                        "w_bg", "b_bg", "w_g", "b_g", "ln_out_g", "ln_out_b", "w_o",
                                        "b_o")]


class BlockDesc(ctypes.Structure):
    _fields_ = [("dtype", c_int32), ("extra_msa", c_int32), ("n_seq", c_int64), ("n_res", c_int64),
                ("c_m", c_int64), ("c_z", c_int64), ("msa_heads", c_int32),
                ("msa_head_dim", c_int32), ("tri_heads", c_int32), ("tri_head_dim", c_int32),
                ("tri_mul_hidden", c_int64), ("opm_hidden", c_int64),
                ("transition_factor", c_int64), ("chunk", c_int64), ("ln_eps", c_float),
                ("opm_eps", c_float), ("global_eps", c_float), ("opm_first", c_int32),
                ("dropout", c_int32), ("drop_row_attn", c_float), ("drop_tri_mul", c_float),
                ("drop_tri_att", c_float), ("drop_seed", c_uint64), ("drop_offset", c_uint64)]


class BlockW(ctypes.Structure):
    _fields_ = [("row_attn", AttnW), ("col_attn", AttnW), ("msa_trans", TransW), ("opm", OpmW),
                ("tri_mul_out", TrimulW), ("tri_mul_in", TrimulW), ("tri_att_start", AttnW),
                ("tri_att_end", AttnW), ("pair_trans", TransW)]


class TemplateDesc(ctypes.Structure):
    _fields_ = [("dtype", c_int32), ("n_res", c_int64), ("c_t", c_int64), ("tri_heads", c_int32),
                ("tri_head_dim", c_int32), ("tri_mul_hidden", c_int64), ("transition_factor", c_int64),
                ("chunk", c_int64), ("ln_eps", c_float), ("dropout", c_int32), ("template_index", c_int32),
                ("drop_tri_mul", c_float), ("drop_tri_att", c_float), ("drop_seed", c_uint64),
                ("drop_offset", c_uint64)]


class TemplateW(ctypes.Structure):
    _fields_ = [("tri_att_start", AttnW), ("tri_att_end", AttnW), ("tri_mul_out", TrimulW),
                ("tri_mul_in", TrimulW), ("pair_trans", TransW)]


SUBOP_STRUCT = {"row_attn": AttnW, "col_attn": AttnW, "msa_trans": TransW, "opm": OpmW,
                "tri_mul_out": TrimulW, "tri_mul_in": TrimulW, "tri_att_start": AttnW,
                "tri_att_end": AttnW, "pair_trans": TransW}

class OptimDesc(ctypes.Structure):
    _fields_ = [("lr", c_double), ("beta1", c_double), ("beta2", c_double), ("eps", c_double),
                ("max_norm", c_double), ("ema_decay", c_double), ("step", c_int64)]


# name -> (argtypes, restype)
_P = c_void_p
_SIGS = {
    "evo_version": ([], c_char_p),
    "evo_last_error": ([], c_char_p),
    "evo_device_check": ([], c_int32),
    "evo_attn_workspace_bytes": ([POINTER(AttnDesc), c_int32], c_size_t),
    "evo_attn_saved_bytes": ([POINTER(AttnDesc)], c_size_t),
    "evo_attn_fwd": ([POINTER(AttnDesc), POINTER(AttnW), _P, _P, _P, _P, _P, _P, c_size_t, _P], c_int32),
    "evo_attn_bwd": ([POINTER(AttnDesc), POINTER(AttnW), _P, _P, _P, _P, _P, _P, _P, POINTER(AttnW), _P,
                      c_size_t, _P], c_int32),
    "evo_transition_workspace_bytes": ([POINTER(TransDesc), c_int32], c_size_t),
    "evo_transition_saved_bytes": ([POINTER(TransDesc)], c_size_t),
    "evo_transition_fwd": ([POINTER(TransDesc), POINTER(TransW), _P, _P, _P, _P, c_size_t, _P], c_int32),
    "evo_transition_bwd": ([POINTER(TransDesc), POINTER(TransW), _P, _P, _P, _P, POINTER(TransW), _P,
                            c_size_t, _P], c_int32),
    "opm_workspace_bytes": ([POINTER(OpmDesc), c_int32], c_size_t),
    "opm_saved_bytes": ([POINTER(OpmDesc)], c_size_t),
    "opm_fwd": ([POINTER(OpmDesc), POINTER(OpmW), _P, _P, _P, _P, _P, _P, c_size_t, _P], c_int32),
    "opm_bwd": ([POINTER(OpmDesc), POINTER(OpmW), _P, _P, _P, _P, _P, POINTER(OpmW), _P, c_size_t, _P],
                c_int32),
    "tri_mul_workspace_bytes": ([POINTER(TrimulDesc), c_int32], c_size_t),
    "tri_mul_saved_bytes": ([POINTER(TrimulDesc)], c_size_t),
    "tri_mul_fwd": ([POINTER(TrimulDesc), POINTER(TrimulW), _P, _P, _P, _P, _P, c_size_t, _P], c_int32),
    "tri_mul_bwd": ([POINTER(TrimulDesc), POINTER(TrimulW), _P, _P, _P, _P, _P, POINTER(TrimulW), _P,
                     c_size_t, _P], c_int32),
    "evoformer_block_workspace_bytes": ([POINTER(BlockDesc), c_int32], c_size_t),
    "evoformer_block_fwd": ([POINTER(BlockDesc), POINTER(BlockW), _P, _P, _P, _P, _P, _P, _P, c_size_t,
                             _P], c_int32),
    "evoformer_block_bwd": ([POINTER(BlockDesc), POINTER(BlockW), _P, _P, _P, _P, _P, _P, _P, _P,
                             POINTER(BlockW), _P, c_size_t, _P], c_int32),
    "evoformer_block_saved_bytes": ([POINTER(BlockDesc)], c_size_t),
    "evoformer_block_save_workspace_bytes": ([POINTER(BlockDesc), c_int32], c_size_t),
    "evoformer_block_fwd_save": ([POINTER(BlockDesc), POINTER(BlockW), _P, _P, _P, _P, _P, _P, _P, c_size_t,
                                  _P, c_size_t, _P], c_int32),
    "evoformer_block_bwd_saved": ([POINTER(BlockDesc), POINTER(BlockW), _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                   POINTER(BlockW), _P, c_size_t, _P], c_int32),
    "template_pair_block_workspace_bytes": ([POINTER(TemplateDesc), c_int32], c_size_t),
    "template_pair_block_fwd": ([POINTER(TemplateDesc), POINTER(TemplateW), _P, _P, _P, _P, c_size_t, _P],
                                c_int32),
    "template_pair_block_bwd": ([POINTER(TemplateDesc), POINTER(TemplateW), _P, _P, _P, _P, POINTER(TemplateW),
                                 _P, c_size_t, _P], c_int32),
    "evo_optim_workspace_bytes": ([c_int64], c_size_t),
    "evo_grad_global_norm": ([_P, c_int64, _P, _P, c_size_t, _P], c_int32),
    "evo_clip_by_global_norm": ([_P, c_int64, c_double, _P, _P, c_size_t, _P], c_int32),
    "evo_adam_step": ([POINTER(OptimDesc), _P, _P, _P, _P, c_int64, _P], c_int32),
    "evo_ema_update": ([_P, _P, c_int64, c_double, _P], c_int32),
    "evo_optimizer_step": ([POINTER(OptimDesc), _P, _P, _P, _P, _P, c_int64, _P, _P, c_size_t, _P],
                           c_int32),
    "evo_optimizer_step_noalloc": ([POINTER(OptimDesc), _P, _P, _P, _P, _P, c_int64, _P, _P], c_int32),
}

EXPORTS = tuple(_SIGS)

_lib = None


def load(path: str = LIB_PATH):
    """Load libevo.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run paper_2207_05477_amd.build.build() "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class EvoError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != EVO_OK:
        raise EvoError(status, where, load().evo_last_error().decode())
