"""Python binding of libevo.so: argument marshalling only.

Every function here has the name of the C entry point it calls.  PyTorch
supplies device memory, the current HIP stream and data pointers; all
arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi as A

DTYPES = {"f32": (A.EVO_F32, torch.float32), "bf16": (A.EVO_BF16, torch.bfloat16)}
BLOCK_SUBOPS = ("row_attn", "col_attn", "msa_trans", "opm", "tri_mul_out", "tri_mul_in",
                "tri_att_start", "tri_att_end", "pair_trans")
TEMPLATE_SUBOPS = ("tri_att_start", "tri_att_end", "tri_mul_out", "tri_mul_in", "pair_trans")
_ALIGN = 64  # FP32 elements = 256 bytes


def _lib():
    return A.load()


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(t, what: str, dtype=None, numel=None, device=None):
    """Raise ValueError unless `t` (None allowed) has the dtype, element count
    and device the descriptor implies: the ABI takes raw pointers and cannot
    tell a wrong buffer from a right one."""
    if t is None:
        return
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} elements, expected {numel}")
    if device is not None and t.device != torch.device(device):
        raise ValueError(f"{what}: on {t.device}, expected {device}")


def _acts(dtype_code: int, device, **tensors):
    """Activation tensors: the descriptor's dtype, the given element counts, one device."""
    dt = torch.bfloat16 if dtype_code == A.EVO_BF16 else torch.float32
    for name, (t, n) in tensors.items():
        _check(t, name, dt, n, device)


def _masks(device, **tensors):
    """Masks: FP32 0/1 arrays of the given element counts (None = all ones)."""
    for name, (t, n) in tensors.items():
        _check(t, name, torch.float32, n, device)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def act_dtype(name: str) -> torch.dtype:
    return DTYPES[name][1]


# ------------------------------------------------------------------ workspaces
_WS: dict = {}


def workspace(nbytes: int, device) -> torch.Tensor:
    """A reusable byte buffer per (device, stream); grows as needed."""
    device = torch.device(device)
    key = (device.index, torch.cuda.current_stream(device).cuda_stream)
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf


def release_workspaces():
    _WS.clear()


# ------------------------------------------------------------------ parameters
class FlatParams:
    """The parameters of one block in one contiguous FP32 device buffer, each
    tensor at a 256-byte aligned offset; C weight structs point into it.  A
    buffer of the same layout holds the parameter gradients."""

    def __init__(self, named: dict, device, subops=BLOCK_SUBOPS):
        self.layout = []
        off = 0
        for sub in subops:
            for name, t in named[sub].items():
                n = int(t.numel())
                self.layout.append((sub, name, off, tuple(t.shape)))
                off += (n + _ALIGN - 1) // _ALIGN * _ALIGN
        self.numel = off
        self.device = torch.device(device)
        self.buffer = torch.zeros(off, dtype=torch.float32, device=self.device)
        for sub, name, o, shape in self.layout:
            src = named[sub][name].detach().to(device=self.device, dtype=torch.float32).reshape(-1)
            self.buffer[o:o + src.numel()].copy_(src)

    def views(self, buffer: torch.Tensor | None = None) -> dict:
        buf = self.buffer if buffer is None else buffer
        out: dict = {}
        for sub, name, o, shape in self.layout:
            n = 1
            for s in shape:
                n *= s
            out.setdefault(sub, {})[name] = buf[o:o + n].view(shape)
        return out

    def zeros_like(self) -> torch.Tensor:
        return torch.zeros_like(self.buffer)

    def substruct(self, sub: str, buffer: torch.Tensor | None = None):
        buf = self.buffer if buffer is None else buffer
        s = A.SUBOP_STRUCT[sub]()
        base = buf.data_ptr()
        for sb, name, o, _ in self.layout:
            if sb == sub:
                setattr(s, name, base + 4 * o)
        return s

    def block_struct(self, buffer: torch.Tensor | None = None) -> A.BlockW:
        w = A.BlockW()
        for sub in BLOCK_SUBOPS:
            setattr(w, sub, self.substruct(sub, buffer))
        w._keep = self.buffer if buffer is None else buffer
        return w

    def template_struct(self, buffer: torch.Tensor | None = None) -> A.TemplateW:
        w = A.TemplateW()
        for sub in TEMPLATE_SUBOPS:
            setattr(w, sub, self.substruct(sub, buffer))
        w._keep = self.buffer if buffer is None else buffer
        return w


def weight_struct(sub: str, params: dict):
    """C weight struct of one sub-op from individual FP32 device tensors."""
    s = A.SUBOP_STRUCT[sub]()
    for name, t in params.items():
        if t.dtype != torch.float32:
            raise ValueError(f"{sub}.{name}: parameters are FP32")
        setattr(s, name, _ptr(t).value)
    s._keep = dict(params)   # the struct holds raw pointers: keep the tensors alive with it
    return s


# ------------------------------------------------------------------ descriptors
def _set_dropout(d, cfg, dropout):
    """dropout: None (off) or (seed, offset) of the counter-based generator."""
    if dropout is None:
        d.dropout = 0
        return
    d.dropout = 1
    d.drop_seed, d.drop_offset = int(dropout[0]), int(dropout[1])
    d.drop_tri_mul, d.drop_tri_att = cfg.drop_tri_mul, cfg.drop_tri_att


def block_desc(cfg, dtype: str | None = None, chunk: int | None = None, dropout=None) -> A.BlockDesc:
    d = A.BlockDesc()
    d.opm_first = 1 if cfg.opm_first else 0
    _set_dropout(d, cfg, dropout)
    if dropout is not None:
        d.drop_row_attn = cfg.drop_row_attn
    d.dtype = DTYPES[dtype or cfg.dtype][0]
    d.extra_msa = 1 if cfg.extra_msa else 0
    d.n_seq, d.n_res, d.c_m, d.c_z = cfg.n_seq, cfg.n_res, cfg.c_m, cfg.c_z
    d.msa_heads, d.msa_head_dim = cfg.msa_heads, cfg.msa_head_dim
    d.tri_heads, d.tri_head_dim = cfg.tri_heads, cfg.tri_head_dim
    d.tri_mul_hidden, d.opm_hidden = cfg.tri_mul_hidden, cfg.opm_hidden
    d.transition_factor = cfg.transition_factor
    d.chunk = cfg.chunk if chunk is None else chunk
    d.ln_eps, d.opm_eps, d.global_eps = cfg.ln_eps, cfg.opm_eps, cfg.global_eps
    return d


def attn_desc(kind: int, dtype: str, n_outer: int, n_inner: int, c_in: int, heads: int, head_dim: int,
              c_pair: int = 0, ln_eps: float = 1e-5, global_eps: float = 1e-10, chunk: int = 0):
    d = A.AttnDesc()
    d.kind, d.dtype = kind, DTYPES[dtype][0]
    d.n_outer, d.n_inner, d.c_in, d.c_pair = n_outer, n_inner, c_in, c_pair
    d.heads, d.head_dim = heads, head_dim
    d.ln_eps, d.global_eps, d.chunk = ln_eps, global_eps, chunk
    return d


def trans_desc(dtype: str, rows: int, c: int, factor: int = 4, ln_eps: float = 1e-5):
    d = A.TransDesc()
    d.dtype, d.rows, d.c, d.factor, d.ln_eps = DTYPES[dtype][0], rows, c, factor, ln_eps
    return d


def opm_desc(dtype: str, n_seq: int, n_res: int, c_m: int, c_hidden: int, c_z: int,
             ln_eps: float = 1e-5, opm_eps: float = 1e-3, chunk: int = 0):
    d = A.OpmDesc()
    d.dtype = DTYPES[dtype][0]
    d.n_seq, d.n_res, d.c_m, d.c_hidden, d.c_z = n_seq, n_res, c_m, c_hidden, c_z
    d.ln_eps, d.opm_eps, d.chunk = ln_eps, opm_eps, chunk
    return d


def trimul_desc(dtype: str, direction: int, n_res: int, c_z: int, c_hidden: int,
                ln_eps: float = 1e-5, chunk: int = 0):
    d = A.TrimulDesc()
    d.dtype, d.dir = DTYPES[dtype][0], direction
    d.n_res, d.c_z, d.c_hidden, d.ln_eps, d.chunk = n_res, c_z, c_hidden, ln_eps, chunk
    return d


# ------------------------------------------------------------------ block
def evoformer_block_fwd(cfg, flat: FlatParams, m, z, msa_mask=None, pair_mask=None, m_out=None,
                        z_out=None, dtype: str | None = None, chunk: int | None = None, dropout=None):
    lib = _lib()
    d = block_desc(cfg, dtype, chunk, dropout)
    w = flat.block_struct()
    m_out = torch.empty_like(m) if m_out is None else m_out
    z_out = torch.empty_like(z) if z_out is None else z_out
    SR, RR = d.n_seq * d.n_res, d.n_res * d.n_res
    _acts(d.dtype, m.device, m=(m, SR * d.c_m), z=(z, RR * d.c_z), m_out=(m_out, SR * d.c_m),
          z_out=(z_out, RR * d.c_z))
    _masks(m.device, msa_mask=(msa_mask, SR), pair_mask=(pair_mask, RR))
    _check(flat.buffer, "parameters", torch.float32, flat.numel, m.device)
    nbytes = lib.evoformer_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_FWD)
    if nbytes == 0:
        A.check(A.EVO_ESHAPE, "evoformer_block_workspace_bytes")
    ws = workspace(nbytes, m.device)
    A.check(lib.evoformer_block_fwd(ctypes.byref(d), ctypes.byref(w), _ptr(m), _ptr(z), _ptr(msa_mask),
                                    _ptr(pair_mask), _ptr(m_out), _ptr(z_out), _ptr(ws), ws.numel(),
                                    _stream(m.device)), "evoformer_block_fwd")
    return m_out, z_out


def evoformer_block_bwd(cfg, flat: FlatParams, m, z, msa_mask, pair_mask, dm_out, dz_out, dflat=None,
                        dm=None, dz=None, dtype: str | None = None, dropout=None):
    """Returns (dm, dz, dflat); dflat (same layout as flat.buffer) is accumulated into."""
    lib = _lib()
    d = block_desc(cfg, dtype, 0, dropout)
    w = flat.block_struct()
    dflat = flat.zeros_like() if dflat is None else dflat
    dw = flat.block_struct(dflat)
    dm = torch.empty_like(dm_out) if dm is None else dm
    dz = torch.empty_like(dz_out) if dz is None else dz
    SR, RR = d.n_seq * d.n_res, d.n_res * d.n_res
    _acts(d.dtype, m.device, m=(m, SR * d.c_m), z=(z, RR * d.c_z), dm_out=(dm_out, SR * d.c_m),
          dz_out=(dz_out, RR * d.c_z), dm=(dm, SR * d.c_m), dz=(dz, RR * d.c_z))
    _masks(m.device, msa_mask=(msa_mask, SR), pair_mask=(pair_mask, RR))
    _check(flat.buffer, "parameters", torch.float32, flat.numel, m.device)
    _check(dflat, "parameter gradients", torch.float32, flat.numel, m.device)
    nbytes = lib.evoformer_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_BWD)
    if nbytes == 0:
        A.check(A.EVO_ESHAPE, "evoformer_block_workspace_bytes")
    ws = workspace(nbytes, m.device)
    A.check(lib.evoformer_block_bwd(ctypes.byref(d), ctypes.byref(w), _ptr(m), _ptr(z), _ptr(msa_mask),
                                    _ptr(pair_mask), _ptr(dm_out), _ptr(dz_out), _ptr(dm), _ptr(dz),
                                    ctypes.byref(dw), _ptr(ws), ws.numel(), _stream(m.device)),
            "evoformer_block_bwd")
    return dm, dz, dflat


def evoformer_block_saved_bytes(cfg, dtype: str | None = None, dropout=None) -> int:
    """Bytes of the state evoformer_block_fwd_save keeps for evoformer_block_bwd_saved."""
    d = block_desc(cfg, dtype, 0, dropout)
    n = _lib().evoformer_block_saved_bytes(ctypes.byref(d))
    if n == 0:
        A.check(A.EVO_ESHAPE, "evoformer_block_saved_bytes")
    return n


def evoformer_block_fwd_save(cfg, flat: FlatParams, m, z, msa_mask=None, pair_mask=None, m_out=None,
                             z_out=None, saved=None, dtype: str | None = None, dropout=None):
    """The block forward without its checkpoint: returns (m_out, z_out, saved), where `saved`
    (a uint8 device tensor) holds what evoformer_block_bwd_saved needs instead of a recomputation."""
    lib = _lib()
    d = block_desc(cfg, dtype, 0, dropout)
    w = flat.block_struct()
    m_out = torch.empty_like(m) if m_out is None else m_out
    z_out = torch.empty_like(z) if z_out is None else z_out
    SR, RR = d.n_seq * d.n_res, d.n_res * d.n_res
    _acts(d.dtype, m.device, m=(m, SR * d.c_m), z=(z, RR * d.c_z), m_out=(m_out, SR * d.c_m),
          z_out=(z_out, RR * d.c_z))
    _masks(m.device, msa_mask=(msa_mask, SR), pair_mask=(pair_mask, RR))
    _check(flat.buffer, "parameters", torch.float32, flat.numel, m.device)
    nsv = evoformer_block_saved_bytes(cfg, dtype, dropout)
    saved = torch.empty(nsv, dtype=torch.uint8, device=m.device) if saved is None else saved
    _check(saved, "saved state", torch.uint8, nsv, m.device)
    nbytes = lib.evoformer_block_save_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_FWD)
    if nbytes == 0:
        A.check(A.EVO_ESHAPE, "evoformer_block_save_workspace_bytes")
    ws = workspace(nbytes, m.device)
    A.check(lib.evoformer_block_fwd_save(ctypes.byref(d), ctypes.byref(w), _ptr(m), _ptr(z), _ptr(msa_mask),
                                         _ptr(pair_mask), _ptr(m_out), _ptr(z_out), _ptr(saved), saved.numel(),
                                         _ptr(ws), ws.numel(), _stream(m.device)), "evoformer_block_fwd_save")
    return m_out, z_out, saved


def evoformer_block_bwd_saved(cfg, flat: FlatParams, m, z, msa_mask, pair_mask, saved, dm_out, dz_out,
                              dflat=None, dm=None, dz=None, dtype: str | None = None, dropout=None):
    """evoformer_block_bwd over the state of evoformer_block_fwd_save (no recomputation);
    returns (dm, dz, dflat), dflat accumulated into."""
    lib = _lib()
    d = block_desc(cfg, dtype, 0, dropout)
    w = flat.block_struct()
    dflat = flat.zeros_like() if dflat is None else dflat
    dw = flat.block_struct(dflat)
    dm = torch.empty_like(dm_out) if dm is None else dm
    dz = torch.empty_like(dz_out) if dz is None else dz
    SR, RR = d.n_seq * d.n_res, d.n_res * d.n_res
    _acts(d.dtype, m.device, m=(m, SR * d.c_m), z=(z, RR * d.c_z), dm_out=(dm_out, SR * d.c_m),
          dz_out=(dz_out, RR * d.c_z), dm=(dm, SR * d.c_m), dz=(dz, RR * d.c_z))
    _masks(m.device, msa_mask=(msa_mask, SR), pair_mask=(pair_mask, RR))
    _check(flat.buffer, "parameters", torch.float32, flat.numel, m.device)
    _check(dflat, "parameter gradients", torch.float32, flat.numel, m.device)
    _check(saved, "saved state", torch.uint8, evoformer_block_saved_bytes(cfg, dtype, dropout), m.device)
    nbytes = lib.evoformer_block_save_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_BWD)
    if nbytes == 0:
        A.check(A.EVO_ESHAPE, "evoformer_block_save_workspace_bytes")
    ws = workspace(nbytes, m.device)
    A.check(lib.evoformer_block_bwd_saved(ctypes.byref(d), ctypes.byref(w), _ptr(m), _ptr(z), _ptr(msa_mask),
                                          _ptr(pair_mask), _ptr(saved), _ptr(dm_out), _ptr(dz_out), _ptr(dm),
                                          _ptr(dz), ctypes.byref(dw), _ptr(ws), ws.numel(), _stream(m.device)),
            "evoformer_block_bwd_saved")
    return dm, dz, dflat


# ------------------------------------------------------------------ template pair stack block
def template_desc(cfg, dtype: str | None = None, chunk: int | None = None, dropout=None,
                  template_index: int = 0) -> A.TemplateDesc:
    d = A.TemplateDesc()
    d.dtype = DTYPES[dtype or cfg.dtype][0]
    d.n_res, d.c_t = cfg.n_res, cfg.c_z
    d.tri_heads, d.tri_head_dim = cfg.tri_heads, cfg.tri_head_dim
    d.tri_mul_hidden, d.transition_factor = cfg.tri_mul_hidden, cfg.transition_factor
    d.chunk = cfg.chunk if chunk is None else chunk
    d.ln_eps = cfg.ln_eps
    d.template_index = template_index
    _set_dropout(d, cfg, dropout)
    return d


def template_pair_block_fwd(cfg, flat: FlatParams, t, pair_mask=None, t_out=None, dtype: str | None = None,
                            chunk: int | None = None, dropout=None, template_index: int = 0):
    """One template's pair features t [R, R, c_t] through one template pair stack block."""
    lib = _lib()
    d = template_desc(cfg, dtype, chunk, dropout, template_index)
    w = flat.template_struct()
    t_out = torch.empty_like(t) if t_out is None else t_out
    RR = d.n_res * d.n_res
    _acts(d.dtype, t.device, t=(t, RR * d.c_t), t_out=(t_out, RR * d.c_t))
    _masks(t.device, pair_mask=(pair_mask, RR))
    _check(flat.buffer, "parameters", torch.float32, flat.numel, t.device)
    nbytes = lib.template_pair_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_FWD)
    if nbytes == 0:
        A.check(A.EVO_ESHAPE, "template_pair_block_workspace_bytes")
    ws = workspace(nbytes, t.device)
    A.check(lib.template_pair_block_fwd(ctypes.byref(d), ctypes.byref(w), _ptr(t), _ptr(pair_mask), _ptr(t_out),
                                        _ptr(ws), ws.numel(), _stream(t.device)), "template_pair_block_fwd")
    return t_out


def template_pair_block_bwd(cfg, flat: FlatParams, t, pair_mask, dt_out, dflat=None, dt=None,
                            dtype: str | None = None, dropout=None, template_index: int = 0):
    """Returns (dt, dflat); dflat is accumulated into."""
    lib = _lib()
    d = template_desc(cfg, dtype, 0, dropout, template_index)
    w = flat.template_struct()
    dflat = flat.zeros_like() if dflat is None else dflat
    dw = flat.template_struct(dflat)
    dt = torch.empty_like(dt_out) if dt is None else dt
    RR = d.n_res * d.n_res
    _acts(d.dtype, t.device, t=(t, RR * d.c_t), dt_out=(dt_out, RR * d.c_t), dt=(dt, RR * d.c_t))
    _masks(t.device, pair_mask=(pair_mask, RR))
    _check(dflat, "parameter gradients", torch.float32, flat.numel, t.device)
    nbytes = lib.template_pair_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_BWD)
    if nbytes == 0:
        A.check(A.EVO_ESHAPE, "template_pair_block_workspace_bytes")
    ws = workspace(nbytes, t.device)
    A.check(lib.template_pair_block_bwd(ctypes.byref(d), ctypes.byref(w), _ptr(t), _ptr(pair_mask), _ptr(dt_out),
                                        _ptr(dt), ctypes.byref(dw), _ptr(ws), ws.numel(), _stream(t.device)),
            "template_pair_block_bwd")
    return dt, dflat


# ------------------------------------------------------------------ per-op entry points
def _attn_check(desc, x, pair, mask, **acts):
    rows = desc.n_outer * desc.n_inner
    _acts(desc.dtype, x.device, x=(x, rows * desc.c_in),
          **{k: (t, rows * desc.c_in) for k, t in acts.items()})
    if desc.kind == A.EVO_ATTN_ROW:
        _acts(desc.dtype, x.device, pair=(pair, desc.n_inner * desc.n_inner * desc.c_pair))
    _masks(x.device, mask=(mask, rows))


def evo_attn_fwd(desc, w_struct, x, pair=None, mask=None, out=None, keep_saved=True):
    lib = _lib()
    out = torch.empty_like(x) if out is None else out
    _attn_check(desc, x, pair, mask, out=out)
    saved = None
    if keep_saved:
        saved = torch.empty(max(lib.evo_attn_saved_bytes(ctypes.byref(desc)), 256), dtype=torch.uint8,
                            device=x.device)
    nbytes = lib.evo_attn_workspace_bytes(ctypes.byref(desc), A.EVO_PHASE_FWD)
    ws = workspace(nbytes, x.device)
    A.check(lib.evo_attn_fwd(ctypes.byref(desc), ctypes.byref(w_struct), _ptr(x), _ptr(pair), _ptr(mask),
                             _ptr(out), _ptr(saved), _ptr(ws), ws.numel(), _stream(x.device)), "evo_attn_fwd")
    return out, saved


def evo_attn_bwd(desc, w_struct, x, pair, mask, saved, d_out, dw_struct, d_x=None, d_pair=None):
    lib = _lib()
    d_x = torch.empty_like(d_out) if d_x is None else d_x
    _attn_check(desc, x, pair, mask, d_out=d_out, d_x=d_x)
    if desc.kind == A.EVO_ATTN_ROW:
        _acts(desc.dtype, x.device, d_pair=(d_pair, desc.n_inner * desc.n_inner * desc.c_pair))
    nbytes = lib.evo_attn_workspace_bytes(ctypes.byref(desc), A.EVO_PHASE_BWD)
    ws = workspace(nbytes, x.device)
    A.check(lib.evo_attn_bwd(ctypes.byref(desc), ctypes.byref(w_struct), _ptr(x), _ptr(pair), _ptr(mask),
                             _ptr(saved), _ptr(d_out), _ptr(d_x), _ptr(d_pair), ctypes.byref(dw_struct),
                             _ptr(ws), ws.numel(), _stream(x.device)), "evo_attn_bwd")
    return d_x


def evo_transition_fwd(desc, w_struct, x, out=None, keep_saved=True):
    lib = _lib()
    out = torch.empty_like(x) if out is None else out
    _acts(desc.dtype, x.device, x=(x, desc.rows * desc.c), out=(out, desc.rows * desc.c))
    saved = None
    if keep_saved:
        saved = torch.empty(max(lib.evo_transition_saved_bytes(ctypes.byref(desc)), 256),
                            dtype=torch.uint8, device=x.device)
    ws = workspace(lib.evo_transition_workspace_bytes(ctypes.byref(desc), A.EVO_PHASE_FWD), x.device)
    A.check(lib.evo_transition_fwd(ctypes.byref(desc), ctypes.byref(w_struct), _ptr(x), _ptr(out),
                                   _ptr(saved), _ptr(ws), ws.numel(), _stream(x.device)),
            "evo_transition_fwd")
    return out, saved


def evo_transition_bwd(desc, w_struct, x, saved, d_out, dw_struct, d_x=None):
    lib = _lib()
    d_x = torch.empty_like(d_out) if d_x is None else d_x
    n = desc.rows * desc.c
    _acts(desc.dtype, x.device, x=(x, n), d_out=(d_out, n), d_x=(d_x, n))
    ws = workspace(lib.evo_transition_workspace_bytes(ctypes.byref(desc), A.EVO_PHASE_BWD), x.device)
    A.check(lib.evo_transition_bwd(ctypes.byref(desc), ctypes.byref(w_struct), _ptr(x), _ptr(saved),
                                   _ptr(d_out), _ptr(d_x), ctypes.byref(dw_struct), _ptr(ws), ws.numel(),
                                   _stream(x.device)), "evo_transition_bwd")
    return d_x


def opm_fwd(desc, w_struct, m, msa_mask, z_in, z_out=None, keep_saved=True):
    lib = _lib()
    z_out = torch.empty_like(z_in) if z_out is None else z_out
    SR, RR = desc.n_seq * desc.n_res, desc.n_res * desc.n_res
    _acts(desc.dtype, m.device, m=(m, SR * desc.c_m), z_in=(z_in, RR * desc.c_z), z_out=(z_out, RR * desc.c_z))
    _masks(m.device, msa_mask=(msa_mask, SR))
    saved = None
    if keep_saved:
        saved = torch.empty(max(lib.opm_saved_bytes(ctypes.byref(desc)), 256), dtype=torch.uint8,
                            device=m.device)
    ws = workspace(lib.opm_workspace_bytes(ctypes.byref(desc), A.EVO_PHASE_FWD), m.device)
    A.check(lib.opm_fwd(ctypes.byref(desc), ctypes.byref(w_struct), _ptr(m), _ptr(msa_mask), _ptr(z_in),
                        _ptr(z_out), _ptr(saved), _ptr(ws), ws.numel(), _stream(m.device)), "opm_fwd")
    return z_out, saved


def opm_bwd(desc, w_struct, m, msa_mask, saved, dz_out, d_m, dw_struct):
    """d_m is accumulated into."""
    lib = _lib()
    SR, RR = desc.n_seq * desc.n_res, desc.n_res * desc.n_res
    _acts(desc.dtype, m.device, m=(m, SR * desc.c_m), dz_out=(dz_out, RR * desc.c_z), d_m=(d_m, SR * desc.c_m))
    _masks(m.device, msa_mask=(msa_mask, SR))
    ws = workspace(lib.opm_workspace_bytes(ctypes.byref(desc), A.EVO_PHASE_BWD), m.device)
    A.check(lib.opm_bwd(ctypes.byref(desc), ctypes.byref(w_struct), _ptr(m), _ptr(msa_mask), _ptr(saved),
                        _ptr(dz_out), _ptr(d_m), ctypes.byref(dw_struct), _ptr(ws), ws.numel(),
                        _stream(m.device)), "opm_bwd")
    return d_m


def tri_mul_fwd(desc, w_struct, z, pair_mask, z_out=None, keep_saved=True):
    lib = _lib()
    z_out = torch.empty_like(z) if z_out is None else z_out
    RR = desc.n_res * desc.n_res
    _acts(desc.dtype, z.device, z=(z, RR * desc.c_z), z_out=(z_out, RR * desc.c_z))
    _masks(z.device, pair_mask=(pair_mask, RR))
    saved = None
    if keep_saved:
        saved = torch.empty(max(lib.tri_mul_saved_bytes(ctypes.byref(desc)), 256), dtype=torch.uint8,
                            device=z.device)
    ws = workspace(lib.tri_mul_workspace_bytes(ctypes.byref(desc), A.EVO_PHASE_FWD), z.device)
    A.check(lib.tri_mul_fwd(ctypes.byref(desc), ctypes.byref(w_struct), _ptr(z), _ptr(pair_mask),
                            _ptr(z_out), _ptr(saved), _ptr(ws), ws.numel(), _stream(z.device)), "tri_mul_fwd")
    return z_out, saved


def tri_mul_bwd(desc, w_struct, z, pair_mask, saved, dz_out, dw_struct, dz=None):
    lib = _lib()
    dz = torch.empty_like(dz_out) if dz is None else dz
    RR = desc.n_res * desc.n_res
    _acts(desc.dtype, z.device, z=(z, RR * desc.c_z), dz_out=(dz_out, RR * desc.c_z), dz=(dz, RR * desc.c_z))
    _masks(z.device, pair_mask=(pair_mask, RR))
    ws = workspace(lib.tri_mul_workspace_bytes(ctypes.byref(desc), A.EVO_PHASE_BWD), z.device)
    A.check(lib.tri_mul_bwd(ctypes.byref(desc), ctypes.byref(w_struct), _ptr(z), _ptr(pair_mask),
                            _ptr(saved), _ptr(dz_out), _ptr(dz), ctypes.byref(dw_struct), _ptr(ws),
                            ws.numel(), _stream(z.device)), "tri_mul_bwd")
    return dz


# ------------------------------------------------------------------ optimizer (fused flat buffers)
def _flat(t, what, n=None, device=None):
    _check(t, what, torch.float32, n, device)


def optim_desc(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-6, max_norm=0.0, ema_decay=0.999, step=1):
    """evo_optim_desc_t; the defaults are AlphaFold2's Adam settings."""
    return A.OptimDesc(lr, beta1, beta2, eps, max_norm, ema_decay, step)


def _optim_ws(n, device):
    return workspace(_lib().evo_optim_workspace_bytes(n), device)


def evo_grad_global_norm(grads):
    """The global norm of a flat FP32 gradient buffer, as a 1-element device tensor."""
    n = grads.numel()
    _flat(grads, "grads")
    out = torch.empty(1, dtype=torch.float32, device=grads.device)
    ws = _optim_ws(n, grads.device)
    A.check(_lib().evo_grad_global_norm(_ptr(grads), n, _ptr(out), _ptr(ws), ws.numel(), _stream(grads.device)),
            "evo_grad_global_norm")
    return out


def evo_clip_by_global_norm(grads, max_norm):
    """Scales grads in place; returns the norm before clipping (device tensor)."""
    n = grads.numel()
    _flat(grads, "grads")
    out = torch.empty(1, dtype=torch.float32, device=grads.device)
    ws = _optim_ws(n, grads.device)
    A.check(_lib().evo_clip_by_global_norm(_ptr(grads), n, float(max_norm), _ptr(out), _ptr(ws), ws.numel(),
                                           _stream(grads.device)), "evo_clip_by_global_norm")
    return out


def evo_adam_step(desc, params, grads, m, v):
    n = params.numel()
    for name, t in (("grads", grads), ("m", m), ("v", v)):
        _flat(t, name, n, params.device)
    _flat(params, "params")
    A.check(_lib().evo_adam_step(ctypes.byref(desc), _ptr(params), _ptr(grads), _ptr(m), _ptr(v), n,
                                 _stream(params.device)), "evo_adam_step")


def evo_ema_update(ema, params, decay):
    n = params.numel()
    _flat(params, "params")
    _flat(ema, "ema", n, params.device)
    A.check(_lib().evo_ema_update(_ptr(ema), _ptr(params), n, float(decay), _stream(params.device)),
            "evo_ema_update")


def evo_optimizer_step(desc, params, grads, m, v, ema=None):
    """Clip (desc.max_norm > 0) + Adam + EMA (ema not None) in place; returns the
    gradient norm before clipping as a device tensor (zeros without clipping)."""
    n = params.numel()
    _flat(params, "params")
    for name, t in (("grads", grads), ("m", m), ("v", v), ("ema", ema)):
        _flat(t, name, n, params.device)
    norm = torch.zeros(1, dtype=torch.float32, device=params.device)
    ws = _optim_ws(n, params.device)
    A.check(_lib().evo_optimizer_step(ctypes.byref(desc), _ptr(params), _ptr(grads), _ptr(m), _ptr(v), _ptr(ema),
                                      n, _ptr(norm), _ptr(ws), ws.numel(), _stream(params.device)),
            "evo_optimizer_step")
    return norm


def evo_optimizer_step_noalloc(desc, params, grads, m, v, ema=None):
    """evo_optimizer_step without a workspace (the library's static scratch)."""
    n = params.numel()
    _flat(params, "params")
    for name, t in (("grads", grads), ("m", m), ("v", v), ("ema", ema)):
        _flat(t, name, n, params.device)
    norm = torch.zeros(1, dtype=torch.float32, device=params.device)
    A.check(_lib().evo_optimizer_step_noalloc(ctypes.byref(desc), _ptr(params), _ptr(grads), _ptr(m), _ptr(v),
                                              _ptr(ema), n, _ptr(norm), _stream(params.device)),
            "evo_optimizer_step_noalloc")
    return norm
