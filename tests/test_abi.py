"""CPU-side checks of the C ABI: libevo.so loads, exports every function that
include/evo.h declares, sizes workspaces, and rejects bad arguments with the
documented status before touching a device (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "evo.h")


def _lib():
    from paper_2207_05477_amd import _abi as A
    return A, A.load()


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(?:evo_status_t|size_t|const char\s*\*|void|int32_t)\s+(\w+)\s*\(", src)
    return sorted(set(names))


def test_header_functions_are_exported_and_bound():
    A, lib = _lib()
    declared = _declared_functions()
    assert len(declared) >= 24
    for name in declared:
        assert hasattr(lib, name), f"libevo.so does not export {name}"
    missing = set(declared) - set(A.EXPORTS) - {"evo_profile_begin", "evo_profile_end", "evo_profile_set_detail"}
    assert not missing, f"binding lacks prototypes for {missing}"


def test_version_and_last_error():
    A, lib = _lib()
    assert lib.evo_version().decode().startswith("evoformer-gfx950")


@pytest.mark.parametrize("name", ["C0", "C1", "C2", "C3", "C4a", "C4b"])
def test_block_workspace_sizes(name):
    A, lib = _lib()
    from paper_2207_05477_amd import binding as B
    cfg = synth.get(name)
    d = B.block_desc(cfg)
    fwd = lib.evoformer_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_FWD)
    bwd = lib.evoformer_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_BWD)
    assert fwd > 0 and bwd > fwd
    # the backward keeps every sub-op's intermediates: at least the nine activations
    act = 2 if cfg.dtype == "bf16" else 4
    assert bwd >= (3 * cfg.n_seq * cfg.n_res * cfg.c_m + 6 * cfg.n_res ** 2 * cfg.c_z) * act


def _fake(n):
    # aligned host-side stand-ins: validation fails before any device access
    return ctypes.c_void_p(0x10000 * n)


def test_block_fwd_rejects_null_and_bad_shape():
    A, lib = _lib()
    from paper_2207_05477_amd import binding as B
    cfg = synth.get("C0")
    d = B.block_desc(cfg)
    w = A.BlockW()
    st = lib.evoformer_block_fwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), None, None,
                                 _fake(3), _fake(4), _fake(5), 1 << 30, None)
    assert st == A.EVO_EINVAL
    assert "null" in lib.evo_last_error().decode()
    d.msa_head_dim = 12
    st = lib.evoformer_block_fwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), None, None,
                                 _fake(3), _fake(4), _fake(5), 1 << 30, None)
    assert st == A.EVO_ESHAPE
    assert "head_dim" in lib.evo_last_error().decode()


def _full_weights(A, struct_cls, n):
    s = struct_cls()
    for i, (name, _) in enumerate(struct_cls._fields_):
        setattr(s, name, 0x100000 + 0x1000 * (n * 64 + i))
    return s


def test_block_fwd_rejects_small_workspace_and_misalignment():
    A, lib = _lib()
    from paper_2207_05477_amd import binding as B
    cfg = synth.get("C0")
    d = B.block_desc(cfg)
    w = A.BlockW()
    for i, (sub, cls) in enumerate(A.BlockW._fields_):
        setattr(w, sub, _full_weights(A, cls, i))
    need = lib.evoformer_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_FWD)
    st = lib.evoformer_block_fwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), None, None,
                                 _fake(3), _fake(4), _fake(5), need - 1, None)
    assert st == A.EVO_EWORKSPACE, lib.evo_last_error()
    st = lib.evoformer_block_fwd(ctypes.byref(d), ctypes.byref(w), ctypes.c_void_p(0x10008), _fake(2), None,
                                 None, _fake(3), _fake(4), _fake(5), need, None)
    assert st == A.EVO_EINVAL
    assert "aligned" in lib.evo_last_error().decode()


@pytest.mark.parametrize("name", ["C0", "C1", "C3"])
def test_saved_block_sizes_and_validation(name):
    # the checkpoint-free pair: the state holds at least the nine activations;
    # chunked descriptors have no state; aliased outputs and a short state
    # buffer are refused before anything runs
    A, lib = _lib()
    from paper_2207_05477_amd import binding as B
    cfg = synth.get(name)
    d = B.block_desc(cfg)
    sv = lib.evoformer_block_saved_bytes(ctypes.byref(d))
    act = 2 if cfg.dtype == "bf16" else 4
    assert sv >= (3 * cfg.n_seq * cfg.n_res * cfg.c_m + 6 * cfg.n_res ** 2 * cfg.c_z) * act
    assert lib.evoformer_block_save_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_BWD) > 0
    # the saved state plus the saved backward's workspace is the checkpointed backward's workspace
    # less the recomputation's scratch: never more than the two together
    ck = lib.evoformer_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_BWD)
    assert sv < ck
    d_chunk = B.block_desc(cfg, chunk=16)
    assert lib.evoformer_block_saved_bytes(ctypes.byref(d_chunk)) == 0
    w = A.BlockW()
    for i, (sub, cls) in enumerate(A.BlockW._fields_):
        setattr(w, sub, _full_weights(A, cls, i))
    st = lib.evoformer_block_fwd_save(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), None, None,
                                      _fake(1), _fake(4), _fake(5), sv, _fake(6), 1 << 40, None)
    assert st == A.EVO_EINVAL and "alias" in lib.evo_last_error().decode()
    st = lib.evoformer_block_fwd_save(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), None, None,
                                      _fake(3), _fake(4), _fake(5), sv - 1, _fake(6), 1 << 40, None)
    assert st == A.EVO_EWORKSPACE and "saved" in lib.evo_last_error().decode()


def test_op_descriptor_validation():
    A, lib = _lib()
    from paper_2207_05477_amd import binding as B
    d = B.attn_desc(A.EVO_ATTN_TRI_START, "f32", 32, 40, 16, 2, 8)
    assert lib.evo_attn_workspace_bytes(ctypes.byref(d), 0) == 0        # not square
    assert "square" in lib.evo_last_error().decode()
    d = B.attn_desc(A.EVO_ATTN_ROW, "bf16", 8, 32, 30, 2, 8, c_pair=16)
    assert lib.evo_attn_workspace_bytes(ctypes.byref(d), 0) == 0        # c_in not a multiple of 8
    d = B.opm_desc("f32", 8, 32, 32, 12, 16)
    assert lib.opm_workspace_bytes(ctypes.byref(d), 0) == 0              # c_hidden not a power of 2
    d = B.trimul_desc("f32", 5, 32, 16, 16)
    assert lib.tri_mul_workspace_bytes(ctypes.byref(d), 0) == 0          # bad direction
    d = B.trimul_desc("f32", A.EVO_TRI_IN, 32, 16, 16)
    assert lib.tri_mul_workspace_bytes(ctypes.byref(d), 0) > 0
    assert lib.tri_mul_saved_bytes(ctypes.byref(d)) > 0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2207_05477_amd import _abi as A
    with pytest.raises(RuntimeError, match="not built"):
        A._lib_saved = A._lib
        A._lib = None
        try:
            A.load(str(tmp_path / "missing.so"))
        finally:
            A._lib = A._lib_saved


@pytest.mark.parametrize("name", ["C0", "C1", "C2", "C3", "C4b"])
def test_workspace_query_matches_a_real_call(name):
    # A call with real (non-null) parameter and gradient pointers carves its
    # workspace in a dry pass before touching the device; with exactly the
    # queried size it must pass the workspace check (and then stop at the
    # device check here, where there is no GPU).
    A, lib = _lib()
    from paper_2207_05477_amd import binding as B
    cfg = synth.get(name)
    d = B.block_desc(cfg)
    w = A.BlockW()
    dw = A.BlockW()
    for i, (sub, cls) in enumerate(A.BlockW._fields_):
        setattr(w, sub, _full_weights(A, cls, i))
        setattr(dw, sub, _full_weights(A, cls, i + 32))
    need_f = lib.evoformer_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_FWD)
    st = lib.evoformer_block_fwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), _fake(3), _fake(4),
                                 _fake(5), _fake(6), _fake(7), need_f, None)
    assert st in (A.EVO_EHIP, A.EVO_EUNSUPPORTED), lib.evo_last_error()
    if cfg.backward:
        need_b = lib.evoformer_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_BWD)
        st = lib.evoformer_block_bwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), _fake(3), _fake(4),
                                     _fake(5), _fake(6), _fake(7), _fake(8), ctypes.byref(dw), _fake(9), need_b,
                                     None)
        assert st in (A.EVO_EHIP, A.EVO_EUNSUPPORTED), lib.evo_last_error()


def test_binding_rejects_wrong_dtype_shape_and_device():
    # the binding checks what the raw-pointer ABI cannot: dtype, element count, device
    import torch
    from paper_2207_05477_amd import binding as B
    m = torch.zeros(2, 8, 8)
    with pytest.raises(ValueError, match="dtype"):
        B._acts(B.A.EVO_BF16, m.device, m=(m, m.numel()))
    with pytest.raises(ValueError, match="elements"):
        B._acts(B.A.EVO_F32, m.device, m=(m, 7))
    with pytest.raises(ValueError, match="dtype"):
        B._masks(m.device, msa_mask=(torch.ones(16, dtype=torch.bool), 16))
    with pytest.raises(ValueError, match="elements"):
        B._masks(m.device, msa_mask=(torch.ones(15), 16))
    with pytest.raises(ValueError, match="on cpu"):
        B._check(m, "m", torch.float32, m.numel(), "meta")
    B._acts(B.A.EVO_F32, m.device, m=(m, m.numel()), z=(None, 3))


@pytest.mark.parametrize("variant", ["dropout", "opm_first+dropout"])
def test_workspace_query_matches_a_real_call_with_dropout(variant):
    # Dropout tables are carved from the workspace; a sizing pass that took
    # them for absent would size the backward short of the live pass (whose
    # per-op gradient scaling carves a buffer of its own) and the call would
    # run past the end of the workspace.  The entry points' shadow pass checks
    # the live carving against the size: with exactly the queried size the
    # call must get past the workspace check (and stop at the device check).
    A, lib = _lib()
    from paper_2207_05477_amd import binding as B
    cfg = synth.get("C0").replace(opm_first="opm_first" in variant, backward=True)
    d = B.block_desc(cfg, dropout=(7, 3))
    w = A.BlockW()
    dw = A.BlockW()
    for i, (sub, cls) in enumerate(A.BlockW._fields_):
        setattr(w, sub, _full_weights(A, cls, i))
        setattr(dw, sub, _full_weights(A, cls, i + 32))
    for phase in (A.EVO_PHASE_FWD, A.EVO_PHASE_BWD):
        need = lib.evoformer_block_workspace_bytes(ctypes.byref(d), phase)
        assert need > 0
        if phase == A.EVO_PHASE_FWD:
            st = lib.evoformer_block_fwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), _fake(3), _fake(4),
                                         _fake(5), _fake(6), _fake(7), need, None)
        else:
            st = lib.evoformer_block_bwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), _fake(3), _fake(4),
                                         _fake(5), _fake(6), _fake(7), _fake(8), ctypes.byref(dw), _fake(9), need,
                                         None)
        assert st in (A.EVO_EHIP, A.EVO_EUNSUPPORTED), lib.evo_last_error()


def test_template_workspace_query_matches_a_real_call_with_dropout():
    A, lib = _lib()
    from paper_2207_05477_amd import binding as B
    cfg = synth.get("T").replace(n_res=40)
    d = B.template_desc(cfg, dropout=(7, 3), template_index=2)
    w = A.TemplateW()
    dw = A.TemplateW()
    for i, (sub, cls) in enumerate(A.TemplateW._fields_):
        setattr(w, sub, _full_weights(A, cls, i))
        setattr(dw, sub, _full_weights(A, cls, i + 32))
    need = lib.template_pair_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_FWD)
    st = lib.template_pair_block_fwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), _fake(3), _fake(4), need,
                                     None)
    assert st in (A.EVO_EHIP, A.EVO_EUNSUPPORTED), lib.evo_last_error()
    need = lib.template_pair_block_workspace_bytes(ctypes.byref(d), A.EVO_PHASE_BWD)
    st = lib.template_pair_block_bwd(ctypes.byref(d), ctypes.byref(w), _fake(1), _fake(2), _fake(3), _fake(4),
                                     ctypes.byref(dw), _fake(6), need, None)
    assert st in (A.EVO_EHIP, A.EVO_EUNSUPPORTED), lib.evo_last_error()
