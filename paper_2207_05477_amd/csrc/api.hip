// C ABI (include/evo.h): argument validation, precision dispatch and
// workspace carving around the ops.
#include <mutex>

#include "ops.h"

namespace evo {

const char* last_error();

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

#define REQ(cond, code, ...) EVO_CHECK_ARG(cond, code, __VA_ARGS__)

static bool mult8(int64_t v) { return v > 0 && v % 8 == 0; }

evo_status_t check_attn_desc(const evo_attn_desc_t* d) {
  REQ(d, EVO_EINVAL, "attention: null descriptor");
  REQ(d->kind >= EVO_ATTN_ROW && d->kind <= EVO_ATTN_TRI_END, EVO_EINVAL, "attention: bad kind %d", d->kind);
  REQ(d->dtype == EVO_F32 || d->dtype == EVO_BF16, EVO_EINVAL, "attention: bad dtype %d", d->dtype);
  REQ(d->head_dim == 8 || d->head_dim == 16 || d->head_dim == 32 || d->head_dim == 64, EVO_ESHAPE,
      "attention: head_dim %d not in {8,16,32,64}", d->head_dim);
  REQ(d->heads >= 1 && d->heads <= 16, EVO_ESHAPE, "attention: heads %d not in [1,16]", d->heads);
  REQ(d->n_outer > 0 && d->n_inner > 0, EVO_ESHAPE, "attention: empty input");
  REQ(mult8(d->c_in), EVO_ESHAPE, "attention: c_in %lld not a positive multiple of 8", (long long)d->c_in);
  REQ(d->c_in <= 512, EVO_ESHAPE, "attention: c_in %lld > 512", (long long)d->c_in);
  if (d->kind == EVO_ATTN_ROW) {
    REQ(mult8(d->c_pair) && d->c_pair <= 256 && 256 % d->c_pair == 0, EVO_ESHAPE,
        "attention: c_pair %lld must divide 256 and be a multiple of 8", (long long)d->c_pair);
  }
  if (d->kind == EVO_ATTN_COL_GLOBAL) {
    // one lane per (column, head) with a column's heads on adjacent lanes of a wave
    REQ(d->heads == 1 || d->heads == 2 || d->heads == 4 || d->heads == 8 || d->heads == 16, EVO_ESHAPE,
        "global attention: heads %d not a power of two <= 16", d->heads);
    REQ(d->head_dim <= 32, EVO_ESHAPE, "global attention: head_dim %d not in {8, 16, 32}", d->head_dim);
  }
  if (d->kind == EVO_ATTN_TRI_START || d->kind == EVO_ATTN_TRI_END) {
    REQ(d->n_outer == d->n_inner, EVO_ESHAPE, "triangle attention: pair representation must be square");
    REQ(d->c_in <= 256 && 256 % d->c_in == 0, EVO_ESHAPE, "triangle attention: c_in must divide 256");
  }
  REQ(d->chunk >= 0, EVO_EINVAL, "attention: negative chunk");
  if (d->chunk > 0 && d->chunk < d->n_inner && (d->kind == EVO_ATTN_TRI_START || d->kind == EVO_ATTN_TRI_END))
    REQ(is_pow2(d->chunk) && d->chunk >= 8 && d->n_inner % d->chunk == 0, EVO_ESHAPE,
        "attention: chunk %lld must be a power of two >= 8 dividing n_inner", (long long)d->chunk);
  return EVO_OK;
}

evo_status_t check_trans_desc(const evo_trans_desc_t* d) {
  REQ(d, EVO_EINVAL, "transition: null descriptor");
  REQ(d->dtype == EVO_F32 || d->dtype == EVO_BF16, EVO_EINVAL, "transition: bad dtype");
  REQ(d->rows > 0 && mult8(d->c) && d->c <= 512 && d->factor >= 1, EVO_ESHAPE, "transition: bad shape");
  return EVO_OK;
}

evo_status_t check_opm_desc(const evo_opm_desc_t* d) {
  REQ(d, EVO_EINVAL, "outer product mean: null descriptor");
  REQ(d->dtype == EVO_F32 || d->dtype == EVO_BF16, EVO_EINVAL, "outer product mean: bad dtype");
  REQ(d->n_seq > 0 && mult8(d->n_res) && mult8(d->c_m) && mult8(d->c_z) && d->c_m <= 512, EVO_ESHAPE,
      "outer product mean: bad shape");
  REQ(is_pow2(d->c_hidden) && d->c_hidden >= 8 && d->c_hidden <= 64, EVO_ESHAPE,
      "outer product mean: c_hidden %lld must be a power of two in [8, 64]", (long long)d->c_hidden);
  REQ(d->chunk >= 0, EVO_EINVAL, "outer product mean: negative chunk");
  if (d->chunk > 0 && d->chunk < d->n_res)
    REQ(d->n_res % d->chunk == 0, EVO_ESHAPE, "outer product mean: chunk must divide n_res");
  return EVO_OK;
}

evo_status_t check_trimul_desc(const evo_trimul_desc_t* d) {
  REQ(d, EVO_EINVAL, "triangle multiplication: null descriptor");
  REQ(d->dtype == EVO_F32 || d->dtype == EVO_BF16, EVO_EINVAL, "triangle multiplication: bad dtype");
  REQ(d->dir == EVO_TRI_OUT || d->dir == EVO_TRI_IN, EVO_EINVAL, "triangle multiplication: bad dir");
  REQ(mult8(d->n_res) && mult8(d->c_z) && mult8(d->c_hidden) && d->c_z <= 512 && d->c_hidden <= 256,
      EVO_ESHAPE, "triangle multiplication: bad shape");
  REQ(d->chunk >= 0, EVO_EINVAL, "triangle multiplication: negative chunk");
  if (d->chunk > 0 && d->chunk < d->n_res)
    REQ(is_pow2(d->chunk) && d->chunk >= 8 && d->n_res % d->chunk == 0, EVO_ESHAPE,
        "triangle multiplication: chunk %lld must be a power of two >= 8 dividing n_res", (long long)d->chunk);
  return EVO_OK;
}

evo_status_t check_block_desc(const evo_block_desc_t* d) {
  REQ(d, EVO_EINVAL, "block: null descriptor");
  evo_attn_desc_t a = block_attn_desc(*d, EVO_ATTN_ROW);
  EVO_TRY(check_attn_desc(&a));
  a = block_attn_desc(*d, d->extra_msa ? EVO_ATTN_COL_GLOBAL : EVO_ATTN_COL);
  EVO_TRY(check_attn_desc(&a));
  a = block_attn_desc(*d, EVO_ATTN_TRI_START);
  EVO_TRY(check_attn_desc(&a));
  evo_trans_desc_t t = block_trans_desc(*d, true);
  EVO_TRY(check_trans_desc(&t));
  t = block_trans_desc(*d, false);
  EVO_TRY(check_trans_desc(&t));
  evo_opm_desc_t o = block_opm_desc(*d);
  EVO_TRY(check_opm_desc(&o));
  evo_trimul_desc_t m = block_trimul_desc(*d, EVO_TRI_OUT);
  EVO_TRY(check_trimul_desc(&m));
  REQ(d->opm_first == 0 || d->opm_first == 1, EVO_EINVAL, "block: opm_first must be 0 or 1");
  REQ(d->dropout == 0 || d->dropout == 1, EVO_EINVAL, "block: dropout must be 0 or 1");
  if (d->dropout) {
    REQ(d->chunk == 0, EVO_EINVAL, "block: dropout (training) with the chunked (inference) forward");
    for (float r : {d->drop_row_attn, d->drop_tri_mul, d->drop_tri_att})
      REQ(r >= 0.f && r < 1.f, EVO_EINVAL, "block: dropout rate %g outside [0, 1)", (double)r);
    REQ(d->c_m % 4 == 0 && d->c_z % 4 == 0, EVO_ESHAPE, "block: dropout needs channels divisible by 4");
  }
  return EVO_OK;
}

evo_status_t check_template_desc(const evo_template_desc_t* d) {
  REQ(d, EVO_EINVAL, "template block: null descriptor");
  const evo_block_desc_t b = template_as_block(*d);
  evo_attn_desc_t a = block_attn_desc(b, EVO_ATTN_TRI_START);
  EVO_TRY(check_attn_desc(&a));
  evo_trans_desc_t t = block_trans_desc(b, false);
  EVO_TRY(check_trans_desc(&t));
  evo_trimul_desc_t m = block_trimul_desc(b, EVO_TRI_OUT);
  EVO_TRY(check_trimul_desc(&m));
  REQ(d->dropout == 0 || d->dropout == 1, EVO_EINVAL, "template block: dropout must be 0 or 1");
  REQ(d->template_index >= 0 && d->template_index < (1 << 24), EVO_EINVAL,
      "template block: template_index %d outside [0, 2^24)", d->template_index);
  if (d->dropout) {
    REQ(d->chunk == 0, EVO_EINVAL, "template block: dropout (training) with the chunked (inference) forward");
    for (float r : {d->drop_tri_mul, d->drop_tri_att})
      REQ(r >= 0.f && r < 1.f, EVO_EINVAL, "template block: dropout rate %g outside [0, 1)", (double)r);
    REQ(d->c_t % 4 == 0, EVO_ESHAPE, "template block: dropout needs c_t divisible by 4");
  }
  return EVO_OK;
}

static evo_status_t device_ok() {
  static std::mutex mu;
  static int cache[64];
  static bool init = false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    set_error("no HIP device");
    return EVO_EHIP;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!init) { for (int i = 0; i < 64; ++i) cache[i] = -1; init = true; }
  if (cache[dev] < 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) { set_error("hipGetDeviceProperties failed"); return EVO_EHIP; }
    cache[dev] = strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
  }
  if (!cache[dev]) { set_error("device is not gfx950"); return EVO_EUNSUPPORTED; }
  return EVO_OK;
}

evo_status_t check_device() { return device_ok(); }

static evo_status_t ptrs_ok(std::initializer_list<const void*> req, std::initializer_list<const void*> opt) {
  for (const void* p : req) {
    REQ(p != nullptr, EVO_EINVAL, "required pointer is null");
    REQ(aligned16(p), EVO_EINVAL, "pointer %p is not 16-byte aligned", p);
  }
  for (const void* p : opt) REQ(aligned16(p), EVO_EINVAL, "pointer %p is not 16-byte aligned", p);
  return EVO_OK;
}

static evo_status_t weights_ok(const evo_attn_w_t* w, const evo_attn_desc_t* d) {
  REQ(w, EVO_EINVAL, "attention: null weights");
  EVO_TRY(ptrs_ok({w->ln_g, w->ln_b, w->w_q, w->w_k, w->w_v, w->w_g, w->b_g, w->w_o, w->b_o}, {}));
  if (d->kind == EVO_ATTN_ROW) EVO_TRY(ptrs_ok({w->ln_z_g, w->ln_z_b, w->w_bias}, {}));
  if (d->kind == EVO_ATTN_TRI_START || d->kind == EVO_ATTN_TRI_END) EVO_TRY(ptrs_ok({w->w_bias}, {}));
  return EVO_OK;
}
static evo_status_t weights_ok(const evo_trans_w_t* w) {
  REQ(w, EVO_EINVAL, "transition: null weights");
  return ptrs_ok({w->ln_g, w->ln_b, w->w_1, w->b_1, w->w_2, w->b_2}, {});
}
static evo_status_t weights_ok(const evo_opm_w_t* w) {
  REQ(w, EVO_EINVAL, "outer product mean: null weights");
  return ptrs_ok({w->ln_g, w->ln_b, w->w_a, w->b_a, w->w_b, w->b_b, w->w_o, w->b_o}, {});
}
static evo_status_t weights_ok(const evo_trimul_w_t* w) {
  REQ(w, EVO_EINVAL, "triangle multiplication: null weights");
  return ptrs_ok({w->ln_g, w->ln_b, w->w_ap, w->b_ap, w->w_ag, w->b_ag, w->w_bp, w->b_bp, w->w_bg,
                  w->b_bg, w->w_g, w->b_g, w->ln_out_g, w->ln_out_b, w->w_o, w->b_o}, {});
}
static evo_status_t weights_ok(const evo_block_w_t* w, const evo_block_desc_t* d) {
  REQ(w, EVO_EINVAL, "block: null weights");
  evo_attn_desc_t a = block_attn_desc(*d, EVO_ATTN_ROW);
  EVO_TRY(weights_ok(&w->row_attn, &a));
  a = block_attn_desc(*d, d->extra_msa ? EVO_ATTN_COL_GLOBAL : EVO_ATTN_COL);
  EVO_TRY(weights_ok(&w->col_attn, &a));
  a = block_attn_desc(*d, EVO_ATTN_TRI_START);
  EVO_TRY(weights_ok(&w->tri_att_start, &a));
  EVO_TRY(weights_ok(&w->tri_att_end, &a));
  EVO_TRY(weights_ok(&w->msa_trans));
  EVO_TRY(weights_ok(&w->pair_trans));
  EVO_TRY(weights_ok(&w->opm));
  EVO_TRY(weights_ok(&w->tri_mul_out));
  EVO_TRY(weights_ok(&w->tri_mul_in));
  return EVO_OK;
}

static evo_status_t weights_ok(const evo_template_w_t* w, const evo_template_desc_t* d) {
  REQ(w, EVO_EINVAL, "template block: null weights");
  const evo_block_desc_t b = template_as_block(*d);
  const evo_attn_desc_t a = block_attn_desc(b, EVO_ATTN_TRI_START);
  EVO_TRY(weights_ok(&w->tri_att_start, &a));
  EVO_TRY(weights_ok(&w->tri_att_end, &a));
  EVO_TRY(weights_ok(&w->tri_mul_out));
  EVO_TRY(weights_ok(&w->tri_mul_in));
  return weights_ok(&w->pair_trans);
}

static Arena live_arena(void* p, size_t bytes) {
  Arena a;
  a.base = (char*)p;
  a.cap = bytes;
  return a;
}

// Run `fn(ctx)` once dry to size the workspace, then for real.
template <typename F>
static evo_status_t run_checked(void* stream, void* ws, size_t ws_bytes, F fn) {
  Ctx dry;
  dry.dry = true;
  Arena dw;
  dw.dry = true;
  EVO_TRY(fn(dry, dw));
  REQ(dw.off <= ws_bytes, EVO_EWORKSPACE, "workspace too small: %zu bytes needed, %zu given", dw.off, ws_bytes);
  REQ(dw.off == 0 || ws != nullptr, EVO_EINVAL, "workspace pointer is null");
  REQ(aligned16(ws), EVO_EINVAL, "workspace not 16-byte aligned");
  {
    // Shadow pass: the same code without launches, carving the caller's real
    // workspace, so that every branch on a carved pointer goes the way the live
    // pass goes.  A live pass needing more than the sizing pass found would
    // write past the end of the workspace: refuse it before anything runs.
    Arena sh = live_arena(ws, ws_bytes);
    EVO_TRY(fn(dry, sh));
    REQ(!sh.overflow(), EVO_EWORKSPACE, "internal: the workspace sizing (%zu bytes) is short of what the call carves "
        "(%zu bytes)", dw.off, sh.off);
  }
  EVO_TRY(device_ok());
  Ctx c;
  c.stream = (hipStream_t)stream;
  Arena a = live_arena(ws, ws_bytes);
  // parameter-gradient reductions of a backward entry point: one launch at its end
  return with_batched_reductions(c, [&](const Ctx& cq) { return fn(cq, a); });
}

}  // namespace evo

using namespace evo;

extern "C" {

const char* evo_version(void) { return "evoformer-gfx950 0.1"; }
const char* evo_last_error(void) { return evo::last_error(); }
evo_status_t evo_device_check(void) { return device_ok(); }

// ------------------------------------------------------------------ attention
size_t evo_attn_saved_bytes(const evo_attn_desc_t* d) {
  if (check_attn_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws, sv; ws.dry = sv.dry = true;
  evo_attn_w_t w; memset(&w, 0, sizeof(w));
  if (d->dtype == EVO_BF16) attn_fwd_op<bf16, bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr);
  else attn_fwd_op<float, float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr);
  return sv.off;
}

size_t evo_attn_workspace_bytes(const evo_attn_desc_t* d, int32_t phase) {
  if (check_attn_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws, sv; ws.dry = sv.dry = true;
  evo_attn_w_t w; memset(&w, 0, sizeof(w));
  if (phase == EVO_PHASE_FWD) {  // sized for saved == NULL: saved tensors live in the workspace
    if (d->dtype == EVO_BF16) attn_fwd_op<bf16, bf16>(c, ws, ws, *d, w, nullptr, nullptr, nullptr, nullptr);
    else attn_fwd_op<float, float>(c, ws, ws, *d, w, nullptr, nullptr, nullptr, nullptr);
  } else {
    if (d->dtype == EVO_BF16) attn_bwd_op<bf16, bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, w);
    else attn_bwd_op<float, float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, w);
  }
  return ws.off;
}

evo_status_t evo_attn_fwd(const evo_attn_desc_t* d, const evo_attn_w_t* w, const void* x, const void* pair,
                          const float* mask, void* out, void* saved, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_attn_desc(d));
  EVO_TRY(weights_ok(w, d));
  EVO_TRY(ptrs_ok({x, out}, {mask, saved}));
  if (d->kind == EVO_ATTN_ROW) EVO_TRY(ptrs_ok({pair}, {}));
  REQ(!(saved && d->chunk > 0), EVO_EINVAL, "attention: chunked forward keeps no saved state");
  const size_t need_sv = evo_attn_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = saved ? live_arena(saved, need_sv) : a;
    if (saved && c.dry) { sv = Arena(); sv.dry = true; }
    Arena& svr = saved ? sv : a;
    if (d->dtype == EVO_BF16)
      return attn_fwd_op<bf16, bf16>(c, a, svr, *d, *w, (const bf16*)x, (const bf16*)pair, mask, (bf16*)out);
    return attn_fwd_op<float, float>(c, a, svr, *d, *w, (const float*)x, (const float*)pair, mask, (float*)out);
  });
}

evo_status_t evo_attn_bwd(const evo_attn_desc_t* d, const evo_attn_w_t* w, const void* x, const void* pair,
                          const float* mask, const void* saved, const void* d_out, void* d_x, void* d_pair,
                          const evo_attn_w_t* d_w, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_attn_desc(d));
  EVO_TRY(weights_ok(w, d));
  EVO_TRY(weights_ok(d_w, d));
  EVO_TRY(ptrs_ok({x, saved, d_out, d_x}, {mask}));
  if (d->kind == EVO_ATTN_ROW) EVO_TRY(ptrs_ok({pair, d_pair}, {}));
  const size_t need_sv = evo_attn_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(const_cast<void*>(saved), need_sv);
    sv.dry = c.dry;
    if (d->dtype == EVO_BF16)
      return attn_bwd_op<bf16, bf16>(c, a, sv, *d, *w, (const bf16*)x, (const bf16*)pair, mask, (const bf16*)d_out,
                               (bf16*)d_x, (bf16*)d_pair, *d_w);
    return attn_bwd_op<float, float>(c, a, sv, *d, *w, (const float*)x, (const float*)pair, mask, (const float*)d_out,
                              (float*)d_x, (float*)d_pair, *d_w);
  });
}

// ------------------------------------------------------------------ transition
size_t evo_transition_saved_bytes(const evo_trans_desc_t* d) {
  if (check_trans_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws, sv; ws.dry = sv.dry = true;
  evo_trans_w_t w; memset(&w, 0, sizeof(w));
  if (d->dtype == EVO_BF16) trans_fwd_op<bf16, bf16>(c, ws, sv, *d, w, nullptr, nullptr);
  else trans_fwd_op<float, float>(c, ws, sv, *d, w, nullptr, nullptr);
  return sv.off;
}

size_t evo_transition_workspace_bytes(const evo_trans_desc_t* d, int32_t phase) {
  if (check_trans_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws, sv; ws.dry = sv.dry = true;
  evo_trans_w_t w; memset(&w, 0, sizeof(w));
  if (phase == EVO_PHASE_FWD) {
    if (d->dtype == EVO_BF16) trans_fwd_op<bf16, bf16>(c, ws, ws, *d, w, nullptr, nullptr);
    else trans_fwd_op<float, float>(c, ws, ws, *d, w, nullptr, nullptr);
  } else {
    if (d->dtype == EVO_BF16) trans_bwd_op<bf16, bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, w);
    else trans_bwd_op<float, float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, w);
  }
  return ws.off;
}

evo_status_t evo_transition_fwd(const evo_trans_desc_t* d, const evo_trans_w_t* w, const void* x, void* out,
                                void* saved, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_trans_desc(d));
  EVO_TRY(weights_ok(w));
  EVO_TRY(ptrs_ok({x, out}, {saved}));
  const size_t need_sv = evo_transition_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(saved, need_sv);
    sv.dry = c.dry;
    Arena& svr = saved ? sv : a;
    if (d->dtype == EVO_BF16) return trans_fwd_op<bf16, bf16>(c, a, svr, *d, *w, (const bf16*)x, (bf16*)out);
    return trans_fwd_op<float, float>(c, a, svr, *d, *w, (const float*)x, (float*)out);
  });
}

evo_status_t evo_transition_bwd(const evo_trans_desc_t* d, const evo_trans_w_t* w, const void* x,
                                const void* saved, const void* d_out, void* d_x, const evo_trans_w_t* d_w,
                                void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_trans_desc(d));
  EVO_TRY(weights_ok(w));
  EVO_TRY(weights_ok(d_w));
  EVO_TRY(ptrs_ok({x, saved, d_out, d_x}, {}));
  const size_t need_sv = evo_transition_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(const_cast<void*>(saved), need_sv);
    sv.dry = c.dry;
    if (d->dtype == EVO_BF16)
      return trans_bwd_op<bf16, bf16>(c, a, sv, *d, *w, (const bf16*)x, (const bf16*)d_out, (bf16*)d_x, *d_w);
    return trans_bwd_op<float, float>(c, a, sv, *d, *w, (const float*)x, (const float*)d_out, (float*)d_x, *d_w);
  });
}

// ------------------------------------------------------------------ outer product mean
size_t opm_saved_bytes(const evo_opm_desc_t* d) {
  if (check_opm_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws, sv; ws.dry = sv.dry = true;
  evo_opm_w_t w; memset(&w, 0, sizeof(w));
  if (d->dtype == EVO_BF16) opm_fwd_op<bf16, bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr);
  else opm_fwd_op<float, float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr);
  return sv.off;
}

size_t opm_workspace_bytes(const evo_opm_desc_t* d, int32_t phase) {
  if (check_opm_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws, sv; ws.dry = sv.dry = true;
  evo_opm_w_t w; memset(&w, 0, sizeof(w));
  if (phase == EVO_PHASE_FWD) {
    if (d->dtype == EVO_BF16) opm_fwd_op<bf16, bf16>(c, ws, ws, *d, w, nullptr, nullptr, nullptr, nullptr);
    else opm_fwd_op<float, float>(c, ws, ws, *d, w, nullptr, nullptr, nullptr, nullptr);
  } else {
    if (d->dtype == EVO_BF16) opm_bwd_op<bf16, bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, w);
    else opm_bwd_op<float, float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, w);
  }
  return ws.off;
}

evo_status_t opm_fwd(const evo_opm_desc_t* d, const evo_opm_w_t* w, const void* m, const float* msa_mask,
                     const void* z_in, void* z_out, void* saved, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_opm_desc(d));
  EVO_TRY(weights_ok(w));
  EVO_TRY(ptrs_ok({m, z_in, z_out}, {msa_mask, saved}));
  REQ(!(saved && d->chunk > 0), EVO_EINVAL, "outer product mean: chunked forward keeps no saved state");
  const size_t need_sv = opm_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(saved, need_sv);
    sv.dry = c.dry;
    Arena& svr = saved ? sv : a;
    if (d->dtype == EVO_BF16)
      return opm_fwd_op<bf16, bf16>(c, a, svr, *d, *w, (const bf16*)m, msa_mask, (const bf16*)z_in, (bf16*)z_out);
    return opm_fwd_op<float, float>(c, a, svr, *d, *w, (const float*)m, msa_mask, (const float*)z_in, (float*)z_out);
  });
}

evo_status_t opm_bwd(const evo_opm_desc_t* d, const evo_opm_w_t* w, const void* m, const float* msa_mask,
                     const void* saved, const void* dz_out, void* d_m, const evo_opm_w_t* d_w, void* ws,
                     size_t ws_bytes, void* stream) {
  EVO_TRY(check_opm_desc(d));
  EVO_TRY(weights_ok(w));
  EVO_TRY(weights_ok(d_w));
  EVO_TRY(ptrs_ok({m, saved, dz_out, d_m}, {msa_mask}));
  const size_t need_sv = opm_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(const_cast<void*>(saved), need_sv);
    sv.dry = c.dry;
    if (d->dtype == EVO_BF16)
      return opm_bwd_op<bf16, bf16>(c, a, sv, *d, *w, (const bf16*)m, msa_mask, (const bf16*)dz_out, (bf16*)d_m, *d_w);
    return opm_bwd_op<float, float>(c, a, sv, *d, *w, (const float*)m, msa_mask, (const float*)dz_out, (float*)d_m, *d_w);
  });
}

// ------------------------------------------------------------------ triangle multiplication
size_t tri_mul_saved_bytes(const evo_trimul_desc_t* d) {
  if (check_trimul_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws, sv; ws.dry = sv.dry = true;
  evo_trimul_w_t w; memset(&w, 0, sizeof(w));
  if (d->dtype == EVO_BF16) trimul_fwd_op<bf16, bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr);
  else trimul_fwd_op<float, float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr);
  return sv.off;
}

size_t tri_mul_workspace_bytes(const evo_trimul_desc_t* d, int32_t phase) {
  if (check_trimul_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws, sv; ws.dry = sv.dry = true;
  evo_trimul_w_t w; memset(&w, 0, sizeof(w));
  if (phase == EVO_PHASE_FWD) {
    if (d->dtype == EVO_BF16) trimul_fwd_op<bf16, bf16>(c, ws, ws, *d, w, nullptr, nullptr, nullptr);
    else trimul_fwd_op<float, float>(c, ws, ws, *d, w, nullptr, nullptr, nullptr);
  } else {
    if (d->dtype == EVO_BF16) trimul_bwd_op<bf16, bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, w);
    else trimul_bwd_op<float, float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, w);
  }
  return ws.off;
}

evo_status_t tri_mul_fwd(const evo_trimul_desc_t* d, const evo_trimul_w_t* w, const void* z,
                         const float* pair_mask, void* z_out, void* saved, void* ws, size_t ws_bytes,
                         void* stream) {
  EVO_TRY(check_trimul_desc(d));
  EVO_TRY(weights_ok(w));
  EVO_TRY(ptrs_ok({z, z_out}, {pair_mask, saved}));
  REQ(!(saved && d->chunk > 0), EVO_EINVAL, "triangle multiplication: chunked forward keeps no saved state");
  const size_t need_sv = tri_mul_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(saved, need_sv);
    sv.dry = c.dry;
    Arena& svr = saved ? sv : a;
    if (d->dtype == EVO_BF16)
      return trimul_fwd_op<bf16, bf16>(c, a, svr, *d, *w, (const bf16*)z, pair_mask, (bf16*)z_out);
    return trimul_fwd_op<float, float>(c, a, svr, *d, *w, (const float*)z, pair_mask, (float*)z_out);
  });
}

evo_status_t tri_mul_bwd(const evo_trimul_desc_t* d, const evo_trimul_w_t* w, const void* z,
                         const float* pair_mask, const void* saved, const void* dz_out, void* dz,
                         const evo_trimul_w_t* d_w, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_trimul_desc(d));
  EVO_TRY(weights_ok(w));
  EVO_TRY(weights_ok(d_w));
  EVO_TRY(ptrs_ok({z, saved, dz_out, dz}, {pair_mask}));
  const size_t need_sv = tri_mul_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(const_cast<void*>(saved), need_sv);
    sv.dry = c.dry;
    if (d->dtype == EVO_BF16)
      return trimul_bwd_op<bf16, bf16>(c, a, sv, *d, *w, (const bf16*)z, pair_mask, (const bf16*)dz_out, (bf16*)dz, *d_w);
    return trimul_bwd_op<float, float>(c, a, sv, *d, *w, (const float*)z, pair_mask, (const float*)dz_out, (float*)dz, *d_w);
  });
}

// ------------------------------------------------------------------ block
size_t evoformer_block_workspace_bytes(const evo_block_desc_t* d, int32_t phase) {
  if (check_block_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws; ws.dry = true;
  evo_block_w_t w; memset(&w, 0, sizeof(w));
  if (phase == EVO_PHASE_FWD) {
    if (d->dtype == EVO_BF16) block_fwd_op<bf16>(c, ws, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    else block_fwd_op<float>(c, ws, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  } else {
    if (d->dtype == EVO_BF16)
      block_bwd_op<bf16>(c, ws, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, w);
    else
      block_bwd_op<float>(c, ws, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, w);
  }
  return ws.off;
}

evo_status_t evoformer_block_fwd(const evo_block_desc_t* d, const evo_block_w_t* w, const void* m, const void* z,
                                 const float* msa_mask, const float* pair_mask, void* m_out, void* z_out,
                                 void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_block_desc(d));
  EVO_TRY(weights_ok(w, d));
  EVO_TRY(ptrs_ok({m, z, m_out, z_out}, {msa_mask, pair_mask}));
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    if (d->dtype == EVO_BF16)
      return block_fwd_op<bf16>(c, a, *d, *w, (const bf16*)m, (const bf16*)z, msa_mask, pair_mask, (bf16*)m_out,
                                (bf16*)z_out);
    return block_fwd_op<float>(c, a, *d, *w, (const float*)m, (const float*)z, msa_mask, pair_mask, (float*)m_out,
                               (float*)z_out);
  });
}

evo_status_t evoformer_block_bwd(const evo_block_desc_t* d, const evo_block_w_t* w, const void* m, const void* z,
                                 const float* msa_mask, const float* pair_mask, const void* dm_out,
                                 const void* dz_out, void* dm, void* dz, const evo_block_w_t* d_w, void* ws,
                                 size_t ws_bytes, void* stream) {
  EVO_TRY(check_block_desc(d));
  EVO_TRY(weights_ok(w, d));
  EVO_TRY(weights_ok(d_w, d));
  EVO_TRY(ptrs_ok({m, z, dm_out, dz_out, dm, dz}, {msa_mask, pair_mask}));
  REQ(d->chunk == 0, EVO_EINVAL, "block backward: chunked execution is forward-only");
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    if (d->dtype == EVO_BF16)
      return block_bwd_op<bf16>(c, a, *d, *w, (const bf16*)m, (const bf16*)z, msa_mask, pair_mask,
                                (const bf16*)dm_out, (const bf16*)dz_out, (bf16*)dm, (bf16*)dz, *d_w);
    return block_bwd_op<float>(c, a, *d, *w, (const float*)m, (const float*)z, msa_mask, pair_mask,
                               (const float*)dm_out, (const float*)dz_out, (float*)dm, (float*)dz, *d_w);
  });
}

// ------------------------------------------------------------------ block without its checkpoint
size_t evoformer_block_saved_bytes(const evo_block_desc_t* d) {
  if (check_block_desc(d) != EVO_OK || d->chunk != 0) return 0;
  Ctx c; c.dry = true;
  Arena ws; ws.dry = true;
  Arena sv; sv.dry = true;
  evo_block_w_t w; memset(&w, 0, sizeof(w));
  if (d->dtype == EVO_BF16)
    block_fwd_save_op<bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  else
    block_fwd_save_op<float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  return sv.off;
}

size_t evoformer_block_save_workspace_bytes(const evo_block_desc_t* d, int32_t phase) {
  if (check_block_desc(d) != EVO_OK || d->chunk != 0) return 0;
  Ctx c; c.dry = true;
  Arena ws; ws.dry = true;
  Arena sv; sv.dry = true;
  evo_block_w_t w; memset(&w, 0, sizeof(w));
  if (phase == EVO_PHASE_FWD) {
    if (d->dtype == EVO_BF16) block_fwd_save_op<bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    else block_fwd_save_op<float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  } else {
    if (d->dtype == EVO_BF16)
      block_bwd_saved_op<bf16>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, w);
    else
      block_bwd_saved_op<float>(c, ws, sv, *d, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, w);
  }
  return ws.off;
}

evo_status_t evoformer_block_fwd_save(const evo_block_desc_t* d, const evo_block_w_t* w, const void* m, const void* z,
                                      const float* msa_mask, const float* pair_mask, void* m_out, void* z_out,
                                      void* saved, size_t saved_bytes, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_block_desc(d));
  EVO_TRY(weights_ok(w, d));
  EVO_TRY(ptrs_ok({m, z, m_out, z_out, saved}, {msa_mask, pair_mask}));
  REQ(d->chunk == 0, EVO_EINVAL, "block forward with saved state: chunked execution keeps no state");
  REQ(m_out != m && z_out != z, EVO_EINVAL, "block forward with saved state: outputs must not alias the inputs");
  const size_t need_sv = evoformer_block_saved_bytes(d);
  REQ(saved_bytes >= need_sv, EVO_EWORKSPACE, "saved buffer too small: %zu bytes needed, %zu given", need_sv,
      saved_bytes);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(saved, need_sv);
    const evo_status_t st =
        d->dtype == EVO_BF16
            ? block_fwd_save_op<bf16>(c, a, sv, *d, *w, (const bf16*)m, (const bf16*)z, msa_mask, pair_mask,
                                      (bf16*)m_out, (bf16*)z_out)
            : block_fwd_save_op<float>(c, a, sv, *d, *w, (const float*)m, (const float*)z, msa_mask, pair_mask,
                                       (float*)m_out, (float*)z_out);
    REQ(st != EVO_OK || !sv.overflow(), EVO_EWORKSPACE, "internal: saved state larger than its sizing");
    return st;
  });
}

evo_status_t evoformer_block_bwd_saved(const evo_block_desc_t* d, const evo_block_w_t* w, const void* m,
                                       const void* z, const float* msa_mask, const float* pair_mask,
                                       const void* saved, const void* dm_out, const void* dz_out, void* dm, void* dz,
                                       const evo_block_w_t* d_w, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_block_desc(d));
  EVO_TRY(weights_ok(w, d));
  EVO_TRY(weights_ok(d_w, d));
  EVO_TRY(ptrs_ok({m, z, saved, dm_out, dz_out, dm, dz}, {msa_mask, pair_mask}));
  REQ(d->chunk == 0, EVO_EINVAL, "block backward: chunked execution is forward-only");
  const size_t need_sv = evoformer_block_saved_bytes(d);
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    Arena sv = live_arena(const_cast<void*>(saved), need_sv);
    const evo_status_t st =
        d->dtype == EVO_BF16
            ? block_bwd_saved_op<bf16>(c, a, sv, *d, *w, (const bf16*)m, (const bf16*)z, msa_mask, pair_mask,
                                       (const bf16*)dm_out, (const bf16*)dz_out, (bf16*)dm, (bf16*)dz, *d_w)
            : block_bwd_saved_op<float>(c, a, sv, *d, *w, (const float*)m, (const float*)z, msa_mask, pair_mask,
                                        (const float*)dm_out, (const float*)dz_out, (float*)dm, (float*)dz, *d_w);
    REQ(st != EVO_OK || !sv.overflow(), EVO_EWORKSPACE, "internal: saved state larger than its sizing");
    return st;
  });
}

// ------------------------------------------------------------------ template pair stack block
size_t template_pair_block_workspace_bytes(const evo_template_desc_t* d, int32_t phase) {
  if (check_template_desc(d) != EVO_OK) return 0;
  Ctx c; c.dry = true;
  Arena ws; ws.dry = true;
  evo_template_w_t w; memset(&w, 0, sizeof(w));
  if (phase == EVO_PHASE_FWD) {
    if (d->dtype == EVO_BF16) template_fwd_op<bf16>(c, ws, *d, w, nullptr, nullptr, nullptr);
    else template_fwd_op<float>(c, ws, *d, w, nullptr, nullptr, nullptr);
  } else {
    if (d->dtype == EVO_BF16) template_bwd_op<bf16>(c, ws, *d, w, nullptr, nullptr, nullptr, nullptr, w);
    else template_bwd_op<float>(c, ws, *d, w, nullptr, nullptr, nullptr, nullptr, w);
  }
  return ws.off;
}

evo_status_t template_pair_block_fwd(const evo_template_desc_t* d, const evo_template_w_t* w, const void* t,
                                     const float* pair_mask, void* t_out, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_template_desc(d));
  EVO_TRY(weights_ok(w, d));
  EVO_TRY(ptrs_ok({t, t_out}, {pair_mask}));
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    if (d->dtype == EVO_BF16)
      return template_fwd_op<bf16>(c, a, *d, *w, (const bf16*)t, pair_mask, (bf16*)t_out);
    return template_fwd_op<float>(c, a, *d, *w, (const float*)t, pair_mask, (float*)t_out);
  });
}

evo_status_t template_pair_block_bwd(const evo_template_desc_t* d, const evo_template_w_t* w, const void* t,
                                     const float* pair_mask, const void* dt_out, void* dt,
                                     const evo_template_w_t* d_w, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_template_desc(d));
  EVO_TRY(weights_ok(w, d));
  EVO_TRY(weights_ok(d_w, d));
  EVO_TRY(ptrs_ok({t, dt_out, dt}, {pair_mask}));
  REQ(d->chunk == 0, EVO_EINVAL, "template block backward: chunked execution is forward-only");
  return run_checked(stream, ws, ws_bytes, [&](const Ctx& c, Arena& a) -> evo_status_t {
    if (d->dtype == EVO_BF16)
      return template_bwd_op<bf16>(c, a, *d, *w, (const bf16*)t, pair_mask, (const bf16*)dt_out, (bf16*)dt, *d_w);
    return template_bwd_op<float>(c, a, *d, *w, (const float*)t, pair_mask, (const float*)dt_out, (float*)dt, *d_w);
  });
}

}  // extern "C"
