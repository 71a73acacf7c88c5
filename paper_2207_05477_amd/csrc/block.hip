// One Evoformer block: the nine residual sub-operations in order.  The block
// is the activation-checkpoint boundary: its forward keeps nothing, its
// backward recomputes the forward (saving every sub-op's intermediates in the
// workspace) and then runs the sub-op backwards in reverse order.
#include "ops.h"

#include <type_traits>

namespace evo {

evo_attn_desc_t block_attn_desc(const evo_block_desc_t& b, int kind) {
  evo_attn_desc_t d;
  memset(&d, 0, sizeof(d));
  d.kind = kind;
  d.dtype = b.dtype;
  d.ln_eps = b.ln_eps;
  d.global_eps = b.global_eps;
  if (kind == EVO_ATTN_ROW || kind == EVO_ATTN_COL || kind == EVO_ATTN_COL_GLOBAL) {
    d.n_outer = b.n_seq; d.n_inner = b.n_res; d.c_in = b.c_m;
    d.c_pair = kind == EVO_ATTN_ROW ? b.c_z : 0;
    d.heads = b.msa_heads; d.head_dim = b.msa_head_dim;
  } else {
    d.n_outer = b.n_res; d.n_inner = b.n_res; d.c_in = b.c_z;
    d.heads = b.tri_heads; d.head_dim = b.tri_head_dim;
    d.chunk = b.chunk;
  }
  return d;
}

evo_trans_desc_t block_trans_desc(const evo_block_desc_t& b, bool msa) {
  evo_trans_desc_t d;
  memset(&d, 0, sizeof(d));
  d.dtype = b.dtype;
  d.rows = msa ? b.n_seq * b.n_res : b.n_res * b.n_res;
  d.c = msa ? b.c_m : b.c_z;
  d.factor = b.transition_factor;
  d.ln_eps = b.ln_eps;
  return d;
}

evo_opm_desc_t block_opm_desc(const evo_block_desc_t& b) {
  evo_opm_desc_t d;
  memset(&d, 0, sizeof(d));
  d.dtype = b.dtype;
  d.n_seq = b.n_seq; d.n_res = b.n_res; d.c_m = b.c_m; d.c_hidden = b.opm_hidden; d.c_z = b.c_z;
  d.ln_eps = b.ln_eps; d.opm_eps = b.opm_eps;
  d.chunk = b.chunk;
  return d;
}

evo_trimul_desc_t block_trimul_desc(const evo_block_desc_t& b, int dir) {
  evo_trimul_desc_t d;
  memset(&d, 0, sizeof(d));
  d.dtype = b.dtype; d.dir = dir;
  d.n_res = b.n_res; d.c_z = b.c_z; d.c_hidden = b.tri_mul_hidden;
  d.ln_eps = b.ln_eps;
  d.chunk = b.chunk;
  return d;
}

// Sequential scratch: every sub-op starts at the same base; the high-water mark is kept.
struct Scratch {
  Arena base;
  size_t high = 0;
  size_t start() const { return (base.off + 255) & ~(size_t)255; }
  Arena fresh() {
    Arena a;
    a.dry = base.dry;
    a.base = base.dry ? nullptr : base.base + start();
    a.cap = base.dry ? 0 : (base.cap > start() ? base.cap - start() : 0);
    return a;
  }
  void done(const Arena& a) { if (a.off > high) high = a.off; }
  size_t end() const { return start() + high; }
};

template <typename T, typename X>
static evo_status_t block_fwd_x(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                                const X* m, const X* z, const float* mm, const float* pm, X* mo, X* zo) {
  Scratch sc;
  sc.base = ws;
  const int col_kind = d.extra_msa ? EVO_ATTN_COL_GLOBAL : EVO_ATTN_COL;
#define EVO_STEP(tag, call)       \
  do {                            \
    ProfTag pt_(tag);             \
    Arena a = sc.fresh();         \
    EVO_TRY(call);                \
    sc.done(a);                   \
  } while (0)
  EVO_STEP("row.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, EVO_ATTN_ROW), w.row_attn, m, z, mm, mo)));
  EVO_STEP("col.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, col_kind), w.col_attn, mo, nullptr, mm, mo)));
  EVO_STEP("msa_trans.fwd", (trans_fwd_op<T, X>(c, a, a, block_trans_desc(d, true), w.msa_trans, mo, mo)));
  EVO_STEP("opm.fwd", (opm_fwd_op<T, X>(c, a, a, block_opm_desc(d), w.opm, mo, mm, z, zo)));
  EVO_STEP("tri_mul_out.fwd", (trimul_fwd_op<T, X>(c, a, a, block_trimul_desc(d, EVO_TRI_OUT), w.tri_mul_out, zo, pm, zo)));
  EVO_STEP("tri_mul_in.fwd", (trimul_fwd_op<T, X>(c, a, a, block_trimul_desc(d, EVO_TRI_IN), w.tri_mul_in, zo, pm, zo)));
  EVO_STEP("tri_att_start.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, EVO_ATTN_TRI_START), w.tri_att_start, zo, nullptr, pm, zo)));
  EVO_STEP("tri_att_end.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, EVO_ATTN_TRI_END), w.tri_att_end, zo, nullptr, pm, zo)));
  EVO_STEP("pair_trans.fwd", (trans_fwd_op<T, X>(c, a, a, block_trans_desc(d, false), w.pair_trans, zo, zo)));
#undef EVO_STEP
  ws.off = sc.end();
  return EVO_OK;
}

template <typename T, typename X>
static evo_status_t block_bwd_x(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                                const X* m, const X* z, const float* mm, const float* pm, const X* dmo,
                                const X* dzo, X* dm, X* dz, const evo_block_w_t& dw) {
  const int64_t SRc = d.n_seq * d.n_res * d.c_m, RRc = d.n_res * d.n_res * d.c_z;
  const int col_kind = d.extra_msa ? EVO_ATTN_COL_GLOBAL : EVO_ATTN_COL;
  const evo_attn_desc_t d_row = block_attn_desc(d, EVO_ATTN_ROW), d_col = block_attn_desc(d, col_kind);
  evo_attn_desc_t d_tas = block_attn_desc(d, EVO_ATTN_TRI_START), d_tae = block_attn_desc(d, EVO_ATTN_TRI_END);
  d_tas.chunk = 0; d_tae.chunk = 0;
  const evo_trans_desc_t d_tm = block_trans_desc(d, true), d_tz = block_trans_desc(d, false);
  evo_opm_desc_t d_opm = block_opm_desc(d);
  d_opm.chunk = 0;
  evo_trimul_desc_t d_mo = block_trimul_desc(d, EVO_TRI_OUT), d_mi = block_trimul_desc(d, EVO_TRI_IN);
  d_mo.chunk = 0; d_mi.chunk = 0;

  // activations between sub-ops
  X* m1 = ws.take_n<X>(SRc);
  X* m2 = ws.take_n<X>(SRc);
  X* m3 = ws.take_n<X>(SRc);
  X* z1 = ws.take_n<X>(RRc);
  X* z2 = ws.take_n<X>(RRc);
  X* z3 = ws.take_n<X>(RRc);
  X* z4 = ws.take_n<X>(RRc);
  X* z5 = ws.take_n<X>(RRc);
  X* z6 = ws.take_n<X>(RRc);
  // saved regions: carved by the ops themselves from per-op sub-arenas
  Arena sv[9];
  for (int i = 0; i < 9; ++i) { sv[i].dry = true; }
  {
    Ctx dry = c; dry.dry = true;
    Arena junk; junk.dry = true;
    attn_fwd_op<T, X>(dry, junk, sv[0], d_row, w.row_attn, m, z, mm, m1);
    attn_fwd_op<T, X>(dry, junk, sv[1], d_col, w.col_attn, m1, nullptr, mm, m2);
    trans_fwd_op<T, X>(dry, junk, sv[2], d_tm, w.msa_trans, m2, m3);
    opm_fwd_op<T, X>(dry, junk, sv[3], d_opm, w.opm, m3, mm, z, z1);
    trimul_fwd_op<T, X>(dry, junk, sv[4], d_mo, w.tri_mul_out, z1, pm, z2);
    trimul_fwd_op<T, X>(dry, junk, sv[5], d_mi, w.tri_mul_in, z2, pm, z3);
    attn_fwd_op<T, X>(dry, junk, sv[6], d_tas, w.tri_att_start, z3, nullptr, pm, z4);
    attn_fwd_op<T, X>(dry, junk, sv[7], d_tae, w.tri_att_end, z4, nullptr, pm, z5);
    trans_fwd_op<T, X>(dry, junk, sv[8], d_tz, w.pair_trans, z5, z6);
  }
  char* svbase[9];
  for (int i = 0; i < 9; ++i) svbase[i] = (char*)ws.take(sv[i].off);
  auto S = [&](int i) {
    Arena a;
    a.dry = c.dry;
    a.base = svbase[i];
    a.cap = sv[i].off;
    return a;
  };
  Scratch sc;
  sc.base = ws;
  // each sub-op's parameter-gradient reductions run as one launch at its end
#define EVO_STEPS(i, tag, call)                                                \
  do {                                                                         \
    ProfTag pt_(tag);                                                          \
    Arena a = sc.fresh();                                                      \
    Arena s = S(i);                                                            \
    EVO_TRY(with_batched_reductions(c, [&](const Ctx& c) { return call; })); \
    sc.done(a);                                                                \
  } while (0)
  // recompute the forward, keeping what the backward needs
  EVO_STEPS(0, "row.recompute", (attn_fwd_op<T, X>(c, a, s, d_row, w.row_attn, m, z, mm, m1)));
  EVO_STEPS(1, "col.recompute", (attn_fwd_op<T, X>(c, a, s, d_col, w.col_attn, m1, nullptr, mm, m2)));
  EVO_STEPS(2, "msa_trans.recompute", (trans_fwd_op<T, X>(c, a, s, d_tm, w.msa_trans, m2, m3)));
  EVO_STEPS(3, "opm.recompute", (opm_fwd_op<T, X>(c, a, s, d_opm, w.opm, m3, mm, z, z1)));
  EVO_STEPS(4, "tri_mul_out.recompute", (trimul_fwd_op<T, X>(c, a, s, d_mo, w.tri_mul_out, z1, pm, z2)));
  EVO_STEPS(5, "tri_mul_in.recompute", (trimul_fwd_op<T, X>(c, a, s, d_mi, w.tri_mul_in, z2, pm, z3)));
  EVO_STEPS(6, "tri_att_start.recompute", (attn_fwd_op<T, X>(c, a, s, d_tas, w.tri_att_start, z3, nullptr, pm, z4)));
  EVO_STEPS(7, "tri_att_end.recompute", (attn_fwd_op<T, X>(c, a, s, d_tae, w.tri_att_end, z4, nullptr, pm, z5)));
  EVO_STEPS(8, "pair_trans.recompute", (trans_fwd_op<T, X>(c, a, s, d_tz, w.pair_trans, z5, z6)));
  // backward in reverse order; the pair gradient is updated in place in dz
  if (!c.dry) {
    EVO_TRY(copy_elems<X>(c, dzo, dz, RRc));
    EVO_TRY(copy_elems<X>(c, dmo, dm, SRc));
  }
  EVO_STEPS(8, "pair_trans.bwd", (trans_bwd_op<T, X>(c, a, s, d_tz, w.pair_trans, z5, dz, dz, dw.pair_trans)));
  EVO_STEPS(7, "tri_att_end.bwd", (attn_bwd_op<T, X>(c, a, s, d_tae, w.tri_att_end, z4, nullptr, pm, dz, dz, nullptr, dw.tri_att_end)));
  EVO_STEPS(6, "tri_att_start.bwd", (attn_bwd_op<T, X>(c, a, s, d_tas, w.tri_att_start, z3, nullptr, pm, dz, dz, nullptr, dw.tri_att_start)));
  EVO_STEPS(5, "tri_mul_in.bwd", (trimul_bwd_op<T, X>(c, a, s, d_mi, w.tri_mul_in, z2, pm, dz, dz, dw.tri_mul_in)));
  EVO_STEPS(4, "tri_mul_out.bwd", (trimul_bwd_op<T, X>(c, a, s, d_mo, w.tri_mul_out, z1, pm, dz, dz, dw.tri_mul_out)));
  EVO_STEPS(3, "opm.bwd", (opm_bwd_op<T, X>(c, a, s, d_opm, w.opm, m3, mm, dz, dm, dw.opm)));
  EVO_STEPS(2, "msa_trans.bwd", (trans_bwd_op<T, X>(c, a, s, d_tm, w.msa_trans, m2, dm, dm, dw.msa_trans)));
  EVO_STEPS(1, "col.bwd", (attn_bwd_op<T, X>(c, a, s, d_col, w.col_attn, m1, nullptr, mm, dm, dm, nullptr, dw.col_attn)));
  EVO_STEPS(0, "row.bwd", (attn_bwd_op<T, X>(c, a, s, d_row, w.row_attn, m, z, mm, dm, dm, dz, dw.row_attn)));
#undef EVO_STEPS
  ws.off = sc.end();
  return EVO_OK;
}

// Public block ops: inputs and outputs in the activation type T.  Inside the
// block the residual streams (m, z and their gradients between sub-ops) are
// FP32; GEMM / attention operands and saved intermediates stay in T.
template <typename T>
evo_status_t block_fwd_op(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                          const T* m, const T* z, const float* mm, const float* pm, T* mo, T* zo) {
  if constexpr (std::is_same<T, float>::value) {
    return block_fwd_x<T, float>(c, ws, d, w, m, z, mm, pm, mo, zo);
  } else {
    const int64_t SRc = d.n_seq * d.n_res * d.c_m, RRc = d.n_res * d.n_res * d.c_z;
    float* mx = ws.take_n<float>(SRc);
    float* zx = ws.take_n<float>(RRc);
    EVO_TRY((convert_elems<T, float>(c, m, mx, SRc)));
    EVO_TRY((convert_elems<T, float>(c, z, zx, RRc)));
    EVO_TRY((block_fwd_x<T, float>(c, ws, d, w, mx, zx, mm, pm, mx, zx)));
    EVO_TRY((convert_elems<float, T>(c, mx, mo, SRc)));
    return convert_elems<float, T>(c, zx, zo, RRc);
  }
}

template <typename T>
evo_status_t block_bwd_op(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                          const T* m, const T* z, const float* mm, const float* pm, const T* dmo,
                          const T* dzo, T* dm, T* dz, const evo_block_w_t& dw) {
  if constexpr (std::is_same<T, float>::value) {
    return block_bwd_x<T, float>(c, ws, d, w, m, z, mm, pm, dmo, dzo, dm, dz, dw);
  } else {
    const int64_t SRc = d.n_seq * d.n_res * d.c_m, RRc = d.n_res * d.n_res * d.c_z;
    float* mx = ws.take_n<float>(SRc);
    float* zx = ws.take_n<float>(RRc);
    float* dmx = ws.take_n<float>(SRc);
    float* dzx = ws.take_n<float>(RRc);
    EVO_TRY((convert_elems<T, float>(c, m, mx, SRc)));
    EVO_TRY((convert_elems<T, float>(c, z, zx, RRc)));
    EVO_TRY((convert_elems<T, float>(c, dmo, dmx, SRc)));
    EVO_TRY((convert_elems<T, float>(c, dzo, dzx, RRc)));
    EVO_TRY((block_bwd_x<T, float>(c, ws, d, w, mx, zx, mm, pm, dmx, dzx, dmx, dzx, dw)));
    EVO_TRY((convert_elems<float, T>(c, dmx, dm, SRc)));
    return convert_elems<float, T>(c, dzx, dz, RRc);
  }
}

#define EVO_INST_B(T)                                                                              \
  template evo_status_t block_fwd_op<T>(const Ctx&, Arena&, const evo_block_desc_t&,               \
                                        const evo_block_w_t&, const T*, const T*, const float*,    \
                                        const float*, T*, T*);                                     \
  template evo_status_t block_bwd_op<T>(const Ctx&, Arena&, const evo_block_desc_t&,               \
                                        const evo_block_w_t&, const T*, const T*, const float*,    \
                                        const float*, const T*, const T*, T*, T*,                  \
                                        const evo_block_w_t&);

EVO_INST_B(float)
EVO_INST_B(bf16)

}  // namespace evo
