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

// Training dropout of a block: the multiplier tables of the sub-operations
// with dropout (counter word = sub-operation number | template << 8), carved
// from the workspace and formed in one launch.  Row attention shares its
// multipliers along the MSA rows, the triangle multiplications and the
// starting-node attention along the first residue axis, the ending-node
// attention along the second.
struct DropCfg {
  bool on = false;
  uint64_t seed = 0, offset = 0;
  float rate_row = 0.f, rate_mul = 0.f, rate_att = 0.f;
  uint32_t tmpl = 0;
};
enum { SUB_ROW = 0, SUB_TMO = 4, SUB_TMI = 5, SUB_TAS = 6, SUB_TAE = 7 };
struct BlockDrop {
  DropSpec row, tmo, tmi, tas, tae;
};

static evo_status_t make_block_drop(const Ctx& c, Arena& ws, const DropCfg& dc, int64_t R, int64_t cm, int64_t cz,
                                    bool msa, BlockDrop* bd, bool fill = true) {
  *bd = BlockDrop();
  if (!dc.on) return EVO_OK;
  float* out[5];
  int64_t len[5];
  uint32_t word[5];
  float rate[5];
  DropSpec* spec[5];
  int n = 0;
  auto add = [&](DropSpec* sp, int sub, float r, int64_t C, int64_t div, int64_t mod) {
    if (r <= 0.f) return;
    float* t = ws.take_n<float>(R * C);   // null in the sizing pass; `on` holds in both
    sp->tbl = t; sp->div = div; sp->mod = mod; sp->on = true;
    out[n] = t; len[n] = R * C; word[n] = (uint32_t)sub | (dc.tmpl << 8); rate[n] = r; spec[n] = sp;
    ++n;
  };
  if (msa) add(&bd->row, SUB_ROW, dc.rate_row, cm, 1, R);
  add(&bd->tmo, SUB_TMO, dc.rate_mul, cz, 1, R);
  add(&bd->tmi, SUB_TMI, dc.rate_mul, cz, 1, R);
  add(&bd->tas, SUB_TAS, dc.rate_att, cz, 1, R);
  add(&bd->tae, SUB_TAE, dc.rate_att, cz, R, 0);
  (void)spec;
  return fill ? dropout_tables(c, dc.seed, dc.offset, n, out, len, word, rate) : EVO_OK;
}

static DropCfg block_drop_cfg(const evo_block_desc_t& d) {
  DropCfg dc;
  dc.on = d.dropout != 0;
  dc.seed = d.drop_seed; dc.offset = d.drop_offset;
  dc.rate_row = d.drop_row_attn; dc.rate_mul = d.drop_tri_mul; dc.rate_att = d.drop_tri_att;
  return dc;
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

// Parameter groups of a block call packed ahead, in a few launches: the
// forward layout (and bias rows) for forwards and recomputed forwards, in a
// backward also the backward layout.  The sub-operations then find their
// groups in the cache instead of packing their own (one launch each).
template <typename T>
static evo_status_t prepack_groups(const Ctx& c, Arena& ws, PackArgs* g, int n, bool bwd, bool fill,
                                   PackCache* pc) {
  PackArgs* list[PackCache::MAX];
  pc->n = 0;
  for (int i = 0; i < n; ++i) {
    int64_t ntot = 0;
    for (int s = 0; s < g[i].nseg; ++s) ntot += g[i].seg[s].n;
    g[i].dst_t = ws.take_n<T>((int64_t)g[i].K * ntot);
    g[i].bias = ws.take_n<float>(ntot);
    g[i].dst = bwd ? ws.take_n<T>((int64_t)g[i].K * ntot) : nullptr;
    list[i] = &g[i];
  }
  if (c.dry) return EVO_OK;
  if (fill) EVO_TRY(pack_groups<T>(c, list, n));
  for (int i = 0; i < n; ++i) pc->e[pc->n++] = g[i];
  return EVO_OK;
}

template <typename T>
static evo_status_t prepack_block(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                                  bool bwd, bool fill, PackCache* pc) {
  PackArgs g[18];
  const int col_kind = d.extra_msa ? EVO_ATTN_COL_GLOBAL : EVO_ATTN_COL;
  attn_pack_groups(block_attn_desc(d, EVO_ATTN_ROW), w.row_attn, &g[0], &g[1]);
  attn_pack_groups(block_attn_desc(d, col_kind), w.col_attn, &g[2], &g[3]);
  trans_pack_groups(block_trans_desc(d, true), w.msa_trans, &g[4], &g[5]);
  opm_pack_groups(block_opm_desc(d), w.opm, &g[6], &g[7]);
  trimul_pack_groups(block_trimul_desc(d, EVO_TRI_OUT), w.tri_mul_out, &g[8], &g[9]);
  trimul_pack_groups(block_trimul_desc(d, EVO_TRI_IN), w.tri_mul_in, &g[10], &g[11]);
  attn_pack_groups(block_attn_desc(d, EVO_ATTN_TRI_START), w.tri_att_start, &g[12], &g[13]);
  attn_pack_groups(block_attn_desc(d, EVO_ATTN_TRI_END), w.tri_att_end, &g[14], &g[15]);
  trans_pack_groups(block_trans_desc(d, false), w.pair_trans, &g[16], &g[17]);
  return prepack_groups<T>(c, ws, g, 18, bwd, fill, pc);
}

template <typename T>
static evo_status_t prepack_template(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_template_w_t& w,
                                     bool bwd, PackCache* pc) {
  PackArgs g[10];
  attn_pack_groups(block_attn_desc(d, EVO_ATTN_TRI_START), w.tri_att_start, &g[0], &g[1]);
  attn_pack_groups(block_attn_desc(d, EVO_ATTN_TRI_END), w.tri_att_end, &g[2], &g[3]);
  trimul_pack_groups(block_trimul_desc(d, EVO_TRI_OUT), w.tri_mul_out, &g[4], &g[5]);
  trimul_pack_groups(block_trimul_desc(d, EVO_TRI_IN), w.tri_mul_in, &g[6], &g[7]);
  trans_pack_groups(block_trans_desc(d, false), w.pair_trans, &g[8], &g[9]);
  return prepack_groups<T>(c, ws, g, 10, bwd, true, pc);
}

template <typename T, typename X>
static evo_status_t block_fwd_x(const Ctx& c0, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                                const X* m, const X* z, const float* mm, const float* pm, X* mo, X* zo) {
  BlockDrop bd;
  EVO_TRY(make_block_drop(c0, ws, block_drop_cfg(d), d.n_res, d.c_m, d.c_z, true, &bd));
  PackCache pc;
  EVO_TRY(prepack_block<T>(c0, ws, d, w, false, true, &pc));
  Ctx c = c0;
  c.packed = &pc;
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
  // the outer-product-mean-first order reads the block's input m and hands
  // z + OPM(m) to both branches (the pair bias of row attention included)
  if (d.opm_first) EVO_STEP("opm.fwd", (opm_fwd_op<T, X>(c, a, a, block_opm_desc(d), w.opm, m, mm, z, zo)));
  const X* zpair = d.opm_first ? zo : z;
  EVO_STEP("row.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, EVO_ATTN_ROW), w.row_attn, m, zpair, mm, mo, &bd.row)));
  EVO_STEP("col.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, col_kind), w.col_attn, mo, nullptr, mm, mo)));
  EVO_STEP("msa_trans.fwd", (trans_fwd_op<T, X>(c, a, a, block_trans_desc(d, true), w.msa_trans, mo, mo)));
  if (!d.opm_first) EVO_STEP("opm.fwd", (opm_fwd_op<T, X>(c, a, a, block_opm_desc(d), w.opm, mo, mm, z, zo)));
  EVO_STEP("tri_mul_out.fwd", (trimul_fwd_op<T, X>(c, a, a, block_trimul_desc(d, EVO_TRI_OUT), w.tri_mul_out, zo, pm, zo, &bd.tmo)));
  EVO_STEP("tri_mul_in.fwd", (trimul_fwd_op<T, X>(c, a, a, block_trimul_desc(d, EVO_TRI_IN), w.tri_mul_in, zo, pm, zo, &bd.tmi)));
  EVO_STEP("tri_att_start.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, EVO_ATTN_TRI_START), w.tri_att_start, zo, nullptr, pm, zo, &bd.tas)));
  EVO_STEP("tri_att_end.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, EVO_ATTN_TRI_END), w.tri_att_end, zo, nullptr, pm, zo, &bd.tae)));
  EVO_STEP("pair_trans.fwd", (trans_fwd_op<T, X>(c, a, a, block_trans_desc(d, false), w.pair_trans, zo, zo)));
#undef EVO_STEP
  ws.off = sc.end();
  return EVO_OK;
}

// A block's training pass.  BLK_FULL: the checkpointed backward (recompute the
// forward into the workspace, then the backward ops in reverse order).
// BLK_SAVE: only the recomputation, as a forward that keeps the block's state
// (dropout tables, packed parameters, the activations between sub-ops and
// every sub-op's saved tensors) in `kp` and writes the block's outputs to
// mo / zo.  BLK_SAVED: only the backward, over the state a BLK_SAVE call left
// in `kp` (carved in the same order, nothing recomputed).  In BLK_FULL `kp` is
// the workspace itself.
enum { BLK_FULL = 0, BLK_SAVE = 1, BLK_SAVED = 2 };

template <typename T, typename X>
static evo_status_t block_train_x(const Ctx& c0, Arena& ws, Arena& kp, int mode, const evo_block_desc_t& d,
                                  const evo_block_w_t& w, const X* m, const X* z, const float* mm, const float* pm,
                                  const X* dmo, const X* dzo, X* dm, X* dz, const evo_block_w_t& dw, X* mo,
                                  X* zo, const X** fin = nullptr) {
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

  const bool fill = mode != BLK_SAVED, save = mode == BLK_SAVE;
  BlockDrop bd;
  EVO_TRY(make_block_drop(c0, kp, block_drop_cfg(d), d.n_res, d.c_m, d.c_z, true, &bd, fill));
  PackCache pc;
  EVO_TRY(prepack_block<T>(c0, kp, d, w, true, fill, &pc));
  Ctx c = c0;
  c.packed = &pc;
  const bool of = d.opm_first != 0;
  // activations between sub-ops.  A0 order: m -> m1 -> m2 -> m3 (row, column,
  // transition), z -> z1 (outer product mean of m3) -> z2 ... z6 (pair stack).
  // Outer-product-mean first: z -> z1 (outer product mean of m), then the MSA
  // stack m -> m1 -> m2 -> m3 with the pair bias from z1, and the pair stack.
  X* m1 = kp.take_n<X>(SRc);
  X* m2 = kp.take_n<X>(SRc);
  X* m3 = kp.take_n<X>(SRc);
  X* z1 = kp.take_n<X>(RRc);
  X* z2 = kp.take_n<X>(RRc);
  X* z3 = kp.take_n<X>(RRc);
  X* z4 = kp.take_n<X>(RRc);
  X* z5 = kp.take_n<X>(RRc);
  X* z6 = kp.take_n<X>(RRc);
  // saved regions: carved by the ops themselves from per-op sub-arenas
  Arena sv[9];
  for (int i = 0; i < 9; ++i) { sv[i].dry = true; }
  {
    Ctx dry = c; dry.dry = true;
    Arena junk; junk.dry = true;
    attn_fwd_op<T, X>(dry, junk, sv[0], d_row, w.row_attn, m, z, mm, m1);
    attn_fwd_op<T, X>(dry, junk, sv[1], d_col, w.col_attn, m1, nullptr, mm, m2);
    trans_fwd_op<T, X>(dry, junk, sv[2], d_tm, w.msa_trans, m2, m3);
    opm_fwd_op<T, X>(dry, junk, sv[3], d_opm, w.opm, m3, mm, z, z1);   // sizes only: order immaterial
    trimul_fwd_op<T, X>(dry, junk, sv[4], d_mo, w.tri_mul_out, z1, pm, z2);
    trimul_fwd_op<T, X>(dry, junk, sv[5], d_mi, w.tri_mul_in, z2, pm, z3);
    attn_fwd_op<T, X>(dry, junk, sv[6], d_tas, w.tri_att_start, z3, nullptr, pm, z4);
    attn_fwd_op<T, X>(dry, junk, sv[7], d_tae, w.tri_att_end, z4, nullptr, pm, z5);
    trans_fwd_op<T, X>(dry, junk, sv[8], d_tz, w.pair_trans, z5, z6);
  }
  char* svbase[9];
  for (int i = 0; i < 9; ++i) svbase[i] = (char*)kp.take(sv[i].off);
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
  const X* m_opm = of ? m : m3;     // the outer product mean's input
  const X* z_row = of ? z1 : z;     // the pair representation row attention reads
  if (mode != BLK_SAVED) {
  if (of) EVO_STEPS(3, save ? "opm.fwd" : "opm.recompute", (opm_fwd_op<T, X>(c, a, s, d_opm, w.opm, m_opm, mm, z, z1)));
  EVO_STEPS(0, save ? "row.fwd" : "row.recompute", (attn_fwd_op<T, X>(c, a, s, d_row, w.row_attn, m, z_row, mm, m1, &bd.row)));
  EVO_STEPS(1, save ? "col.fwd" : "col.recompute", (attn_fwd_op<T, X>(c, a, s, d_col, w.col_attn, m1, nullptr, mm, m2)));
  EVO_STEPS(2, save ? "msa_trans.fwd" : "msa_trans.recompute", (trans_fwd_op<T, X>(c, a, s, d_tm, w.msa_trans, m2, m3)));
  if (!of) EVO_STEPS(3, save ? "opm.fwd" : "opm.recompute", (opm_fwd_op<T, X>(c, a, s, d_opm, w.opm, m_opm, mm, z, z1)));
  EVO_STEPS(4, save ? "tri_mul_out.fwd" : "tri_mul_out.recompute", (trimul_fwd_op<T, X>(c, a, s, d_mo, w.tri_mul_out, z1, pm, z2, &bd.tmo)));
  EVO_STEPS(5, save ? "tri_mul_in.fwd" : "tri_mul_in.recompute", (trimul_fwd_op<T, X>(c, a, s, d_mi, w.tri_mul_in, z2, pm, z3, &bd.tmi)));
  EVO_STEPS(6, save ? "tri_att_start.fwd" : "tri_att_start.recompute", (attn_fwd_op<T, X>(c, a, s, d_tas, w.tri_att_start, z3, nullptr, pm, z4, &bd.tas)));
  EVO_STEPS(7, save ? "tri_att_end.fwd" : "tri_att_end.recompute", (attn_fwd_op<T, X>(c, a, s, d_tae, w.tri_att_end, z4, nullptr, pm, z5, &bd.tae)));
  EVO_STEPS(8, save ? "pair_trans.fwd" : "pair_trans.recompute", (trans_fwd_op<T, X>(c, a, s, d_tz, w.pair_trans, z5, z6)));
  }
  if (mode == BLK_SAVE) {
    // outputs: copied to mo / zo, or handed back in place (fin)
    if (fin) { fin[0] = m3; fin[1] = z6; }
    if (!c.dry && mo) EVO_TRY(copy_elems<X>(c, m3, mo, SRc));
    if (!c.dry && zo) EVO_TRY(copy_elems<X>(c, z6, zo, RRc));
    ws.off = sc.end();
    return EVO_OK;
  }
  // backward in reverse order; the pair gradient moves from dz_out into dz at
  // the pair transition and is then updated in place in dz
  if (!c.dry) EVO_TRY(copy_elems<X>(c, dmo, dm, SRc));
  EVO_STEPS(8, "pair_trans.bwd", (trans_bwd_op<T, X>(c, a, s, d_tz, w.pair_trans, z5, dzo, dz, dw.pair_trans)));
  EVO_STEPS(7, "tri_att_end.bwd", (attn_bwd_op<T, X>(c, a, s, d_tae, w.tri_att_end, z4, nullptr, pm, dz, dz, nullptr, dw.tri_att_end, &bd.tae)));
  EVO_STEPS(6, "tri_att_start.bwd", (attn_bwd_op<T, X>(c, a, s, d_tas, w.tri_att_start, z3, nullptr, pm, dz, dz, nullptr, dw.tri_att_start, &bd.tas)));
  EVO_STEPS(5, "tri_mul_in.bwd", (trimul_bwd_op<T, X>(c, a, s, d_mi, w.tri_mul_in, z2, pm, dz, dz, dw.tri_mul_in, &bd.tmi)));
  EVO_STEPS(4, "tri_mul_out.bwd", (trimul_bwd_op<T, X>(c, a, s, d_mo, w.tri_mul_out, z1, pm, dz, dz, dw.tri_mul_out, &bd.tmo)));
  // dz now holds the gradient at z1; the outer product mean passes it on to z
  if (!of) EVO_STEPS(3, "opm.bwd", (opm_bwd_op<T, X>(c, a, s, d_opm, w.opm, m_opm, mm, dz, dm, dw.opm)));
  EVO_STEPS(2, "msa_trans.bwd", (trans_bwd_op<T, X>(c, a, s, d_tm, w.msa_trans, m2, dm, dm, dw.msa_trans)));
  EVO_STEPS(1, "col.bwd", (attn_bwd_op<T, X>(c, a, s, d_col, w.col_attn, m1, nullptr, mm, dm, dm, nullptr, dw.col_attn)));
  EVO_STEPS(0, "row.bwd", (attn_bwd_op<T, X>(c, a, s, d_row, w.row_attn, m, z_row, mm, dm, dm, dz, dw.row_attn, &bd.row)));
  if (of) EVO_STEPS(3, "opm.bwd", (opm_bwd_op<T, X>(c, a, s, d_opm, w.opm, m_opm, mm, dz, dm, dw.opm)));
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

// The training pass in the activation type T: FP32 residual streams inside
// (BF16 inputs converted into FP32: in the workspace for a checkpointed
// backward, in the saved state, ahead of everything else the state holds, for
// a BLK_SAVE call, whose BLK_SAVED backward takes them from there).
template <typename T>
static evo_status_t block_train_op(const Ctx& c, Arena& ws, Arena& kp, int mode, const evo_block_desc_t& d,
                                   const evo_block_w_t& w, const T* m, const T* z, const float* mm, const float* pm,
                                   const T* dmo, const T* dzo, T* dm, T* dz, const evo_block_w_t& dw, T* mo, T* zo) {
  if constexpr (std::is_same<T, float>::value) {
    return block_train_x<T, float>(c, ws, kp, mode, d, w, m, z, mm, pm, dmo, dzo, dm, dz, dw, mo, zo);
  } else {
    const int64_t SRc = d.n_seq * d.n_res * d.c_m, RRc = d.n_res * d.n_res * d.c_z;
    const bool bwd = mode != BLK_SAVE;
    Arena& ia = mode == BLK_FULL ? ws : kp;
    float* mx = ia.take_n<float>(SRc);
    float* zx = ia.take_n<float>(RRc);
    float* dmx = bwd ? ws.take_n<float>(SRc) : nullptr;
    float* dzx = bwd ? ws.take_n<float>(RRc) : nullptr;
    if (mode != BLK_SAVED) {
      EVO_TRY((convert_elems<T, float>(c, m, mx, SRc)));
      EVO_TRY((convert_elems<T, float>(c, z, zx, RRc)));
    }
    if (bwd) {
      EVO_TRY((convert_elems<T, float>(c, dmo, dmx, SRc)));
      EVO_TRY((convert_elems<T, float>(c, dzo, dzx, RRc)));
    }
    const float* fin[2] = {nullptr, nullptr};
    EVO_TRY((block_train_x<T, float>(c, ws, kp, mode, d, w, mx, zx, mm, pm, dmx, dzx, dmx, dzx, dw, nullptr, nullptr,
                                     fin)));
    if (!bwd) {
      EVO_TRY((convert_elems<float, T>(c, fin[0], mo, SRc)));
      return convert_elems<float, T>(c, fin[1], zo, RRc);
    }
    EVO_TRY((convert_elems<float, T>(c, dmx, dm, SRc)));
    return convert_elems<float, T>(c, dzx, dz, RRc);
  }
}

template <typename T>
evo_status_t block_bwd_op(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                          const T* m, const T* z, const float* mm, const float* pm, const T* dmo,
                          const T* dzo, T* dm, T* dz, const evo_block_w_t& dw) {
  return block_train_op<T>(c, ws, ws, BLK_FULL, d, w, m, z, mm, pm, dmo, dzo, dm, dz, dw, nullptr, nullptr);
}

template <typename T>
evo_status_t block_fwd_save_op(const Ctx& c, Arena& ws, Arena& saved, const evo_block_desc_t& d,
                               const evo_block_w_t& w, const T* m, const T* z, const float* mm, const float* pm,
                               T* mo, T* zo) {
  return block_train_op<T>(c, ws, saved, BLK_SAVE, d, w, m, z, mm, pm, nullptr, nullptr, nullptr, nullptr, w, mo,
                           zo);
}

template <typename T>
evo_status_t block_bwd_saved_op(const Ctx& c, Arena& ws, Arena& saved, const evo_block_desc_t& d,
                                const evo_block_w_t& w, const T* m, const T* z, const float* mm, const float* pm,
                                const T* dmo, const T* dzo, T* dm, T* dz, const evo_block_w_t& dw) {
  return block_train_op<T>(c, ws, saved, BLK_SAVED, d, w, m, z, mm, pm, dmo, dzo, dm, dz, dw, nullptr, nullptr);
}

// ============================================================== template pair stack block
// The pair-stack sub-operations on one template's pair features, in the
// template order (attention around the starting and the ending node, outgoing
// and incoming multiplication, transition); sub-op descriptors come from an
// Evoformer block descriptor with c_z = c_t.
evo_block_desc_t template_as_block(const evo_template_desc_t& t) {
  evo_block_desc_t b;
  memset(&b, 0, sizeof(b));
  b.dtype = t.dtype;
  b.n_seq = 1; b.n_res = t.n_res; b.c_m = 8; b.c_z = t.c_t;
  b.msa_heads = 1; b.msa_head_dim = 8;
  b.tri_heads = t.tri_heads; b.tri_head_dim = t.tri_head_dim;
  b.tri_mul_hidden = t.tri_mul_hidden; b.opm_hidden = 8; b.transition_factor = t.transition_factor;
  b.chunk = t.chunk;
  b.ln_eps = t.ln_eps; b.opm_eps = 1e-3f; b.global_eps = 1e-10f;
  return b;
}

static DropCfg template_drop_cfg(const evo_template_desc_t& d) {
  DropCfg dc;
  dc.on = d.dropout != 0;
  dc.seed = d.drop_seed; dc.offset = d.drop_offset;
  dc.rate_mul = d.drop_tri_mul; dc.rate_att = d.drop_tri_att;
  dc.tmpl = (uint32_t)d.template_index;
  return dc;
}

template <typename T, typename X>
static evo_status_t template_fwd_x(const Ctx& c0, Arena& ws, const evo_template_desc_t& td, const evo_template_w_t& w,
                                   const X* t, const float* pm, X* to) {
  const evo_block_desc_t d = template_as_block(td);
  BlockDrop bd;
  EVO_TRY(make_block_drop(c0, ws, template_drop_cfg(td), d.n_res, 0, d.c_z, false, &bd));
  PackCache pc;
  EVO_TRY(prepack_template<T>(c0, ws, d, w, false, &pc));
  Ctx c = c0;
  c.packed = &pc;
  Scratch sc;
  sc.base = ws;
#define EVO_STEP(tag, call)       \
  do {                            \
    ProfTag pt_(tag);             \
    Arena a = sc.fresh();         \
    EVO_TRY(call);                \
    sc.done(a);                   \
  } while (0)
  EVO_STEP("tri_att_start.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, EVO_ATTN_TRI_START), w.tri_att_start, t, nullptr, pm, to, &bd.tas)));
  EVO_STEP("tri_att_end.fwd", (attn_fwd_op<T, X>(c, a, a, block_attn_desc(d, EVO_ATTN_TRI_END), w.tri_att_end, to, nullptr, pm, to, &bd.tae)));
  EVO_STEP("tri_mul_out.fwd", (trimul_fwd_op<T, X>(c, a, a, block_trimul_desc(d, EVO_TRI_OUT), w.tri_mul_out, to, pm, to, &bd.tmo)));
  EVO_STEP("tri_mul_in.fwd", (trimul_fwd_op<T, X>(c, a, a, block_trimul_desc(d, EVO_TRI_IN), w.tri_mul_in, to, pm, to, &bd.tmi)));
  EVO_STEP("pair_trans.fwd", (trans_fwd_op<T, X>(c, a, a, block_trans_desc(d, false), w.pair_trans, to, to)));
#undef EVO_STEP
  ws.off = sc.end();
  return EVO_OK;
}

template <typename T, typename X>
static evo_status_t template_bwd_x(const Ctx& c0, Arena& ws, const evo_template_desc_t& td, const evo_template_w_t& w,
                                   const X* t, const float* pm, const X* dto, X* dt, const evo_template_w_t& dw) {
  evo_block_desc_t d = template_as_block(td);
  d.chunk = 0;
  const int64_t RRc = d.n_res * d.n_res * d.c_z;
  const evo_attn_desc_t d_tas = block_attn_desc(d, EVO_ATTN_TRI_START), d_tae = block_attn_desc(d, EVO_ATTN_TRI_END);
  const evo_trimul_desc_t d_mo = block_trimul_desc(d, EVO_TRI_OUT), d_mi = block_trimul_desc(d, EVO_TRI_IN);
  const evo_trans_desc_t d_tz = block_trans_desc(d, false);
  BlockDrop bd;
  EVO_TRY(make_block_drop(c0, ws, template_drop_cfg(td), d.n_res, 0, d.c_z, false, &bd));
  PackCache pc;
  EVO_TRY(prepack_template<T>(c0, ws, d, w, true, &pc));
  Ctx c = c0;
  c.packed = &pc;
  // t -> t1 (start) -> t2 (end) -> t3 (out) -> t4 (in) -> t5 (transition)
  X* t1 = ws.take_n<X>(RRc);
  X* t2 = ws.take_n<X>(RRc);
  X* t3 = ws.take_n<X>(RRc);
  X* t4 = ws.take_n<X>(RRc);
  X* t5 = ws.take_n<X>(RRc);
  Arena sv[5];
  for (int i = 0; i < 5; ++i) sv[i].dry = true;
  {
    Ctx dry = c; dry.dry = true;
    Arena junk; junk.dry = true;
    attn_fwd_op<T, X>(dry, junk, sv[0], d_tas, w.tri_att_start, t, nullptr, pm, t1);
    attn_fwd_op<T, X>(dry, junk, sv[1], d_tae, w.tri_att_end, t1, nullptr, pm, t2);
    trimul_fwd_op<T, X>(dry, junk, sv[2], d_mo, w.tri_mul_out, t2, pm, t3);
    trimul_fwd_op<T, X>(dry, junk, sv[3], d_mi, w.tri_mul_in, t3, pm, t4);
    trans_fwd_op<T, X>(dry, junk, sv[4], d_tz, w.pair_trans, t4, t5);
  }
  char* svbase[5];
  for (int i = 0; i < 5; ++i) svbase[i] = (char*)ws.take(sv[i].off);
  auto S = [&](int i) {
    Arena a;
    a.dry = c.dry;
    a.base = svbase[i];
    a.cap = sv[i].off;
    return a;
  };
  Scratch sc;
  sc.base = ws;
#define EVO_STEPS(i, tag, call)                                                \
  do {                                                                         \
    ProfTag pt_(tag);                                                          \
    Arena a = sc.fresh();                                                      \
    Arena s = S(i);                                                            \
    EVO_TRY(with_batched_reductions(c, [&](const Ctx& c) { return call; })); \
    sc.done(a);                                                                \
  } while (0)
  EVO_STEPS(0, "tri_att_start.recompute", (attn_fwd_op<T, X>(c, a, s, d_tas, w.tri_att_start, t, nullptr, pm, t1, &bd.tas)));
  EVO_STEPS(1, "tri_att_end.recompute", (attn_fwd_op<T, X>(c, a, s, d_tae, w.tri_att_end, t1, nullptr, pm, t2, &bd.tae)));
  EVO_STEPS(2, "tri_mul_out.recompute", (trimul_fwd_op<T, X>(c, a, s, d_mo, w.tri_mul_out, t2, pm, t3, &bd.tmo)));
  EVO_STEPS(3, "tri_mul_in.recompute", (trimul_fwd_op<T, X>(c, a, s, d_mi, w.tri_mul_in, t3, pm, t4, &bd.tmi)));
  EVO_STEPS(4, "pair_trans.recompute", (trans_fwd_op<T, X>(c, a, s, d_tz, w.pair_trans, t4, t5)));
  if (!c.dry) EVO_TRY(copy_elems<X>(c, dto, dt, RRc));
  EVO_STEPS(4, "pair_trans.bwd", (trans_bwd_op<T, X>(c, a, s, d_tz, w.pair_trans, t4, dt, dt, dw.pair_trans)));
  EVO_STEPS(3, "tri_mul_in.bwd", (trimul_bwd_op<T, X>(c, a, s, d_mi, w.tri_mul_in, t3, pm, dt, dt, dw.tri_mul_in, &bd.tmi)));
  EVO_STEPS(2, "tri_mul_out.bwd", (trimul_bwd_op<T, X>(c, a, s, d_mo, w.tri_mul_out, t2, pm, dt, dt, dw.tri_mul_out, &bd.tmo)));
  EVO_STEPS(1, "tri_att_end.bwd", (attn_bwd_op<T, X>(c, a, s, d_tae, w.tri_att_end, t1, nullptr, pm, dt, dt, nullptr, dw.tri_att_end, &bd.tae)));
  EVO_STEPS(0, "tri_att_start.bwd", (attn_bwd_op<T, X>(c, a, s, d_tas, w.tri_att_start, t, nullptr, pm, dt, dt, nullptr, dw.tri_att_start, &bd.tas)));
#undef EVO_STEPS
  ws.off = sc.end();
  return EVO_OK;
}

template <typename T>
evo_status_t template_fwd_op(const Ctx& c, Arena& ws, const evo_template_desc_t& d, const evo_template_w_t& w,
                             const T* t, const float* pm, T* to) {
  if constexpr (std::is_same<T, float>::value) {
    return template_fwd_x<T, float>(c, ws, d, w, t, pm, to);
  } else {
    const int64_t RRc = d.n_res * d.n_res * d.c_t;
    float* tx = ws.take_n<float>(RRc);
    EVO_TRY((convert_elems<T, float>(c, t, tx, RRc)));
    EVO_TRY((template_fwd_x<T, float>(c, ws, d, w, tx, pm, tx)));
    return convert_elems<float, T>(c, tx, to, RRc);
  }
}

template <typename T>
evo_status_t template_bwd_op(const Ctx& c, Arena& ws, const evo_template_desc_t& d, const evo_template_w_t& w,
                             const T* t, const float* pm, const T* dto, T* dt, const evo_template_w_t& dw) {
  if constexpr (std::is_same<T, float>::value) {
    return template_bwd_x<T, float>(c, ws, d, w, t, pm, dto, dt, dw);
  } else {
    const int64_t RRc = d.n_res * d.n_res * d.c_t;
    float* tx = ws.take_n<float>(RRc);
    float* dtx = ws.take_n<float>(RRc);
    EVO_TRY((convert_elems<T, float>(c, t, tx, RRc)));
    EVO_TRY((convert_elems<T, float>(c, dto, dtx, RRc)));
    EVO_TRY((template_bwd_x<T, float>(c, ws, d, w, tx, pm, dtx, dtx, dw)));
    return convert_elems<float, T>(c, dtx, dt, RRc);
  }
}

template evo_status_t template_fwd_op<float>(const Ctx&, Arena&, const evo_template_desc_t&, const evo_template_w_t&,
                                             const float*, const float*, float*);
template evo_status_t template_fwd_op<bf16>(const Ctx&, Arena&, const evo_template_desc_t&, const evo_template_w_t&,
                                            const bf16*, const float*, bf16*);
template evo_status_t template_bwd_op<float>(const Ctx&, Arena&, const evo_template_desc_t&, const evo_template_w_t&,
                                             const float*, const float*, const float*, float*,
                                             const evo_template_w_t&);
template evo_status_t template_bwd_op<bf16>(const Ctx&, Arena&, const evo_template_desc_t&, const evo_template_w_t&,
                                            const bf16*, const float*, const bf16*, bf16*, const evo_template_w_t&);

#define EVO_INST_B(T)                                                                              \
  template evo_status_t block_fwd_op<T>(const Ctx&, Arena&, const evo_block_desc_t&,               \
                                        const evo_block_w_t&, const T*, const T*, const float*,    \
                                        const float*, T*, T*);                                     \
  template evo_status_t block_bwd_op<T>(const Ctx&, Arena&, const evo_block_desc_t&,               \
                                        const evo_block_w_t&, const T*, const T*, const float*,    \
                                        const float*, const T*, const T*, T*, T*,                  \
                                        const evo_block_w_t&);                                     \
  template evo_status_t block_fwd_save_op<T>(const Ctx&, Arena&, Arena&, const evo_block_desc_t&,  \
                                             const evo_block_w_t&, const T*, const T*,             \
                                             const float*, const float*, T*, T*);                  \
  template evo_status_t block_bwd_saved_op<T>(const Ctx&, Arena&, Arena&, const evo_block_desc_t&, \
                                              const evo_block_w_t&, const T*, const T*,            \
                                              const float*, const float*, const T*, const T*, T*,  \
                                              T*, const evo_block_w_t&);

EVO_INST_B(float)
EVO_INST_B(bf16)

}  // namespace evo
