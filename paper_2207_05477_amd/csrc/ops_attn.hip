// Gated self-attention op (all kinds): LayerNorm -> fused q|k|v|gate
// projection (one GEMM, sigmoid gate in the epilogue) -> pair-bias projection
// -> attention core -> output projection with bias and residual in the
// epilogue; and its backward.
#include "ops.h"

namespace evo {

namespace {

struct AttnShape {
  int kind;
  int64_t no, ni, rows, cin, cpair;
  int H, D, HC, NQ;
  bool global, row, tri;
};

AttnShape attn_shape(const evo_attn_desc_t& d) {
  AttnShape s;
  s.kind = d.kind;
  s.no = d.n_outer; s.ni = d.n_inner; s.rows = d.n_outer * d.n_inner;
  s.cin = d.c_in; s.cpair = d.c_pair;
  s.H = d.heads; s.D = d.head_dim; s.HC = d.heads * d.head_dim;
  s.global = d.kind == EVO_ATTN_COL_GLOBAL;
  s.row = d.kind == EVO_ATTN_ROW;
  s.tri = d.kind == EVO_ATTN_TRI_START || d.kind == EVO_ATTN_TRI_END;
  s.NQ = s.global ? 2 * s.HC + 2 * s.D : 4 * s.HC;
  return s;
}

template <typename T>
struct AttnSaved {
  T* y; float* mean; float* rstd;
  T* yz; float* zmean; float* zrstd;
  T* qkvg;
  float* bias;
  float* o;   // pre-gate context, FP32
  T* go;
  float* st_max; float* st_inv;
  float* gctx; float* qbar; float* minv;
  void carve(Arena& a, const AttnShape& s) {
    y = a.take_n<T>(s.rows * s.cin);
    mean = a.take_n<float>(s.rows);
    rstd = a.take_n<float>(s.rows);
    yz = nullptr; zmean = zrstd = nullptr; bias = nullptr; gctx = qbar = minv = nullptr;
    if (s.row) bias = a.take_n<float>((int64_t)s.H * s.ni * s.ni);
    if (s.tri) bias = a.take_n<float>((int64_t)s.H * s.rows);
    qkvg = a.take_n<T>(s.rows * s.NQ);
    if (s.global) {
      gctx = a.take_n<float>(s.ni * s.HC);
      qbar = a.take_n<float>(s.ni * s.HC);
      minv = a.take_n<float>(s.ni);
      st_max = a.take_n<float>(s.ni * s.H);
      st_inv = a.take_n<float>(s.ni * s.H);
      o = nullptr;
    } else {
      o = a.take_n<float>(s.rows * s.HC);
      st_max = a.take_n<float>(s.rows * s.H);
      st_inv = a.take_n<float>(s.rows * s.H);
    }
    go = a.take_n<T>(s.rows * s.HC);
  }
};

// Strides of the attention core for each kind (see evo.h for the index maps).
AttnCore core_for(const AttnShape& s, const void* qkvg, void* o, void* go, const float* bias,
                  const float* mask, float* smax, float* sinv) {
  AttnCore a;
  const int64_t ld = s.NQ, HC = s.HC;
  const char* base = (const char*)qkvg;
  (void)base;
  a.H = s.H; a.D = s.D;
  a.o = o; a.go = go;
  a.bias = bias; a.mask = mask;
  a.st_max = smax; a.st_inv = sinv;
  const bool batch_outer = s.kind == EVO_ATTN_ROW || s.kind == EVO_ATTN_TRI_START;
  if (batch_outer) {
    a.nbatch = s.no; a.Lq = a.Lk = s.ni;
    a.sb = s.ni * ld; a.sp = ld; a.osb = s.ni * HC; a.osp = HC;
    a.stb = s.ni; a.stq = 1;
    a.mb = s.ni; a.mk = 1;
    a.bh = s.ni * s.ni; a.bq = s.ni; a.bk = 1;
  } else {  // COL, TRI_END: batch is the inner index, queries/keys run over the outer index
    a.nbatch = s.ni; a.Lq = a.Lk = s.no;
    a.sb = ld; a.sp = s.ni * ld; a.osb = HC; a.osp = s.ni * HC;
    a.stb = 1; a.stq = s.ni;
    a.mb = 1; a.mk = s.ni;
    // TRI_END: the bias b_ki of query i, key k is stored transposed (see
    // pair_bias), so that it has unit stride along keys like the other kinds
    a.bh = s.no * s.no; a.bq = s.no; a.bk = 1;
  }
  return a;
}

// Pair bias of the attention core, log2(e) * (LayerNorm(x) W_bias), [H][n][n]:
// b[h][q][k] for the row and starting-node kinds; the ending-node kind's bias of
// query i and key k is the projection of pair entry (k, i), written transposed
// so that the core reads it at q*n + k as well.  The bias gradient comes back
// in the projection's own row order (AttnGrad dbq, dbk).
template <typename X, typename T>
evo_status_t pair_bias(const Ctx& c, bool tri_end, const X* x, int64_t n, int C, const float* ln_g,
                       const float* ln_b, float eps, const float* W, int H, float* bias) {
  return ln_rowproj<X, T>(c, x, n * n, C, ln_g, ln_b, eps, W, H, bias, kLog2e, tri_end ? n : 0);
}

template <typename T>
void set_qkvg(AttnCore& a, const T* qkvg, const AttnShape& s) {
  a.q = qkvg;
  a.k = qkvg + s.HC;
  a.v = qkvg + 2 * s.HC;
  a.g = qkvg + 3 * s.HC;
}

}  // namespace

// Global column attention (gattn.hip): forward scratch size in FP32 elements,
// forward and backward.  qbar [R][H*D] is the masked-mean query, minv[i] =
// 1 / (sum_s M_si + eps), gctx [R][H*D] the context, smax / sinv [R][H] the
// softmax statistics.
int64_t gattn_fwd_scratch(int64_t S, int64_t R, int H, int D);
template <typename T>
evo_status_t gattn_fwd(const Ctx& c, float* scratch, int64_t S, int64_t R, int H, int D, const T* qkvg,
                       const float* mask, float eps, float* qbar, float* minv, float* gctx, float* smax,
                       float* sinv, T* go);
template <typename T>
evo_status_t gattn_bwd(const Ctx& c, Arena& ws, int64_t S, int64_t R, int H, int D, const T* qkvg,
                       const float* mask, const float* qbar, const float* minv, const float* gctx,
                       const float* smax, const float* sinv, const float* dgo, T* dqkvg);

// Parameter groups of an attention op: the fused q|k|v|g projection (the
// gate bias as its bias row) and the output projection.
void attn_pack_groups(const evo_attn_desc_t& d, const evo_attn_w_t& w, PackArgs* in, PackArgs* out) {
  const AttnShape s = attn_shape(d);
  *in = PackArgs();
  in->K = (int)s.cin;
  in->seg[0] = {w.w_q, nullptr, s.HC};
  in->seg[1] = {w.w_k, nullptr, s.global ? s.D : s.HC};
  in->seg[2] = {w.w_v, nullptr, s.global ? s.D : s.HC};
  in->seg[3] = {w.w_g, w.b_g, s.HC};
  in->nseg = 4;
  *out = PackArgs();
  out->K = s.HC;
  out->seg[0] = {w.w_o, nullptr, (int)s.cin};
  out->nseg = 1;
}

// Forward of triangle attention in chunks of `chunk` batch rows (starting node:
// rows i; ending node: columns j), keeping no saved state.  Only the chunk's
// LayerNorm / projection / context buffers exist; the pair bias (all rows) is
// formed once.  Equal to the unchunked forward (same per-row arithmetic).
template <typename T, typename X>
static evo_status_t attn_fwd_tri_chunked(const Ctx& c, Arena& ws, const evo_attn_desc_t& d,
                                         const AttnShape& s, const evo_attn_w_t& w, const X* x,
                                         const float* mask, X* out) {
  const int64_t R = s.ni, C = d.chunk, CR = C * R, cin = s.cin;
  const int sh = ilog2(C);
  const bool start = s.kind == EVO_ATTN_TRI_START;
  T* wt_qkvg = ws.take_n<T>((int64_t)s.NQ * cin);
  float* b_qkvg = ws.take_n<float>(s.NQ);
  T* wt_o = ws.take_n<T>(cin * s.HC);
  float* bias = ws.take_n<float>((int64_t)s.H * R * R);
  T* y = ws.take_n<T>(CR * cin);
  float* mean = ws.take_n<float>(CR);
  float* rstd = ws.take_n<float>(CR);
  T* qkvg = ws.take_n<T>(CR * s.NQ);
  T* go = ws.take_n<T>(CR * s.HC);
  if (c.dry) return EVO_OK;
  PackArgs pk, po;
  attn_pack_groups(d, w, &pk, &po);
  pk.dst_t = wt_qkvg;
  pk.bias = b_qkvg;
  po.dst_t = wt_o;
  EVO_TRY(pack_params<T>(c, {&pk, &po}));
  wt_qkvg = (T*)pk.dst_t;
  b_qkvg = pk.bias;
  wt_o = (T*)po.dst_t;
  EVO_TRY((pair_bias<X, T>(c, !start, x, R, (int)cin, w.ln_g, w.ln_b, d.ln_eps, w.w_bias, s.H, bias)));
  for (int64_t c0 = 0; c0 < R; c0 += C) {
    // chunk rows: starting node (i, j) = (c0 + ii, j) contiguous; ending node
    // (i, j) = (i, c0 + jj) with local row i*C + jj
    const X* xs = start ? x + c0 * R * cin : x + c0 * cin;
    EVO_TRY((ln_fwd_rows<X, T>(c, xs, CR, (int)cin, start ? -1 : sh, R * cin, w.ln_g, w.ln_b, d.ln_eps, y,
                               mean, rstd)));
    GemmArgs g;
    g.M = CR; g.N = s.NQ; g.K = cin;
    g.A = op_rowmajor(y, cin);
    g.B = op_rowmajor(wt_qkvg, cin);
    g.epi = epi_rowmajor(qkvg, s.NQ, false);
    g.epi.bias = b_qkvg;
    g.epi.act = ACT_SIGMOID;
    g.epi.act_n0 = s.NQ - s.HC;
    EVO_TRY(gemm<T>(c, g));
    AttnCore a;
    a.H = s.H; a.D = s.D; a.o = nullptr; a.go = go; a.bias = bias; a.bh = R * R;
    a.nbatch = C; a.Lq = a.Lk = R;
    a.bq = R; a.bk = 1;   // both kinds (pair_bias)
    if (start) {
      a.sb = R * s.NQ; a.sp = s.NQ; a.osb = R * s.HC; a.osp = s.HC;
      a.mask = mask ? mask + c0 * R : nullptr; a.mb = R; a.mk = 1;
    } else {
      a.sb = s.NQ; a.sp = C * s.NQ; a.osb = s.HC; a.osp = C * s.HC;
      a.mask = mask ? mask + c0 : nullptr; a.mb = 1; a.mk = R;
    }
    set_qkvg<T>(a, qkvg, s);
    EVO_TRY(attn_fwd<T>(c, a));
    GemmArgs go_;
    go_.M = CR; go_.N = cin; go_.K = s.HC;
    go_.A = op_rowmajor(go, s.HC);
    go_.B = op_rowmajor(wt_o, s.HC);
    go_.epi.out_f32 = is_f32<X>() ? 1 : 0;
    go_.epi.resid_f32 = is_f32<X>() ? 1 : 0;
    go_.epi.bias = w.b_o;
    go_.epi.r_m = -1;   // residual addressed like the output
    if (start) {
      go_.epi.out = out + c0 * R * cin; go_.epi.m_lo = cin; go_.epi.n_lo = 1;
      go_.epi.resid = x + c0 * R * cin;
    } else {
      go_.epi.out = out + c0 * cin; go_.epi.m_lo = cin; go_.epi.m_hi = R * cin; go_.epi.m_shift = sh;
      go_.epi.n_lo = 1;
      go_.epi.resid = x + c0 * cin;
    }
    EVO_TRY(gemm<T>(c, go_));
  }
  return EVO_OK;
}

template <typename T, typename X>
evo_status_t attn_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_attn_desc_t& d,
                         const evo_attn_w_t& w, const X* x, const X* pair, const float* mask, X* out,
                         const DropSpec* drop) {
  const AttnShape s = attn_shape(d);
  if (s.tri && d.chunk > 0 && d.chunk < s.ni) {
    if (drop && drop->on) { set_error("attention: the chunked forward has no dropout"); return EVO_EINVAL; }
    return attn_fwd_tri_chunked<T, X>(c, ws, d, s, w, x, mask, out);
  }
  // saved state handed to a backward only when it has an arena of its own; a
  // forward whose intermediates live in its workspace (a checkpointed block's
  // forward, an op called without saved state) skips the context and statistics
  const bool keep = &sv != &ws;
  AttnSaved<T> S;
  S.carve(sv, s);
  T* wt_qkvg = ws.take_n<T>((int64_t)s.NQ * s.cin);
  float* b_qkvg = ws.take_n<float>(s.NQ);
  T* wt_o = ws.take_n<T>((int64_t)s.cin * s.HC);
  float* ga_scratch = s.global ? ws.take_n<float>(gattn_fwd_scratch(s.no, s.ni, s.H, s.D)) : nullptr;
  if (c.dry) return EVO_OK;

  // parameters: forward operands [n][k] in the compute type
  PackArgs pk, po;
  attn_pack_groups(d, w, &pk, &po);
  pk.dst_t = wt_qkvg;
  pk.bias = b_qkvg;
  po.dst_t = wt_o;
  EVO_TRY(pack_params<T>(c, {&pk, &po}));
  wt_qkvg = (T*)pk.dst_t;
  b_qkvg = pk.bias;
  wt_o = (T*)po.dst_t;

  EVO_TRY((ln_fwd<X, T>(c, x, s.rows, (int)s.cin, w.ln_g, w.ln_b, d.ln_eps, S.y, S.mean, S.rstd)));
  {
    GemmArgs g;
    g.M = s.rows; g.N = s.NQ; g.K = s.cin;
    g.A = op_rowmajor(S.y, s.cin);
    g.B = op_rowmajor(wt_qkvg, s.cin);
    g.epi = epi_rowmajor(S.qkvg, s.NQ, false);
    g.epi.bias = b_qkvg;
    g.epi.act = ACT_SIGMOID;
    g.epi.act_n0 = s.NQ - s.HC;
    EVO_TRY(gemm<T>(c, g));
  }
  if (s.row) {
    EVO_TRY((pair_bias<X, T>(c, false, pair, s.ni, (int)s.cpair, w.ln_z_g, w.ln_z_b, d.ln_eps, w.w_bias, s.H,
                             S.bias)));
  } else if (s.tri) {
    EVO_TRY((pair_bias<X, T>(c, s.kind == EVO_ATTN_TRI_END, x, s.ni, (int)s.cin, w.ln_g, w.ln_b, d.ln_eps,
                             w.w_bias, s.H, S.bias)));
  }
  if (s.global) {
    EVO_TRY(gattn_fwd<T>(c, ga_scratch, s.no, s.ni, s.H, s.D, S.qkvg, mask, d.global_eps, S.qbar, S.minv,
                         S.gctx, S.st_max, S.st_inv, S.go));
  } else {
    AttnCore a = core_for(s, S.qkvg, keep ? S.o : nullptr, S.go, S.bias, mask, keep ? S.st_max : nullptr,
                          keep ? S.st_inv : nullptr);
    set_qkvg<T>(a, S.qkvg, s);
    EVO_TRY(attn_fwd<T>(c, a));
  }
  {
    GemmArgs g;
    g.M = s.rows; g.N = s.cin; g.K = s.HC;
    g.A = op_rowmajor(S.go, s.HC);
    g.B = op_rowmajor(wt_o, s.HC);
    epi_out<X>(g.epi, out, s.cin);
    g.epi.bias = w.b_o;
    epi_dropout(g.epi, drop, s.cin);
    epi_resid<X>(g.epi, x, s.cin, 1);
    EVO_TRY(gemm<T>(c, g));
  }
  return EVO_OK;
}

template <typename T, typename X>
evo_status_t attn_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_attn_desc_t& d,
                         const evo_attn_w_t& w, const X* x, const X* pair, const float* mask,
                         const X* dout, X* dx, X* dpair, const evo_attn_w_t& dw, const DropSpec* drop) {
  const AttnShape s = attn_shape(d);
  AttnSaved<T> S;
  S.carve(sv, s);
  // with dropout the update's gradient is drop * dout; the residual passes dout on
  const X* dres = dout;
  if (drop && drop->on) {
    X* dd = ws.take_n<X>(s.rows * s.cin);
    EVO_TRY(dropout_apply<X>(c, dout, dd, s.rows, (int)s.cin, *drop));
    dout = dd;
  }
  evo_status_t cst;
  const T* dout_t = as_compute<T, X>(c, ws, dout, s.rows * s.cin, &cst);
  EVO_TRY(cst);
  T* w_qkvg = ws.take_n<T>((int64_t)s.cin * s.NQ);     // [c_in][NQ]
  T* w_o = ws.take_n<T>((int64_t)s.HC * s.cin);        // [HC][c_in]
  float* dgo = ws.take_n<float>(s.rows * s.HC);   // FP32: consumed by the gate backward only
  T* dctx = s.global ? nullptr : ws.take_n<T>(s.rows * s.HC);
  T* dqkvg = ws.take_n<T>(s.rows * s.NQ);
  float* Dsum = s.global ? nullptr : ws.take_n<float>(s.rows * s.H);
  float* dy = ws.take_n<float>(s.rows * s.cin);
  float* dbias = nullptr;
  float* dbias_part = nullptr;
  float* ds = nullptr;   // FP32 logit gradients (see AttnGrad::ds)
  AttnCore a;
  int64_t ngroups = 0;
  if (!s.global) {
    a = core_for(s, S.qkvg, S.o, S.go, S.bias, mask, S.st_max, S.st_inv);
    set_qkvg<T>(a, S.qkvg, s);
    if (s.row || s.tri) {
      ngroups = attn_bwd_groups<T>(a);
      dbias_part = ws.take_n<float>((size_t)ngroups * s.H * a.Lq * a.Lk);
      dbias = ws.take_n<float>((size_t)s.H * a.Lq * a.Lk);
    }
    const int64_t nds = attn_bwd_ds_elems<T>(a);
    ds = nds ? ws.take_n<float>(nds) : nullptr;
  }
  const int64_t mark = ws.off;   // scratch below is reused by each step
  (void)mark;

  if (!c.dry) {
    PackArgs pk, po;
    attn_pack_groups(d, w, &pk, &po);
    pk.dst = w_qkvg;
    po.dst = w_o;
    EVO_TRY(pack_params<T>(c, {&pk, &po}));
    w_qkvg = (T*)pk.dst;
    w_o = (T*)po.dst;
  }

  // output projection
  {
    ProfTag t_("out_proj");
    float* const ob[1] = {dw.b_o};
    EVO_TRY(wgrad<T>(c, ws, S.go, s.HC, dout_t, s.cin, s.rows, s.HC, s.cin, dw.w_o, ob));
    GemmArgs g;
    g.M = s.rows; g.N = s.HC; g.K = s.cin;
    g.A = op_rowmajor(dout_t, s.cin);
    g.B = op_rowmajor(w_o, s.cin);
    g.epi = epi_rowmajor(dgo, s.HC, true);
    EVO_TRY(gemm<T>(c, g));
  }
  if (s.global) {
    ProfTag t_("core");
    EVO_TRY(gattn_bwd<T>(c, ws, s.no, s.ni, s.H, s.D, S.qkvg, mask, S.qbar, S.minv, S.gctx, S.st_max,
                         S.st_inv, dgo, dqkvg));
  } else {
    // gate and attention core
    ProfTag t_("core");
    EVO_TRY(gate_bwd<T>(c, s.rows, s.H, s.D, dgo, s.HC, S.o, s.HC, S.qkvg + 3 * s.HC, s.NQ, dctx,
                        s.HC, dqkvg + 3 * s.HC, s.NQ, Dsum));
    AttnGrad gr;
    gr.dctx = dctx;
    gr.Dsum = Dsum;
    gr.dq = dqkvg; gr.dk = dqkvg + s.HC; gr.dv = dqkvg + 2 * s.HC;
    gr.dsb = a.sb; gr.dsp = a.sp;
    gr.dbias_part = dbias_part;
    gr.ds = ds;
    // partials in the projection's row order: (q, k) -> pair entry (k, q) for the ending node
    const bool tend = s.kind == EVO_ATTN_TRI_END;
    gr.dbq = tend ? 1 : a.bq;
    gr.dbk = tend ? a.Lq : a.bk;
    EVO_TRY(attn_bwd<T>(c, a, gr));
    if (dbias_part) {
      const int64_t nb = s.H * a.Lq * a.Lk;
      EVO_TRY(reduce_partials(c, dbias_part, ngroups, nb, nb, dbias, false));
    }
  }
  // gate bias and projection weights
  {
    ProfTag t_("in_proj");
    const int kv = s.global ? s.D : s.HC;
    const int woff[4] = {0, s.HC, s.HC + kv, (int)(s.NQ - s.HC)};
    const int wn[4] = {s.HC, kv, kv, s.HC};
    float* const wout[4] = {dw.w_q, dw.w_k, dw.w_v, dw.w_g};
    float* const bout[4] = {nullptr, nullptr, nullptr, dw.b_g};
    EVO_TRY(wgrad_segments<T>(c, ws, S.y, s.cin, dqkvg, s.NQ, s.rows, s.cin, 4, woff, wn, wout, bout));
    GemmArgs g;
    g.M = s.rows; g.N = s.cin; g.K = s.NQ;
    g.A = op_rowmajor(dqkvg, s.NQ);
    g.B = op_rowmajor(w_qkvg, s.NQ);
    g.epi = epi_rowmajor(dy, s.cin, true);
    EVO_TRY(gemm<T>(c, g));
  }
  // pair bias
  if (s.row) {
    ProfTag t_("pair_bias");
    // the pair LayerNorm output is recomputed here (the forward projects it without storing it)
    const int64_t P = s.ni * s.ni;
    S.yz = ws.take_n<T>(P * s.cpair);
    S.zmean = ws.take_n<float>(P);
    S.zrstd = ws.take_n<float>(P);
    EVO_TRY((ln_fwd<X, T>(c, pair, P, (int)s.cpair, w.ln_z_g, w.ln_z_b, d.ln_eps, S.yz, S.zmean, S.zrstd)));
    float* dyz = ws.take_n<float>(P * s.cpair);
    EVO_TRY(rowproj_bwd<T>(c, ws, S.yz, P, (int)s.cpair, w.w_bias, s.H, dbias, dyz, false, dw.w_bias));
    float* part = ws.take_n<float>((size_t)ln_bwd_partials(P) * 2 * s.cpair);
    int nb = 0;
    EVO_TRY(ln_bwd<X>(c, pair, S.zmean, S.zrstd, w.ln_z_g, dyz, P, (int)s.cpair, nullptr, true, dpair,
                      part, &nb));
    if (!c.dry) EVO_TRY(reduce_partials2(c, part, nb, (int)s.cpair, dw.ln_z_g, dw.ln_z_b));
  } else if (s.tri) {
    ProfTag t_("pair_bias");
    EVO_TRY(rowproj_bwd<T>(c, ws, S.y, s.rows, (int)s.cin, w.w_bias, s.H, dbias, dy, true, dw.w_bias));
  }
  // input LayerNorm and residual
  float* part = ws.take_n<float>((size_t)ln_bwd_partials(s.rows) * 2 * s.cin);
  int nb = 0;
  EVO_TRY(ln_bwd<X>(c, x, S.mean, S.rstd, w.ln_g, dy, s.rows, (int)s.cin, dres, false, dx, part, &nb));
  if (!c.dry) EVO_TRY(reduce_partials2(c, part, nb, (int)s.cin, dw.ln_g, dw.ln_b));
  return EVO_OK;
}

#define EVO_INST_A(T, X)                                                                           \
  template evo_status_t attn_fwd_op<T, X>(const Ctx&, Arena&, Arena&, const evo_attn_desc_t&,      \
                                          const evo_attn_w_t&, const X*, const X*, const float*, X*, \
                                          const DropSpec*);                                          \
  template evo_status_t attn_bwd_op<T, X>(const Ctx&, Arena&, Arena&, const evo_attn_desc_t&,      \
                                          const evo_attn_w_t&, const X*, const X*, const float*,   \
                                          const X*, X*, X*, const evo_attn_w_t&, const DropSpec*);

EVO_INST_A(float, float)
EVO_INST_A(bf16, bf16)
EVO_INST_A(bf16, float)

}  // namespace evo
