// Transition, outer product mean and triangle multiplicative update ops.
#include "ops.h"

namespace evo {

// Parameter groups of the pair-stack ops (segments only; callers add the
// destinations).  Transition: W_1 with b_1 as its bias row, W_2.
void trans_pack_groups(const evo_trans_desc_t& d, const evo_trans_w_t& w, PackArgs* p1, PackArgs* p2) {
  const int C = (int)d.c, HID = (int)(d.c * d.factor);
  *p1 = PackArgs(); p1->K = C; p1->seg[0] = {w.w_1, w.b_1, HID}; p1->nseg = 1;
  *p2 = PackArgs(); p2->K = HID; p2->seg[0] = {w.w_2, nullptr, C}; p2->nseg = 1;
}
// Outer product mean: W_a | W_b with their biases, the output projection.
void opm_pack_groups(const evo_opm_desc_t& d, const evo_opm_w_t& w, PackArgs* pa, PackArgs* po) {
  const int ch = (int)d.c_hidden;
  *pa = PackArgs(); pa->K = (int)d.c_m; pa->seg[0] = {w.w_a, w.b_a, ch}; pa->seg[1] = {w.w_b, w.b_b, ch};
  pa->nseg = 2;
  *po = PackArgs(); po->K = ch * ch; po->seg[0] = {w.w_o, nullptr, (int)d.c_z}; po->nseg = 1;
}
// Triangle multiplication: a, b projections and gates with the output gate
// (one GEMM), the output projection.
void trimul_pack_groups(const evo_trimul_desc_t& d, const evo_trimul_w_t& w, PackArgs* pp, PackArgs* po) {
  const int ch = (int)d.c_hidden, cz = (int)d.c_z;
  *pp = PackArgs();
  pp->K = cz;
  pp->seg[0] = {w.w_ap, w.b_ap, ch};
  pp->seg[1] = {w.w_ag, w.b_ag, ch};
  pp->seg[2] = {w.w_bp, w.b_bp, ch};
  pp->seg[3] = {w.w_bg, w.b_bg, ch};
  pp->seg[4] = {w.w_g, w.b_g, cz};
  pp->nseg = 5;
  *po = PackArgs(); po->K = ch; po->seg[0] = {w.w_o, nullptr, cz}; po->nseg = 1;
}

// ============================================================== transition
template <typename T>
static void trans_carve(Arena& a, const evo_trans_desc_t& d, T** y, float** mean, float** rstd, T** h) {
  *y = a.take_n<T>(d.rows * d.c);
  *mean = a.take_n<float>(d.rows);
  *rstd = a.take_n<float>(d.rows);
  *h = a.take_n<T>(d.rows * d.c * d.factor);
}

template <typename T, typename X>
evo_status_t trans_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trans_desc_t& d,
                          const evo_trans_w_t& w, const X* x, X* out) {
  T *y, *h; float *mean, *rstd;
  trans_carve<T>(sv, d, &y, &mean, &rstd, &h);
  const int64_t C = d.c, HID = d.c * d.factor;
  T* wt1 = ws.take_n<T>(HID * C);
  T* wt2 = ws.take_n<T>(C * HID);
  float* b1 = ws.take_n<float>(HID);
  if (c.dry) return EVO_OK;
  PackArgs p1, p2;
  trans_pack_groups(d, w, &p1, &p2);
  p1.dst_t = wt1; p1.bias = b1;
  p2.dst_t = wt2;
  EVO_TRY(pack_params<T>(c, {&p1, &p2}));
  wt1 = (T*)p1.dst_t; b1 = p1.bias;
  wt2 = (T*)p2.dst_t;
  EVO_TRY((ln_fwd<X, T>(c, x, d.rows, (int)C, w.ln_g, w.ln_b, d.ln_eps, y, mean, rstd)));
  {
    GemmArgs g;
    g.M = d.rows; g.N = HID; g.K = C;
    g.A = op_rowmajor(y, C);
    g.B = op_rowmajor(wt1, C);
    g.epi = epi_rowmajor(h, HID, false);
    g.epi.bias = b1;
    g.epi.act = ACT_RELU;
    EVO_TRY(gemm<T>(c, g));
  }
  GemmArgs g;
  g.M = d.rows; g.N = C; g.K = HID;
  g.A = op_rowmajor(h, HID);
  g.B = op_rowmajor(wt2, HID);
  epi_out<X>(g.epi, out, C);
  g.epi.bias = w.b_2;
  epi_resid<X>(g.epi, x, C, 1);
  return gemm<T>(c, g);
}

template <typename T, typename X>
evo_status_t trans_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trans_desc_t& d,
                          const evo_trans_w_t& w, const X* x, const X* dout, X* dx,
                          const evo_trans_w_t& dw) {
  T *y, *h; float *mean, *rstd;
  trans_carve<T>(sv, d, &y, &mean, &rstd, &h);
  evo_status_t cst;
  const T* dout_t = as_compute<T, X>(c, ws, dout, d.rows * d.c, &cst);
  EVO_TRY(cst);
  const int64_t C = d.c, HID = d.c * d.factor;
  T* w1 = ws.take_n<T>(C * HID);     // [C][HID]
  T* w2 = ws.take_n<T>(HID * C);     // [HID][C]
  T* dh = ws.take_n<T>(d.rows * HID);
  float* dy = ws.take_n<float>(d.rows * C);
  if (!c.dry) {
    PackArgs p1, p2;
    trans_pack_groups(d, w, &p1, &p2);
    p1.dst = w1;
    p2.dst = w2;
    EVO_TRY(pack_params<T>(c, {&p1, &p2}));
    w1 = (T*)p1.dst;
    w2 = (T*)p2.dst;
  }
  float* const ob2[1] = {dw.b_2};
  EVO_TRY(wgrad<T>(c, ws, h, HID, dout_t, C, d.rows, HID, C, dw.w_2, ob2));
  {
    GemmArgs g;
    g.M = d.rows; g.N = HID; g.K = C;
    g.A = op_rowmajor(dout_t, C);
    g.B = op_rowmajor(w2, C);
    g.epi = epi_rowmajor(dh, HID, false);
    g.epi.relu_ref = h; g.epi.r_m = HID; g.epi.r_n = 1;
    if (!c.dry) EVO_TRY(gemm<T>(c, g));
  }
  float* const ob1[1] = {dw.b_1};
  EVO_TRY(wgrad<T>(c, ws, y, C, dh, HID, d.rows, C, HID, dw.w_1, ob1));
  {
    GemmArgs g;
    g.M = d.rows; g.N = C; g.K = HID;
    g.A = op_rowmajor(dh, HID);
    g.B = op_rowmajor(w1, HID);
    g.epi = epi_rowmajor(dy, C, true);
    if (!c.dry) EVO_TRY(gemm<T>(c, g));
  }
  float* part = ws.take_n<float>((size_t)ln_bwd_partials(d.rows) * 2 * C);
  int nb = 0;
  EVO_TRY(ln_bwd<X>(c, x, mean, rstd, w.ln_g, dy, d.rows, (int)C, dout, false, dx, part, &nb));
  if (!c.dry) EVO_TRY(reduce_partials2(c, part, nb, (int)C, dw.ln_g, dw.ln_b));
  return EVO_OK;
}

// ============================================================== outer product mean
template <typename T>
struct OpmSaved {
  T* y; float* mean; float* rstd; T* ab; T* on; float* scale;
  void carve(Arena& a, const evo_opm_desc_t& d) {
    const int64_t SR = d.n_seq * d.n_res, RR = d.n_res * d.n_res, ch = d.c_hidden;
    y = a.take_n<T>(SR * d.c_m);
    mean = a.take_n<float>(SR);
    rstd = a.take_n<float>(SR);
    ab = a.take_n<T>(SR * 2 * ch);
    on = a.take_n<T>(RR * ch * ch);
    scale = a.take_n<float>(RR);
  }
};

template <typename T, typename X>
evo_status_t opm_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_opm_desc_t& d,
                        const evo_opm_w_t& w, const X* m, const float* mask, const X* zin, X* zout) {
  OpmSaved<T> S;
  const bool chunked = d.chunk > 0 && d.chunk < d.n_res;
  if (chunked) {
    // no saved state: the outer product exists only for `chunk` rows i at a time
    S.y = ws.take_n<T>(d.n_seq * d.n_res * d.c_m);
    S.mean = ws.take_n<float>(d.n_seq * d.n_res);
    S.rstd = ws.take_n<float>(d.n_seq * d.n_res);
    S.ab = ws.take_n<T>(d.n_seq * d.n_res * 2 * d.c_hidden);
    S.on = ws.take_n<T>(d.chunk * d.n_res * d.c_hidden * d.c_hidden);
    S.scale = ws.take_n<float>(d.n_res * d.n_res);
  } else {
    S.carve(sv, d);
  }
  const int64_t S_ = d.n_seq, R = d.n_res, SR = S_ * R, RR = R * R, ch = d.c_hidden, cm = d.c_m,
                cz = d.c_z, ch2 = ch * ch;
  const int sh = ilog2(ch);
  T* wt_ab = ws.take_n<T>(2 * ch * cm);
  float* b_ab = ws.take_n<float>(2 * ch);
  T* wt_o = ws.take_n<T>(cz * ch2);
  if (c.dry) return EVO_OK;
  PackArgs pa, po;
  opm_pack_groups(d, w, &pa, &po);
  pa.dst_t = wt_ab; pa.bias = b_ab;
  po.dst_t = wt_o;
  EVO_TRY(pack_params<T>(c, {&pa, &po}));
  wt_ab = (T*)pa.dst_t; b_ab = pa.bias;
  wt_o = (T*)po.dst_t;
  EVO_TRY((ln_fwd<X, T>(c, m, SR, (int)cm, w.ln_g, w.ln_b, d.ln_eps, S.y, S.mean, S.rstd)));
  {  // a | b = mask * (y W + b)
    GemmArgs g;
    g.M = SR; g.N = 2 * ch; g.K = cm;
    g.A = op_rowmajor(S.y, cm);
    g.B = op_rowmajor(wt_ab, cm);
    g.epi = epi_rowmajor(S.ab, 2 * ch, false);
    g.epi.bias = b_ab;
    if (mask) { g.epi.scale = mask; g.epi.sm_shift = 0; g.epi.sm_ld = 1; g.epi.sn_shift = 31; g.epi.sn_ld = 0; }
    EVO_TRY(gemm<T>(c, g));
  }
  EVO_TRY(opm_norm(c, mask, S_, R, d.opm_eps, S.scale));
  const int64_t C = chunked ? d.chunk : R;
  for (int64_t i0 = 0; i0 < R; i0 += C) {
    {  // On[i][j][p][q] = sum_s a[s][i][p] b[s][j][q] / (eps + n_ij), rows i of this chunk
      GemmArgs g;
      g.M = C * ch; g.N = R * ch; g.K = S_;
      g.A.ptr = S.ab + i0 * 2 * ch; g.A.r_lo = 1; g.A.r_hi = 2 * ch; g.A.r_shift = sh;
      g.A.k_lo = R * 2 * ch; g.A.k_contig = 0;
      g.B = g.A; g.B.ptr = S.ab + ch;
      g.epi.out = S.on; g.epi.out_f32 = 0;
      g.epi.m_lo = ch; g.epi.m_hi = R * ch2; g.epi.m_shift = sh;
      g.epi.n_lo = 1; g.epi.n_hi = ch2; g.epi.n_shift = sh;
      g.epi.scale = S.scale + i0 * R; g.epi.sm_shift = sh; g.epi.sm_ld = R; g.epi.sn_shift = sh; g.epi.sn_ld = 1;
      EVO_TRY(gemm<T>(c, g));
    }
    GemmArgs g;
    g.M = C * R; g.N = cz; g.K = ch2;
    g.A = op_rowmajor(S.on, ch2);
    g.B = op_rowmajor(wt_o, ch2);
    epi_out<X>(g.epi, zout + i0 * R * cz, cz);
    g.epi.bias = w.b_o;
    epi_resid<X>(g.epi, zin + i0 * R * cz, cz, 1);
    EVO_TRY(gemm<T>(c, g));
  }
  return EVO_OK;
}

template <typename T, typename X>
evo_status_t opm_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_opm_desc_t& d,
                        const evo_opm_w_t& w, const X* m, const float* mask, const X* dz_x, X* dm,
                        const evo_opm_w_t& dw) {
  OpmSaved<T> S;
  S.carve(sv, d);
  evo_status_t cst;
  const T* dz = as_compute<T, X>(c, ws, dz_x, d.n_res * d.n_res * d.c_z, &cst);
  EVO_TRY(cst);
  const int64_t S_ = d.n_seq, R = d.n_res, SR = S_ * R, RR = R * R, ch = d.c_hidden, cm = d.c_m,
                cz = d.c_z, ch2 = ch * ch;
  const int sh = ilog2(ch);
  T* w_ab = ws.take_n<T>(cm * 2 * ch);   // [cm][2ch]
  T* w_o = ws.take_n<T>(ch2 * cz);       // [ch2][cz]
  T* dO = ws.take_n<T>(RR * ch2);
  T* dab = ws.take_n<T>(SR * 2 * ch);
  float* dy = ws.take_n<float>(SR * cm);
  // da and db have only S_ rows: 128 x 128 tiles split OPM_SPLIT ways along
  // their R * ch reduction (FP32 partials), summed with the mask in one pass
  constexpr int OPM_SPLIT = 4;
  float* dpart = ws.take_n<float>((size_t)OPM_SPLIT * SR * ch);
  if (!c.dry) {
    PackArgs pa, po;
    opm_pack_groups(d, w, &pa, &po);
    pa.dst = w_ab;
    po.dst = w_o;
    EVO_TRY(pack_params<T>(c, {&pa, &po}));
    w_ab = (T*)pa.dst;
    w_o = (T*)po.dst;
  }
  float* const obo[1] = {dw.b_o};
  EVO_TRY(wgrad<T>(c, ws, S.on, ch2, dz, cz, RR, ch2, cz, dw.w_o, obo));
  if (!c.dry) {
    {  // dO = (dz W_o^T) / (eps + n_ij)
      GemmArgs g;
      g.M = RR; g.N = ch2; g.K = cz;
      g.A = op_rowmajor(dz, cz);
      g.B = op_rowmajor(w_o, cz);
      g.epi = epi_rowmajor(dO, ch2, false);
      g.epi.scale = S.scale; g.epi.sm_shift = 0; g.epi.sm_ld = 1; g.epi.sn_shift = 31; g.epi.sn_ld = 0;
      EVO_TRY(gemm<T>(c, g));
    }
    // da and db as [s][(i, p)] products (rows s, columns (i, p) contiguous within
    // blocks of ch), so that the partials move as row vectors.
    {  // da[s][i][p] = mask_si * sum_{j,q} b[s][j][q] dO[i][j][p][q]
      GemmArgs g;
      g.M = S_; g.N = R * ch; g.K = R * ch;
      g.split_k = OPM_SPLIT; g.big_tiles = 1;
      g.A.ptr = S.ab + ch; g.A.r_lo = R * 2 * ch;
      g.A.k_lo = 1; g.A.k_hi = 2 * ch; g.A.k_shift = sh; g.A.k_contig = 1;
      g.B.ptr = dO; g.B.r_lo = ch; g.B.r_hi = R * ch2; g.B.r_shift = sh;
      g.B.k_lo = 1; g.B.k_hi = ch2; g.B.k_shift = sh; g.B.k_contig = 1;
      g.epi = epi_rowmajor(dpart, R * ch, true);
      g.epi.batch = SR * ch;
      EVO_TRY(gemm<T>(c, g));
      EVO_TRY(opm_dab_reduce<T>(c, dpart, OPM_SPLIT, S_, R, (int)ch, mask, dab, 0));
    }
    {  // db[s][j][q] = mask_sj * sum_{i,p} a[s][i][p] dO[i][j][p][q]
      GemmArgs g;
      g.M = S_; g.N = R * ch; g.K = R * ch;
      g.split_k = OPM_SPLIT; g.big_tiles = 1;
      g.A.ptr = S.ab; g.A.r_lo = R * 2 * ch;
      g.A.k_lo = 1; g.A.k_hi = 2 * ch; g.A.k_shift = sh; g.A.k_contig = 1;
      g.B.ptr = dO; g.B.r_lo = 1; g.B.r_hi = ch2; g.B.r_shift = sh;
      g.B.k_lo = ch; g.B.k_hi = R * ch2; g.B.k_shift = sh; g.B.k_contig = 0;
      g.epi = epi_rowmajor(dpart, R * ch, true);
      g.epi.batch = SR * ch;
      EVO_TRY(gemm<T>(c, g));
      EVO_TRY(opm_dab_reduce<T>(c, dpart, OPM_SPLIT, S_, R, (int)ch, mask, dab, (int)ch));
    }
  }
  {
    const int woff[2] = {0, (int)ch}, wn[2] = {(int)ch, (int)ch};
    float* const wout[2] = {dw.w_a, dw.w_b};
    float* const bout[2] = {dw.b_a, dw.b_b};
    EVO_TRY(wgrad_segments<T>(c, ws, S.y, cm, dab, 2 * ch, SR, cm, 2, woff, wn, wout, bout));
  }
  if (!c.dry) {
    GemmArgs g;
    g.M = SR; g.N = cm; g.K = 2 * ch;
    g.A = op_rowmajor(dab, 2 * ch);
    g.B = op_rowmajor(w_ab, 2 * ch);
    g.epi = epi_rowmajor(dy, cm, true);
    EVO_TRY(gemm<T>(c, g));
  }
  float* part = ws.take_n<float>((size_t)ln_bwd_partials(SR) * 2 * cm);
  int nb = 0;
  EVO_TRY(ln_bwd<X>(c, m, S.mean, S.rstd, w.ln_g, dy, SR, (int)cm, nullptr, true, dm, part, &nb));
  if (!c.dry) EVO_TRY(reduce_partials2(c, part, nb, (int)cm, dw.ln_g, dw.ln_b));
  return EVO_OK;
}

// ============================================================== triangle multiplication
template <typename T>
struct TriSaved {
  // raw: projection output in the compute type (its last cz columns hold the
  // output gate after the sigmoid); x (contraction output, channel-major) feeds
  // only the output LayerNorm, in the compute type like its operands.
  T* y; float* mean; float* rstd; T* raw; T* a; T* b; T* x; T* xn; float* mean2;
  float* rstd2;
  void carve(Arena& ar, const evo_trimul_desc_t& d) {
    const int64_t P = d.n_res * d.n_res, ch = d.c_hidden, cz = d.c_z;
    y = ar.take_n<T>(P * cz);
    mean = ar.take_n<float>(P);
    rstd = ar.take_n<float>(P);
    raw = ar.take_n<T>(P * (4 * ch + cz));
    a = ar.take_n<T>(P * ch);
    b = ar.take_n<T>(P * ch);
    x = ar.take_n<T>(P * ch);
    xn = ar.take_n<T>(P * ch);
    mean2 = ar.take_n<float>(P);
    rstd2 = ar.take_n<float>(P);
  }
};

// Forward in chunks of `chunk` output rows i, keeping no saved state: the
// projections run over row chunks into the full channel-major a, b and the
// gate g; contraction, output LayerNorm and output projection then run per
// chunk of output rows (x_ij for i in the chunk needs a's rows i and all of b).
template <typename T, typename X>
static evo_status_t trimul_fwd_chunked(const Ctx& c, Arena& ws, const evo_trimul_desc_t& d,
                                       const evo_trimul_w_t& w, const X* z, const float* mask, X* zout) {
  const int64_t R = d.n_res, P = R * R, ch = d.c_hidden, cz = d.c_z, NP = 4 * ch + cz, C = d.chunk,
                CR = C * R;
  T* wt_p = ws.take_n<T>(NP * cz);
  float* b_p = ws.take_n<float>(NP);
  T* wt_o = ws.take_n<T>(cz * ch);
  T* a = ws.take_n<T>(P * ch);
  T* b = ws.take_n<T>(P * ch);
  float* g = ws.take_n<float>(P * cz);
  T* y = ws.take_n<T>(CR * cz);
  float* mean = ws.take_n<float>(CR);
  float* rstd = ws.take_n<float>(CR);
  T* raw = ws.take_n<T>(CR * NP);
  T* x = ws.take_n<T>(CR * ch);
  T* xn = ws.take_n<T>(CR * ch);
  if (c.dry) return EVO_OK;
  PackArgs pp, po;
  trimul_pack_groups(d, w, &pp, &po);
  pp.dst_t = wt_p;
  pp.bias = b_p;
  po.dst_t = wt_o;
  EVO_TRY(pack_params<T>(c, {&pp, &po}));
  wt_p = (T*)pp.dst_t;
  b_p = pp.bias;
  wt_o = (T*)po.dst_t;
  for (int64_t c0 = 0; c0 < R; c0 += C) {
    const int64_t p0 = c0 * R;
    EVO_TRY((ln_fwd<X, T>(c, z + p0 * cz, CR, (int)cz, w.ln_g, w.ln_b, d.ln_eps, y, mean, rstd)));
    GemmArgs gp;
    gp.M = CR; gp.N = NP; gp.K = cz;
    gp.A = op_rowmajor(y, cz);
    gp.B = op_rowmajor(wt_p, cz);
    gp.epi = epi_rowmajor(raw, NP, false);
    gp.epi.bias = b_p;
    gp.epi.act = ACT_SIGMOID;   // output gate columns, as in the unchunked forward
    gp.epi.act_n0 = 4 * ch;
    EVO_TRY(gemm<T>(c, gp));
    EVO_TRY(trimul_proj<T>(c, CR, (int)ch, (int)cz, raw, mask ? mask + p0 : nullptr, a + p0, b + p0, P,
                           g + p0 * cz));   // (raw is per chunk: the gate is copied apart)
  }
  float* mean2 = mean;
  float* rstd2 = rstd;
  for (int64_t c0 = 0; c0 < R; c0 += C) {
    const int64_t p0 = c0 * R;
    GemmArgs gx;
    gx.M = C; gx.N = R; gx.K = R; gx.batch = (int)ch;
    if (d.dir == EVO_TRI_OUT) {
      gx.A = op_rowmajor(a + c0 * R, R);
      gx.B = op_rowmajor(b, R);
    } else {
      gx.A = op_colmajor(a + c0, R);
      gx.B = op_colmajor(b, R);
    }
    gx.A.batch = P; gx.B.batch = P;
    gx.epi = epi_rowmajor(x, R, false);
    gx.epi.batch = CR;
    EVO_TRY(gemm<T>(c, gx));
    EVO_TRY(ln_fwd_cm<T>(c, x, CR, (int)ch, w.ln_out_g, w.ln_out_b, d.ln_eps, xn, mean2, rstd2));
    GemmArgs go;
    go.M = CR; go.N = cz; go.K = ch;
    go.A = op_rowmajor(xn, ch);
    go.B = op_rowmajor(wt_o, ch);
    epi_out<X>(go.epi, zout + p0 * cz, cz);
    go.epi.bias = w.b_o;
    go.epi.gate = g + p0 * cz; go.epi.g_m = cz; go.epi.g_n = 1; go.epi.gate_f32 = 1;
    epi_resid<X>(go.epi, z + p0 * cz, cz, 1);
    EVO_TRY(gemm<T>(c, go));
  }
  return EVO_OK;
}

template <typename T, typename X>
evo_status_t trimul_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trimul_desc_t& d,
                           const evo_trimul_w_t& w, const X* z, const float* mask, X* zout,
                           const DropSpec* drop) {
  if (d.chunk > 0 && d.chunk < d.n_res) {
    if (drop && drop->on) {
      set_error("triangle multiplication: the chunked forward has no dropout");
      return EVO_EINVAL;
    }
    return trimul_fwd_chunked<T, X>(c, ws, d, w, z, mask, zout);
  }
  TriSaved<T> S;
  S.carve(sv, d);
  const int64_t R = d.n_res, P = R * R, ch = d.c_hidden, cz = d.c_z, NP = 4 * ch + cz;
  T* wt_p = ws.take_n<T>(NP * cz);
  float* b_p = ws.take_n<float>(NP);
  T* wt_o = ws.take_n<T>(cz * ch);
  if (c.dry) return EVO_OK;
  PackArgs pp, po;
  trimul_pack_groups(d, w, &pp, &po);
  pp.dst_t = wt_p;
  pp.bias = b_p;
  po.dst_t = wt_o;
  EVO_TRY(pack_params<T>(c, {&pp, &po}));
  wt_p = (T*)pp.dst_t;
  b_p = pp.bias;
  wt_o = (T*)po.dst_t;
  EVO_TRY((ln_fwd<X, T>(c, z, P, (int)cz, w.ln_g, w.ln_b, d.ln_eps, S.y, S.mean, S.rstd)));
  {
    GemmArgs g;
    g.M = P; g.N = NP; g.K = cz;
    g.A = op_rowmajor(S.y, cz);
    g.B = op_rowmajor(wt_p, cz);
    g.epi = epi_rowmajor(S.raw, NP, false);
    g.epi.bias = b_p;
    g.epi.act = ACT_SIGMOID;   // output gate columns: sigmoid in the epilogue
    g.epi.act_n0 = 4 * ch;
    EVO_TRY(gemm<T>(c, g));
  }
  EVO_TRY(trimul_proj<T>(c, P, (int)ch, (int)cz, S.raw, mask, S.a, S.b, P, nullptr));
  {  // per-channel contraction, channel-major operands [ch][R][R]
    ProfTag t_("contract");
    GemmArgs g;
    g.M = R; g.N = R; g.K = R; g.batch = (int)ch;
    if (d.dir == EVO_TRI_OUT) {   // X_c = A_c B_c^T
      g.A = op_rowmajor(S.a, R);
      g.B = op_rowmajor(S.b, R);
    } else {                      // X_c = A_c^T B_c
      g.A = op_colmajor(S.a, R);
      g.B = op_colmajor(S.b, R);
    }
    g.A.batch = P; g.B.batch = P;
    g.epi = epi_rowmajor(S.x, R, false);
    g.epi.batch = P;
    EVO_TRY(gemm<T>(c, g));
  }
  EVO_TRY(ln_fwd_cm<T>(c, S.x, P, (int)ch, w.ln_out_g, w.ln_out_b, d.ln_eps, S.xn, S.mean2, S.rstd2));
  GemmArgs g;
  g.M = P; g.N = cz; g.K = ch;
  g.A = op_rowmajor(S.xn, ch);
  g.B = op_rowmajor(wt_o, ch);
  epi_out<X>(g.epi, zout, cz);
  g.epi.bias = w.b_o;
  g.epi.gate = S.raw + 4 * ch; g.epi.g_m = NP; g.epi.g_n = 1; g.epi.gate_f32 = 0;
  epi_dropout(g.epi, drop, cz);
  epi_resid<X>(g.epi, z, cz, 1);
  return gemm<T>(c, g);
}

template <typename T, typename X>
evo_status_t trimul_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trimul_desc_t& d,
                           const evo_trimul_w_t& w, const X* z, const float* mask, const X* dzo,
                           X* dz, const evo_trimul_w_t& dw, const DropSpec* drop) {
  TriSaved<T> S;
  S.carve(sv, d);
  const int64_t R = d.n_res, P = R * R, ch = d.c_hidden, cz = d.c_z, NP = 4 * ch + cz;
  // with dropout the update's gradient is drop * dzo; the residual passes dzo on
  const X* dres = dzo;
  if (drop && drop->on) {
    X* dd = ws.take_n<X>(P * cz);
    EVO_TRY(dropout_apply<X>(c, dzo, dd, P, (int)cz, *drop));
    dzo = dd;
  }
  T* w_p = ws.take_n<T>(cz * NP);      // [cz][NP]
  T* wt_o = ws.take_n<T>(cz * ch);     // [cz][ch]
  T* w_o = ws.take_n<T>(ch * cz);      // [ch][cz]
  float* t = ws.take_n<float>(P * cz);
  T* dt = ws.take_n<T>(P * cz);
  T* draw = ws.take_n<T>(P * NP);
  float* dxn = ws.take_n<float>(P * ch);
  T* dx = ws.take_n<T>(P * ch);
  float* da = ws.take_n<float>(P * ch);
  float* db = ws.take_n<float>(P * ch);
  float* dy = ws.take_n<float>(P * cz);
  if (!c.dry) {
    PackArgs pp, po;
    trimul_pack_groups(d, w, &pp, &po);
    pp.dst = w_p;
    po.dst_t = wt_o;
    po.dst = w_o;
    EVO_TRY(pack_params<T>(c, {&pp, &po}));
    w_p = (T*)pp.dst;
    wt_o = (T*)po.dst_t;
    w_o = (T*)po.dst;
    {  // t = LN_out(x) W_o + b_o
      GemmArgs g;
      g.M = P; g.N = cz; g.K = ch;
      g.A = op_rowmajor(S.xn, ch);
      g.B = op_rowmajor(wt_o, ch);
      g.epi = epi_rowmajor(t, cz, true);
      g.epi.bias = w.b_o;
      EVO_TRY(gemm<T>(c, g));
    }
    EVO_TRY((trimul_gate_bwd<T, X>(c, P, (int)ch, (int)cz, dzo, t, S.raw + 4 * ch, NP, dt, draw)));
  }
  float* const obo[1] = {dw.b_o};
  EVO_TRY(wgrad<T>(c, ws, S.xn, ch, dt, cz, P, ch, cz, dw.w_o, obo));
  if (!c.dry) {
    GemmArgs g;
    g.M = P; g.N = ch; g.K = cz;
    g.A = op_rowmajor(dt, cz);
    g.B = op_rowmajor(w_o, cz);
    g.epi = epi_rowmajor(dxn, ch, true);
    EVO_TRY(gemm<T>(c, g));
  }
  {
    float* part = ws.take_n<float>((size_t)ln_bwd_cm_partials(P) * 2 * ch);
    int nb = 0;
    EVO_TRY(ln_bwd_cm<T>(c, S.x, S.mean2, S.rstd2, w.ln_out_g, dxn, P, (int)ch, dx, part, &nb));
    if (!c.dry) EVO_TRY(reduce_partials2(c, part, nb, (int)ch, dw.ln_out_g, dw.ln_out_b));
  }
  if (!c.dry) {
    ProfTag t_("contract");
    GemmArgs g;
    g.M = R; g.N = R; g.K = R; g.batch = (int)ch;
    if (d.dir == EVO_TRI_OUT) {
      // da_c[i][k] = sum_j dx_c[i][j] b_c[j][k]
      g.A = op_rowmajor(dx, R);
      g.B = op_colmajor(S.b, R);
      g.A.batch = P; g.B.batch = P;
      g.epi = epi_rowmajor(da, R, true); g.epi.batch = P;
      EVO_TRY(gemm<T>(c, g));
      // db_c[j][k] = sum_i dx_c[i][j] a_c[i][k]
      g.A = op_colmajor(dx, R);
      g.B = op_colmajor(S.a, R);
      g.A.batch = P; g.B.batch = P;
      g.epi = epi_rowmajor(db, R, true); g.epi.batch = P;
      EVO_TRY(gemm<T>(c, g));
    } else {
      // da_c[k][i] = sum_j b_c[k][j] dx_c[i][j]
      g.A = op_rowmajor(S.b, R);
      g.B = op_rowmajor(dx, R);
      g.A.batch = P; g.B.batch = P;
      g.epi = epi_rowmajor(da, R, true); g.epi.batch = P;
      EVO_TRY(gemm<T>(c, g));
      // db_c[k][j] = sum_i a_c[k][i] dx_c[i][j]
      g.A = op_rowmajor(S.a, R);
      g.B = op_colmajor(dx, R);
      g.A.batch = P; g.B.batch = P;
      g.epi = epi_rowmajor(db, R, true); g.epi.batch = P;
      EVO_TRY(gemm<T>(c, g));
    }
    EVO_TRY(trimul_proj_bwd<T>(c, P, (int)ch, (int)cz, S.raw, mask, da, db, draw));
  }
  int offs[5] = {0, (int)ch, (int)(2 * ch), (int)(3 * ch), (int)(4 * ch)};
  int ns[5] = {(int)ch, (int)ch, (int)ch, (int)ch, (int)cz};
  float* const obp[5] = {dw.b_ap, dw.b_ag, dw.b_bp, dw.b_bg, dw.b_g};
  float* owp[5] = {dw.w_ap, dw.w_ag, dw.w_bp, dw.w_bg, dw.w_g};
  {
    ProfTag t_("wgrad_proj");
    EVO_TRY(wgrad_segments<T>(c, ws, S.y, cz, draw, NP, P, cz, 5, offs, ns, owp, obp));
  }
  if (!c.dry) {
    GemmArgs g;
    g.M = P; g.N = cz; g.K = NP;
    g.A = op_rowmajor(draw, NP);
    g.B = op_rowmajor(w_p, NP);
    g.epi = epi_rowmajor(dy, cz, true);
    EVO_TRY(gemm<T>(c, g));
  }
  float* part = ws.take_n<float>((size_t)ln_bwd_partials(P) * 2 * cz);
  int nb = 0;
  EVO_TRY(ln_bwd<X>(c, z, S.mean, S.rstd, w.ln_g, dy, P, (int)cz, dres, false, dz, part, &nb));
  if (!c.dry) EVO_TRY(reduce_partials2(c, part, nb, (int)cz, dw.ln_g, dw.ln_b));
  return EVO_OK;
}

#define EVO_INST_P(T, X)                                                                           \
  template evo_status_t trans_fwd_op<T, X>(const Ctx&, Arena&, Arena&, const evo_trans_desc_t&,    \
                                           const evo_trans_w_t&, const X*, X*);                    \
  template evo_status_t trans_bwd_op<T, X>(const Ctx&, Arena&, Arena&, const evo_trans_desc_t&,    \
                                           const evo_trans_w_t&, const X*, const X*, X*,           \
                                           const evo_trans_w_t&);                                  \
  template evo_status_t opm_fwd_op<T, X>(const Ctx&, Arena&, Arena&, const evo_opm_desc_t&,        \
                                         const evo_opm_w_t&, const X*, const float*, const X*, X*); \
  template evo_status_t opm_bwd_op<T, X>(const Ctx&, Arena&, Arena&, const evo_opm_desc_t&,        \
                                         const evo_opm_w_t&, const X*, const float*, const X*, X*, \
                                         const evo_opm_w_t&);                                      \
  template evo_status_t trimul_fwd_op<T, X>(const Ctx&, Arena&, Arena&, const evo_trimul_desc_t&,  \
                                            const evo_trimul_w_t&, const X*, const float*, X*,     \
                                            const DropSpec*);                                      \
  template evo_status_t trimul_bwd_op<T, X>(const Ctx&, Arena&, Arena&, const evo_trimul_desc_t&,  \
                                            const evo_trimul_w_t&, const X*, const float*,         \
                                            const X*, X*, const evo_trimul_w_t&, const DropSpec*);

EVO_INST_P(float, float)
EVO_INST_P(bf16, bf16)
EVO_INST_P(bf16, float)

}  // namespace evo
