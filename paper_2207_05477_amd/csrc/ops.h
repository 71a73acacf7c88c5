// Host-side composition of the Evoformer sub-operations from the kernels.
// Every op takes two arenas: `ws` (scratch, reusable after the call) and
// `sv` (tensors the backward needs; may be the scratch arena for inference).
// The same functions run in dry mode to size both.
#pragma once
#include "attn.h"
#include "gemm.h"
#include "misc.h"

#include <type_traits>

namespace evo {

// ---- helpers shared by the ops
// dW[M][N] += X^T dY over `rows` rows; X[row][m] (pitch ldx), dY[row][n] (pitch ldy);
// with dB (a pointer to one output, itself nullable) also the bias gradient
// dB[0][n] += sum over rows of dY, from the same GEMM.
template <typename T>
evo_status_t wgrad(const Ctx& c, Arena& ws, const T* X, int64_t ldx, const T* dY, int64_t ldy,
                   int64_t rows, int64_t M, int64_t N, float* dW, float* const* dB = nullptr);
// Segments of one weight-gradient GEMM: dW_s[M][n_s] += X^T dY[:, off_s : off_s + n_s]
// for each s (one GEMM over the span of all segments, one segmented reduction),
// and with dB the bias gradients dB_s[n] += column sums of the same dY columns
// (null entries skipped).
template <typename T>
evo_status_t wgrad_segments(const Ctx& c, Arena& ws, const T* X, int64_t ldx, const T* dY, int64_t ldy,
                            int64_t rows, int64_t M, int nseg, const int* seg_off, const int* seg_n,
                            float* const* dW, float* const* dB = nullptr);
// out[h][row] = sum_c x[row][c] W[c][h]  (H <= 16), FP32 out.
template <typename T>
evo_status_t rowproj(const Ctx& c, const T* x, int64_t rows, int C, const float* W, int H, float* out);
// dx[row][c] (+)= sum_h dout[h][row] W[c][h]  (FP32);   dW[c][h] += sum_row x[row][c] dout[h][row]
template <typename T>
evo_status_t rowproj_bwd(const Ctx& c, Arena& ws, const T* x, int64_t rows, int C, const float* W,
                         int H, const float* dout, float* dx, bool accumulate, float* dW);
inline int ilog2(int64_t v) { int s = 0; while ((1LL << s) < v) ++s; return s; }

// Residual-stream type X (x, out, d_out, d_x) may be wider than the compute
// type T (GEMM operands, saved intermediates): FP32 residuals around BF16 compute.
template <typename X> constexpr bool is_f32() { return std::is_same<X, float>::value; }
template <typename X> inline void epi_out(GemmEpilogue& e, X* out, int64_t ld) {
  e.out = out; e.m_lo = ld; e.n_lo = 1; e.out_f32 = is_f32<X>() ? 1 : 0;
}
template <typename X> inline void epi_resid(GemmEpilogue& e, const X* r, int64_t r_m, int64_t r_n) {
  e.resid = r; e.r_m = r_m; e.r_n = r_n; e.resid_f32 = is_f32<X>() ? 1 : 0;
}
// p as a compute-type tensor: itself, or a converted copy in the workspace.
template <typename T, typename X>
inline const T* as_compute(const Ctx& c, Arena& ws, const X* p, int64_t n, evo_status_t* st) {
  *st = EVO_OK;
  if constexpr (std::is_same<T, X>::value) {
    (void)c; (void)ws; (void)n;
    return p;
  } else {
    T* b = ws.take_n<T>(n);
    *st = convert_elems<X, T>(c, p, b, n);
    return b;
  }
}
inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// ---- training dropout of a residual update (dropout.hip)
// Multiplier of update element (row r, channel c): tbl[((r / div) % mod) * C + c]
// (mod = 0: no modulo).  On z rows r = i * R + j: shared along i (a table over
// j) is div = 1, mod = R; shared along j (a table over i) is div = R, mod = 0.
// `on` says whether the op has dropout at all: it holds in the sizing pass too,
// where tbl (carved from a dry arena) is null, so that both passes carve the
// same scratch.
struct DropSpec {
  const float* tbl = nullptr;
  int64_t div = 1, mod = 0;
  bool on = false;
};
// Multiplier tables from Philox4x32-10: table t has len[t] entries drawn at
// counter word word[t] (0 or 1 / (1 - rate[t])); one launch for all tables.
evo_status_t dropout_tables(const Ctx& c, uint64_t seed, uint64_t offset, int n, float* const* out,
                            const int64_t* len, const uint32_t* word, const float* rate);
// dst = src * multiplier (rows x C, C a multiple of 4); dst may alias src.
template <typename X>
evo_status_t dropout_apply(const Ctx& c, const X* src, X* dst, int64_t rows, int C, const DropSpec& d);
inline void epi_dropout(GemmEpilogue& e, const DropSpec* d, int64_t C) {
  if (!d || !d->on) return;
  e.scale = d->tbl; e.sm_shift = 0; e.sm_div = d->div; e.sm_mod = d->mod; e.sm_ld = C;
  e.sn_shift = 0; e.sn_ld = 1;
}

// ---- ops (T = float or bf16; X = residual-stream type, T or float)
// drop: optional training dropout of the op's residual update (attention of
// the MSA rows and both triangle kinds, both triangle multiplications).
template <typename T, typename X = T>
evo_status_t attn_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_attn_desc_t& d,
                         const evo_attn_w_t& w, const X* x, const X* pair, const float* mask, X* out,
                         const DropSpec* drop = nullptr);
template <typename T, typename X = T>
evo_status_t attn_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_attn_desc_t& d,
                         const evo_attn_w_t& w, const X* x, const X* pair, const float* mask,
                         const X* dout, X* dx, X* dpair, const evo_attn_w_t& dw,
                         const DropSpec* drop = nullptr);

template <typename T, typename X = T>
evo_status_t trans_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trans_desc_t& d,
                          const evo_trans_w_t& w, const X* x, X* out);
template <typename T, typename X = T>
evo_status_t trans_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trans_desc_t& d,
                          const evo_trans_w_t& w, const X* x, const X* dout, X* dx,
                          const evo_trans_w_t& dw);

template <typename T, typename X = T>
evo_status_t opm_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_opm_desc_t& d,
                        const evo_opm_w_t& w, const X* m, const float* mask, const X* zin, X* zout);
template <typename T, typename X = T>
evo_status_t opm_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_opm_desc_t& d,
                        const evo_opm_w_t& w, const X* m, const float* mask, const X* dz, X* dm,
                        const evo_opm_w_t& dw);

template <typename T, typename X = T>
evo_status_t trimul_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trimul_desc_t& d,
                           const evo_trimul_w_t& w, const X* z, const float* mask, X* zout,
                           const DropSpec* drop = nullptr);
template <typename T, typename X = T>
evo_status_t trimul_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trimul_desc_t& d,
                           const evo_trimul_w_t& w, const X* z, const float* mask, const X* dzo,
                           X* dz, const evo_trimul_w_t& dw, const DropSpec* drop = nullptr);

// Parameter groups of each op (segments only; see PackArgs in misc.h).
void attn_pack_groups(const evo_attn_desc_t& d, const evo_attn_w_t& w, PackArgs* in, PackArgs* out);
void trans_pack_groups(const evo_trans_desc_t& d, const evo_trans_w_t& w, PackArgs* p1, PackArgs* p2);
void opm_pack_groups(const evo_opm_desc_t& d, const evo_opm_w_t& w, PackArgs* pa, PackArgs* po);
void trimul_pack_groups(const evo_trimul_desc_t& d, const evo_trimul_w_t& w, PackArgs* pp, PackArgs* po);

// ---- argument validation shared by the ABI entry points
evo_status_t check_attn_desc(const evo_attn_desc_t* d);
evo_status_t check_trans_desc(const evo_trans_desc_t* d);
evo_status_t check_opm_desc(const evo_opm_desc_t* d);
evo_status_t check_trimul_desc(const evo_trimul_desc_t* d);
evo_status_t check_block_desc(const evo_block_desc_t* d);

// Sub-op descriptors derived from a block descriptor.
evo_attn_desc_t block_attn_desc(const evo_block_desc_t& b, int kind);
evo_trans_desc_t block_trans_desc(const evo_block_desc_t& b, bool msa);
evo_opm_desc_t block_opm_desc(const evo_block_desc_t& b);
evo_trimul_desc_t block_trimul_desc(const evo_block_desc_t& b, int dir);

template <typename T>
evo_status_t block_fwd_op(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                          const T* m, const T* z, const float* mm, const float* pm, T* mo, T* zo);
template <typename T>
evo_status_t block_bwd_op(const Ctx& c, Arena& ws, const evo_block_desc_t& d, const evo_block_w_t& w,
                          const T* m, const T* z, const float* mm, const float* pm, const T* dmo,
                          const T* dzo, T* dm, T* dz, const evo_block_w_t& dw);
// The block without its checkpoint: a forward that keeps the block's state in
// `saved` (sized by a dry call) and a backward that consumes it instead of
// recomputing the forward.
template <typename T>
evo_status_t block_fwd_save_op(const Ctx& c, Arena& ws, Arena& saved, const evo_block_desc_t& d,
                               const evo_block_w_t& w, const T* m, const T* z, const float* mm, const float* pm,
                               T* mo, T* zo);
template <typename T>
evo_status_t block_bwd_saved_op(const Ctx& c, Arena& ws, Arena& saved, const evo_block_desc_t& d,
                                const evo_block_w_t& w, const T* m, const T* z, const float* mm, const float* pm,
                                const T* dmo, const T* dzo, T* dm, T* dz, const evo_block_w_t& dw);

// Template pair stack block (block.hip).
evo_block_desc_t template_as_block(const evo_template_desc_t& t);
evo_status_t check_template_desc(const evo_template_desc_t* d);
template <typename T>
evo_status_t template_fwd_op(const Ctx& c, Arena& ws, const evo_template_desc_t& d, const evo_template_w_t& w,
                             const T* t, const float* pm, T* to);
template <typename T>
evo_status_t template_bwd_op(const Ctx& c, Arena& ws, const evo_template_desc_t& d, const evo_template_w_t& w,
                             const T* t, const float* pm, const T* dto, T* dt, const evo_template_w_t& dw);

}  // namespace evo
