// Host-side composition of the Evoformer sub-operations from the kernels.
// Every op takes two arenas: `ws` (scratch, reusable after the call) and
// `sv` (tensors the backward needs; may be the scratch arena for inference).
// The same functions run in dry mode to size both.
#pragma once
#include "attn.h"
#include "gemm.h"
#include "misc.h"

namespace evo {

// ---- helpers shared by the ops
// dW[M][N] += X^T dY over `rows` rows; X[row][m] (pitch ldx), dY[row][n] (pitch ldy).
template <typename T>
evo_status_t wgrad(const Ctx& c, Arena& ws, const T* X, int64_t ldx, const T* dY, int64_t ldy,
                   int64_t rows, int64_t M, int64_t N, float* dW);
// out[h][row] = sum_c x[row][c] W[c][h]  (H <= 16), FP32 out.
template <typename T>
evo_status_t rowproj(const Ctx& c, const T* x, int64_t rows, int C, const float* W, int H, float* out);
// dx[row][c] (+)= sum_h dout[h][row] W[c][h]  (FP32);   dW[c][h] += sum_row x[row][c] dout[h][row]
template <typename T>
evo_status_t rowproj_bwd(const Ctx& c, Arena& ws, const T* x, int64_t rows, int C, const float* W,
                         int H, const float* dout, float* dx, bool accumulate, float* dW);
// Column sums of x[rows][ld] restricted to segments, accumulated into outs[i] (+=).
template <typename T>
evo_status_t colsum_segments(const Ctx& c, Arena& ws, const T* x, int64_t rows, int64_t ld,
                             int nseg, const int* seg_off, const int* seg_n, float* const* outs);

inline int ilog2(int64_t v) { int s = 0; while ((1LL << s) < v) ++s; return s; }
inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// ---- ops (T = float or bf16)
template <typename T>
evo_status_t attn_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_attn_desc_t& d,
                         const evo_attn_w_t& w, const T* x, const T* pair, const float* mask, T* out);
template <typename T>
evo_status_t attn_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_attn_desc_t& d,
                         const evo_attn_w_t& w, const T* x, const T* pair, const float* mask,
                         const T* dout, T* dx, T* dpair, const evo_attn_w_t& dw);

template <typename T>
evo_status_t trans_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trans_desc_t& d,
                          const evo_trans_w_t& w, const T* x, T* out);
template <typename T>
evo_status_t trans_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trans_desc_t& d,
                          const evo_trans_w_t& w, const T* x, const T* dout, T* dx,
                          const evo_trans_w_t& dw);

template <typename T>
evo_status_t opm_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_opm_desc_t& d,
                        const evo_opm_w_t& w, const T* m, const float* mask, const T* zin, T* zout);
template <typename T>
evo_status_t opm_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_opm_desc_t& d,
                        const evo_opm_w_t& w, const T* m, const float* mask, const T* dz, T* dm,
                        const evo_opm_w_t& dw);

template <typename T>
evo_status_t trimul_fwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trimul_desc_t& d,
                           const evo_trimul_w_t& w, const T* z, const float* mask, T* zout);
template <typename T>
evo_status_t trimul_bwd_op(const Ctx& c, Arena& ws, Arena& sv, const evo_trimul_desc_t& d,
                           const evo_trimul_w_t& w, const T* z, const float* mask, const T* dzo,
                           T* dz, const evo_trimul_w_t& dw);

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

}  // namespace evo
