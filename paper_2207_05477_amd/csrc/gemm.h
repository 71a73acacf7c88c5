// Generic MFMA GEMM for the Evoformer block: C[m, n] = sum_k A[m, k] B[k, n].
//
// Operands are addressed through two-level strides so that the projections,
// their transposed (weight-gradient) forms, the per-channel triangle
// contraction and the outer-product-mean products run on one kernel without
// layout copies:  offset(r) = (r >> shift) * hi + (r & (2^shift - 1)) * lo,
// or r * lo when shift < 0.  Each operand is contiguous either along k
// (vector loads along k) or along its row index (vector loads along rows,
// transposed into LDS).
#pragma once
#include "common.h"

namespace evo {

struct GemmOperand {
  const void* ptr = nullptr;
  int64_t batch = 0;          // elements between batches (blockIdx.z)
  int64_t r_lo = 0, r_hi = 0;  // row (m for A, n for B) addressing
  int32_t r_shift = -1;
  int64_t k_lo = 0, k_hi = 0;  // reduction-index addressing
  int32_t k_shift = -1;
  int32_t k_contig = 1;       // 1: k_lo == 1; 0: r_lo == 1
};

enum { ACT_NONE = 0, ACT_RELU = 1, ACT_SIGMOID = 2 };

// Epilogue, applied per output element in this order:
//   v = alpha * acc;  v += bias[n];  v *= scale[...];  v = act(v) (n >= act_n0);
//   v = relu_ref > 0 ? v : 0;  v *= gate;  v += resid;  out (+)= v
struct GemmEpilogue {
  void* out = nullptr;
  int64_t batch = 0;                   // elements between batches / split-K slices
  int64_t m_lo = 0, m_hi = 0; int32_t m_shift = -1;
  int64_t n_lo = 1, n_hi = 0; int32_t n_shift = -1;
  int32_t out_f32 = 0;                 // 1: out is FP32, 0: out is the kernel type
  int32_t accumulate = 0;              // out += v (FP32 out only)
  float alpha = 1.0f;
  const float* bias = nullptr;         // [N]
  int32_t act = ACT_NONE;
  int32_t act_n0 = 0;
  const float* scale = nullptr;        // scale[srow(m) * sm_ld + (n >> sn_shift) * sn_ld],
  int32_t sm_shift = 0, sn_shift = 0;  // srow(m) = ((m >> sm_shift) / sm_div) % sm_mod
  int64_t sm_ld = 0, sn_ld = 0;        // (sm_mod = 0: no modulo)
  int64_t sm_div = 1, sm_mod = 0;
  const void* relu_ref = nullptr;      // kernel type, addressed like resid
  const void* gate = nullptr;          // kernel type (FP32 if gate_f32), gate[m * g_m + n * g_n]
  int64_t g_m = 0, g_n = 0;
  int32_t gate_f32 = 0;
  const void* resid = nullptr;         // kernel type (FP32 if resid_f32), resid[m * r_m + n * r_n]
                                       // (r_m < 0 / g_m < 0: addressed like the output)
  int64_t r_m = 0, r_n = 0;
  int32_t resid_f32 = 0;
};

// Row index of the epilogue scale table (32-bit: output rows stay below 2^31).
EVO_DEV int64_t scale_row(const GemmEpilogue& e, int64_t m) {
  uint32_t q = (uint32_t)(m >> e.sm_shift);
  if (e.sm_div > 1) q /= (uint32_t)e.sm_div;
  if (e.sm_mod > 0) q %= (uint32_t)e.sm_mod;
  return (int64_t)q;
}

struct GemmArgs {
  int64_t M = 0, N = 0, K = 0;
  int32_t batch = 1;       // independent problems (blockIdx.z)
  int32_t split_k = 1;     // > 1: blockIdx.z splits K, partial results to out + z * epi.batch
  int32_t big_tiles = 0;   // 1: 128 x 128 tiles whatever M x N (split-K problems with few tiles)
  GemmOperand A, B;        // A rows = m, B rows = n
  GemmEpilogue epi;
  // Optional: column sums of B over the reduction, colsum[z * N + n] =
  // sum_k B[n][k] over slice z's k range (split-K) or problem z's (batch),
  // FP32.  Plain operand layouts with B row-contiguous (not along k) only.
  float* colsum = nullptr;
};

template <typename T>
evo_status_t gemm(const Ctx& ctx, const GemmArgs& g);

// ---- convenience builders (dense row-major matrices)
// A = X[m, k] with row stride ld (k contiguous)
inline GemmOperand op_rowmajor(const void* p, int64_t ld) {
  GemmOperand o; o.ptr = p; o.r_lo = ld; o.k_lo = 1; o.k_contig = 1; return o;
}
// A = X^T where X is [k, m] with row stride ld (m contiguous)
inline GemmOperand op_colmajor(const void* p, int64_t ld) {
  GemmOperand o; o.ptr = p; o.r_lo = 1; o.k_lo = ld; o.k_contig = 0; return o;
}
inline GemmEpilogue epi_rowmajor(void* out, int64_t ld, bool f32) {
  GemmEpilogue e; e.out = out; e.m_lo = ld; e.n_lo = 1; e.out_f32 = f32 ? 1 : 0; return e;
}

}  // namespace evo
