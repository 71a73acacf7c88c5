// Attention core kernels (gfx950): gated self-attention with an additive
// per-head bias shared across the batch axis ("nonbatched_bias") and key masks,
// with an online softmax so that the [batch, H, Lq, Lk] logits never exist in
// memory.  One kernel family serves MSA row, MSA column and both triangle
// attentions through strides.
#pragma once
#include "common.h"

namespace evo {

// Logit given to masked keys (replaces the logit; fully masked rows average uniformly).
constexpr float kMaskLogit = -1e30f;
// The kernels work in the log2 domain: logits and the bias are scaled by log2(e).
constexpr float kLog2e = 1.4426950408889634f;

struct AttnCore {
  // q, k, v, g element (b, p, h, d) at ptr + b*sb + p*sp + h*D + d
  const void* q = nullptr; const void* k = nullptr; const void* v = nullptr; const void* g = nullptr;
  int64_t sb = 0, sp = 0;
  // per-(b, p, h) output rows: o (pre-gate context, FP32: the backward's row sums
  // of the context gradient with it need more than 16-bit precision; null: not
  // kept), go (gated context), stride osb/osp
  void* o = nullptr; void* go = nullptr;
  int64_t osb = 0, osp = 0;
  // log2(e) * bias, at [h*bh + q*bq + k*bk] (FP32), or null
  const float* bias = nullptr; int64_t bh = 0, bq = 0, bk = 0;
  // key mask[b*mb + k*mk] (FP32 0/1) or null
  const float* mask = nullptr; int64_t mb = 0, mk = 0;
  // per-query statistics [(b*stb + q*stq)*H + h]: row max (log2 domain) and 1/rowsum
  float* st_max = nullptr; float* st_inv = nullptr; int64_t stb = 0, stq = 0;
  int H = 0, D = 0;
  int64_t Lq = 0, Lk = 0, nbatch = 0;
  int64_t q_begin = 0, q_count = -1;     // query sub-range (chunked forward); count < 0: all
};

struct AttnGrad {
  // dctx (gradient of the pre-gate context), same addressing as o
  const void* dctx = nullptr;
  const float* Dsum = nullptr;   // [(b*stb + q*stq)*H + h] = sum_d dctx * o
  // outputs: dq, dk, dv with addressing (b, p, h, d) -> ptr + b*dsb + p*dsp + h*D + d
  void* dq = nullptr; void* dk = nullptr; void* dv = nullptr;
  int64_t dsb = 0, dsp = 0;
  // bias-gradient partials [group][H][Lq*Lk] FP32, element (q, k) of a slice at
  // q*dbq + k*dbk (null: no bias gradient); the gradient is with respect to the
  // bias itself, not log2(e) * bias
  float* dbias_part = nullptr;
  int64_t dbq = 0, dbk = 0;
  int64_t group = 1;             // batches summed per partial
  // FP32 only: buffer of the logit gradients dS, keys-major [b][h][k][q] (FP32,
  // attn_bwd_ds_elems elements).  Set: the dK/dV kernel stores dS and dQ and
  // the bias partials are taken from it; null: the dQ kernel recomputes them.
  float* ds = nullptr;
};

template <typename T> evo_status_t attn_fwd(const Ctx& c, const AttnCore& a);
template <typename T> evo_status_t attn_bwd(const Ctx& c, const AttnCore& a, const AttnGrad& g);
template <typename T> int64_t attn_bwd_groups(const AttnCore& a);   // number of bias-gradient partial slices
// Elements of the logit-gradient buffer (AttnGrad::ds) the backward of `a` uses,
// 0 when it recomputes the logits in the dQ kernel instead.
template <typename T> int64_t attn_bwd_ds_elems(const AttnCore& a);

}  // namespace evo
