// Global column attention of the extra-MSA stack (gfx950).
//
// Per residue column i: one query per head, the masked mean over MSA rows of
// q; single-head keys and values shared by all heads; softmax over the rows t;
// the context is broadcast back to every row through the per-row gate.  The
// work per column is tiny (H x S logits), so one workgroup owns one column and
// keeps logits, probabilities and their gradients in LDS.
// q | k | v | g live in one projection buffer [S*R][2*H*D + 2*D].
#include "ops.h"

namespace evo {

constexpr int GA_THREADS = 256;

EVO_DEV float block_reduce(float v, float* red, bool is_max) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = is_max ? wave_max(v) : wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  float r = red[0];
  for (int w = 1; w < GA_THREADS / 64; ++w) r = is_max ? fmaxf(r, red[w]) : r + red[w];
  return r;
}

// logits[h][t] (masked, scaled) and qbar[h*D + d] for column i; returns in LDS.
template <typename T>
EVO_DEV void gattn_logits(int64_t S, int64_t R, int H, int D, const T* qkvg, const float* mask, float eps,
                          int64_t i, float* qbar, float* logit, float* red) {
  const int HC = H * D, NQ = 2 * HC + 2 * D;
  float msum = 0.f;
  for (int64_t s = threadIdx.x; s < S; s += GA_THREADS) msum += mask ? mask[s * R + i] : 1.f;
  msum = block_reduce(msum, red, false);
  for (int e = threadIdx.x; e < HC; e += GA_THREADS) {
    float acc = 0.f;
    for (int64_t s = 0; s < S; ++s) {
      const float mk = mask ? mask[s * R + i] : 1.f;
      acc += mk * to_f32(qkvg[(s * R + i) * NQ + e]);
    }
    qbar[e] = acc / (msum + eps);
  }
  __syncthreads();
  const float sc = 1.0f / sqrtf((float)D);
  for (int64_t e = threadIdx.x; e < (int64_t)H * S; e += GA_THREADS) {
    const int h = (int)(e / S);
    const int64_t t = e % S;
    const T* kr = qkvg + (t * R + i) * NQ + HC;
    float acc = 0.f;
    for (int d = 0; d < D; ++d) acc += qbar[h * D + d] * to_f32(kr[d]);
    float x = acc * sc;
    if (mask && mask[t * R + i] == 0.f) x = -1e30f;
    logit[h * S + t] = x;
  }
  __syncthreads();
}

// In-place softmax over t of each head's logits.
EVO_DEV void gattn_softmax(int64_t S, int H, float* logit, float* red, float* smax, float* sinv) {
  for (int h = 0; h < H; ++h) {
    float* l = logit + h * S;
    float mx = -INFINITY;
    for (int64_t t = threadIdx.x; t < S; t += GA_THREADS) mx = fmaxf(mx, l[t]);
    mx = block_reduce(mx, red, true);
    float sm = 0.f;
    for (int64_t t = threadIdx.x; t < S; t += GA_THREADS) sm += __expf(l[t] - mx);
    sm = block_reduce(sm, red, false);
    const float inv = 1.0f / sm;
    for (int64_t t = threadIdx.x; t < S; t += GA_THREADS) l[t] = __expf(l[t] - mx) * inv;
    if (threadIdx.x == 0 && smax) { smax[h] = mx; sinv[h] = inv; }
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(GA_THREADS) void gattn_fwd_kernel(int64_t S, int64_t R, int H, int D,
                                                               const T* qkvg, const float* mask, float eps,
                                                               float* gctx, float* smax, float* sinv) {
  extern __shared__ float sm[];
  float* red = sm;                 // [4]
  float* qbar = sm + 8;            // [HC]
  float* logit = qbar + H * D;     // [H][S]
  const int64_t i = blockIdx.x;
  const int HC = H * D, NQ = 2 * HC + 2 * D;
  gattn_logits<T>(S, R, H, D, qkvg, mask, eps, i, qbar, logit, red);
  gattn_softmax(S, H, logit, red, smax + i * H, sinv + i * H);
  for (int e = threadIdx.x; e < HC; e += GA_THREADS) {
    const int h = e / D, d = e % D;
    float acc = 0.f;
    for (int64_t t = 0; t < S; ++t) acc += logit[h * S + t] * to_f32(qkvg[(t * R + i) * NQ + HC + D + d]);
    gctx[i * HC + e] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gattn_gate_kernel(int64_t S, int64_t R, int H, int D, const T* qkvg,
                                                         const float* gctx, T* go) {
  const int HC = H * D, NQ = 2 * HC + 2 * D;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= S * R * HC) return;
  const int64_t row = e / HC;
  const int c = (int)(e % HC);
  const int64_t i = row % R;
  go[e] = from_f32<T>(to_f32(qkvg[row * NQ + HC + 2 * D + c]) * gctx[i * HC + c]);
}

template <typename T>
evo_status_t gattn_fwd(const Ctx& c, int64_t S, int64_t R, int H, int D, const T* qkvg, const float* mask,
                       float eps, float* gctx, float* smax, float* sinv, T* go) {
  if (c.dry) return EVO_OK;
  const size_t lds = (8 + (size_t)H * D + (size_t)H * S) * sizeof(float);
  if (lds > 150 * 1024) { set_error("global attention: %lld rows exceed LDS", (long long)S); return EVO_ESHAPE; }
  EVO_LAUNCH(EVO_KNAME("gattn_fwd_kernel", T), 4.0 * (double)S * R * H * D, (double)S * R * (2 * H * D + 2 * D) * sizeof(T), (gattn_fwd_kernel<T>), dim3((unsigned)R), dim3(GA_THREADS), lds, c.stream, S, R, H, D,
                     qkvg, mask, eps, gctx, smax, sinv);
  EVO_TRY(check_launch("gattn_fwd"));
  const int64_t n = S * R * H * D;
  EVO_LAUNCH(EVO_KNAME("gattn_gate_kernel", T), 0.0, (double)n * 2 * sizeof(T), (gattn_gate_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, S, R,
                     H, D, qkvg, gctx, go);
  return check_launch("gattn_gate");
}

// dg (pre-sigmoid) for every row; dctx[i][h][d] = sum_s dgo * g.
template <typename T>
__global__ __launch_bounds__(256) void gattn_gate_bwd_kernel(int64_t S, int64_t R, int H, int D, const T* qkvg,
                                                             const float* gctx, const float* dgo, T* dqkvg) {
  const int HC = H * D, NQ = 2 * HC + 2 * D;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= S * R * HC) return;
  const int64_t row = e / HC;
  const int c = (int)(e % HC);
  const int64_t i = row % R;
  const float g = to_f32(qkvg[row * NQ + HC + 2 * D + c]);
  dqkvg[row * NQ + HC + 2 * D + c] = from_f32<T>(dgo[e] * gctx[i * HC + c] * g * (1.f - g));
}

template <typename T>
__global__ __launch_bounds__(GA_THREADS) void gattn_bwd_kernel(int64_t S, int64_t R, int H, int D, const T* qkvg,
                                                               const float* mask, float eps, const float* dgo,
                                                               T* dqkvg) {
  extern __shared__ float sm[];
  const int HC = H * D, NQ = 2 * HC + 2 * D;
  float* red = sm;
  float* qbar = sm + 8;
  float* dctx = qbar + HC;
  float* dqbar = dctx + HC;
  float* p = dqbar + HC;            // [H][S]
  float* dl = p + H * S;            // [H][S]
  const int64_t i = blockIdx.x;
  gattn_logits<T>(S, R, H, D, qkvg, mask, eps, i, qbar, p, red);
  gattn_softmax(S, H, p, red, nullptr, nullptr);
  float msum = 0.f;
  for (int64_t s = threadIdx.x; s < S; s += GA_THREADS) msum += mask ? mask[s * R + i] : 1.f;
  msum = block_reduce(msum, red, false);
  // gradient of the context
  for (int e = threadIdx.x; e < HC; e += GA_THREADS) {
    float acc = 0.f;
    for (int64_t s = 0; s < S; ++s)
      acc += dgo[(s * R + i) * HC + e] * to_f32(qkvg[(s * R + i) * NQ + HC + 2 * D + e]);
    dctx[e] = acc;
  }
  __syncthreads();
  // dp[h][t] = sum_d dctx[h][d] v[t][d];  dv[t][d] = sum_h p[h][t] dctx[h][d]
  for (int64_t e = threadIdx.x; e < (int64_t)H * S; e += GA_THREADS) {
    const int h = (int)(e / S);
    const int64_t t = e % S;
    const T* vr = qkvg + (t * R + i) * NQ + HC + D;
    float acc = 0.f;
    for (int d = 0; d < D; ++d) acc += dctx[h * D + d] * to_f32(vr[d]);
    dl[e] = acc;
  }
  for (int64_t e = threadIdx.x; e < S * D; e += GA_THREADS) {
    const int64_t t = e / D;
    const int d = (int)(e % D);
    float acc = 0.f;
    for (int h = 0; h < H; ++h) acc += p[h * S + t] * dctx[h * D + d];
    dqkvg[(t * R + i) * NQ + HC + D + d] = from_f32<T>(acc);
  }
  __syncthreads();
  // softmax backward (no gradient through masked logits)
  for (int h = 0; h < H; ++h) {
    float s1 = 0.f;
    for (int64_t t = threadIdx.x; t < S; t += GA_THREADS) s1 += p[h * S + t] * dl[h * S + t];
    s1 = block_reduce(s1, red, false);
    for (int64_t t = threadIdx.x; t < S; t += GA_THREADS) {
      const bool masked = mask && mask[t * R + i] == 0.f;
      dl[h * S + t] = masked ? 0.f : p[h * S + t] * (dl[h * S + t] - s1);
    }
  }
  __syncthreads();
  const float sc = 1.0f / sqrtf((float)D);
  // dqbar and dk
  for (int e = threadIdx.x; e < HC; e += GA_THREADS) {
    const int h = e / D, d = e % D;
    float acc = 0.f;
    for (int64_t t = 0; t < S; ++t) acc += dl[h * S + t] * to_f32(qkvg[(t * R + i) * NQ + HC + d]);
    dqbar[e] = acc * sc;
  }
  for (int64_t e = threadIdx.x; e < S * D; e += GA_THREADS) {
    const int64_t t = e / D;
    const int d = (int)(e % D);
    float acc = 0.f;
    for (int h = 0; h < H; ++h) acc += dl[h * S + t] * qbar[h * D + d];
    dqkvg[(t * R + i) * NQ + HC + d] = from_f32<T>(acc * sc);
  }
  __syncthreads();
  // dq[s][h][d] = mask_si / (sum_s mask + eps) * dqbar[h][d]
  const float inv = 1.0f / (msum + eps);
  for (int64_t e = threadIdx.x; e < S * HC; e += GA_THREADS) {
    const int64_t s = e / HC;
    const int c = (int)(e % HC);
    const float mk = mask ? mask[s * R + i] : 1.f;
    dqkvg[(s * R + i) * NQ + c] = from_f32<T>(mk * inv * dqbar[c]);
  }
}

template <typename T>
evo_status_t gattn_bwd(const Ctx& c, Arena& ws, int64_t S, int64_t R, int H, int D, const T* qkvg,
                       const float* mask, float eps, const float* gctx, const float* smax, const float* sinv,
                       const float* dgo, T* dqkvg) {
  (void)ws; (void)smax; (void)sinv;
  if (c.dry) return EVO_OK;
  const size_t lds = (8 + 3 * (size_t)H * D + 2 * (size_t)H * S) * sizeof(float);
  if (lds > 150 * 1024) { set_error("global attention bwd: %lld rows exceed LDS", (long long)S); return EVO_ESHAPE; }
  const int64_t n = S * R * H * D;
  EVO_LAUNCH(EVO_KNAME("gattn_gate_bwd_kernel", T), 0.0, (double)n * (4.0 + 2 * sizeof(T)), (gattn_gate_bwd_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, S, R,
                     H, D, qkvg, gctx, dgo, dqkvg);
  EVO_TRY(check_launch("gattn_gate_bwd"));
  EVO_LAUNCH(EVO_KNAME("gattn_bwd_kernel", T), 8.0 * (double)S * R * H * D, (double)S * R * (3 * H * D + 4 * D) * sizeof(T), (gattn_bwd_kernel<T>), dim3((unsigned)R), dim3(GA_THREADS), lds, c.stream, S, R, H, D, qkvg,
                     mask, eps, dgo, dqkvg);
  return check_launch("gattn_bwd");
}

template evo_status_t gattn_fwd<float>(const Ctx&, int64_t, int64_t, int, int, const float*, const float*, float,
                                       float*, float*, float*, float*);
template evo_status_t gattn_fwd<bf16>(const Ctx&, int64_t, int64_t, int, int, const bf16*, const float*, float,
                                      float*, float*, float*, bf16*);
template evo_status_t gattn_bwd<float>(const Ctx&, Arena&, int64_t, int64_t, int, int, const float*, const float*,
                                       float, const float*, const float*, const float*, const float*, float*);
template evo_status_t gattn_bwd<bf16>(const Ctx&, Arena&, int64_t, int64_t, int, int, const bf16*, const float*,
                                      float, const float*, const float*, const float*, const float*, bf16*);

}  // namespace evo
