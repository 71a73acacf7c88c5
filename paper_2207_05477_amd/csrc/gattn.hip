// Global column attention of the extra-MSA stack (gfx950).
//
// Per residue column i: one query per head, the masked mean over the MSA rows
// s of q; single-head keys and values shared by all heads; softmax over the
// rows t; the context is broadcast back to every row through the per-row
// gate.  The work is a few streaming passes over the projection buffer
// (HBM-bound): the rows are split into chunks of GA_CHUNK, each pass leaves
// per-chunk partial results (sums, or the softmax's local max, sum and
// context), and small reduction kernels combine them in a fixed order, so any
// number of rows works (no column has to fit in LDS) and results are
// deterministic.
//   forward   qbar partials -> qbar (+ 1 / (sum_s M_si + eps)) -> softmax partials
//             -> context, row max, 1 / row sum -> gated output
//   backward  gate backward + dctx partials -> dctx, D_ih = dctx . ctx ->
//             softmax backward (dk, dv per row; dqbar partials) -> dqbar -> dq
// q | k | v | g live in one projection buffer [S*R][NQ], NQ = 2*H*D + 2*D,
// row s*R + i.  Threads of the row-streaming passes own 8 consecutive
// channels of one column; threads of the softmax passes own one (column,
// head), with the H heads of a column on adjacent lanes.
#include "ops.h"

namespace evo {

constexpr int GA_THREADS = 64;   // one wave per workgroup: many workgroups in flight
constexpr int GA_CHUNK = 32;     // rows per chunk

int64_t gattn_chunks(int64_t S) { return (S + GA_CHUNK - 1) / GA_CHUNK; }

// ============================================================== forward
// part_q[ch][i][c] = sum_{s in chunk ch} M_si q[s, i, c];  part_m[ch][i] = sum M_si
template <typename T>
__global__ __launch_bounds__(GA_THREADS) void gattn_qbar_partial_kernel(int64_t S, int64_t R, int HC, int NQ,
                                                                        const T* qkvg, const float* mask,
                                                                        float* part_q, float* part_m) {
  const int vpc = HC / 8, cpw = GA_THREADS / vpc;
  const int64_t i = (int64_t)blockIdx.x * cpw + threadIdx.x / vpc;
  const int c0 = (threadIdx.x % vpc) * 8;
  const int64_t ch = blockIdx.y;
  if (i >= R) return;
  const int64_t s0 = ch * GA_CHUNK, s1 = s0 + GA_CHUNK < S ? s0 + GA_CHUNK : S;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float msum = 0.f;
#pragma unroll 4
  for (int64_t s = s0; s < s1; ++s) {
    const float mk = mask ? mask[s * R + i] : 1.f;
    float q[8];
    ld8(qkvg + (s * R + i) * NQ + c0, q);
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] += mk * q[e];
    msum += mk;
  }
  st8(part_q + (ch * R + i) * HC + c0, acc);
  if (c0 == 0) part_m[ch * R + i] = msum;
}

// qbar[i][c] = sum_ch part_q / (sum_ch part_m + eps);  minv[i] = 1 / (sum_ch part_m + eps)
__global__ __launch_bounds__(256) void gattn_qbar_reduce_kernel(int64_t R, int HC, int64_t nch, const float* part_q,
                                                                const float* part_m, float eps, float* qbar,
                                                                float* minv) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= R * HC) return;
  const int64_t i = e / HC;
  float q = 0.f, m = 0.f;
  for (int64_t ch = 0; ch < nch; ++ch) {
    q += part_q[ch * R * HC + e];
    m += part_m[ch * R + i];
  }
  const float inv = 1.0f / (m + eps);
  qbar[e] = q * inv;
  if (e % HC == 0) minv[i] = inv;
}

// Per chunk of rows t, per (i, h): local max, sum of exp and context of the
// masked softmax over t of qbar_ih . k_ti * scale.  Masked keys get kMaskLogit.
template <typename T, int D>
__global__ __launch_bounds__(GA_THREADS) void gattn_softmax_partial_kernel(int64_t S, int64_t R, int H, int NQ,
                                                                           const T* qkvg, const float* mask,
                                                                           const float* qbar, float scale,
                                                                           float* part_ml, float* part_ctx) {
  const int HC = H * D, cpw = GA_THREADS / H;
  const int64_t i = (int64_t)blockIdx.x * cpw + threadIdx.x / H;
  const int h = threadIdx.x % H;
  const int64_t ch = blockIdx.y;
  if (i >= R) return;
  float qb[D];
#pragma unroll
  for (int d = 0; d < D; d += 8) ld8(qbar + i * HC + h * D + d, qb + d);
  const int64_t t0 = ch * GA_CHUNK, t1 = t0 + GA_CHUNK < S ? t0 + GA_CHUNK : S;
  float m = -INFINITY, l = 0.f, ctx[D];
#pragma unroll
  for (int d = 0; d < D; ++d) ctx[d] = 0.f;
  for (int64_t t = t0; t < t1; ++t) {
    const T* row = qkvg + (t * R + i) * NQ + HC;
    float k[D], v[D];
#pragma unroll
    for (int d = 0; d < D; d += 8) { ld8(row + d, k + d); ld8(row + D + d, v + d); }
    float x = 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) x = fmaf(qb[d], k[d], x);
    x *= scale;
    if (mask && mask[t * R + i] == 0.f) x = kMaskLogit;
    if (x > m) {
      const float a = __expf(m - x);   // m = -inf: a = 0
      l *= a;
#pragma unroll
      for (int d = 0; d < D; ++d) ctx[d] *= a;
      m = x;
    }
    const float p = __expf(x - m);
    l += p;
#pragma unroll
    for (int d = 0; d < D; ++d) ctx[d] = fmaf(p, v[d], ctx[d]);
  }
  const int64_t o = (ch * R + i) * H + h;
  part_ml[2 * o] = m;
  part_ml[2 * o + 1] = l;
#pragma unroll
  for (int d = 0; d < D; d += 8) st8(part_ctx + o * D + d, ctx + d);
}

// Combine the chunks: row max M, 1/L and the normalised context per (i, h).
template <int D>
__global__ __launch_bounds__(256) void gattn_combine_kernel(int64_t R, int H, int64_t nch, const float* part_ml,
                                                            const float* part_ctx, float* gctx, float* smax,
                                                            float* sinv) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (i, h)
  if (e >= R * H) return;
  float M = -INFINITY;
  for (int64_t ch = 0; ch < nch; ++ch) M = fmaxf(M, part_ml[2 * (ch * R * H + e)]);
  float L = 0.f, ctx[D];
#pragma unroll
  for (int d = 0; d < D; ++d) ctx[d] = 0.f;
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int64_t o = ch * R * H + e;
    const float a = __expf(part_ml[2 * o] - M);
    L = fmaf(a, part_ml[2 * o + 1], L);
    float c[D];
#pragma unroll
    for (int d = 0; d < D; d += 8) ld8(part_ctx + o * D + d, c + d);
#pragma unroll
    for (int d = 0; d < D; ++d) ctx[d] = fmaf(a, c[d], ctx[d]);
  }
  const float inv = 1.0f / L;
#pragma unroll
  for (int d = 0; d < D; ++d) ctx[d] *= inv;
#pragma unroll
  for (int d = 0; d < D; d += 8) st8(gctx + e * D + d, ctx + d);
  smax[e] = M;
  sinv[e] = inv;
}

// go[s, i, c] = g[s, i, c] * ctx[i, c], 8 channels per thread.
template <typename T>
__global__ __launch_bounds__(256) void gattn_gate_kernel(int64_t S, int64_t R, int HC, int NQ, const T* qkvg,
                                                         const float* gctx, T* go) {
  const int vpc = HC / 8;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= S * R * vpc) return;
  const int64_t row = e / vpc;
  const int c0 = (int)(e % vpc) * 8;
  const int64_t i = row % R;
  float g[8], cx[8], o[8];
  ld8(qkvg + row * NQ + (NQ - HC) + c0, g);   // gate columns
  ld8(gctx + i * HC + c0, cx);
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = g[k] * cx[k];
  st8(go + row * HC + c0, o);
}

// Scratch (FP32 elements) of the forward: per-chunk partials of qbar, the mask
// sums, the softmax statistics and the contexts.
int64_t gattn_fwd_scratch(int64_t S, int64_t R, int H, int D) {
  const int64_t nch = gattn_chunks(S), HC = (int64_t)H * D;
  return nch * R * (HC + 1 + 2 * H + HC) + 64;
}

template <typename T, int D>
static evo_status_t gattn_fwd_d(const Ctx& c, float* scratch, int64_t S, int64_t R, int H, const T* qkvg,
                                const float* mask, float eps, float* qbar, float* minv, float* gctx, float* smax,
                                float* sinv, T* go) {
  const int HC = H * D, NQ = 2 * HC + 2 * D;
  const int64_t nch = gattn_chunks(S);
  auto align = [](int64_t n) { return (n + 63) & ~(int64_t)63; };   // 256-byte aligned pieces
  float* part_q = scratch;
  float* part_m = part_q + align(nch * R * HC);
  float* part_ml = part_m + align(nch * R);
  float* part_ctx = part_ml + align(nch * R * H * 2);
  if (c.dry) return EVO_OK;
  const int vpc = HC / 8, cpw = GA_THREADS / vpc, cpw2 = GA_THREADS / H;
  const double qb = (double)S * R * HC * sizeof(T), kvb = (double)S * R * 2 * D * sizeof(T);
  EVO_LAUNCH(EVO_KNAME("gattn_qbar_partial_kernel", T), 2.0 * S * R * HC, qb, (gattn_qbar_partial_kernel<T>),
             dim3((unsigned)((R + cpw - 1) / cpw), (unsigned)nch), dim3(GA_THREADS), 0, c.stream, S, R, HC, NQ,
             qkvg, mask, part_q, part_m);
  EVO_TRY(check_launch("gattn_qbar_partial"));
  EVO_LAUNCH("gattn_qbar_reduce_kernel", 0.0, (double)nch * R * (HC + 1) * 4, gattn_qbar_reduce_kernel,
             dim3((unsigned)((R * HC + 255) / 256)), dim3(256), 0, c.stream, R, HC, nch, part_q, part_m, eps, qbar,
             minv);
  EVO_TRY(check_launch("gattn_qbar_reduce"));
  EVO_LAUNCH(EVO_KNAME("gattn_softmax_partial_kernel", T), 4.0 * S * R * HC, kvb,
             (gattn_softmax_partial_kernel<T, D>), dim3((unsigned)((R + cpw2 - 1) / cpw2), (unsigned)nch),
             dim3(GA_THREADS), 0, c.stream, S, R, H, NQ, qkvg, mask, qbar, 1.0f / sqrtf((float)D), part_ml,
             part_ctx);
  EVO_TRY(check_launch("gattn_softmax_partial"));
  EVO_LAUNCH("gattn_combine_kernel", 0.0, (double)nch * R * (HC + 2 * H) * 4, (gattn_combine_kernel<D>),
             dim3((unsigned)((R * H + 255) / 256)), dim3(256), 0, c.stream, R, H, nch, part_ml, part_ctx, gctx,
             smax, sinv);
  EVO_TRY(check_launch("gattn_combine"));
  const int64_t n = S * R * vpc;
  EVO_LAUNCH(EVO_KNAME("gattn_gate_kernel", T), 0.0, (double)S * R * HC * 2 * sizeof(T), (gattn_gate_kernel<T>),
             dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, S, R, HC, NQ, qkvg, gctx, go);
  return check_launch("gattn_gate");
}

template <typename T>
evo_status_t gattn_fwd(const Ctx& c, float* scratch, int64_t S, int64_t R, int H, int D, const T* qkvg,
                       const float* mask, float eps, float* qbar, float* minv, float* gctx, float* smax,
                       float* sinv, T* go) {
  switch (D) {
    case 8: return gattn_fwd_d<T, 8>(c, scratch, S, R, H, qkvg, mask, eps, qbar, minv, gctx, smax, sinv, go);
    case 16: return gattn_fwd_d<T, 16>(c, scratch, S, R, H, qkvg, mask, eps, qbar, minv, gctx, smax, sinv, go);
    case 32: return gattn_fwd_d<T, 32>(c, scratch, S, R, H, qkvg, mask, eps, qbar, minv, gctx, smax, sinv, go);
    default: set_error("global attention: head_dim %d not in {8, 16, 32}", D); return EVO_ESHAPE;
  }
}

// ============================================================== backward
// Gate backward per row (dg before the sigmoid into dqkvg's gate columns) and
// part_dctx[ch][i][c] = sum_{s in chunk} dgo[s, i, c] g[s, i, c].
template <typename T>
__global__ __launch_bounds__(GA_THREADS) void gattn_gate_bwd_partial_kernel(int64_t S, int64_t R, int HC, int NQ,
                                                                            const T* qkvg, const float* gctx,
                                                                            const float* dgo, T* dqkvg,
                                                                            float* part_dctx) {
  const int vpc = HC / 8, cpw = GA_THREADS / vpc;
  const int64_t i = (int64_t)blockIdx.x * cpw + threadIdx.x / vpc;
  const int c0 = (threadIdx.x % vpc) * 8;
  const int64_t ch = blockIdx.y;
  if (i >= R) return;
  const int gofs = NQ - HC;   // gate columns
  float cx[8];
  ld8(gctx + i * HC + c0, cx);
  const int64_t s0 = ch * GA_CHUNK, s1 = s0 + GA_CHUNK < S ? s0 + GA_CHUNK : S;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int64_t s = s0; s < s1; ++s) {
    const int64_t row = s * R + i;
    float g[8], dg[8], out[8];
    ld8(qkvg + row * NQ + gofs + c0, g);
    ld8(dgo + row * HC + c0, dg);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      acc[e] = fmaf(dg[e], g[e], acc[e]);
      out[e] = dg[e] * cx[e] * g[e] * (1.f - g[e]);
    }
    st8(dqkvg + row * NQ + gofs + c0, out);
  }
  st8(part_dctx + (ch * R + i) * HC + c0, acc);
}

// dctx[i][c] = sum_ch part_dctx;  Dh[i][h] = sum_d dctx[i][h][d] ctx[i][h][d]
template <int D>
__global__ __launch_bounds__(256) void gattn_dctx_reduce_kernel(int64_t R, int H, int64_t nch, const float* part,
                                                                const float* gctx, float* dctx, float* Dh) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (i, h)
  if (e >= R * H) return;
  const int64_t HC = (int64_t)H * D;
  float acc[D];
#pragma unroll
  for (int d = 0; d < D; ++d) acc[d] = 0.f;
  for (int64_t ch = 0; ch < nch; ++ch) {
    float v[D];
#pragma unroll
    for (int d = 0; d < D; d += 8) ld8(part + ch * R * HC + e * D + d, v + d);
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] += v[d];
  }
  float cx[D], dsum = 0.f;
#pragma unroll
  for (int d = 0; d < D; d += 8) ld8(gctx + e * D + d, cx + d);
#pragma unroll
  for (int d = 0; d < D; ++d) dsum = fmaf(acc[d], cx[d], dsum);
#pragma unroll
  for (int d = 0; d < D; d += 8) st8(dctx + e * D + d, acc + d);
  Dh[e] = dsum;
}

// Softmax backward per chunk of rows t and (i, h): p recomputed from the
// saved max and 1/sum; ds = p (dctx . v - D_ih), zero at masked keys; dv and
// dk of row t summed over the H heads (adjacent lanes); dqbar partials.
template <typename T, int D>
__global__ __launch_bounds__(GA_THREADS) void gattn_softmax_bwd_kernel(int64_t S, int64_t R, int H, int NQ,
                                                                       const T* qkvg, const float* mask,
                                                                       const float* qbar, const float* dctx,
                                                                       const float* Dh, const float* smax,
                                                                       const float* sinv, float scale, T* dqkvg,
                                                                       float* part_dqbar) {
  const int HC = H * D, cpw = GA_THREADS / H;
  const int64_t i0 = (int64_t)blockIdx.x * cpw + threadIdx.x / H;
  const bool ok = i0 < R;
  const int64_t i = ok ? i0 : R - 1;   // lanes past the end shadow the last column, write nothing
  const int h = threadIdx.x % H;
  const int64_t ch = blockIdx.y;
  const int64_t e = i * H + h;
  float qb[D], dc[D], acc[D];
#pragma unroll
  for (int d = 0; d < D; d += 8) { ld8(qbar + e * D + d, qb + d); ld8(dctx + e * D + d, dc + d); }
#pragma unroll
  for (int d = 0; d < D; ++d) acc[d] = 0.f;
  const float M = smax[e], inv = sinv[e], Dsum = Dh[e];
  const int64_t t0 = ch * GA_CHUNK, t1 = t0 + GA_CHUNK < S ? t0 + GA_CHUNK : S;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row = t * R + i;
    float k[D], v[D];
#pragma unroll
    for (int d = 0; d < D; d += 8) { ld8(qkvg + row * NQ + HC + d, k + d); ld8(qkvg + row * NQ + HC + D + d, v + d); }
    float x = 0.f, dp = 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) { x = fmaf(qb[d], k[d], x); dp = fmaf(dc[d], v[d], dp); }
    const bool masked = mask && mask[row] == 0.f;
    x = masked ? kMaskLogit : x * scale;
    const float p = __expf(x - M) * inv;
    const float ds = masked ? 0.f : p * (dp - Dsum);
    float dv[D], dk[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      acc[d] = fmaf(ds * scale, k[d], acc[d]);
      dv[d] = p * dc[d];
      dk[d] = ds * scale * qb[d];
    }
    for (int o = 1; o < H; o <<= 1) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        dv[d] += __shfl_xor(dv[d], o, 64);
        dk[d] += __shfl_xor(dk[d], o, 64);
      }
    }
    if (ok && h == 0) {
#pragma unroll
      for (int d = 0; d < D; d += 8) {
        st8(dqkvg + row * NQ + HC + d, dk + d);
        st8(dqkvg + row * NQ + HC + D + d, dv + d);
      }
    }
  }
  if (ok) {
#pragma unroll
    for (int d = 0; d < D; d += 8) st8(part_dqbar + (ch * R * H + e) * D + d, acc + d);
  }
}

// dqbar[i][c] = sum_ch part (plain sum; the 1/(sum M + eps) factor is applied per row in dq)
__global__ __launch_bounds__(256) void gattn_sum_chunks_kernel(int64_t n, int64_t nch, const float* part, float* out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  float acc = 0.f;
  for (int64_t ch = 0; ch < nch; ++ch) acc += part[ch * n + e];
  out[e] = acc;
}

// dq[s, i, c] = M_si * minv[i] * dqbar[i, c], 8 channels per thread.
template <typename T>
__global__ __launch_bounds__(256) void gattn_dq_kernel(int64_t S, int64_t R, int HC, int NQ, const float* mask,
                                                       const float* minv, const float* dqbar, T* dqkvg) {
  const int vpc = HC / 8;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= S * R * vpc) return;
  const int64_t row = e / vpc;
  const int c0 = (int)(e % vpc) * 8;
  const int64_t i = row % R;
  const float f = (mask ? mask[row] : 1.f) * minv[i];
  float v[8];
  ld8(dqbar + i * HC + c0, v);
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] *= f;
  st8(dqkvg + row * NQ + c0, v);
}

template <typename T, int D>
static evo_status_t gattn_bwd_d(const Ctx& c, Arena& ws, int64_t S, int64_t R, int H, const T* qkvg,
                                const float* mask, const float* qbar, const float* minv, const float* gctx,
                                const float* smax, const float* sinv, const float* dgo, T* dqkvg) {
  const int HC = H * D, NQ = 2 * HC + 2 * D;
  const int64_t nch = gattn_chunks(S);
  float* part = ws.take_n<float>(nch * R * HC);   // dctx partials, then dqbar partials
  float* dctx = ws.take_n<float>(R * HC);
  float* Dh = ws.take_n<float>(R * H);
  float* dqbar = ws.take_n<float>(R * HC);
  if (c.dry) return EVO_OK;
  const int vpc = HC / 8, cpw = GA_THREADS / vpc, cpw2 = GA_THREADS / H;
  const double rowb = (double)S * R;
  EVO_LAUNCH(EVO_KNAME("gattn_gate_bwd_partial_kernel", T), 0.0, rowb * HC * (2 * sizeof(T) + 4),
             (gattn_gate_bwd_partial_kernel<T>), dim3((unsigned)((R + cpw - 1) / cpw), (unsigned)nch),
             dim3(GA_THREADS), 0, c.stream, S, R, HC, NQ, qkvg, gctx, dgo, dqkvg, part);
  EVO_TRY(check_launch("gattn_gate_bwd_partial"));
  EVO_LAUNCH("gattn_dctx_reduce_kernel", 0.0, (double)nch * R * HC * 4, (gattn_dctx_reduce_kernel<D>),
             dim3((unsigned)((R * H + 255) / 256)), dim3(256), 0, c.stream, R, H, nch, part, gctx, dctx, Dh);
  EVO_TRY(check_launch("gattn_dctx_reduce"));
  EVO_LAUNCH(EVO_KNAME("gattn_softmax_bwd_kernel", T), 8.0 * S * R * HC, rowb * 4 * D * sizeof(T),
             (gattn_softmax_bwd_kernel<T, D>), dim3((unsigned)((R + cpw2 - 1) / cpw2), (unsigned)nch),
             dim3(GA_THREADS), 0, c.stream, S, R, H, NQ, qkvg, mask, qbar, dctx, Dh, smax, sinv,
             1.0f / sqrtf((float)D), dqkvg, part);
  EVO_TRY(check_launch("gattn_softmax_bwd"));
  EVO_LAUNCH("gattn_sum_chunks_kernel", 0.0, (double)nch * R * HC * 4, gattn_sum_chunks_kernel,
             dim3((unsigned)((R * HC + 255) / 256)), dim3(256), 0, c.stream, R * HC, nch, part, dqbar);
  EVO_TRY(check_launch("gattn_sum_chunks"));
  const int64_t n = S * R * vpc;
  EVO_LAUNCH(EVO_KNAME("gattn_dq_kernel", T), 0.0, rowb * HC * sizeof(T), (gattn_dq_kernel<T>),
             dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, S, R, HC, NQ, mask, minv, dqbar, dqkvg);
  return check_launch("gattn_dq");
}

template <typename T>
evo_status_t gattn_bwd(const Ctx& c, Arena& ws, int64_t S, int64_t R, int H, int D, const T* qkvg,
                       const float* mask, const float* qbar, const float* minv, const float* gctx,
                       const float* smax, const float* sinv, const float* dgo, T* dqkvg) {
  switch (D) {
    case 8: return gattn_bwd_d<T, 8>(c, ws, S, R, H, qkvg, mask, qbar, minv, gctx, smax, sinv, dgo, dqkvg);
    case 16: return gattn_bwd_d<T, 16>(c, ws, S, R, H, qkvg, mask, qbar, minv, gctx, smax, sinv, dgo, dqkvg);
    case 32: return gattn_bwd_d<T, 32>(c, ws, S, R, H, qkvg, mask, qbar, minv, gctx, smax, sinv, dgo, dqkvg);
    default: set_error("global attention: head_dim %d not in {8, 16, 32}", D); return EVO_ESHAPE;
  }
}

#define EVO_INST_G(T)                                                                                          \
  template evo_status_t gattn_fwd<T>(const Ctx&, float*, int64_t, int64_t, int, int, const T*, const float*,  \
                                     float, float*, float*, float*, float*, float*, T*);                       \
  template evo_status_t gattn_bwd<T>(const Ctx&, Arena&, int64_t, int64_t, int, int, const T*, const float*, \
                                     const float*, const float*, const float*, const float*, const float*,     \
                                     const float*, T*);
EVO_INST_G(float)
EVO_INST_G(bf16)

}  // namespace evo
