// LayerNorm (wave-per-row, FP32 statistics), deterministic column reductions,
// parameter packing and the elementwise kernels of the gated ops.
#include "misc.h"

namespace evo {

// ============================================================== LayerNorm forward
template <typename TI, typename T, int NV>
__global__ __launch_bounds__(256) void ln_fwd_kernel(const TI* __restrict__ x, int64_t rows, int C,
                                                     const float* __restrict__ g,
                                                     const float* __restrict__ b, float eps,
                                                     T* __restrict__ y, float* __restrict__ mean,
                                                     float* __restrict__ rstd, int rshift, int64_t rhi) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const TI* xr = x + (rshift < 0 ? row * C : (row >> rshift) * rhi + (row & ((1LL << rshift) - 1)) * C);
  float v[NV];
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int c = lane + 64 * i;
    v[i] = c < C ? to_f32(xr[c]) : 0.f;
    s += v[i];
  }
  const float mu = wave_sum(s) / (float)C;
  float q = 0.f;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int c = lane + 64 * i;
    const float d = c < C ? v[i] - mu : 0.f;
    q += d * d;
  }
  const float rs = 1.0f / sqrtf(wave_sum(q) / (float)C + eps);
  T* yr = y + row * C;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int c = lane + 64 * i;
    if (c < C) yr[c] = from_f32<T>((v[i] - mu) * rs * g[c] + b[c]);
  }
  if (lane == 0) {
    if (mean) mean[row] = mu;
    if (rstd) rstd[row] = rs;
  }
}

// Vectorised form (C % 8 == 0, C <= 1024, 16-byte aligned rows): LPR lanes
// share a row, lane l owning the 8-channel chunks j*LPR + l (j < NC), so a wave
// normalises 64 / LPR rows at once with 16-byte accesses.
constexpr int LNF_ROWS = 2;   // rows per lane group in the vectorised LayerNorm forward
template <typename TI, typename T, int LPR, int NC>
__global__ __launch_bounds__(256) void ln_fwd_vec_kernel(const TI* __restrict__ x, int64_t rows, int C,
                                                         const float* __restrict__ g,
                                                         const float* __restrict__ b, float eps,
                                                         T* __restrict__ y, float* __restrict__ mean,
                                                         float* __restrict__ rstd, int rshift, int64_t rhi) {
  // LNF_ROWS rows per lane group, RPB rows apart: all their loads are issued
  // before any is used (rows past the end read the last row, never stored)
  constexpr int RPB = 256 / LPR;
  const int l = threadIdx.x & (LPR - 1);
  float v[LNF_ROWS][NC][8];
#pragma unroll
  for (int q = 0; q < LNF_ROWS; ++q) {
    int64_t row = ((int64_t)blockIdx.x * LNF_ROWS + q) * RPB + threadIdx.x / LPR;
    row = row < rows ? row : rows - 1;
    const TI* xr = x + (rshift < 0 ? row * C : (row >> rshift) * rhi + (row & ((1LL << rshift) - 1)) * C);
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c0 = (j * LPR + l) * 8;
      if (c0 < C) ld8(xr + c0, v[q][j]);
      else
#pragma unroll
        for (int i = 0; i < 8; ++i) v[q][j][i] = 0.f;
    }
  }
#pragma unroll
  for (int q = 0; q < LNF_ROWS; ++q) {
    const int64_t row = ((int64_t)blockIdx.x * LNF_ROWS + q) * RPB + threadIdx.x / LPR;
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < NC; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) s += v[q][j][i];
    const float mu = group_sum<LPR>(s) / (float)C;
    float sq = 0.f;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c0 = (j * LPR + l) * 8;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float d = c0 < C ? v[q][j][i] - mu : 0.f;
        sq += d * d;
      }
    }
    const float rs = 1.0f / sqrtf(group_sum<LPR>(sq) / (float)C + eps);
    if (row >= rows) continue;
    T* yr = y + row * C;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c0 = (j * LPR + l) * 8;
      if (c0 < C) {
        float gg[8], bb[8], o[8];
        ld8(g + c0, gg);
        ld8(b + c0, bb);
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = (v[q][j][i] - mu) * rs * gg[i] + bb[i];
        st8(yr + c0, o);
      }
    }
    if (l == 0) {
      if (mean) mean[row] = mu;
      if (rstd) rstd[row] = rs;
    }
  }
}

// Lanes per row of the vectorised LayerNorm kernels: the smallest power of two
// >= C / 8, at least 4 and at most 64.
static int ln_lanes(int C) {
  int l = 4;
  while (l < 64 && l * 8 < C) l <<= 1;
  return l;
}

template <typename TI, typename T, int LPR>
static void ln_fwd_vec_launch(const Ctx& c, double bytes, const TI* x, int64_t rows, int C, int rshift,
                              int64_t rhi, const float* g, const float* b, float eps, T* y, float* mean,
                              float* rstd) {
  constexpr int RPB = 256 / LPR * LNF_ROWS;
  dim3 grid((unsigned)((rows + RPB - 1) / RPB));
  if (C <= 8 * LPR)
    EVO_LAUNCH(EVO_KNAME("ln_fwd_vec_kernel", TI), 0.0, bytes, (ln_fwd_vec_kernel<TI, T, LPR, 1>), grid, dim3(256), 0, c.stream, x, rows, C, g, b, eps, y, mean, rstd, rshift, rhi);
  else
    EVO_LAUNCH(EVO_KNAME("ln_fwd_vec_kernel", TI), 0.0, bytes, (ln_fwd_vec_kernel<TI, T, LPR, 2>), grid, dim3(256), 0, c.stream, x, rows, C, g, b, eps, y, mean, rstd, rshift, rhi);
}

template <typename TI, typename T>
evo_status_t ln_fwd_rows(const Ctx& c, const TI* x, int64_t rows, int C, int rshift, int64_t rhi,
                         const float* g, const float* b, float eps, T* y, float* mean, float* rstd) {
  if (c.dry || rows == 0) return EVO_OK;
  dim3 grid((unsigned)((rows + 3) / 4));
  const double bytes = (double)rows * C * (sizeof(TI) + sizeof(T)) + rows * 8.0;
  if (C % 8 == 0 && C <= 1024 && (rshift < 0 || rhi % 8 == 0) && aligned16(x) && aligned16(y) &&
      aligned16(g) && aligned16(b)) {
    switch (ln_lanes(C)) {
      case 4: ln_fwd_vec_launch<TI, T, 4>(c, bytes, x, rows, C, rshift, rhi, g, b, eps, y, mean, rstd); break;
      case 8: ln_fwd_vec_launch<TI, T, 8>(c, bytes, x, rows, C, rshift, rhi, g, b, eps, y, mean, rstd); break;
      case 16: ln_fwd_vec_launch<TI, T, 16>(c, bytes, x, rows, C, rshift, rhi, g, b, eps, y, mean, rstd); break;
      case 32: ln_fwd_vec_launch<TI, T, 32>(c, bytes, x, rows, C, rshift, rhi, g, b, eps, y, mean, rstd); break;
      default: ln_fwd_vec_launch<TI, T, 64>(c, bytes, x, rows, C, rshift, rhi, g, b, eps, y, mean, rstd); break;
    }
    return check_launch("ln_fwd");
  }
  if (C <= 64) EVO_LAUNCH(EVO_KNAME("ln_fwd_kernel", TI), 0.0, bytes, (ln_fwd_kernel<TI, T, 1>), grid, dim3(256), 0, c.stream, x, rows, C, g, b, eps, y, mean, rstd, rshift, rhi);
  else if (C <= 128) EVO_LAUNCH(EVO_KNAME("ln_fwd_kernel", TI), 0.0, bytes, (ln_fwd_kernel<TI, T, 2>), grid, dim3(256), 0, c.stream, x, rows, C, g, b, eps, y, mean, rstd, rshift, rhi);
  else if (C <= 256) EVO_LAUNCH(EVO_KNAME("ln_fwd_kernel", TI), 0.0, bytes, (ln_fwd_kernel<TI, T, 4>), grid, dim3(256), 0, c.stream, x, rows, C, g, b, eps, y, mean, rstd, rshift, rhi);
  else if (C <= 1024) EVO_LAUNCH(EVO_KNAME("ln_fwd_kernel", TI), 0.0, bytes, (ln_fwd_kernel<TI, T, 16>), grid, dim3(256), 0, c.stream, x, rows, C, g, b, eps, y, mean, rstd, rshift, rhi);
  else { set_error("layernorm: C=%d > 1024", C); return EVO_ESHAPE; }
  return check_launch("ln_fwd");
}

template <typename TI, typename T>
evo_status_t ln_fwd(const Ctx& c, const TI* x, int64_t rows, int C, const float* g, const float* b,
                    float eps, T* y, float* mean, float* rstd) {
  return ln_fwd_rows<TI, T>(c, x, rows, C, -1, 0, g, b, eps, y, mean, rstd);
}

// Output index of head h, row `row` of the projection: [H][rows], or with
// tr_n > 0 (rows = tr_n^2, row = a * tr_n + b) the transposed [H][b][a].
EVO_DEV int64_t rowproj_dst(int h, int64_t rows, int64_t row, int64_t tr_n) {
  if (tr_n <= 0) return (int64_t)h * rows + row;
  // rows = tr_n^2 < 2^31 (checked by the launcher): 32-bit division
  const uint32_t r = (uint32_t)row, n = (uint32_t)tr_n, a = r / n;
  return (int64_t)h * rows + (int64_t)(r - a * n) * tr_n + a;
}

// Fused LayerNorm + small projection (pair bias): a block owns RPB rows; the
// row tile goes through LDS (coalesced loads), then 256 / RPB lanes share a
// row: each reduces an interleaved share of the channels for the statistics
// and the H dot products, and xor-shuffles combine the shares.
template <typename TI, typename T, int RPB>
__global__ __launch_bounds__(256) void ln_rowproj_kernel(const TI* __restrict__ x, int64_t rows, int C,
                                                         const float* __restrict__ g,
                                                         const float* __restrict__ b, float eps,
                                                         const float* __restrict__ W, int H,
                                                         float* __restrict__ out, float out_scale,
                                                         int64_t tr_n) {
  constexpr int LPR = 256 / RPB;          // lanes per row
  extern __shared__ float sm[];           // tile [RPB][C + 4], then W [C][H]
  const int ldt = C + 4;
  float* tile = sm;
  float* sW = sm + RPB * ldt;
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * RPB;
  const int nrow = rows - r0 < RPB ? (int)(rows - r0) : RPB;
  for (int e = tid; e < C * H; e += 256) sW[e] = W[e];
  for (int e = tid; e < RPB * C; e += 256) {
    const int rr = e / C, cc = e - rr * C;
    tile[rr * ldt + cc] = rr < nrow ? to_f32(x[(r0 + rr) * C + cc]) : 0.f;
  }
  __syncthreads();
  const int rr = tid / LPR, q = tid % LPR;
  const float* t = tile + rr * ldt;
  float s = 0.f;
  for (int cc = q; cc < C; cc += LPR) s += t[cc];
#pragma unroll
  for (int o = 1; o < LPR; o <<= 1) s += __shfl_xor(s, o, 64);
  const float mu = s / (float)C;
  float v = 0.f;
  for (int cc = q; cc < C; cc += LPR) {
    const float d = t[cc] - mu;
    v += d * d;
  }
#pragma unroll
  for (int o = 1; o < LPR; o <<= 1) v += __shfl_xor(v, o, 64);
  const float rs = 1.0f / sqrtf(v / (float)C + eps);
  float acc[16];
#pragma unroll
  for (int h = 0; h < 16; ++h) acc[h] = 0.f;
  for (int cc = q; cc < C; cc += LPR) {
    // the projection reads the LayerNorm output in the storage precision
    const float yv = to_f32(from_f32<T>((t[cc] - mu) * rs * g[cc] + b[cc]));
#pragma unroll
    for (int h = 0; h < 16; ++h)
      if (h < H) acc[h] += yv * sW[cc * H + h];
  }
#pragma unroll
  for (int h = 0; h < 16; ++h) {
    if (h < H) {
#pragma unroll
      for (int o = 1; o < LPR; o <<= 1) acc[h] += __shfl_xor(acc[h], o, 64);
    }
  }
  if (rr < nrow) {
#pragma unroll
    for (int h = 0; h < 16; ++h)
      if (h < H && h % LPR == q) out[rowproj_dst(h, rows, r0 + rr, tr_n)] = acc[h] * out_scale;
  }
}

// Vectorised form (C % 8 == 0, C <= 512, H <= HM): the lane layout of
// ln_fwd_vec_kernel with one 8-channel chunk per lane; the lane's W slice
// (8 channels x HM heads) stays in registers while a thread walks RIT rows
// spaced 256 / LPR apart; the H dot products are summed over the row's lanes by
// xor shuffles.
constexpr int LRP_RIT = 4;   // rows per thread: all their loads are issued first
template <typename TI, typename T, int LPR, int HM>
__global__ __launch_bounds__(256) void ln_rowproj_vec_kernel(const TI* __restrict__ x, int64_t rows, int C,
                                                             const float* __restrict__ g,
                                                             const float* __restrict__ b, float eps,
                                                             const float* __restrict__ W, int H,
                                                             float* __restrict__ out, float out_scale,
                                                             int64_t tr_n) {
  constexpr int RPI = 256 / LPR;   // rows per iteration of the block
  // W staged once per block as [c][HM] (coalesced), the lane's slice read back as vectors
  __shared__ __attribute__((aligned(16))) float sw[8 * LPR * HM];
  const int l = threadIdx.x & (LPR - 1);
  const int c0 = l * 8;
  const bool cok = c0 < C;
  for (int e = threadIdx.x; e < 8 * LPR * HM; e += 256) {
    const int cc = e / HM, h = e - cc * HM;
    sw[e] = (cc < C && h < H) ? W[cc * H + h] : 0.f;
  }
  float w[8][HM], gg[8], bb[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    gg[i] = cok ? g[c0 + i] : 0.f;
    bb[i] = cok ? b[c0 + i] : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int h = 0; h < HM; h += 4) {
      const f32x4 q = *(const f32x4*)(sw + (c0 + i) * HM + h);
      w[i][h] = q[0]; w[i][h + 1] = q[1]; w[i][h + 2] = q[2]; w[i][h + 3] = q[3];
    }
  float vr[LRP_RIT][8];
#pragma unroll
  for (int it = 0; it < LRP_RIT; ++it) {
    const int64_t row = ((int64_t)blockIdx.x * LRP_RIT + it) * RPI + threadIdx.x / LPR;
    if (row < rows && cok) ld8(x + row * C + c0, vr[it]);
    else
#pragma unroll
      for (int i = 0; i < 8; ++i) vr[it][i] = 0.f;
  }
#pragma unroll
  for (int it = 0; it < LRP_RIT; ++it) {
    const int64_t row = ((int64_t)blockIdx.x * LRP_RIT + it) * RPI + threadIdx.x / LPR;
    const bool ok = row < rows;
    const float* v = vr[it];
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += v[i];
    const float mu = group_sum<LPR>(s) / (float)C;
    float q = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float d = cok ? v[i] - mu : 0.f;
      q += d * d;
    }
    const float rs = 1.0f / sqrtf(group_sum<LPR>(q) / (float)C + eps);
    float acc[HM];
#pragma unroll
    for (int h = 0; h < HM; ++h) acc[h] = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      // the projection reads the LayerNorm output in the storage precision
      const float yv = to_f32(from_f32<T>((v[i] - mu) * rs * gg[i] + bb[i]));
#pragma unroll
      for (int h = 0; h < HM; ++h) acc[h] += yv * w[i][h];
    }
#pragma unroll
    for (int h = 0; h < HM; ++h) {
      acc[h] = group_sum<LPR>(acc[h]);
      if (ok && h < H && l == h % LPR) out[rowproj_dst(h, rows, row, tr_n)] = acc[h] * out_scale;
    }
  }
}

template <typename TI, typename T, int LPR>
static void ln_rowproj_vec_launch(const Ctx& c, double flops, double bytes, const TI* x, int64_t rows, int C,
                                  const float* g, const float* b, float eps, const float* W, int H, float* out,
                                  float out_scale, int64_t tr_n) {
  constexpr int RPB = 256 / LPR * LRP_RIT;
  const dim3 grid((unsigned)((rows + RPB - 1) / RPB));
  if (H <= 4)
    EVO_LAUNCH(EVO_KNAME("ln_rowproj_vec_kernel", TI), flops, bytes, (ln_rowproj_vec_kernel<TI, T, LPR, 4>), grid, dim3(256), 0, c.stream, x, rows, C, g, b, eps, W, H, out, out_scale, tr_n);
  else
    EVO_LAUNCH(EVO_KNAME("ln_rowproj_vec_kernel", TI), flops, bytes, (ln_rowproj_vec_kernel<TI, T, LPR, 8>), grid, dim3(256), 0, c.stream, x, rows, C, g, b, eps, W, H, out, out_scale, tr_n);
}

template <typename TI, typename T>
evo_status_t ln_rowproj(const Ctx& c, const TI* x, int64_t rows, int C, const float* g, const float* b,
                        float eps, const float* W, int H, float* out, float out_scale, int64_t tr_n) {
  if (c.dry || rows == 0) return EVO_OK;
  if (C > 256 || H > 16) { set_error("layernorm projection: C=%d H=%d unsupported", C, H); return EVO_ESHAPE; }
  if (tr_n < 0 || (tr_n > 0 && (tr_n * tr_n != rows || rows >= (1LL << 31)))) {
    set_error("layernorm projection: transposed output needs rows = n^2 (rows=%lld, n=%lld)", (long long)rows,
              (long long)tr_n);
    return EVO_ESHAPE;
  }
  const double bytes = (double)rows * C * sizeof(TI) + (double)rows * H * 4.0;
  const double flops = 2.0 * rows * C * H;
  if (C % 8 == 0 && H <= 8 && aligned16(x)) {
    switch (C / 8 <= 4 ? 4 : C / 8 <= 8 ? 8 : C / 8 <= 16 ? 16 : 32) {
      case 4: ln_rowproj_vec_launch<TI, T, 4>(c, flops, bytes, x, rows, C, g, b, eps, W, H, out, out_scale, tr_n); break;
      case 8: ln_rowproj_vec_launch<TI, T, 8>(c, flops, bytes, x, rows, C, g, b, eps, W, H, out, out_scale, tr_n); break;
      case 16: ln_rowproj_vec_launch<TI, T, 16>(c, flops, bytes, x, rows, C, g, b, eps, W, H, out, out_scale, tr_n); break;
      default: ln_rowproj_vec_launch<TI, T, 32>(c, flops, bytes, x, rows, C, g, b, eps, W, H, out, out_scale, tr_n); break;
    }
    return check_launch("ln_rowproj");
  }
  if (C <= 128) {
    const size_t lds = ((size_t)64 * (C + 4) + (size_t)C * H) * sizeof(float);
    EVO_LAUNCH(EVO_KNAME("ln_rowproj_kernel", TI), flops, bytes, (ln_rowproj_kernel<TI, T, 64>),
               dim3((unsigned)((rows + 63) / 64)), dim3(256), lds, c.stream, x, rows, C, g, b, eps, W, H, out,
               out_scale, tr_n);
  } else {
    const size_t lds = ((size_t)32 * (C + 4) + (size_t)C * H) * sizeof(float);
    EVO_LAUNCH(EVO_KNAME("ln_rowproj_kernel", TI), flops, bytes, (ln_rowproj_kernel<TI, T, 32>),
               dim3((unsigned)((rows + 31) / 32)), dim3(256), lds, c.stream, x, rows, C, g, b, eps, W, H, out,
               out_scale, tr_n);
  }
  return check_launch("ln_rowproj");
}

// Channel-major forward: a block owns 64 positions; x tile [C][64] staged in LDS.
template <typename T>
__global__ __launch_bounds__(256) void ln_fwd_cm_kernel(const T* __restrict__ x, int64_t P, int C,
                                                        const float* __restrict__ g,
                                                        const float* __restrict__ b, float eps,
                                                        T* __restrict__ y, float* __restrict__ mean,
                                                        float* __restrict__ rstd) {
  extern __shared__ float tile[];  // [C][65]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  for (int e = tid; e < C * 64; e += 256) {
    const int cc = e >> 6, pp = e & 63;
    const int64_t p = p0 + pp;
    tile[cc * 65 + pp] = p < P ? to_f32(x[(int64_t)cc * P + p]) : 0.f;
  }
  __syncthreads();
  for (int pp = wave * 16; pp < wave * 16 + 16; ++pp) {
    const int64_t p = p0 + pp;
    if (p >= P) break;
    float s = 0.f;
    for (int cc = lane; cc < C; cc += 64) s += tile[cc * 65 + pp];
    const float mu = wave_sum(s) / (float)C;
    float q = 0.f;
    for (int cc = lane; cc < C; cc += 64) {
      const float d = tile[cc * 65 + pp] - mu;
      q += d * d;
    }
    const float rs = 1.0f / sqrtf(wave_sum(q) / (float)C + eps);
    for (int cc = lane; cc < C; cc += 64)
      y[p * C + cc] = from_f32<T>((tile[cc * 65 + pp] - mu) * rs * g[cc] + b[cc]);
    if (lane == 0) { mean[p] = mu; rstd[p] = rs; }
  }
}

// Channel-major tile of 64 positions: x[c][p0 .. p0 + 63] -> tile[c * 65 + pp] (FP32)
// and back, moving 16-byte vectors of 8 positions when the rows allow it
// (P % 8 == 0, x 16-byte aligned) and single elements otherwise; positions
// from P on read as zeros and are not written.
template <typename T>
EVO_DEV void cm_tile_load(const T* __restrict__ x, int64_t P, int C, int64_t p0, float* tile, int tid) {
  const bool vec = (P & 7) == 0 && (((uintptr_t)x) & 15) == 0;
  for (int e = tid; e < C * 8; e += 256) {
    const int cc = e >> 3, pv = (e & 7) * 8;
    const int64_t p = p0 + pv;
    const T* src = x + (int64_t)cc * P + p;
    float v[8];
    if (vec && p + 8 <= P) {
      ld8(src, v);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = p + i < P ? to_f32(src[i]) : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) tile[cc * 65 + pv + i] = v[i];
  }
}
template <typename T>
EVO_DEV void cm_tile_store(T* __restrict__ x, int64_t P, int C, int64_t p0, const float* tile, int tid) {
  const bool vec = (P & 7) == 0 && (((uintptr_t)x) & 15) == 0;
  for (int e = tid; e < C * 8; e += 256) {
    const int cc = e >> 3, pv = (e & 7) * 8;
    const int64_t p = p0 + pv;
    T* dst = x + (int64_t)cc * P + p;
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = tile[cc * 65 + pv + i];
    if (vec && p + 8 <= P) {
      st8(dst, v);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (p + i < P) dst[i] = from_f32<T>(v[i]);
    }
  }
}

// Vectorised form (C % 8 == 0, C <= 256): the 4 waves split the channels for
// the per-position sums (partials combined through LDS in a fixed order), and
// the output moves as 8-channel row vectors of y[P][C].
template <typename T>
__global__ __launch_bounds__(256) void ln_fwd_cm_vec_kernel(const T* __restrict__ x, int64_t P, int C,
                                                            const float* __restrict__ g,
                                                            const float* __restrict__ b, float eps,
                                                            T* __restrict__ y, float* __restrict__ mean,
                                                            float* __restrict__ rstd) {
  extern __shared__ float tile[];  // [C][65], then red [4][64], mu [64], rs [64]
  float* red = tile + C * 65;
  float* smu = red + 4 * 64;
  float* srs = smu + 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int np = P - p0 < 64 ? (int)(P - p0) : 64;
  cm_tile_load(x, P, C, p0, tile, tid);
  __syncthreads();
  const int cq = C / 4, c0 = wave * cq;   // this wave's channels, position = lane
  float s = 0.f;
  for (int cc = c0; cc < c0 + cq; ++cc) s += tile[cc * 65 + lane];
  red[wave * 64 + lane] = s;
  __syncthreads();
  if (wave == 0) smu[lane] = ((red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane])) / (float)C;
  __syncthreads();
  const float mu = smu[lane];
  float q = 0.f;
  for (int cc = c0; cc < c0 + cq; ++cc) {
    const float d = tile[cc * 65 + lane] - mu;
    q += d * d;
  }
  red[wave * 64 + lane] = q;
  __syncthreads();
  if (wave == 0) {
    const float rs = 1.0f / sqrtf(((red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane])) / (float)C + eps);
    srs[lane] = rs;
    if (lane < np) {
      mean[p0 + lane] = smu[lane];
      rstd[p0 + lane] = rs;
    }
  }
  __syncthreads();
  const int cv = C / 8;
  for (int e = tid; e < 64 * cv; e += 256) {
    const int pp = e / cv, cb = (e - pp * cv) * 8;
    if (pp >= np) continue;
    const float m = smu[pp], r = srs[pp];
    float gg[8], bb[8], o[8];
    ld8(g + cb, gg);
    ld8(b + cb, bb);
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = (tile[(cb + i) * 65 + pp] - m) * r * gg[i] + bb[i];
    st8(y + (p0 + pp) * C + cb, o);
  }
}

template <typename T>
evo_status_t ln_fwd_cm(const Ctx& c, const T* x, int64_t P, int C, const float* g, const float* b,
                       float eps, T* y, float* mean, float* rstd) {
  if (c.dry || P == 0) return EVO_OK;
  if (C % 8 == 0 && C <= 256 && aligned16(y) && aligned16(g) && aligned16(b)) {
    const size_t lds = ((size_t)C * 65 + 6 * 64) * sizeof(float);
    EVO_LAUNCH(EVO_KNAME("ln_fwd_cm_vec_kernel", T), 0.0, (double)P * C * 2.0 * sizeof(T) + P * 8.0, (ln_fwd_cm_vec_kernel<T>), dim3((unsigned)((P + 63) / 64)), dim3(256), lds, c.stream,
               x, P, C, g, b, eps, y, mean, rstd);
    return check_launch("ln_fwd_cm");
  }
  if (C > 512) { set_error("layernorm(cm): C=%d > 512", C); return EVO_ESHAPE; }
  size_t lds = (size_t)C * 65 * sizeof(float);
  EVO_LAUNCH(EVO_KNAME("ln_fwd_cm_kernel", T), 0.0, (double)P * C * 2.0 * sizeof(T) + P * 8.0, (ln_fwd_cm_kernel<T>), dim3((unsigned)((P + 63) / 64)), dim3(256), lds, c.stream,
                     x, P, C, g, b, eps, y, mean, rstd);
  return check_launch("ln_fwd_cm");
}

// ============================================================== LayerNorm backward
// A block owns 64 rows (16 per wave); per-lane gamma/beta partials are reduced
// across the 4 waves through LDS and written to part[blk][2C].
constexpr int LNB_ROWS = 64;

int64_t ln_bwd_partials(int64_t rows) { return (rows + LNB_ROWS - 1) / LNB_ROWS; }

template <typename T, int NV>
__global__ __launch_bounds__(256) void ln_bwd_kernel(const T* __restrict__ x,
                                                     const float* __restrict__ mean,
                                                     const float* __restrict__ rstd,
                                                     const float* __restrict__ g,
                                                     const float* __restrict__ dy, int64_t rows,
                                                     int C, const T* resid, int accumulate, T* dx,
                                                     float* __restrict__ part) {
  __shared__ float red[4][2][NV * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float dg[NV], db[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) { dg[i] = 0.f; db[i] = 0.f; }
  const int64_t r0 = (int64_t)blockIdx.x * LNB_ROWS + wave * (LNB_ROWS / 4);
  for (int rr = 0; rr < LNB_ROWS / 4; ++rr) {
    const int64_t row = r0 + rr;
    if (row >= rows) break;
    const float mu = mean[row], rs = rstd[row];
    float xh[NV], gd[NV];
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int c = lane + 64 * i;
      if (c < C) {
        const float d = dy[row * C + c];
        xh[i] = (to_f32(x[row * C + c]) - mu) * rs;
        gd[i] = d * g[c];
        s1 += gd[i];
        s2 += gd[i] * xh[i];
        dg[i] += d * xh[i];
        db[i] += d;
      } else {
        xh[i] = 0.f; gd[i] = 0.f;
      }
    }
    const float a = wave_sum(s1) / (float)C, bb = wave_sum(s2) / (float)C;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int c = lane + 64 * i;
      if (c < C) {
        float v = rs * (gd[i] - a - xh[i] * bb);
        if (resid) v += to_f32(resid[row * C + c]);
        else if (accumulate) v += to_f32(dx[row * C + c]);
        dx[row * C + c] = from_f32<T>(v);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) { red[wave][0][lane + 64 * i] = dg[i]; red[wave][1][lane + 64 * i] = db[i]; }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += 256) {
    float sg = red[0][0][c] + red[1][0][c] + red[2][0][c] + red[3][0][c];
    float sb = red[0][1][c] + red[1][1][c] + red[2][1][c] + red[3][1][c];
    part[(int64_t)blockIdx.x * 2 * C + c] = sg;
    part[(int64_t)blockIdx.x * 2 * C + C + c] = sb;
  }
}

// Vectorised backward (C % 8 == 0, C <= 1024, 16-byte aligned): the lane
// layout of ln_fwd_vec_kernel, 64 rows per block as 64 / (4 * 64 / LPR)
// iterations of 256 / LPR rows.  The gamma/beta partials are summed over the
// row groups of a wave by xor shuffles, then over the 4 waves through LDS, in a
// fixed order.
template <typename T, int LPR, int NC>
__global__ __launch_bounds__(256) void ln_bwd_vec_kernel(const T* __restrict__ x,
                                                         const float* __restrict__ mean,
                                                         const float* __restrict__ rstd,
                                                         const float* __restrict__ g,
                                                         const float* __restrict__ dy, int64_t rows,
                                                         int C, const T* resid, int accumulate, T* dx,
                                                         float* __restrict__ part) {
  constexpr int RPI = 256 / LPR;  // rows per iteration of the block
  static_assert(LNB_ROWS % RPI == 0, "row groups must tile the block's rows");
  __shared__ float red[4][2][NC * LPR * 8];
  const int l = threadIdx.x & (LPR - 1), wave = threadIdx.x >> 6;
  float dg[NC][8], db[NC][8], gam[NC][8];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int c0 = (j * LPR + l) * 8;
    if (c0 < C) ld8(g + c0, gam[j]);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      dg[j][i] = 0.f;
      db[j][i] = 0.f;
      if (c0 >= C) gam[j][i] = 0.f;
    }
  }
  for (int it = 0; it < LNB_ROWS / RPI; ++it) {
    const int64_t row = (int64_t)blockIdx.x * LNB_ROWS + it * RPI + threadIdx.x / LPR;
    const bool ok = row < rows;
    const float mu = ok ? mean[row] : 0.f, rs = ok ? rstd[row] : 0.f;
    float xh[NC][8], d[NC][8];
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c0 = (j * LPR + l) * 8;
      if (ok && c0 < C) {
        ld8(x + row * C + c0, xh[j]);
        ld8(dy + row * C + c0, d[j]);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) { xh[j][i] = mu; d[j][i] = 0.f; }
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        xh[j][i] = (xh[j][i] - mu) * rs;
        const float gd = d[j][i] * gam[j][i];
        s1 += gd;
        s2 += gd * xh[j][i];
        dg[j][i] += d[j][i] * xh[j][i];
        db[j][i] += d[j][i];
      }
    }
    const float a = group_sum<LPR>(s1) / (float)C, bb = group_sum<LPR>(s2) / (float)C;
    if (!ok) continue;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c0 = (j * LPR + l) * 8;
      if (c0 >= C) continue;
      float v[8], r[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = rs * (d[j][i] * gam[j][i] - a - xh[j][i] * bb);
      if (resid) {
        ld8(resid + row * C + c0, r);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] += r[i];
      } else if (accumulate) {
        ld8(dx + row * C + c0, r);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] += r[i];
      }
      st8(dx + row * C + c0, v);
    }
  }
  // row groups of the wave -> lanes 0..LPR-1
#pragma unroll
  for (int o = LPR; o < 64; o <<= 1)
#pragma unroll
    for (int j = 0; j < NC; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        dg[j][i] += __shfl_xor(dg[j][i], o, 64);
        db[j][i] += __shfl_xor(db[j][i], o, 64);
      }
  if ((threadIdx.x & 63) < LPR)
#pragma unroll
    for (int j = 0; j < NC; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        red[wave][0][(j * LPR + l) * 8 + i] = dg[j][i];
        red[wave][1][(j * LPR + l) * 8 + i] = db[j][i];
      }
  __syncthreads();
  for (int cc = threadIdx.x; cc < C; cc += 256) {
    const float sg = (red[0][0][cc] + red[1][0][cc]) + (red[2][0][cc] + red[3][0][cc]);
    const float sb = (red[0][1][cc] + red[1][1][cc]) + (red[2][1][cc] + red[3][1][cc]);
    part[(int64_t)blockIdx.x * 2 * C + cc] = sg;
    part[(int64_t)blockIdx.x * 2 * C + C + cc] = sb;
  }
}

template <typename T, int LPR>
static void ln_bwd_vec_launch(const Ctx& c, double bytes, unsigned nblk, const T* x, const float* mean,
                              const float* rstd, const float* g, const float* dy, int64_t rows, int C,
                              const T* resid, int acc, T* dx, float* part) {
  if (C <= 8 * LPR)
    EVO_LAUNCH(EVO_KNAME("ln_bwd_vec_kernel", T), 0.0, bytes, (ln_bwd_vec_kernel<T, LPR, 1>), dim3(nblk), dim3(256), 0, c.stream, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part);
  else
    EVO_LAUNCH(EVO_KNAME("ln_bwd_vec_kernel", T), 0.0, bytes, (ln_bwd_vec_kernel<T, LPR, 2>), dim3(nblk), dim3(256), 0, c.stream, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part);
}

template <typename T>
evo_status_t ln_bwd(const Ctx& c, const T* x, const float* mean, const float* rstd, const float* g,
                    const float* dy, int64_t rows, int C, const T* resid, bool accumulate, T* dx,
                    float* part, int* nblk) {
  *nblk = (int)ln_bwd_partials(rows);
  if (c.dry || rows == 0) return EVO_OK;
  dim3 grid((unsigned)*nblk);
  const int acc = accumulate ? 1 : 0;
  if (C % 8 == 0 && C <= 1024 && aligned16(x) && aligned16(g) && aligned16(dy) && aligned16(dx) &&
      (!resid || aligned16(resid))) {
    const double bytes = (double)rows * C * (2 * sizeof(T) + 4.0 + ((resid || acc) ? sizeof(T) : 0)) + rows * 8.0;
    switch (ln_lanes(C)) {
      case 4: ln_bwd_vec_launch<T, 4>(c, bytes, grid.x, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part); break;
      case 8: ln_bwd_vec_launch<T, 8>(c, bytes, grid.x, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part); break;
      case 16: ln_bwd_vec_launch<T, 16>(c, bytes, grid.x, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part); break;
      case 32: ln_bwd_vec_launch<T, 32>(c, bytes, grid.x, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part); break;
      default: ln_bwd_vec_launch<T, 64>(c, bytes, grid.x, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part); break;
    }
    return check_launch("ln_bwd");
  }
  if (C <= 64) EVO_LAUNCH(EVO_KNAME("ln_bwd_kernel", T), 0.0, (double)rows * C * (2 * sizeof(T) + 4.0 + ((resid || acc) ? sizeof(T) : 0)) + rows * 8.0, (ln_bwd_kernel<T, 1>), grid, dim3(256), 0, c.stream, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part);
  else if (C <= 128) EVO_LAUNCH(EVO_KNAME("ln_bwd_kernel", T), 0.0, (double)rows * C * (2 * sizeof(T) + 4.0 + ((resid || acc) ? sizeof(T) : 0)) + rows * 8.0, (ln_bwd_kernel<T, 2>), grid, dim3(256), 0, c.stream, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part);
  else if (C <= 256) EVO_LAUNCH(EVO_KNAME("ln_bwd_kernel", T), 0.0, (double)rows * C * (2 * sizeof(T) + 4.0 + ((resid || acc) ? sizeof(T) : 0)) + rows * 8.0, (ln_bwd_kernel<T, 4>), grid, dim3(256), 0, c.stream, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part);
  else if (C <= 512) EVO_LAUNCH(EVO_KNAME("ln_bwd_kernel", T), 0.0, (double)rows * C * (2 * sizeof(T) + 4.0 + ((resid || acc) ? sizeof(T) : 0)) + rows * 8.0, (ln_bwd_kernel<T, 8>), grid, dim3(256), 0, c.stream, x, mean, rstd, g, dy, rows, C, resid, acc, dx, part);
  else { set_error("layernorm bwd: C=%d > 512", C); return EVO_ESHAPE; }
  return check_launch("ln_bwd");
}

// Channel-major backward: x[C][P] (compute type), dy[P][C] -> dx[C][P]; 64 positions per block.
int64_t ln_bwd_cm_partials(int64_t P) { return (P + 63) / 64; }

template <typename T>
__global__ __launch_bounds__(256) void ln_bwd_cm_kernel(const T* __restrict__ x,
                                                        const float* __restrict__ mean,
                                                        const float* __restrict__ rstd,
                                                        const float* __restrict__ g,
                                                        const float* __restrict__ dy, int64_t P,
                                                        int C, T* __restrict__ dx,
                                                        float* __restrict__ part) {
  extern __shared__ float sm[];  // tile [C][65] then red [4][2][C]
  float* tile = sm;
  float* red = sm + C * 65;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  cm_tile_load(x, P, C, p0, tile, tid);
  __syncthreads();
  // channels lane, lane + 64, ... (C <= 256): the parameter-gradient sums of
  // this wave's 16 positions stay in registers
  float rgs[4] = {0.f, 0.f, 0.f, 0.f}, rbs[4] = {0.f, 0.f, 0.f, 0.f}, gl[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) gl[k] = lane + 64 * k < C ? g[lane + 64 * k] : 0.f;
  for (int pp = wave * 16; pp < wave * 16 + 16; ++pp) {
    const int64_t p = p0 + pp;
    if (p >= P) break;
    const float mu = mean[p], rs = rstd[p];
    float d[4], xh[4];
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int cc = lane + 64 * k;
      d[k] = cc < C ? dy[p * C + cc] : 0.f;
      xh[k] = cc < C ? (tile[cc * 65 + pp] - mu) * rs : 0.f;
      const float gd = d[k] * gl[k];
      s1 += gd;
      s2 += gd * xh[k];
      rgs[k] += d[k] * xh[k];
      rbs[k] += d[k];
    }
    const float a = wave_sum(s1) / (float)C, bb = wave_sum(s2) / (float)C;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int cc = lane + 64 * k;
      if (cc < C) tile[cc * 65 + pp] = rs * (d[k] * gl[k] - a - xh[k] * bb);
    }
  }
  float* myred = red + wave * 2 * C;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int cc = lane + 64 * k;
    if (cc < C) { myred[cc] = rgs[k]; myred[C + cc] = rbs[k]; }
  }
  __syncthreads();
  cm_tile_store(dx, P, C, p0, tile, tid);
  for (int cc = tid; cc < C; cc += 256) {
    float sg = 0.f, sb = 0.f;
    for (int w = 0; w < 4; ++w) { sg += red[w * 2 * C + cc]; sb += red[w * 2 * C + C + cc]; }
    part[(int64_t)blockIdx.x * 2 * C + cc] = sg;
    part[(int64_t)blockIdx.x * 2 * C + C + cc] = sb;
  }
}

template <typename T>
evo_status_t ln_bwd_cm(const Ctx& c, const T* x, const float* mean, const float* rstd, const float* g,
                       const float* dy, int64_t P, int C, T* dx, float* part, int* nblk) {
  *nblk = (int)ln_bwd_cm_partials(P);
  if (c.dry || P == 0) return EVO_OK;
  if (C > 256) { set_error("layernorm bwd(cm): C=%d > 256", C); return EVO_ESHAPE; }
  size_t lds = ((size_t)C * 65 + 8 * C) * sizeof(float);
  EVO_LAUNCH(EVO_KNAME("ln_bwd_cm_kernel", T), 0.0, (double)P * C * (4.0 + 2.0 * sizeof(T)) + P * 8.0, (ln_bwd_cm_kernel<T>), dim3((unsigned)*nblk), dim3(256), lds, c.stream, x, mean,
                     rstd, g, dy, P, C, dx, part);
  return check_launch("ln_bwd_cm");
}

// ============================================================== reductions
// Deterministic column reductions out[j] (+)= sum_{i<n} part[i*ld + j] in a
// fixed order.  Wide problems: one thread per column.  Narrow, deep problems
// (few columns, many partials): a block of 8 columns x 32 row groups, each
// thread summing a strided subset of rows, then a fixed tree over the groups.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const float* __restrict__ part, int64_t n,
                                                              int64_t C, int64_t ld, float* out,
                                                              int accumulate) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= C) return;
  float s = 0.f;
  int64_t i = 0;
  for (; i + 4 <= n; i += 4) {   // four partials in flight, summed in order
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[(i + u) * ld + j];
#pragma unroll
    for (int u = 0; u < 4; ++u) s += v[u];
  }
  for (; i < n; ++i) s += part[i * ld + j];
  out[j] = accumulate ? out[j] + s : s;
}

constexpr int RN_COLS = 8, RN_ROWS = 32;

__global__ __launch_bounds__(256) void reduce_partials_narrow_kernel(const float* __restrict__ part, int64_t n,
                                                                     int64_t C, int64_t ld, float* out,
                                                                     int accumulate) {
  __shared__ float red[RN_ROWS][RN_COLS + 1];
  const int tc = threadIdx.x % RN_COLS, tr = threadIdx.x / RN_COLS;
  const int64_t j = (int64_t)blockIdx.x * RN_COLS + tc;
  float s = 0.f;
  if (j < C)
    for (int64_t i = tr; i < n; i += RN_ROWS) s += part[i * ld + j];
  red[tr][tc] = s;
  __syncthreads();
  for (int w = RN_ROWS / 2; w > 0; w >>= 1) {
    if (tr < w) red[tr][tc] += red[tr + w][tc];
    __syncthreads();
  }
  if (tr == 0 && j < C) out[j] = accumulate ? out[j] + red[0][tc] : red[0][tc];
}

evo_status_t reduce_partials(const Ctx& c, const float* part, int64_t n, int64_t C, int64_t ld,
                             float* out, bool accumulate) {
  if (c.dry || C == 0) return EVO_OK;
  const double bytes = ((double)n + 1) * C * 4.0;
  if (C >= 65536 || n < 64) {
    EVO_LAUNCH("reduce_partials_kernel", 0.0, bytes, reduce_partials_kernel, dim3((unsigned)((C + 255) / 256)),
               dim3(256), 0, c.stream, part, n, C, ld, out, accumulate ? 1 : 0);
  } else {
    EVO_LAUNCH("reduce_partials_narrow_kernel", 0.0, bytes, reduce_partials_narrow_kernel,
               dim3((unsigned)((C + RN_COLS - 1) / RN_COLS)), dim3(256), 0, c.stream, part, n, C, ld, out,
               accumulate ? 1 : 0);
  }
  return check_launch("reduce_partials");
}

// Segmented version: flattened column e = m * ld + c of a [M][ld] slice; each
// column finds its segment (if any) and writes out_s[m * n_s + c - off_s].
EVO_DEV int seg_of(const RedSegs& s, int c) {
  int r = -1;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k < s.nseg && c >= s.off[k] && c < s.off[k] + s.n[k]) r = k;
  return r;
}

__global__ __launch_bounds__(256) void reduce_segments_kernel(const float* __restrict__ part, int64_t n,
                                                              int64_t M, int64_t ld, RedSegs segs,
                                                              int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M * ld) return;
  const int64_t m = e / ld;
  const int c = (int)(e - m * ld);
  const int k = seg_of(segs, c);
  if (k < 0 || !segs.out[k]) return;
  float s = 0.f;
  for (int64_t i = 0; i < n; ++i) s += part[i * M * ld + e];
  float* o = segs.out[k] + m * segs.n[k] + (c - segs.off[k]);
  *o = accumulate ? *o + s : s;
}

__global__ __launch_bounds__(256) void reduce_segments_narrow_kernel(const float* __restrict__ part, int64_t n,
                                                                     int64_t M, int64_t ld, RedSegs segs,
                                                                     int accumulate) {
  __shared__ float red[RN_ROWS][RN_COLS + 1];
  const int tc = threadIdx.x % RN_COLS, tr = threadIdx.x / RN_COLS;
  const int64_t e = (int64_t)blockIdx.x * RN_COLS + tc;
  const bool in = e < M * ld;
  float s = 0.f;
  if (in)
    for (int64_t i = tr; i < n; i += RN_ROWS) s += part[i * M * ld + e];
  red[tr][tc] = s;
  __syncthreads();
  for (int w = RN_ROWS / 2; w > 0; w >>= 1) {
    if (tr < w) red[tr][tc] += red[tr + w][tc];
    __syncthreads();
  }
  if (tr != 0 || !in) return;
  const int64_t m = e / ld;
  const int c = (int)(e - m * ld);
  const int k = seg_of(segs, c);
  if (k < 0 || !segs.out[k]) return;
  float* o = segs.out[k] + m * segs.n[k] + (c - segs.off[k]);
  *o = accumulate ? *o + red[0][tc] : red[0][tc];
}

// Batched form: blocks [start_j, start_{j+1}) serve job j.  A job's block is
// (256 / rg) column threads x rg row groups; each thread sums 4 consecutive
// flattened columns over the partial rows i = tr (mod rg), and the rg group
// sums are added in order by the first group.
struct RedJobDev {
  const float* part;
  int64_t n, stride;
  int32_t E, ld, rg, vec4;
  RedSegs segs;
};
struct RedBatchArgs {
  int32_t njobs;
  int32_t start[RED_MAX_JOBS + 1];
  RedJobDev jobs[RED_MAX_JOBS];
};

__global__ __launch_bounds__(256) void reduce_batch_kernel(const RedBatchArgs a) {
  __shared__ f32x4 red[256];
  int j = 0;
  while (j + 1 < a.njobs && (int)blockIdx.x >= a.start[j + 1]) ++j;
  const float* part = a.jobs[j].part;
  const int64_t n = a.jobs[j].n, stride = a.jobs[j].stride;
  const int E = a.jobs[j].E, rg = a.jobs[j].rg;
  const int cw = 256 / rg;
  const int tc = threadIdx.x % cw, tr = threadIdx.x / cw;
  const int e0 = ((int)blockIdx.x - a.start[j]) * cw * 4 + tc * 4;
  f32x4 s = {0.f, 0.f, 0.f, 0.f};
  if (e0 < E) {
    if (a.jobs[j].vec4) {
      // four partials per lane in flight (same summation order): indices past
      // the end read partial n - 1 and count 0
      for (int64_t i0 = tr; i0 < n; i0 += 4 * rg) {
        f32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t i = i0 + u * rg;
          v[u] = *(const f32x4*)(part + (i < n ? i : n - 1) * stride + e0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float f = i0 + u * rg < n ? 1.f : 0.f;
#pragma unroll
          for (int q = 0; q < 4; ++q) s[q] = fmaf(v[u][q], f, s[q]);
        }
      }
    } else {
      for (int64_t i = tr; i < n; i += rg)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (e0 + q < E) s[q] += part[i * stride + e0 + q];
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (tr != 0 || e0 >= E) return;
  f32x4 t = red[tc];
  for (int r = 1; r < rg; ++r) t += red[r * cw + tc];
  const int ld = a.jobs[j].ld;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = e0 + q;
    if (e >= E) break;
    const int m = e / ld, cc = e - m * ld;
    const int k = seg_of(a.jobs[j].segs, cc);
    if (k < 0 || !a.jobs[j].segs.out[k]) continue;
    float* o = a.jobs[j].segs.out[k] + (int64_t)m * a.jobs[j].segs.n[k] + (cc - a.jobs[j].segs.off[k]);
    *o += t[q];
  }
}

evo_status_t flush_reductions(const Ctx& c, RedQueue& q) {
  if (c.dry || q.njobs == 0) { q.njobs = 0; return EVO_OK; }
  RedBatchArgs a;
  memset(&a, 0, sizeof(a));
  a.njobs = q.njobs;
  double bytes = 0.0;
  int nblk = 0;
  for (int j = 0; j < q.njobs; ++j) {
    const RedJob& J = q.jobs[j];
    RedJobDev& D = a.jobs[j];
    const int64_t E = J.M * J.ld;
    if (E >= (1LL << 30)) { set_error("reduce: %lld columns too many", (long long)E); return EVO_EINVAL; }
    D.part = J.part; D.n = J.n; D.stride = E; D.E = (int32_t)E; D.ld = (int32_t)J.ld; D.segs = J.segs;
    D.vec4 = (E % 4 == 0 && aligned16(J.part)) ? 1 : 0;
    // row groups: about 16 partial rows per thread, 1..64 groups
    int rg = 1;
    while (rg < 64 && J.n > 16 * rg) rg <<= 1;
    D.rg = rg;
    const int64_t cols_per_blk = (int64_t)(256 / rg) * 4;
    a.start[j] = nblk;
    nblk += (int)((E + cols_per_blk - 1) / cols_per_blk);
    bytes += ((double)J.n + 2.0) * E * 4.0;
  }
  a.start[q.njobs] = nblk;
  q.njobs = 0;
  EVO_LAUNCH("reduce_batch_kernel", 0.0, bytes, reduce_batch_kernel, dim3((unsigned)nblk), dim3(256), 0,
             c.stream, a);
  return check_launch("reduce_batch");
}

// Whether an output range of segs ([M][n_t] from out_t) overlaps one of a queued job.
static bool overlaps_queued(const RedQueue& q, int64_t M, const RedSegs& segs) {
  for (int j = 0; j < q.njobs; ++j)
    for (int s = 0; s < q.jobs[j].segs.nseg; ++s)
      for (int t = 0; t < segs.nseg; ++t) {
        const float* a0 = q.jobs[j].segs.out[s];
        const float* b0 = segs.out[t];
        if (!a0 || !b0) continue;
        const float* a1 = a0 + q.jobs[j].M * q.jobs[j].segs.n[s];
        const float* b1 = b0 + M * segs.n[t];
        if (a0 < b1 && b0 < a1) return true;
      }
  return false;
}

evo_status_t reduce_segments(const Ctx& c, const float* part, int64_t n, int64_t M, int64_t ld,
                             const RedSegs& segs, bool accumulate) {
  if (c.dry || M * ld == 0 || segs.nseg == 0) return EVO_OK;
  if (segs.nseg > 8) { set_error("reduce: %d segments > 8", segs.nseg); return EVO_EINVAL; }
  if (c.defer && accumulate && n > 0) {
    RedQueue& q = *c.defer;
    if (q.njobs == RED_MAX_JOBS || overlaps_queued(q, M, segs)) EVO_TRY(flush_reductions(c, q));
    RedJob& J = q.jobs[q.njobs++];
    J.part = part; J.n = n; J.M = M; J.ld = ld; J.segs = segs;
    return EVO_OK;
  }
  const int64_t C = M * ld;
  const double bytes = ((double)n + 1) * C * 4.0;
  if (C >= 65536 || n < 64) {
    EVO_LAUNCH("reduce_segments_kernel", 0.0, bytes, reduce_segments_kernel, dim3((unsigned)((C + 255) / 256)),
               dim3(256), 0, c.stream, part, n, M, ld, segs, accumulate ? 1 : 0);
  } else {
    EVO_LAUNCH("reduce_segments_narrow_kernel", 0.0, bytes, reduce_segments_narrow_kernel,
               dim3((unsigned)((C + RN_COLS - 1) / RN_COLS)), dim3(256), 0, c.stream, part, n, M, ld, segs,
               accumulate ? 1 : 0);
  }
  return check_launch("reduce_segments");
}

evo_status_t reduce_partials2(const Ctx& c, const float* part, int64_t n, int C, float* out_a,
                              float* out_b) {
  RedSegs s;
  s.nseg = 2;
  s.off[0] = 0; s.n[0] = C; s.out[0] = out_a;
  s.off[1] = C; s.n[1] = C; s.out[1] = out_b;
  return reduce_segments(c, part, n, 1, 2 * C, s, true);
}


// ============================================================== packing / fill
// Up to PACK_MAX parameter groups in one launch: blocks [start_g, start_{g+1})
// pack group g, one element (k, n) of its [K][sum n] concatenation per thread.
constexpr int PACK_MAX = 10;
struct PackBatch {
  PackArgs a[PACK_MAX];
  int32_t ntot[PACK_MAX];
  int32_t start[PACK_MAX + 1];
  int32_t n;
};

template <typename T>
__global__ __launch_bounds__(256) void pack_kernel(const PackBatch b) {
  int q = 0;
  while (q + 1 < b.n && (int)blockIdx.x >= b.start[q + 1]) ++q;
  const PackArgs& a = b.a[q];
  const int ntot = b.ntot[q];
  const int e = ((int)blockIdx.x - b.start[q]) * 256 + (int)threadIdx.x;
  if (e >= a.K * ntot) return;
  const int k = e / ntot, n = e - k * ntot;
  int s = 0, nl = n;
  while (s < a.nseg - 1 && nl >= a.seg[s].n) { nl -= a.seg[s].n; ++s; }
  const float v = a.seg[s].w[(int64_t)k * a.seg[s].n + nl];
  if (a.dst) ((T*)a.dst)[(int64_t)k * ntot + n] = from_f32<T>(v);
  if (a.dst_t) ((T*)a.dst_t)[(int64_t)n * a.K + k] = from_f32<T>(v);
  if (a.bias && k == 0) a.bias[n] = a.seg[s].bias ? a.seg[s].bias[nl] : 0.f;
}

bool PackCache::find(PackArgs& a) const {
  for (int i = 0; i < n; ++i) {
    const PackArgs& h = e[i];
    if (h.K != a.K || h.nseg != a.nseg) continue;
    if ((a.dst && !h.dst) || (a.dst_t && !h.dst_t) || (a.bias && !h.bias)) continue;
    bool same = true;
    for (int s = 0; s < a.nseg; ++s)
      same = same && h.seg[s].w == a.seg[s].w && h.seg[s].n == a.seg[s].n &&
             (!a.bias || h.seg[s].bias == a.seg[s].bias);
    if (!same) continue;
    if (a.dst) a.dst = h.dst;
    if (a.dst_t) a.dst_t = h.dst_t;
    if (a.bias) a.bias = h.bias;
    return true;
  }
  return false;
}

template <typename T>
evo_status_t pack_groups(const Ctx& c, PackArgs* const* g, int ng) {
  if (c.dry) return EVO_OK;
  for (int i0 = 0; i0 < ng; i0 += PACK_MAX) {
    PackBatch b;
    memset(&b, 0, sizeof(b));
    double bytes = 0.0;
    int nblk = 0;
    for (int i = i0; i < ng && i < i0 + PACK_MAX; ++i) {
      const PackArgs* a = g[i];
      EVO_CHECK_ARG(a->nseg >= 1 && a->nseg <= 5, EVO_EINVAL, "pack: %d segments", a->nseg);
      int ntot = 0;
      for (int s = 0; s < a->nseg; ++s) {
        EVO_CHECK_ARG(a->seg[s].w != nullptr, EVO_EINVAL, "null parameter pointer (segment %d)", s);
        ntot += a->seg[s].n;
      }
      const int64_t n = (int64_t)a->K * ntot;
      EVO_CHECK_ARG(n < (1LL << 30), EVO_EINVAL, "pack: %lld elements too many", (long long)n);
      b.a[b.n] = *a;
      b.ntot[b.n] = ntot;
      b.start[b.n] = nblk;
      ++b.n;
      nblk += (int)((n + 255) / 256);
      bytes += (double)n * (4.0 + sizeof(T) * ((a->dst ? 1 : 0) + (a->dst_t ? 1 : 0)));
    }
    b.start[b.n] = nblk;
    if (nblk == 0) continue;
    EVO_LAUNCH(EVO_KNAME("pack_kernel", T), 0.0, bytes, (pack_kernel<T>), dim3((unsigned)nblk), dim3(256), 0, c.stream, b);
    EVO_TRY(check_launch("pack_params"));
  }
  return EVO_OK;
}

template <typename T>
evo_status_t pack_params(const Ctx& c, std::initializer_list<PackArgs*> list) {
  if (c.dry) return EVO_OK;
  PackArgs* todo[8];
  int n = 0;
  EVO_CHECK_ARG(list.size() <= 8, EVO_EINVAL, "pack: %zu groups", list.size());
  for (PackArgs* a : list)
    if (!(c.packed && c.packed->find(*a))) todo[n++] = a;
  return pack_groups<T>(c, todo, n);
}

template <typename T>
__global__ __launch_bounds__(256) void fill_zero_kernel(T* p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = from_f32<T>(0.f);
}

template <typename T>
evo_status_t fill_zero(const Ctx& c, T* p, int64_t n) {
  if (c.dry || n == 0) return EVO_OK;
  EVO_LAUNCH(EVO_KNAME("fill_zero_kernel", T), 0.0, (double)n * sizeof(T), (fill_zero_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, p, n);
  return check_launch("fill_zero");
}

template <typename T>
__global__ __launch_bounds__(256) void copy_kernel(const T* __restrict__ s, T* __restrict__ d, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) d[e] = s[e];
}

template <typename T>
evo_status_t copy_elems(const Ctx& c, const T* src, T* dst, int64_t n) {
  if (c.dry || n == 0 || src == dst) return EVO_OK;
  if (n % 8 == 0 && aligned16(src) && aligned16(dst)) return convert_elems<T, T>(c, src, dst, n);
  EVO_LAUNCH(EVO_KNAME("copy_kernel", T), 0.0, (double)n * 2 * sizeof(T), (copy_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, src, dst, n);
  return check_launch("copy");
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void convert_kernel(const TI* __restrict__ s, TO* __restrict__ d, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) d[e] = from_f32<TO>(to_f32(s[e]));
}

// EPT elements per thread: 8 when narrowing, 4 when widening, so that a
// wave's widening stores are contiguous 16-byte pieces lane after lane
// (measured faster; narrowing measured faster with 8).
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void convert_vec_kernel(const TI* __restrict__ s, TO* __restrict__ d, int64_t nv) {
  constexpr int EPT = sizeof(TI) < sizeof(TO) ? 4 : 8;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nv) return;
  if constexpr (EPT == 4) {
    const bf16x4 a = *(const bf16x4*)(s + e * 4);
    store4<TO>(d + e * 4, f32x4{(float)a[0], (float)a[1], (float)a[2], (float)a[3]});
  } else {
    float v[8];
    ld8(s + e * 8, v);
    st8(d + e * 8, v);
  }
}

template <typename TI, typename TO>
evo_status_t convert_elems(const Ctx& c, const TI* src, TO* dst, int64_t n) {
  if (c.dry || n == 0) return EVO_OK;
  constexpr int EPT = sizeof(TI) < sizeof(TO) ? 4 : 8;
  if (n % 8 == 0 && aligned16(src) && aligned16(dst)) {
    const int64_t nv = n / EPT;
    EVO_LAUNCH(EVO_KNAME("convert_vec_kernel", TO), 0.0, (double)n * (sizeof(TI) + sizeof(TO)),
               (convert_vec_kernel<TI, TO>), dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, c.stream, src, dst, nv);
    return check_launch("convert");
  }
  EVO_LAUNCH(EVO_KNAME("convert_kernel", TO), 0.0, (double)n * (sizeof(TI) + sizeof(TO)),
             (convert_kernel<TI, TO>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, src, dst, n);
  return check_launch("convert");
}

// ============================================================== attention gate backward
template <typename T>
__global__ __launch_bounds__(256) void gate_bwd_kernel(int64_t rows, int H, int hd, const float* dgo,
                                                       int64_t ld_dgo, const float* o,
                                                       int64_t ld_o,
                                                       const T* g, int64_t ld_g, T* dctx,
                                                       int64_t ld_dctx, T* dgp, int64_t ld_dg,
                                                       float* D) {
  const int HC = H * hd;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = e / HC;
  const int col = (int)(e % HC);
  float contrib = 0.f;
  if (row < rows) {
    const float dy = dgo[row * ld_dgo + col];
    const float ov = to_f32(o[row * ld_o + col]);
    const float gv = to_f32(g[row * ld_g + col]);
    const float dc = dy * gv;
    dctx[row * ld_dctx + col] = from_f32<T>(dc);
    dgp[row * ld_dg + col] = from_f32<T>(dy * ov * gv * (1.f - gv));
    contrib = to_f32(from_f32<T>(dc)) * ov;
  }
  // head_dim lanes are consecutive and aligned inside the wave (hd | 64)
  for (int off = hd >> 1; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off, 64);
  if (row < rows && (col % hd) == 0) D[row * H + col / hd] = contrib;
}

// Vector form: a lane takes 8 consecutive columns of one head (hd / 8 = LPH
// lanes per head, consecutive and aligned inside the wave).
template <typename T, int LPH>
__global__ __launch_bounds__(256) void gate_bwd_vec_kernel(int64_t rows, int H, int hd, const float* dgo,
                                                           int64_t ld_dgo, const float* o,
                                                           int64_t ld_o,
                                                           const T* g, int64_t ld_g, T* dctx,
                                                           int64_t ld_dctx, T* dgp, int64_t ld_dg,
                                                           float* D) {
  const int HC8 = H * hd / 8;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = e / HC8;
  const int col = (int)(e % HC8) * 8;
  float contrib = 0.f;
  if (row < rows) {
    float dy[8], ov[8], gv[8], dc[8], dg[8];
    ld8(dgo + row * ld_dgo + col, dy);
    ld8(o + row * ld_o + col, ov);
    ld8(g + row * ld_g + col, gv);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      dc[i] = dy[i] * gv[i];
      dg[i] = dy[i] * ov[i] * gv[i] * (1.f - gv[i]);
      contrib += to_f32(from_f32<T>(dc[i])) * ov[i];
    }
    st8(dctx + row * ld_dctx + col, dc);
    st8(dgp + row * ld_dg + col, dg);
  }
  contrib = group_sum<LPH>(contrib);
  if (row < rows && (col % hd) == 0) D[row * H + col / hd] = contrib;
}

template <typename T>
evo_status_t gate_bwd(const Ctx& c, int64_t rows, int H, int hd, const float* dgo, int64_t ld_dgo,
                      const float* o, int64_t ld_o, const T* g, int64_t ld_g, T* dctx,
                      int64_t ld_dctx, T* dgpre, int64_t ld_dg, float* D) {
  if (c.dry || rows == 0) return EVO_OK;
  const int64_t n = rows * H * hd;
  const bool vec = (hd == 8 || hd == 16 || hd == 32 || hd == 64) && ld_dgo % 8 == 0 && ld_o % 8 == 0 && ld_g % 8 == 0 &&
                   ld_dctx % 8 == 0 && ld_dg % 8 == 0 && aligned16(dgo) && aligned16(o) && aligned16(g) &&
                   aligned16(dctx) && aligned16(dgpre);
  if (vec) {
    const int64_t n8 = n / 8;
    const dim3 grid((unsigned)((n8 + 255) / 256));
    const double bytes = (double)n * (8.0 + 3 * sizeof(T)) + rows * H * 4.0;
    switch (hd / 8) {
      case 1:
        EVO_LAUNCH(EVO_KNAME("gate_bwd_vec_kernel", T), 0.0, bytes, (gate_bwd_vec_kernel<T, 1>), grid, dim3(256), 0,
                   c.stream, rows, H, hd, dgo, ld_dgo, o, ld_o, g, ld_g, dctx, ld_dctx, dgpre, ld_dg, D);
        break;
      case 2:
        EVO_LAUNCH(EVO_KNAME("gate_bwd_vec_kernel", T), 0.0, bytes, (gate_bwd_vec_kernel<T, 2>), grid, dim3(256), 0,
                   c.stream, rows, H, hd, dgo, ld_dgo, o, ld_o, g, ld_g, dctx, ld_dctx, dgpre, ld_dg, D);
        break;
      case 4:
        EVO_LAUNCH(EVO_KNAME("gate_bwd_vec_kernel", T), 0.0, bytes, (gate_bwd_vec_kernel<T, 4>), grid, dim3(256), 0,
                   c.stream, rows, H, hd, dgo, ld_dgo, o, ld_o, g, ld_g, dctx, ld_dctx, dgpre, ld_dg, D);
        break;
      default:
        EVO_LAUNCH(EVO_KNAME("gate_bwd_vec_kernel", T), 0.0, bytes, (gate_bwd_vec_kernel<T, 8>), grid, dim3(256), 0,
                   c.stream, rows, H, hd, dgo, ld_dgo, o, ld_o, g, ld_g, dctx, ld_dctx, dgpre, ld_dg, D);
        break;
    }
    return check_launch("gate_bwd");
  }
  EVO_LAUNCH(EVO_KNAME("gate_bwd_kernel", T), 0.0, (double)n * (4.0 + 4 * sizeof(T)) + rows * H * 4.0, (gate_bwd_kernel<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream,
                     rows, H, hd, dgo, ld_dgo, o, ld_o, g, ld_g, dctx, ld_dctx, dgpre, ld_dg, D);
  return check_launch("gate_bwd");
}

// ============================================================== triangle multiplication glue
// Tiles of 64 positions x 32 channels, transposed through LDS so that both the
// row-major projection output and the channel-major operands move coalesced.
template <typename T>
__global__ __launch_bounds__(256) void trimul_proj_kernel(int64_t P, int ch, int cz, const T* raw,
                                                          const float* mask, T* a, T* b, int64_t ld_ab) {
  __shared__ float ta[32][65], tb[32][65];
  const int tid = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 32;
  const int ld = 4 * ch + cz;
  for (int e = tid; e < 64 * 32; e += 256) {
    const int pp = e >> 5, cc = e & 31;
    const int64_t p = p0 + pp;
    const int c = c0 + cc;
    float va = 0.f, vb = 0.f;
    if (p < P && c < ch) {
      const T* r = raw + p * ld;
      const float mk = mask ? mask[p] : 1.f;
      va = mk * sigmoidf_(to_f32(r[ch + c])) * to_f32(r[c]);
      vb = mk * sigmoidf_(to_f32(r[3 * ch + c])) * to_f32(r[2 * ch + c]);
    }
    ta[cc][pp] = va;
    tb[cc][pp] = vb;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 32; e += 256) {
    const int cc = e >> 6, pp = e & 63;
    const int64_t p = p0 + pp;
    const int c = c0 + cc;
    if (p < P && c < ch) {
      a[(int64_t)c * ld_ab + p] = from_f32<T>(ta[cc][pp]);
      b[(int64_t)c * ld_ab + p] = from_f32<T>(tb[cc][pp]);
    }
  }
}

// Vector form (ch, cz multiples of 8; ld_ab a multiple of 8; 16-byte
// aligned): tiles of 64 positions x 64 channels; raw is read as 16-byte
// vectors of 8 channels, a and b are written as 16-byte vectors of 8
// positions.
template <typename T>
__global__ __launch_bounds__(256) void trimul_proj_vec_kernel(int64_t P, int ch, int cz, const T* raw,
                                                              const float* mask, T* a, T* b, int64_t ld_ab) {
  __shared__ float ta[64][65], tb[64][65];
  const int tid = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int ld = 4 * ch + cz;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int item = tid + 256 * k;
    const int pp = item >> 3, cg = (item & 7) * 8;
    const int64_t p = p0 + pp;
    const int c = c0 + cg;
    float va[8], vb[8];
    if (p < P && c < ch) {
      const T* r = raw + p * ld;
      const float mk = mask ? mask[p] : 1.f;
      float ap[8], ag[8], bp[8], bg[8];
      ld8(r + c, ap);
      ld8(r + ch + c, ag);
      ld8(r + 2 * ch + c, bp);
      ld8(r + 3 * ch + c, bg);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        va[i] = mk * sigmoidf_(ag[i]) * ap[i];
        vb[i] = mk * sigmoidf_(bg[i]) * bp[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) va[i] = vb[i] = 0.f;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      ta[cg + i][pp] = va[i];
      tb[cg + i][pp] = vb[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int item = tid + 256 * k;
    const int cc = item >> 3, pg = (item & 7) * 8;
    const int64_t p = p0 + pg;
    const int c = c0 + cc;
    if (c >= ch || p >= P) continue;
    float va[8], vb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      va[i] = ta[cc][pg + i];
      vb[i] = tb[cc][pg + i];
    }
    if (p + 8 <= P) {
      st8(a + (int64_t)c * ld_ab + p, va);
      st8(b + (int64_t)c * ld_ab + p, vb);
    } else {
      for (int i = 0; p + i < P; ++i) {
        a[(int64_t)c * ld_ab + p + i] = from_f32<T>(va[i]);
        b[(int64_t)c * ld_ab + p + i] = from_f32<T>(vb[i]);
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gate_cols_kernel(int64_t P, int ch, int cz, const T* raw, float* g) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= P * cz) return;
  const int64_t p = e / cz;
  const int n = (int)(e % cz);
  g[e] = to_f32(raw[p * (4 * ch + cz) + 4 * ch + n]);
}

template <typename T>
evo_status_t trimul_proj(const Ctx& c, int64_t P, int ch, int cz, const T* raw, const float* mask,
                         T* a, T* b, int64_t ld_ab, float* g) {
  if (c.dry || P == 0) return EVO_OK;
  if (ch % 8 == 0 && cz % 8 == 0 && ld_ab % 8 == 0 && aligned16(raw) && aligned16(a) && aligned16(b)) {
    dim3 grid((unsigned)((P + 63) / 64), (unsigned)((ch + 63) / 64));
    EVO_LAUNCH(EVO_KNAME("trimul_proj_vec_kernel", T), 0.0, (double)P * ch * (16.0 + 2 * sizeof(T)),
               (trimul_proj_vec_kernel<T>), grid, dim3(256), 0, c.stream, P, ch, cz, raw, mask, a, b, ld_ab);
  } else {
    dim3 grid((unsigned)((P + 63) / 64), (unsigned)((ch + 31) / 32));
    EVO_LAUNCH(EVO_KNAME("trimul_proj_kernel", T), 0.0, (double)P * ch * (16.0 + 2 * sizeof(T)), (trimul_proj_kernel<T>), grid, dim3(256), 0, c.stream, P, ch, cz, raw, mask, a, b, ld_ab);
  }
  EVO_TRY(check_launch("trimul_proj"));
  if (!g) return EVO_OK;
  const int64_t n = P * cz;
  EVO_LAUNCH(EVO_KNAME("gate_cols_kernel", T), 0.0, (double)n * (4.0 + sizeof(T)), (gate_cols_kernel<T>),
             dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, P, ch, cz, raw, g);
  return check_launch("trimul_gate");
}

template <typename T>
__global__ __launch_bounds__(256) void trimul_proj_bwd_kernel(int64_t P, int ch, int cz, const T* raw,
                                                              const float* mask, const float* da,
                                                              const float* db, T* draw) {
  __shared__ float ta[32][65], tb[32][65];
  const int tid = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 32;
  const int ld = 4 * ch + cz;
  for (int e = tid; e < 64 * 32; e += 256) {
    const int cc = e >> 6, pp = e & 63;
    const int64_t p = p0 + pp;
    const int c = c0 + cc;
    ta[cc][pp] = (p < P && c < ch) ? da[(int64_t)c * P + p] : 0.f;
    tb[cc][pp] = (p < P && c < ch) ? db[(int64_t)c * P + p] : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 32; e += 256) {
    const int pp = e >> 5, cc = e & 31;
    const int64_t p = p0 + pp;
    const int c = c0 + cc;
    if (p < P && c < ch) {
      const T* r = raw + p * ld;
      T* d = draw + p * ld;
      const float mk = mask ? mask[p] : 1.f;
      const float ap = to_f32(r[c]), sa = sigmoidf_(to_f32(r[ch + c]));
      const float bp = to_f32(r[2 * ch + c]), sb = sigmoidf_(to_f32(r[3 * ch + c]));
      const float dav = ta[cc][pp] * mk, dbv = tb[cc][pp] * mk;
      d[c] = from_f32<T>(dav * sa);
      d[ch + c] = from_f32<T>(dav * ap * sa * (1.f - sa));
      d[2 * ch + c] = from_f32<T>(dbv * sb);
      d[3 * ch + c] = from_f32<T>(dbv * bp * sb * (1.f - sb));
    }
  }
}

template <typename T>
evo_status_t trimul_proj_bwd(const Ctx& c, int64_t P, int ch, int cz, const T* raw,
                             const float* mask, const float* da, const float* db, T* draw) {
  if (c.dry || P == 0) return EVO_OK;
  dim3 grid((unsigned)((P + 63) / 64), (unsigned)((ch + 31) / 32));
  EVO_LAUNCH(EVO_KNAME("trimul_proj_bwd_kernel", T), 0.0, (double)P * ch * (24.0 + 4 * sizeof(T)), (trimul_proj_bwd_kernel<T>), grid, dim3(256), 0, c.stream, P, ch, cz, raw, mask, da, db, draw);
  return check_launch("trimul_proj_bwd");
}

template <typename T, typename X>
__global__ __launch_bounds__(256) void trimul_gate_bwd_kernel(int64_t P, int ch, int cz, const X* dz,
                                                              const float* t, const T* g, int64_t ld_g,
                                                              T* dt, T* draw) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= P * cz) return;
  const int64_t p = e / cz;
  const int n = (int)(e % cz);
  const float d = to_f32(dz[e]), gv = to_f32(g[p * ld_g + n]), tv = t[e];
  dt[e] = from_f32<T>(d * gv);
  draw[p * (4 * ch + cz) + 4 * ch + n] = from_f32<T>(d * tv * gv * (1.f - gv));
}

// Vector form: 8 consecutive channels per lane (cz, ch, ld_g multiples of 8).
template <typename T, typename X>
__global__ __launch_bounds__(256) void trimul_gate_bwd_vec_kernel(int64_t P, int ch, int cz, const X* dz,
                                                                  const float* t, const T* g, int64_t ld_g,
                                                                  T* dt, T* draw) {
  const int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8;
  if (e >= P * cz) return;
  const int64_t p = e / cz;
  const int n = (int)(e - p * cz);
  float d[8], gv[8], tv[8], o1[8], o2[8];
  ld8(dz + e, d);
  ld8(g + p * ld_g + n, gv);
  ld8(t + e, tv);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    o1[i] = d[i] * gv[i];
    o2[i] = d[i] * tv[i] * gv[i] * (1.f - gv[i]);
  }
  st8(dt + e, o1);
  st8(draw + p * (4 * ch + cz) + 4 * ch + n, o2);
}

template <typename T, typename X>
evo_status_t trimul_gate_bwd(const Ctx& c, int64_t P, int ch, int cz, const X* dz, const float* t,
                             const T* g, int64_t ld_g, T* dt, T* draw) {
  if (c.dry || P == 0) return EVO_OK;
  const int64_t n = P * cz;
  if (cz % 8 == 0 && ch % 8 == 0 && ld_g % 8 == 0 && aligned16(dz) && aligned16(t) && aligned16(g) &&
      aligned16(dt) && aligned16(draw)) {
    const int64_t n8 = n / 8;
    EVO_LAUNCH(EVO_KNAME("trimul_gate_bwd_vec_kernel", X), 0.0, (double)n * (sizeof(X) + 8.0 + 2 * sizeof(T)),
               (trimul_gate_bwd_vec_kernel<T, X>), dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, c.stream, P,
               ch, cz, dz, t, g, ld_g, dt, draw);
    return check_launch("trimul_gate_bwd");
  }
  EVO_LAUNCH(EVO_KNAME("trimul_gate_bwd_kernel", X), 0.0, (double)n * (sizeof(X) + 8.0 + 2 * sizeof(T)), (trimul_gate_bwd_kernel<T, X>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     c.stream, P, ch, cz, dz, t, g, ld_g, dt, draw);
  return check_launch("trimul_gate_bwd");
}

// ============================================================== outer product mean count
// One thread per 4 consecutive p of one (s, i): the split partials are summed in order.
template <typename T>
__global__ __launch_bounds__(256) void opm_dab_reduce_kernel(const float* __restrict__ part, int nsplit,
                                                             int64_t S, int64_t R, int ch,
                                                             const float* __restrict__ mask, T* dab, int off) {
  const int64_t n = S * R * ch;
  const int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (e >= n) return;
  f32x4 v = *(const f32x4*)(part + e);
  for (int k = 1; k < nsplit; ++k) v += *(const f32x4*)(part + (int64_t)k * n + e);
  const int64_t si = e / ch;           // s * R + i
  const int p = (int)(e - si * ch);
  if (mask) v *= mask[si];
  store4<T>(dab + si * 2 * ch + off + p, v);
}

template <typename T>
evo_status_t opm_dab_reduce(const Ctx& c, const float* part, int nsplit, int64_t S, int64_t R, int ch,
                            const float* mask, T* dab, int off) {
  if (c.dry) return EVO_OK;
  if (ch % 4) { set_error("outer product mean: c_hidden %d not a multiple of 4", ch); return EVO_ESHAPE; }
  const int64_t q = S * R * ch / 4;
  EVO_LAUNCH(EVO_KNAME("opm_dab_reduce_kernel", T), 0.0, (double)S * R * ch * (4.0 * nsplit + sizeof(T)),
             (opm_dab_reduce_kernel<T>), dim3((unsigned)((q + 255) / 256)), dim3(256), 0, c.stream, part, nsplit,
             S, R, ch, mask, dab, off);
  return check_launch("opm_dab_reduce");
}

// A block owns 16 x 16 outputs (i, j); chunks of 64 mask rows s for its 16
// columns i and 16 columns j are staged in LDS, and each thread sums its
// products over s in order.
constexpr int OPN_S = 64;
__global__ __launch_bounds__(256) void opm_norm_kernel(const float* __restrict__ mask, int64_t S, int64_t R,
                                                       float eps, float* __restrict__ scale) {
  __shared__ float si[OPN_S][16], sj[OPN_S][16];
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  const int64_t i0 = (int64_t)blockIdx.y * 16, j0 = (int64_t)blockIdx.x * 16;
  const int64_t i = i0 + ti, j = j0 + tj;
  float n = 0.f;
  if (mask) {
    for (int64_t s0 = 0; s0 < S; s0 += OPN_S) {
      __syncthreads();
      for (int e = tid; e < OPN_S * 16; e += 256) {
        const int ss = e >> 4, t = e & 15;
        const bool sok = s0 + ss < S;
        si[ss][t] = (sok && i0 + t < R) ? mask[(s0 + ss) * R + i0 + t] : 0.f;
        sj[ss][t] = (sok && j0 + t < R) ? mask[(s0 + ss) * R + j0 + t] : 0.f;
      }
      __syncthreads();
      const int ns = S - s0 < OPN_S ? (int)(S - s0) : OPN_S;
      for (int ss = 0; ss < ns; ++ss) n += si[ss][ti] * sj[ss][tj];
    }
  } else {
    n = (float)S;
  }
  if (i < R && j < R) scale[i * R + j] = 1.0f / (eps + n);
}

evo_status_t opm_norm(const Ctx& c, const float* mask, int64_t S, int64_t R, float eps, float* scale) {
  if (c.dry) return EVO_OK;
  const unsigned nb = (unsigned)((R + 15) / 16);
  EVO_LAUNCH("opm_norm_kernel", 2.0 * (double)S * R * R, (double)R * R * 4.0 + (mask ? (double)S * R * 4.0 : 0.0), opm_norm_kernel, dim3(nb, nb), dim3(256), 0, c.stream, mask, S,
                     R, eps, scale);
  return check_launch("opm_norm");
}

// ============================================================== instantiations
#define EVO_INST(T)                                                                                \
  template evo_status_t ln_fwd<T, T>(const Ctx&, const T*, int64_t, int, const float*, const float*, \
                                     float, T*, float*, float*);                                   \
  template evo_status_t ln_fwd_rows<T, T>(const Ctx&, const T*, int64_t, int, int, int64_t,         \
                                          const float*, const float*, float, T*, float*, float*);  \
  template evo_status_t ln_rowproj<T, T>(const Ctx&, const T*, int64_t, int, const float*,         \
                                         const float*, float, const float*, int, float*, float,    \
                                         int64_t);                                                 \
  template evo_status_t ln_fwd_cm<T>(const Ctx&, const T*, int64_t, int, const float*,             \
                                     const float*, float, T*, float*, float*);                     \
  template evo_status_t ln_bwd<T>(const Ctx&, const T*, const float*, const float*, const float*,  \
                                  const float*, int64_t, int, const T*, bool, T*, float*, int*);   \
  template evo_status_t ln_bwd_cm<T>(const Ctx&, const T*, const float*, const float*,             \
                                     const float*, const float*, int64_t, int, T*, float*, int*);  \
  template evo_status_t opm_dab_reduce<T>(const Ctx&, const float*, int, int64_t, int64_t, int,       \
                                          const float*, T*, int);                                  \
  template evo_status_t pack_params<T>(const Ctx&, std::initializer_list<PackArgs*>);              \
  template evo_status_t pack_groups<T>(const Ctx&, PackArgs* const*, int);                         \
  template evo_status_t fill_zero<T>(const Ctx&, T*, int64_t);                                     \
  template evo_status_t copy_elems<T>(const Ctx&, const T*, T*, int64_t);                          \
  template evo_status_t gate_bwd<T>(const Ctx&, int64_t, int, int, const float*, int64_t,                \
                                    const float*, int64_t, const T*, int64_t, T*,   \
                                    int64_t, T*, int64_t, float*);                                       \
  template evo_status_t trimul_proj<T>(const Ctx&, int64_t, int, int, const T*, const float*,      \
                                       T*, T*, int64_t, float*);                                   \
  template evo_status_t trimul_proj_bwd<T>(const Ctx&, int64_t, int, int, const T*,               \
                                           const float*, const float*, const float*, T*);          \
  template evo_status_t trimul_gate_bwd<T, T>(const Ctx&, int64_t, int, int, const T*,           \
                                              const float*, const T*, int64_t, T*, T*);

EVO_INST(float)
EVO_INST(bf16)

// mixed: FP32 residual stream around BF16 compute
template evo_status_t ln_fwd<float, bf16>(const Ctx&, const float*, int64_t, int, const float*, const float*,
                                          float, bf16*, float*, float*);
template evo_status_t ln_fwd_rows<float, bf16>(const Ctx&, const float*, int64_t, int, int, int64_t,
                                               const float*, const float*, float, bf16*, float*, float*);
template evo_status_t ln_rowproj<float, bf16>(const Ctx&, const float*, int64_t, int, const float*,
                                              const float*, float, const float*, int, float*, float, int64_t);
template evo_status_t trimul_gate_bwd<bf16, float>(const Ctx&, int64_t, int, int, const float*, const float*,
                                                   const bf16*, int64_t, bf16*, bf16*);
template evo_status_t convert_elems<float, bf16>(const Ctx&, const float*, bf16*, int64_t);
template evo_status_t convert_elems<bf16, float>(const Ctx&, const bf16*, float*, int64_t);
template evo_status_t convert_elems<float, float>(const Ctx&, const float*, float*, int64_t);
template evo_status_t convert_elems<bf16, bf16>(const Ctx&, const bf16*, bf16*, int64_t);

}  // namespace evo
