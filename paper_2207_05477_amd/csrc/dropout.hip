// Training dropout of the residual updates (AlphaFold2's shared dropout, which
// the paper keeps by following AlphaFold2's settings, Section "Hyperparameter
// setting"): one multiplier per (row or column index, channel), shared along
// the other axis of the update, 0 for a dropped element and 1 / (1 - rate) for
// a kept one.
//
// The multipliers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011), a counter-based
// generator: element e of a sub-operation's table draws output word 0 at the
// counter (e, word, offset_lo, offset_hi) under the key (seed_lo, seed_hi),
// where word = sub-operation number | template index << 8, and is kept when
// that 32-bit draw is at least floor(rate * 2^32).  A table is tiny ([R, C])
// and is formed once per call; the GEMM epilogue that adds the update to the
// residual multiplies by it (a broadcast read from L2), and the backward scales
// the incoming gradient by it before the sub-operation's own backward.
#include "ops.h"

namespace evo {

// Ten rounds: multiply counter words 0 and 2 by the round constants, swap, xor
// the high halves with the other words and the key; the key is bumped by the
// Weyl constants between rounds.
EVO_DEV uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += kW0; k1 += kW1; }
    const uint32_t lo0 = kM0 * c.x, hi0 = __umulhi(kM0, c.x);
    const uint32_t lo1 = kM1 * c.z, hi1 = __umulhi(kM1, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

struct DropTableArgs {
  int32_t n = 0;
  float* out[8];
  int64_t len[8];
  uint32_t word[8];
  uint32_t thresh[8];
  float scale[8];
  uint32_t key0, key1, off0, off1;
};

__global__ __launch_bounds__(256) void dropout_table_kernel(DropTableArgs a) {
  const int t = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.len[t]) return;
  const uint4 r = philox4x32_10(make_uint4((uint32_t)e, a.word[t], a.off0, a.off1), a.key0, a.key1);
  a.out[t][e] = r.x >= a.thresh[t] ? a.scale[t] : 0.0f;
}

// Integer threshold of a rate given as FP32: keep when the draw >= floor(rate * 2^32).
static uint32_t keep_threshold(float rate) {
  const double t = floor((double)rate * 4294967296.0);
  return t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
}

evo_status_t dropout_tables(const Ctx& c, uint64_t seed, uint64_t offset, int n, float* const* out,
                            const int64_t* len, const uint32_t* word, const float* rate) {
  if (c.dry || n == 0) return EVO_OK;
  if (n > 8) { set_error("dropout: more than 8 tables"); return EVO_EINVAL; }
  DropTableArgs a;
  a.n = n;
  int64_t mx = 0;
  double bytes = 0;
  for (int i = 0; i < n; ++i) {
    a.out[i] = out[i];
    a.len[i] = len[i];
    a.word[i] = word[i];
    a.thresh[i] = keep_threshold(rate[i]);
    a.scale[i] = (float)(1.0 / (1.0 - (double)rate[i]));
    mx = len[i] > mx ? len[i] : mx;
    bytes += 4.0 * len[i];
  }
  a.key0 = (uint32_t)seed; a.key1 = (uint32_t)(seed >> 32);
  a.off0 = (uint32_t)offset; a.off1 = (uint32_t)(offset >> 32);
  if (mx == 0) return EVO_OK;
  EVO_LAUNCH("dropout_table_kernel", 0.0, bytes, dropout_table_kernel, dim3((unsigned)((mx + 255) / 256), (unsigned)n),
             dim3(256), 0, c.stream, a);
  return check_launch("dropout tables");
}

// dst[r][c] = src[r][c] * tbl[((r / div) % mod)][c]  (mod = 0: no modulo), 4 channels per thread.
template <typename X>
__global__ __launch_bounds__(256) void dropout_apply_kernel(const X* src, X* dst, int64_t rows, int C,
                                                            const float* tbl, int64_t div, int64_t mod) {
  const int C4 = C / 4;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * C4) return;
  const int64_t r = e / C4;
  const int c0 = (int)(e - r * C4) * 4;
  uint32_t q = (uint32_t)r;
  if (div > 1) q /= (uint32_t)div;
  if (mod > 0) q %= (uint32_t)mod;
  const float* t = tbl + (int64_t)q * C + c0;
  const X* s = src + r * C + c0;
  X* d = dst + r * C + c0;
#pragma unroll
  for (int i = 0; i < 4; ++i) d[i] = from_f32<X>(to_f32(s[i]) * t[i]);
}

template <typename X>
evo_status_t dropout_apply(const Ctx& c, const X* src, X* dst, int64_t rows, int C, const DropSpec& d) {
  if (c.dry) return EVO_OK;
  if (C % 4) { set_error("dropout: channels %d not a multiple of 4", C); return EVO_ESHAPE; }
  const int64_t n = rows * (C / 4);
  EVO_LAUNCH(EVO_KNAME("dropout_apply_kernel", X), 0.0, (double)rows * C * (2 * sizeof(X)),
             (dropout_apply_kernel<X>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, src, dst, rows,
             C, d.tbl, d.div, d.mod);
  return check_launch("dropout apply");
}

template evo_status_t dropout_apply<float>(const Ctx&, const float*, float*, int64_t, int, const DropSpec&);
template evo_status_t dropout_apply<bf16>(const Ctx&, const bf16*, bf16*, int64_t, int, const DropSpec&);

}  // namespace evo
