// Attention core kernels for gfx950.
//
// Forward: a workgroup owns 64 queries of one (batch, head), 16 per wave64.
// Key/value tiles of 64 keys are staged in LDS (keys row-major for the
// logit product, values transposed for the context product).  Logits are
// formed as S^T = K Q^T on MFMA so that every lane holds the 16 logits of a
// single query; the online softmax (exp2 domain, FP32 statistics) needs only
// a 4-lane reduction, and the context O^T = V^T P^T is accumulated with P
// taken straight from registers.  Masked keys get the logit kMaskLogit
// (replacement); keys past the end get -inf; both through a per-key
// multiplier and addend, two operations per logit.  The running maximum moves
// lazily (only by more than kLazy), and in BF16 the row sums come out of the
// context product as one more MFMA tile.  The bias tile layout (which stride
// is 1, whether vector loads apply) is a template parameter fixed per launch.
//
// Backward: probabilities are recomputed from the saved row max and
// 1/row-sum.  One kernel produces dQ and, summed over a group of batches
// in LDS, partial pair-bias gradients (deterministic, no atomics); a second
// kernel produces dK and dV with the roles of queries and keys swapped.
#include "attn.h"

#include <string>
#include <type_traits>

namespace evo {

constexpr int KB = 64;   // keys (or queries, in the dK/dV kernel) per LDS tile
constexpr float kLazy = 8.0f;   // forward: log2 headroom before the running maximum moves

template <typename T, int D>
struct DF {
  static constexpr bool BF = sizeof(T) == 2;
  static constexpr int NKS = BF ? (D >= 32 ? D / 32 : 1) : D / 4;  // MFMA steps over d
  static constexpr int NDT = (D + 15) / 16;                          // 16-row tiles over d
  static constexpr int VEC = BF ? 8 : 4;                              // elements per 16 B
  static constexpr int DP = D + VEC;                                  // LDS pitch, row-major tiles
  static constexpr int TP = KB + VEC;                                 // LDS pitch, transposed tiles
  static constexpr int DR = NDT * 16;                                 // rows of transposed tiles
  using Frag = typename std::conditional<BF, bf16x8, float>::type;
};

// Operand fragment over d of one (position, head) row: lane group lg holds
// d = 32*ks + 8*lg + 0..7 (BF16) or d = lg*D/4 + ks (FP32).
template <typename T, int D>
EVO_DEV void load_dfrag(const T* row, int lg, bool ok, typename DF<T, D>::Frag* f) {
  if constexpr (DF<T, D>::BF) {
#pragma unroll
    for (int ks = 0; ks < DF<T, D>::NKS; ++ks) {
      const int d0 = 32 * ks + 8 * lg;
      if (ok && d0 < D) f[ks] = *(const bf16x8*)(row + d0);
      else f[ks] = bf16x8{};
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < D / 4; ++ks) f[ks] = ok ? (float)row[lg * (D / 4) + ks] : 0.f;
  }
}

template <typename T, int D>
EVO_DEV f32x4 mfma_d(const typename DF<T, D>::Frag* a, const typename DF<T, D>::Frag* b) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < DF<T, D>::NKS; ++ks) {
    if constexpr (DF<T, D>::BF) acc = mfma_bf16(a[ks], b[ks], acc);
    else acc = mfma_f32(a[ks], b[ks], acc);
  }
  return acc;
}

// acc += A * B where A rows come from a transposed LDS tile (row `r`, 64
// contiguous columns) and B is the 64 x 16 matrix whose 16x16 blocks t are
// held in the MFMA output layout p[t] (lane holds rows 4*lg+i of column lr).
template <typename T, int D>
EVO_DEV f32x4 contract64(const T* trow, bool rok, const f32x4* p, int lg, f32x4 acc) {
  if constexpr (DF<T, D>::BF) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      bf16x8 a = bf16x8{};
      if (rok) {
        const bf16x4 lo = *(const bf16x4*)(trow + 32 * u + 4 * lg);
        const bf16x4 hi = *(const bf16x4*)(trow + 32 * u + 16 + 4 * lg);
        a = bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      }
      const f32x4 p0 = p[2 * u], p1 = p[2 * u + 1];
      bf16x8 b = bf16x8{(bf16)p0[0], (bf16)p0[1], (bf16)p0[2], (bf16)p0[3],
                        (bf16)p1[0], (bf16)p1[1], (bf16)p1[2], (bf16)p1[3]};
      acc = mfma_bf16(a, b, acc);
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 a = rok ? *(const f32x4*)(trow + 16 * t + 4 * lg) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i) acc = mfma_f32(a[i], p[t][i], acc);
    }
  }
  return acc;
}

// exp2 on the hardware unit (one instruction; results below 2^-126 flush to
// zero: probabilities that small relative to the row maximum do not matter).
EVO_DEV float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }

// Register staging of a 64-row tile of (position, head) rows [p0, p0 + 64) of
// `src` (rows from pend on read as zeros): load() issues all global loads of
// the tile, store() writes the LDS copies, so that the loads of a stage are in
// flight together.  Row-major copy [64][DP]; with TR also a transposed copy
// [DR][TP], taken two rows per lane so that each store moves a pair of rows
// of one d (4 or 8 bytes) into consecutive LDS words.
EVO_DEV uint32_t u4word(const uint4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

template <typename T, int D, bool TR>
struct RowsStage {
  using F = DF<T, D>;
  static constexpr int VPR = D / F::VEC;                        // vectors per row
  static constexpr int NV = TR ? (KB / 2) * VPR : KB * VPR;     // row pairs or rows x vectors
  static constexpr int NI = (NV + 255) / 256;
  uint4 v0[NI], v1[TR ? NI : 1];

  EVO_DEV void load(const T* src, int64_t sp, int64_t p0, int64_t pend, int tid) {
    const int lim = pend - p0 < KB ? (int)(pend - p0) : KB;
    const T* base = src + p0 * sp;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int e = tid + 256 * it;
      v0[it] = make_uint4(0, 0, 0, 0);
      if constexpr (TR) v1[it] = make_uint4(0, 0, 0, 0);
      if (e < NV) {
        if constexpr (TR) {
          const int r = 2 * (e % (KB / 2)), dv = (e / (KB / 2)) * F::VEC;
          if (r < lim) v0[it] = *(const uint4*)(base + (int64_t)r * sp + dv);
          if (r + 1 < lim) v1[it] = *(const uint4*)(base + (int64_t)(r + 1) * sp + dv);
        } else {
          const int r = e / VPR, dv = (e % VPR) * F::VEC;
          if (r < lim) v0[it] = *(const uint4*)(base + (int64_t)r * sp + dv);
        }
      }
    }
  }
  // Like load(), but rows from pend on repeat row pend - 1 (pend > p0): for
  // kernels whose logits of keys past the end are -inf whatever the key row
  // holds, so that no lane branches or zero-fills.
  EVO_DEV void load_clamped(const T* src, int64_t sp, int64_t p0, int64_t pend, int tid) {
    const int last = (pend - p0 < KB ? (int)(pend - p0) : KB) - 1;
    const T* base = src + p0 * sp;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int e = tid + 256 * it;
      // (zero-filled first: without it the compiler keeps the stage in scratch)
      v0[it] = make_uint4(0, 0, 0, 0);
      if constexpr (TR) v1[it] = make_uint4(0, 0, 0, 0);
      if (NV % 256 == 0 || e < NV) {
        if constexpr (TR) {
          const int r = 2 * (e % (KB / 2)), dv = (e / (KB / 2)) * F::VEC;
          v0[it] = *(const uint4*)(base + (int64_t)(r < last ? r : last) * sp + dv);
          v1[it] = *(const uint4*)(base + (int64_t)(r + 1 < last ? r + 1 : last) * sp + dv);
        } else {
          const int r = e / VPR, dv = (e % VPR) * F::VEC;
          v0[it] = *(const uint4*)(base + (int64_t)(r < last ? r : last) * sp + dv);
        }
      }
    }
  }
  EVO_DEV void store(T* dst_rm, T* dst_t, int tid) const {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int e = tid + 256 * it;
      if (e >= NV) continue;
      if constexpr (TR) {
        const int r = 2 * (e % (KB / 2)), dv = (e / (KB / 2)) * F::VEC;
        if (dst_rm) {
          *(uint4*)(dst_rm + r * F::DP + dv) = v0[it];
          *(uint4*)(dst_rm + (r + 1) * F::DP + dv) = v1[it];
        }
#pragma unroll
        for (int i = 0; i < F::VEC; ++i) {
          T* d = dst_t + (dv + i) * F::TP + r;
          if constexpr (F::BF) {
            // element i of a row is half i & 1 of word i >> 1
            const uint32_t w0 = u4word(v0[it], i >> 1), w1 = u4word(v1[it], i >> 1);
            *(uint32_t*)d = (i & 1) ? ((w0 >> 16) | (w1 & 0xffff0000u)) : ((w0 & 0xffffu) | (w1 << 16));
          } else {
            *(uint2*)d = make_uint2(u4word(v0[it], i), u4word(v1[it], i));
          }
        }
      } else {
        const int r = e / VPR, dv = (e % VPR) * F::VEC;
        *(uint4*)(dst_rm + r * F::DP + dv) = v0[it];
      }
    }
  }
};

constexpr int BP = 68;   // LDS row pitch of the bias tile (floats)

// XCD-aware workgroup coordinates (see xcd_order): each XCD receives a
// contiguous run of (x, y, z), x fastest, so the x blocks of one (y, z) --
// which read the same key/value (or query) rows -- and neighbouring heads y,
// whose rows share cache lines, meet in one L2.
struct WgCoord { int x, y, z; };
EVO_DEV WgCoord xcd_coord() {
  const int gx = gridDim.x, gy = gridDim.y;
  int l = xcd_order(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
  WgCoord c;
  c.x = l % gx;
  l /= gx;
  c.y = l % gy;
  c.z = l / gy;
  return c;
}

template <typename T, int D>
EVO_DEV void zero_pad_rows(T* dst_t, int tid) {
  using F = DF<T, D>;
  if constexpr (F::DR > D) {
    for (int e = tid; e < (F::DR - D) * F::TP; e += 256) dst_t[D * F::TP + e] = from_f32<T>(0.f);
  }
}


// Forward logits, log2 domain: x = (s * km[k] + xb[q][k]) + ka[k], s = q . k,
// with per-key (km, ka) = (scale, 0) for a valid key, (0, kMaskLogit) for a
// masked key and (0, -inf) for a key past the end, and xb = log2(e) * bias
// (0 without bias; finite for every staged column).  Two operations per
// logit; s and xb are finite and |xb| is far below |kMaskLogit|, so masked and
// out-of-range logits are the replacement values exactly, and a valid key's
// logit is fma(s, scale, xb) + 0, bit for bit the backward's recomputation.
EVO_DEV void key_fold(const float* mask, int64_t mk, int64_t k, int64_t kend, float scale, float& mul,
                      float& add) {
  const bool in = k < kend;
  const float mv = mask ? mask[(in ? k : kend - 1) * mk] : 1.f;   // clamped: no divergent load
  mul = (in && mv != 0.f) ? scale : 0.f;
  add = !in ? -INFINITY : (mv == 0.f ? kMaskLogit : 0.f);
}

// Layout of the bias tile load, fixed per launch: none; unit stride along
// keys (tile rows contiguous) or along queries (tile columns contiguous), both
// with 16-byte vector loads and every tile whole along the unit-stride axis;
// anything else (general strides, ragged tiles, unaligned rows) with clamped
// scalar loads.
enum { BIAS_NONE = 0, BIAS_ROWS = 1, BIAS_COLS = 2, BIAS_STRIDED = 3 };

// 64 x 64 bias tile in LDS (the bias is stored in the log2 domain):
// sb[r * BP + c] = bias[(r0 + r) * sr + (c0 + c) * sc].  Loads clamp
// rows and columns into range (out-of-range entries are finite copies, never
// used: their keys get -inf, their queries are discarded), so no lane
// zero-fills or branches per element.  Register staged like RowsStage: load()
// issues the global loads, store() writes LDS.  Element (r, c) of slot `it` of
// thread `tid` (4 consecutive elements along the unit-stride axis per slot):
//   BIAS_ROWS: row r = e >> 4 (e = tid + 256 it), columns c = 4 (e & 15) .. + 3;
//   otherwise: column c = 16 it + (tid & 15), rows r = 4 (tid >> 4) .. + 3, so
//              that the 16 lanes of a group store 16 consecutive columns of
//              one row (transposing stores without bank conflicts).
template <int BM>
struct LogBiasStage {
  f32x4 v[4];
  EVO_DEV void load(const float* bias, int64_t sr, int64_t sc, int64_t r0, int64_t rend, int64_t c0,
                    int64_t cend, int tid) {
    if constexpr (BM == BIAS_ROWS) {
      const int nr = rend - r0 < 64 ? (int)(rend - r0) : 64;
      const float* base = bias + r0 * sr + c0;
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int e = tid + 256 * it;
        const int r = (e >> 4) < nr ? (e >> 4) : nr - 1;
        v[it] = *(const f32x4*)(base + r * sr + (e & 15) * 4);
      }
    } else if constexpr (BM == BIAS_COLS) {
      const int nc = cend - c0 < 64 ? (int)(cend - c0) : 64;
      const float* base = bias + r0 + c0 * sc;
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        int c = 16 * it + (tid & 15);
        c = c < nc ? c : nc - 1;
        v[it] = *(const f32x4*)(base + c * sc + (tid >> 4) * 4);
      }
    } else if constexpr (BM == BIAS_STRIDED) {
      const int nr = rend - r0 < 64 ? (int)(rend - r0) : 64;
      const int nc = cend - c0 < 64 ? (int)(cend - c0) : 64;
      const int cb = tid & 15, rb = (tid >> 4) * 4;
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int c = 16 * it + cb, cc = c < nc ? c : nc - 1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rr = rb + i < nr ? rb + i : nr - 1;
          v[it][i] = bias[(c0 + cc) * sc + (r0 + rr) * sr];
        }
      }
    }
  }
  EVO_DEV void store(float* sb, int tid) const {
    if constexpr (BM == BIAS_ROWS) {
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int e = tid + 256 * it;
        *(f32x4*)(sb + (e >> 4) * BP + (e & 15) * 4) = v[it];
      }
    } else if constexpr (BM != BIAS_NONE) {
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int c = 16 * it + (tid & 15), r = (tid >> 4) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) sb[(r + i) * BP + c] = v[it][i];
      }
    }
  }
};

// ============================================================== forward
// Four waves per SIMD requested: at head dim 32 the FP32 kernel then fits 128
// registers (without the request it took 132, three waves): 121 -> 112 us per
// row-attention launch at N_seq = 128, N_res = 256.
template <typename T, int D, int BM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void attn_fwd_kernel(AttnCore a, float scale_log2) {
  using F = DF<T, D>;
  __shared__ __attribute__((aligned(16))) T sK[KB * F::DP];
  __shared__ __attribute__((aligned(16))) T sVt[F::DR * F::TP];
  __shared__ __attribute__((aligned(16))) float sB[BM != BIAS_NONE ? 64 * BP : 4];
  __shared__ __attribute__((aligned(16))) float sKs[KB];
  __shared__ __attribute__((aligned(16))) float sKa[KB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const WgCoord wg = xcd_coord();
  const int64_t b = wg.z;
  const int h = wg.y;
  const int64_t qend0 = a.q_count < 0 ? a.Lq : a.q_begin + a.q_count;
  const int64_t qend = qend0 < a.Lq ? qend0 : a.Lq;
  const int64_t q0 = a.q_begin + (int64_t)wg.x * 64;
  const int ql = wave * 16 + lr;
  const int64_t qi = q0 + ql;
  const bool qok = qi < qend;

  const T* Q = (const T*)a.q + b * a.sb + h * D;
  const T* K = (const T*)a.k + b * a.sb + h * D;
  const T* V = (const T*)a.v + b * a.sb + h * D;

  typename F::Frag qf[F::NKS];
  load_dfrag<T, D>(Q + qi * a.sp, lg, qok, qf);

  zero_pad_rows<T, D>(sVt, tid);
  float m_run = -INFINITY, l_run = 0.f;
  f32x4 oacc[F::NDT];
#pragma unroll
  for (int dt = 0; dt < F::NDT; ++dt) oacc[dt] = f32x4{0.f, 0.f, 0.f, 0.f};
  // BF16: the row sum of the probabilities comes out of the context product
  // as row 0 of one more 16-row tile whose V^T rows are (1, 0, ..., 0), so
  // that it sums the same BF16 probabilities as the context.
  f32x4 lacc = f32x4{0.f, 0.f, 0.f, 0.f};

  const float* bias = BM != BIAS_NONE ? a.bias + h * a.bh : nullptr;
  const float* mask = a.mask ? a.mask + b * a.mb : nullptr;

  // all global loads of a key tile are issued together, then stored to LDS
  // (a tile-ahead prefetch measured slower: its registers cost occupancy)
  RowsStage<T, D, false> stK;
  RowsStage<T, D, true> stV;
  LogBiasStage<BM> stB;
  for (int64_t kb0 = 0; kb0 < a.Lk; kb0 += KB) {
    stK.load_clamped(K, a.sp, kb0, a.Lk, tid);
    stV.load_clamped(V, a.sp, kb0, a.Lk, tid);
    if constexpr (BM != BIAS_NONE) stB.load(bias, a.bq, a.bk, q0, qend, kb0, a.Lk, tid);
    float kmul = 0.f, kadd = 0.f;
    if (tid < KB) key_fold(mask, a.mk, kb0 + tid, a.Lk, scale_log2, kmul, kadd);
    __syncthreads();
    stK.store(sK, nullptr, tid);
    stV.store(nullptr, sVt, tid);
    if constexpr (BM != BIAS_NONE) stB.store(sB, tid);
    if (tid < KB) { sKs[tid] = kmul; sKa[tid] = kadd; }
    __syncthreads();
    f32x4 s[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      typename F::Frag kf[F::NKS];
      load_dfrag<T, D>(sK + (16 * t + lr) * F::DP, lg, true, kf);
      s[t] = mfma_d<T, D>(kf, qf);
    }
    // logits in the log2 domain (see key_fold)
    float mloc = -INFINITY;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const f32x4 km = *(const f32x4*)(sKs + 16 * t + 4 * lg);
      const f32x4 ka = *(const f32x4*)(sKa + 16 * t + 4 * lg);
      const f32x4 xb = BM != BIAS_NONE ? *(const f32x4*)(sB + ql * BP + 16 * t + 4 * lg) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float x = BM != BIAS_NONE ? fmaf(s[t][i], km[i], xb[i]) + ka[i] : fmaf(s[t][i], km[i], ka[i]);
        s[t][i] = x;
        mloc = fmaxf(mloc, x);
      }
    }
    mloc = fmaxf(mloc, __shfl_xor(mloc, 16, 64));
    mloc = fmaxf(mloc, __shfl_xor(mloc, 32, 64));
    // Lazy rescaling: the reference point m_run moves only when a logit
    // exceeds it by more than kLazy (probabilities relative to it then stay
    // below 2^kLazy), and the wave rescales its accumulators only when one of
    // its queries moved.  Any reference point gives the same normalized
    // result; the saved statistics are taken relative to the final one.
    const bool grow = mloc > m_run + kLazy;
    if (__builtin_amdgcn_ballot_w64(grow)) {
      const float m_new = grow ? mloc : m_run;
      const float alpha = exp2_hw(m_run - m_new);
      m_run = m_new;
#pragma unroll
      for (int dt = 0; dt < F::NDT; ++dt) oacc[dt] = oacc[dt] * alpha;
      if constexpr (F::BF) lacc = lacc * alpha;
      else l_run = l_run * alpha;
    }
    float lsum = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float p = exp2_hw(s[t][i] - m_run);
        s[t][i] = p;
        if constexpr (!F::BF) lsum += p;
      }
#pragma unroll
    for (int dt = 0; dt < F::NDT; ++dt) {
      const int dr = 16 * dt + lr;
      oacc[dt] = contract64<T, D>(sVt + dr * F::TP, true, s, lg, oacc[dt]);
    }
    if constexpr (F::BF) {
      const bf16 one = lr == 0 ? (bf16)1.0f : (bf16)0.0f;
      const bf16x8 ones = bf16x8{one, one, one, one, one, one, one, one};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const f32x4 p0 = s[2 * u], p1 = s[2 * u + 1];
        const bf16x8 pb = bf16x8{(bf16)p0[0], (bf16)p0[1], (bf16)p0[2], (bf16)p0[3],
                                 (bf16)p1[0], (bf16)p1[1], (bf16)p1[2], (bf16)p1[3]};
        lacc = mfma_bf16(ones, pb, lacc);
      }
    } else {
      lsum += __shfl_xor(lsum, 16, 64);
      lsum += __shfl_xor(lsum, 32, 64);
      l_run += lsum;
    }
  }
  if constexpr (F::BF) l_run = __shfl(lacc[0], lr, 64);   // row 0 of the sum tile: lanes 0..15

  if (!qok) return;
  const float inv = 1.0f / l_run;
  float* O = a.o ? (float*)a.o + b * a.osb + qi * a.osp + h * D : nullptr;
  T* GO = a.go ? (T*)a.go + b * a.osb + qi * a.osp + h * D : nullptr;
  const T* G = a.g ? (const T*)a.g + b * a.sb + qi * a.sp + h * D : nullptr;
#pragma unroll
  for (int dt = 0; dt < F::NDT; ++dt) {
    const int d0 = 16 * dt + 4 * lg;
    if (d0 < D) {
      f32x4 o = oacc[dt] * inv;
      if (O) store4<float>(O + d0, o);
      if (GO) {
        f32x4 gv;
#pragma unroll
        for (int i = 0; i < 4; ++i) gv[i] = to_f32(G[d0 + i]) * o[i];
        store4<T>(GO + d0, gv);
      }
    }
  }
  if (lg == 0 && a.st_max) {
    const int64_t si = (b * a.stb + qi * a.stq) * a.H + h;
    a.st_max[si] = m_run;
    a.st_inv[si] = inv;
  }
}

// ============================================================== forward, keys resident in LDS
// When all keys of one (batch, head) fit in LDS (BF16), a workgroup stages K
// (row-major), V^T and the per-key multipliers once, behind one barrier, and
// its waves then run on their own: wave w takes the 16-query subtiles w,
// w + 4, ... of the workgroup's qb queries, each through every key tile.  The
// bias has unit stride along keys, so every lane reads the 16 bias values of
// its query's logits in a tile as four 16-byte vectors straight from memory,
// one tile ahead of their use.  Key tiles with no masked key and no key past
// the end (a per-tile flag) form their logits as fma(s, scale, bias) without
// the per-key multipliers.  Logits, the lazily moved maximum, the BF16 row
// sums and the epilogue are those of attn_fwd_kernel, operation for operation.
struct ResLayout {
  int64_t lkp;          // keys rounded up to whole 64-key tiles
  int64_t tp;           // pitch of V^T rows (elements)
  int64_t off_vt, off_ks, off_ka, off_flag, bytes;
};
template <int D>
__host__ __device__ inline ResLayout res_layout(int64_t Lk) {
  using F = DF<bf16, D>;
  ResLayout L;
  L.lkp = (Lk + 63) / 64 * 64;
  L.tp = L.lkp + 4;   // row pitch 2 lkp + 8 bytes: the 8-byte reads of 16 rows fall on distinct banks
  L.off_vt = L.lkp * F::DP * 2;
  L.off_ks = L.off_vt + (int64_t)F::DR * L.tp * 2;
  L.off_ka = L.off_ks + L.lkp * 4;
  L.off_flag = L.off_ka + L.lkp * 4;
  L.bytes = (L.off_flag + L.lkp / 64 * 4 + 15) / 16 * 16;
  return L;
}

// Transposed store of two key rows r, r + 1 (8 elements of d from dv each)
// into V^T: consecutive keys of one d share a 4-byte word.
EVO_DEV void store_vt_pair(bf16* dst_t, int64_t pitch, int r, int dv, const uint4& v0, const uint4& v1) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t w0 = u4word(v0, i >> 1), w1 = u4word(v1, i >> 1);
    *(uint32_t*)(dst_t + (dv + i) * pitch + r) =
        (i & 1) ? ((w0 >> 16) | (w1 & 0xffff0000u)) : ((w0 & 0xffffu) | (w1 << 16));
  }
}

// Maximum over the four lanes l, l ^ 16, l ^ 32, l ^ 48 (the 16-lane rows of a
// wave), with the row swaps of gfx950 (v_permlane16_swap: rows 0 <-> 1 and
// 2 <-> 3; v_permlane32_swap: rows 0, 1 <-> 2, 3) instead of LDS permutes.
EVO_DEV float rows_max(float v) {
  const auto p16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = fmaxf(__uint_as_float(p16[0]), __uint_as_float(p16[1]));
  const auto p32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(p32[0]), __uint_as_float(p32[1]));
}

// Raw buffer resource over `bytes` bytes (loads past the extent return zeros).
EVO_DEV __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}
EVO_DEV f32x4 buf_load_f32x4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4_t;
  const i32x4_t q = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  return f32x4{__int_as_float(q[0]), __int_as_float(q[1]), __int_as_float(q[2]), __int_as_float(q[3])};
}

template <int D, int BM, int NB>
__global__ __launch_bounds__(256 * NB) __attribute__((amdgpu_waves_per_eu(4))) void attn_fwd_res_kernel(
    AttnCore a, float scale_log2, int qb) {
  using T = bf16;
  using F = DF<T, D>;
  static_assert(BM == BIAS_NONE || BM == BIAS_ROWS, "resident-key forward: bias with unit key stride only");
  constexpr int NT = 256 * NB, NW = 4 * NB;   // threads and waves of the workgroup
  extern __shared__ __attribute__((aligned(16))) unsigned char res_smem[];
  const ResLayout L = res_layout<D>(a.Lk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const WgCoord wg = xcd_coord();
  const int64_t b0 = (int64_t)wg.z * NB;
  const int nb = a.nbatch - b0 < NB ? (int)(a.nbatch - b0) : NB;   // batches of this workgroup
  const int h = wg.y;
  const int lkp = (int)L.lkp, nkt = lkp / 64, Lk = (int)a.Lk;
  auto sK = [&](int g) { return (T*)(res_smem + g * L.bytes); };
  auto sVt = [&](int g) { return (T*)(res_smem + g * L.bytes + L.off_vt); };
  auto sKs = [&](int g) { return (float*)(res_smem + g * L.bytes + L.off_ks); };
  auto sKa = [&](int g) { return (float*)(res_smem + g * L.bytes + L.off_ka); };
  auto sFlag = [&](int g) { return (int*)(res_smem + g * L.bytes + L.off_flag); };

  // ---- stage K, V^T and the key multipliers of each batch (rows from Lk on
  // repeat row Lk - 1: finite, and their keys get -inf)
  constexpr int VPR = D / F::VEC;
  const int nk = lkp * VPR, nv = (lkp / 2) * VPR, half = lkp / 2;
#pragma unroll
  for (int g = 0; g < NB; ++g) {
    if (g >= nb) break;
    const T* K = (const T*)a.k + (b0 + g) * a.sb + h * D;
    const T* V = (const T*)a.v + (b0 + g) * a.sb + h * D;
    for (int e0 = 0; e0 < nk; e0 += 4 * NT) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + NT * u + tid, r = e / VPR, dv = (e % VPR) * F::VEC;
        v[u] = make_uint4(0, 0, 0, 0);
        if (e < nk) v[u] = *(const uint4*)(K + (int64_t)(r < Lk ? r : Lk - 1) * a.sp + dv);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + NT * u + tid, r = e / VPR, dv = (e % VPR) * F::VEC;
        if (e < nk) *(uint4*)(sK(g) + r * F::DP + dv) = v[u];
      }
    }
    for (int e0 = 0; e0 < nv; e0 += 2 * NT) {
      uint4 v0[2], v1[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = e0 + NT * u + tid, r = 2 * (e % half), dv = (e / half) * F::VEC;
        v0[u] = v1[u] = make_uint4(0, 0, 0, 0);
        if (e < nv) {
          v0[u] = *(const uint4*)(V + (int64_t)(r < Lk ? r : Lk - 1) * a.sp + dv);
          v1[u] = *(const uint4*)(V + (int64_t)(r + 1 < Lk ? r + 1 : Lk - 1) * a.sp + dv);
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = e0 + NT * u + tid, r = 2 * (e % half), dv = (e / half) * F::VEC;
        if (e < nv) store_vt_pair(sVt(g), L.tp, r, dv, v0[u], v1[u]);
      }
    }
    if constexpr (F::DR > D) {
      for (int e = tid; e < (F::DR - D) * L.tp; e += NT) sVt(g)[D * L.tp + e] = from_f32<T>(0.f);
    }
    const float* mask = a.mask ? a.mask + (b0 + g) * a.mb : nullptr;
    // key k = tid + NT i: the 64 lanes of a wave cover exactly one key tile
    for (int k = tid; k < lkp; k += NT) {
      float km, ka;
      key_fold(mask, a.mk, k, a.Lk, scale_log2, km, ka);
      sKs(g)[k] = km;
      sKa(g)[k] = ka;
      const bool all_valid = __builtin_amdgcn_ballot_w64(km == 0.f) == 0;
      if (lane == 0) sFlag(g)[k >> 6] = all_valid ? 1 : 0;
    }
  }
  __syncthreads();
  uint64_t fastmask[NB];
#pragma unroll
  for (int g = 0; g < NB; ++g)
    fastmask[g] = g < nb ? __builtin_amdgcn_ballot_w64(lane < nkt && sFlag(g)[lane < nkt ? lane : 0] != 0) : 0;

  // ---- this wave's subtiles (wave-uniform counters live in scalar registers)
  const int64_t qend0 = a.q_count < 0 ? a.Lq : a.q_begin + a.q_count;
  const int64_t qend = qend0 < a.Lq ? qend0 : a.Lq;
  const int64_t qw0 = a.q_begin + (int64_t)wg.x * qb;
  const int64_t qw1 = qw0 + qb < qend ? qw0 + qb : qend;
  const int nsub = (int)((qw1 - qw0 + 15) / 16);
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  if (wv >= nsub) return;

  // Bias of this head through a buffer resource: a lane's query row and key
  // group as the vector offset, the subtile and key tile as scalar offsets.
  // Rows past qend and keys past Lk read zeros or neighbouring finite values
  // (results discarded, logits -inf), so the loads need no clamping or branch:
  // the next tile's bias is fetched on every step, past the last one too.  One
  // load serves all batches of the workgroup.
  const __amdgpu_buffer_rsrc_t brs =
      buf_rsrc(BM != BIAS_NONE ? a.bias + h * a.bh : nullptr,
               BM != BIAS_NONE ? (uint32_t)(((a.Lq - 1) * a.bq + a.Lk) * 4) : 0u);
  uint32_t bvo = 0, bsub = 0;
  if constexpr (BM != BIAS_NONE) {
    bvo = (uint32_t)(((qw0 + lr) * a.bq + 4 * lg) * 4);
    bsub = (uint32_t)(16 * a.bq * 4);
  }
  auto load_bias = [&](int j, int kt, f32x4* xb) {
    if constexpr (BM != BIAS_NONE) {
      const uint32_t so = (uint32_t)j * bsub + (uint32_t)kt * 256u;
#pragma unroll
      for (int t = 0; t < 4; ++t) xb[t] = buf_load_f32x4(brs, bvo + 64u * t, so);
    }
  };
  // query row of subtile j for this lane, clamped into the workgroup's range
  auto qrow = [&](int j) -> int64_t {
    const int64_t q = qw0 + 16 * j + lr;
    return q < qw1 ? q : qw1 - 1;
  };
  auto qbase = [&](int g) { return (const T*)a.q + (b0 + g) * a.sb + h * D; };
  auto gbase = [&](int g) { return (const T*)a.g + (b0 + g) * a.sb + h * D; };

  int j = wv, kt = 0;              // current subtile and key tile
  int jn = wv, ktn = 0;            // next bias to fetch
  typename F::Frag qf[NB][F::NKS], qn[NB][F::NKS];
  float m_run[NB];
  f32x4 oacc[NB][F::NDT], lacc[NB];
#pragma unroll
  for (int g = 0; g < NB; ++g) {
    load_dfrag<T, D>(qbase(g < nb ? g : 0) + qrow(j) * a.sp, lg, true, qf[g]);
    m_run[g] = -INFINITY;
#pragma unroll
    for (int dt = 0; dt < F::NDT; ++dt) oacc[g][dt] = f32x4{0.f, 0.f, 0.f, 0.f};
    lacc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  f32x4 xb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) xb[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  load_bias(jn, ktn, xb);
  if (++ktn == nkt) { ktn = 0; jn += NW; }

  // One key tile of subtile j for every batch in turn.  Once the last batch's
  // logits are formed the bias registers are free and take the next tile's
  // bias, whose load runs under that batch's softmax and context products and
  // the next tile's first products.
  while (j < nsub) {
    if (kt == 0 && j + NW < nsub) {
      // the next subtile's queries, a whole subtile ahead of their use
#pragma unroll
      for (int g = 0; g < NB; ++g) load_dfrag<T, D>(qbase(g < nb ? g : 0) + qrow(j + NW) * a.sp, lg, true, qn[g]);
    }
#pragma unroll
    for (int g = 0; g < NB; ++g) {
      if (g >= nb) break;
      f32x4 s[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        typename F::Frag kf[F::NKS];
        load_dfrag<T, D>(sK(g) + (kt * 64 + 16 * t + lr) * F::DP, lg, true, kf);
        s[t] = mfma_d<T, D>(kf, qf[g]);
      }
      float mloc = -INFINITY;
      if ((fastmask[g] >> kt) & 1) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float x = BM != BIAS_NONE ? fmaf(s[t][i], scale_log2, xb[t][i]) : s[t][i] * scale_log2;
            s[t][i] = x;
            mloc = fmaxf(mloc, x);
          }
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const f32x4 km = *(const f32x4*)(sKs(g) + kt * 64 + 16 * t + 4 * lg);
          const f32x4 ka = *(const f32x4*)(sKa(g) + kt * 64 + 16 * t + 4 * lg);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float x =
                BM != BIAS_NONE ? fmaf(s[t][i], km[i], xb[t][i]) + ka[i] : fmaf(s[t][i], km[i], ka[i]);
            s[t][i] = x;
            mloc = fmaxf(mloc, x);
          }
        }
      }
      if (g == nb - 1) {
        load_bias(jn, ktn, xb);
        if (++ktn == nkt) { ktn = 0; jn += NW; }
      }
      mloc = rows_max(mloc);
      const bool grow = mloc > m_run[g] + kLazy;
      if (__builtin_amdgcn_ballot_w64(grow)) {
        const float m_new = grow ? mloc : m_run[g];
        const float alpha = exp2_hw(m_run[g] - m_new);
        m_run[g] = m_new;
#pragma unroll
        for (int dt = 0; dt < F::NDT; ++dt) oacc[g][dt] = oacc[g][dt] * alpha;
        lacc[g] = lacc[g] * alpha;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) s[t][i] = exp2_hw(s[t][i] - m_run[g]);
#pragma unroll
      for (int dt = 0; dt < F::NDT; ++dt) {
        const int dr = 16 * dt + lr;
        oacc[g][dt] = contract64<T, D>(sVt(g) + dr * L.tp + kt * 64, true, s, lg, oacc[g][dt]);
      }
      const bf16 one = lr == 0 ? (bf16)1.0f : (bf16)0.0f;
      const bf16x8 ones = bf16x8{one, one, one, one, one, one, one, one};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const f32x4 p0 = s[2 * u], p1 = s[2 * u + 1];
        const bf16x8 pb = bf16x8{(bf16)p0[0], (bf16)p0[1], (bf16)p0[2], (bf16)p0[3],
                                 (bf16)p1[0], (bf16)p1[1], (bf16)p1[2], (bf16)p1[3]};
        lacc[g] = mfma_bf16(ones, pb, lacc[g]);
      }
    }
    if (kt == nkt - 1) {
      const int64_t qi = qw0 + 16 * j + lr;
#pragma unroll
      for (int g = 0; g < NB; ++g) {
        if (g >= nb) break;
        const int64_t b = b0 + g;
        const float l_run = __shfl(lacc[g][0], lr, 64);   // row 0 of the sum tile: lanes 0..15
        if (qi < qw1) {
          const float inv = 1.0f / l_run;
          float* O = a.o ? (float*)a.o + b * a.osb + qi * a.osp + h * D : nullptr;
          T* GO = a.go ? (T*)a.go + b * a.osb + qi * a.osp + h * D : nullptr;
          const T* G = a.g ? gbase(g) + qi * a.sp : nullptr;
#pragma unroll
          for (int dt = 0; dt < F::NDT; ++dt) {
            const int d0 = 16 * dt + 4 * lg;
            if (d0 < D) {
              const f32x4 o = oacc[g][dt] * inv;
              if (O) store4<float>(O + d0, o);
              if (GO) {
                const bf16x4 gq = *(const bf16x4*)(G + d0);
                f32x4 gv;
#pragma unroll
                for (int i = 0; i < 4; ++i) gv[i] = to_f32(gq[i]) * o[i];
                store4<T>(GO + d0, gv);
              }
            }
          }
          if (lg == 0 && a.st_max) {
            const int64_t si = (b * a.stb + qi * a.stq) * a.H + h;
            a.st_max[si] = m_run[g];
            a.st_inv[si] = inv;
          }
        }
        // next subtile
#pragma unroll
        for (int ks = 0; ks < F::NKS; ++ks) qf[g][ks] = qn[g][ks];
        m_run[g] = -INFINITY;
#pragma unroll
        for (int dt = 0; dt < F::NDT; ++dt) oacc[g][dt] = f32x4{0.f, 0.f, 0.f, 0.f};
        lacc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      kt = 0;
      j += NW;
    } else {
      ++kt;
    }
  }
}

// ============================================================== backward: dQ and bias partials
// A workgroup owns 64 queries of one head for a group of up to GM batches
// (bias shared across the batch axis).  Key tiles run in the outer loop so
// that the bias tile is staged once and the bias gradient of the tile, summed
// over the group's batches in registers, is written once as this group's
// partial; the dQ accumulators of the group's batches stay in registers.
// Batches per dQ workgroup: FP32 halves the group (its fragments are twice as
// large; a larger group costs occupancy, measured slower).  Groups of 8 at
// head dims 8 and 16, and of 4 at head dim 64, spilled registers to scratch.
template <typename T, int D> struct DqGroup {
  static constexpr int GM = (D >= 64 ? 2 : 4) / (sizeof(T) == 2 ? 1 : 2);
};

template <typename T, int D, int BM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void attn_bwd_dq_kernel(AttnCore a, AttnGrad gr, float scale_log2,
                                                          float scale) {
  using F = DF<T, D>;
  constexpr int GM = DqGroup<T, D>::GM;
  __shared__ __attribute__((aligned(16))) T sK[KB * F::DP];
  __shared__ __attribute__((aligned(16))) T sV[KB * F::DP];
  __shared__ __attribute__((aligned(16))) T sKt[F::DR * F::TP];
  __shared__ __attribute__((aligned(16))) float sB[64 * BP];
  __shared__ __attribute__((aligned(16))) float sKa[KB];
  // BF16 at head dims up to 32: the query and context-gradient rows of the
  // group's batches, staged in LDS once, since they are the same for every key tile
  constexpr bool QO_LDS = F::BF && D <= 32;
  __shared__ __attribute__((aligned(16))) T sQO[QO_LDS ? 2 * GM * KB * F::DP : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const WgCoord wg = xcd_coord();
  const int h = wg.y;
  const int64_t grp = wg.z;
  const int64_t b0 = grp * gr.group;
  const int64_t b1 = b0 + gr.group < a.nbatch ? b0 + gr.group : a.nbatch;
  const int qloc = wave * 16 + lr;
  const int64_t q0 = (int64_t)wg.x * 64;
  const int64_t qi = q0 + qloc;
  const bool qok = qi < a.Lq;
  const bool dbias = gr.dbias_part != nullptr;
  const float* bias = BM != BIAS_NONE ? a.bias + h * a.bh : nullptr;
  float* dbp = dbias ? gr.dbias_part + (grp * a.H + h) * a.Lq * a.Lk : nullptr;

  zero_pad_rows<T, D>(sKt, tid);
  f32x4 dq[GM][F::NDT];
#pragma unroll
  for (int bi = 0; bi < GM; ++bi)
#pragma unroll
    for (int dt = 0; dt < F::NDT; ++dt) dq[bi][dt] = f32x4{0.f, 0.f, 0.f, 0.f};

  if constexpr (QO_LDS) {
#pragma unroll
    for (int bi = 0; bi < GM; ++bi) {
      const int64_t b = b0 + bi;
      if (b >= b1) break;
      RowsStage<T, D, false> sq, so;
      sq.load((const T*)a.q + b * a.sb + h * D, a.sp, q0, a.Lq, tid);
      so.load((const T*)gr.dctx + b * a.osb + h * D, a.osp, q0, a.Lq, tid);
      sq.store(sQO + (2 * bi) * KB * F::DP, nullptr, tid);
      so.store(sQO + (2 * bi + 1) * KB * F::DP, nullptr, tid);
    }
  }
  for (int64_t kb0 = 0; kb0 < a.Lk; kb0 += KB) {
    f32x4 dbacc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) dbacc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int bi = 0; bi < GM; ++bi) {
      const int64_t b = b0 + bi;
      if (b >= b1) break;
      const T* Q = (const T*)a.q + b * a.sb + h * D;
      const T* K = (const T*)a.k + b * a.sb + h * D;
      const T* V = (const T*)a.v + b * a.sb + h * D;
      const T* DO = (const T*)gr.dctx + b * a.osb + h * D;
      const float* mask = a.mask ? a.mask + b * a.mb : nullptr;
      // every global load of the stage first, then the LDS stores
      RowsStage<T, D, true> stK;
      RowsStage<T, D, false> stV;
      LogBiasStage<BM> stB;
      stK.load(K, a.sp, kb0, a.Lk, tid);
      stV.load(V, a.sp, kb0, a.Lk, tid);
      if (BM != BIAS_NONE && bi == 0) stB.load(bias, a.bq, a.bk, q0, a.Lq, kb0, a.Lk, tid);
      // Per-key addend of the logits: 0 for a valid key, -inf for a masked key
      // or one past the end, whose probability is then exactly 0.  (In the
      // forward a masked key has the replacement logit, which gives it
      // probability 0 unless the whole row is masked; a wholly masked row,
      // recognisable by its maximum, has no logit gradient at all and gets
      // irow = 0 below.)
      float kadd = 0.f;
      if (tid < KB) {
        const bool in = kb0 + tid < a.Lk;
        kadd = (in && !(mask && mask[(kb0 + tid) * a.mk] == 0.f)) ? 0.f : -INFINITY;
      }
      typename F::Frag qf[F::NKS], of[F::NKS];
      if constexpr (!QO_LDS) {
        load_dfrag<T, D>(Q + qi * a.sp, lg, qok, qf);
        load_dfrag<T, D>(DO + qi * a.osp, lg, qok, of);
      }
      // queries past the end: mrow = +inf and irow = 0 give dS = 0 exactly
      float mrow = INFINITY, irow = 0.f, drow = 0.f;
      if (qok) {
        const int64_t si = (b * a.stb + qi * a.stq) * a.H + h;
        mrow = a.st_max[si];
        irow = a.st_inv[si];
        drow = gr.Dsum[si];
        if (mrow < 0.5f * kMaskLogit) irow = 0.f;
      }
      __syncthreads();
      stK.store(sK, sKt, tid);
      stV.store(sV, nullptr, tid);
      if (BM != BIAS_NONE && bi == 0) stB.store(sB, tid);
      if (tid < KB) sKa[tid] = kadd;
      __syncthreads();
      if constexpr (QO_LDS) {   // (rows past the end were staged as zeros)
        load_dfrag<T, D>(sQO + (2 * bi) * KB * F::DP + qloc * F::DP, lg, true, qf);
        load_dfrag<T, D>(sQO + (2 * bi + 1) * KB * F::DP + qloc * F::DP, lg, true, of);
      }
      // dS = P (dP - D); exactly 0 for masked keys, keys past the end and
      // queries past the end (see kadd, mrow, irow)
      f32x4 ds[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        typename F::Frag kf[F::NKS], vf[F::NKS];
        load_dfrag<T, D>(sK + (16 * t + lr) * F::DP, lg, true, kf);
        load_dfrag<T, D>(sV + (16 * t + lr) * F::DP, lg, true, vf);
        const f32x4 sv = mfma_d<T, D>(kf, qf);
        const f32x4 dp = mfma_d<T, D>(vf, of);
        const f32x4 bv = BM != BIAS_NONE ? *(const f32x4*)(sB + qloc * BP + 16 * t + 4 * lg)
                                         : f32x4{0.f, 0.f, 0.f, 0.f};
        const f32x4 ka = *(const f32x4*)(sKa + 16 * t + 4 * lg);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float x = fmaf(sv[i], scale_log2, bv[i]) + ka[i];
          ds[t][i] = exp2_hw(x - mrow) * irow * (dp[i] - drow);
        }
        dbacc[t] = dbacc[t] + ds[t];
      }
#pragma unroll
      for (int dt = 0; dt < F::NDT; ++dt) {
        const int dr = 16 * dt + lr;
        dq[bi][dt] = contract64<T, D>(sKt + dr * F::TP, true, ds, lg, dq[bi][dt]);
      }
    }
    // this group's bias-gradient partial for the tile (layout: dbq, dbk)
    if (dbias && qok) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t key = kb0 + 16 * t + 4 * lg;
        const int64_t off = qi * gr.dbq + key * gr.dbk;
        if (gr.dbk == 1 && key + 3 < a.Lk && (off & 3) == 0) {
          *(f32x4*)(dbp + off) = dbacc[t];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (key + i < a.Lk) dbp[off + i * gr.dbk] = dbacc[t][i];
        }
      }
    }
  }
  if (!qok) return;
#pragma unroll
  for (int bi = 0; bi < GM; ++bi) {
    const int64_t b = b0 + bi;
    if (b >= b1) break;
    T* DQ = (T*)gr.dq + b * gr.dsb + qi * gr.dsp + h * D;
#pragma unroll
    for (int dt = 0; dt < F::NDT; ++dt) {
      const int d0 = 16 * dt + 4 * lg;
      if (d0 < D) store4<T>(DQ + d0, dq[bi][dt] * scale);
    }
  }
}

// ============================================================== backward: dK, dV
// Roles of queries and keys swapped: a workgroup owns 64 keys of one head for
// a group of up to GM batches; query tiles run in the outer loop so that the
// bias tile (keys x queries) is staged once for the group.  GM = 1: measured
// on gfx950, the registers of more batches cost more occupancy than the shared
// bias tile saves.
// BF16 at head dim 32 requests four waves per SIMD (127 registers, 81 -> 74 us
// per row-attention launch at N_seq = 128, N_res = 256); at head dims 8 and 16,
// and with a strided bias, that request spills, and FP32 needs 160: three waves.
template <int D> struct DkvGroup { static constexpr int GM = 1; };

template <typename T, int D, int BM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 2 && D == 32 && BM != BIAS_STRIDED ? 4 : 3))) void attn_bwd_dkdv_kernel(AttnCore a, AttnGrad gr, float scale_log2,
                                                            float scale, int32_t group) {
  using F = DF<T, D>;
  constexpr int GM = DkvGroup<D>::GM;
  __shared__ __attribute__((aligned(16))) T sQ[KB * F::DP];
  __shared__ __attribute__((aligned(16))) T sO[KB * F::DP];
  __shared__ __attribute__((aligned(16))) T sQt[F::DR * F::TP];
  __shared__ __attribute__((aligned(16))) T sOt[F::DR * F::TP];
  __shared__ __attribute__((aligned(16))) float sB[64 * BP];
  __shared__ __attribute__((aligned(16))) float sM[KB];
  __shared__ __attribute__((aligned(16))) float sI[KB];
  __shared__ __attribute__((aligned(16))) float sD[KB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const WgCoord wg = xcd_coord();
  const int h = wg.y;
  const int64_t b0 = (int64_t)wg.z * group;
  const int64_t b1 = b0 + group < a.nbatch ? b0 + group : a.nbatch;
  const int kl = wave * 16 + lr;
  const int64_t k0 = (int64_t)wg.x * 64;
  const int64_t key = k0 + kl;
  const bool kok = key < a.Lk;
  const float* bias = BM != BIAS_NONE ? a.bias + h * a.bh : nullptr;

  zero_pad_rows<T, D>(sQt, tid);
  zero_pad_rows<T, D>(sOt, tid);
  f32x4 dk[GM][F::NDT], dv[GM][F::NDT];
#pragma unroll
  for (int bi = 0; bi < GM; ++bi)
#pragma unroll
    for (int dt = 0; dt < F::NDT; ++dt) { dk[bi][dt] = f32x4{0.f, 0.f, 0.f, 0.f}; dv[bi][dt] = dk[bi][dt]; }

  // one batch per workgroup: its key and value fragments and the key's mask
  // stay in registers across the query tiles
  typename F::Frag kf1[F::NKS], vf1[F::NKS];
  bool kmasked1 = false;
  if constexpr (GM == 1) {
    kmasked1 = kok && a.mask && a.mask[b0 * a.mb + key * a.mk] == 0.f;
    load_dfrag<T, D>((const T*)a.k + b0 * a.sb + h * D + key * a.sp, lg, kok, kf1);
    load_dfrag<T, D>((const T*)a.v + b0 * a.sb + h * D + key * a.sp, lg, kok, vf1);
  }
  for (int64_t qb0 = 0; qb0 < a.Lq; qb0 += KB) {
#pragma unroll
    for (int bi = 0; bi < GM; ++bi) {
      const int64_t b = b0 + bi;
      if (b >= b1) break;
      const T* Q = (const T*)a.q + b * a.sb + h * D;
      const T* K = (const T*)a.k + b * a.sb + h * D;
      const T* V = (const T*)a.v + b * a.sb + h * D;
      const T* DO = (const T*)gr.dctx + b * a.osb + h * D;
      const bool kmasked = GM == 1 ? kmasked1 : kok && a.mask && a.mask[b * a.mb + key * a.mk] == 0.f;
      // a masked key's logit is the replacement value, a key past the end
      // (its lane's results are discarded) gets -inf so that P stays finite
      const bool krep = kmasked || !kok;
      const float xrep = kok ? kMaskLogit : -INFINITY;
      // every global load of the stage first, then the LDS stores
      RowsStage<T, D, true> stQ, stO;
      LogBiasStage<BM> stB;
      stQ.load(Q, a.sp, qb0, a.Lq, tid);
      stO.load(DO, a.osp, qb0, a.Lq, tid);
      if (BM != BIAS_NONE && bi == 0) stB.load(bias, a.bk, a.bq, k0, a.Lk, qb0, a.Lq, tid);
      // queries past the end: m = +inf and 1/l = 0 give P = dS = 0 exactly
      float mv = INFINITY, iv = 0.f, dvv = 0.f;
      if (tid < KB && qb0 + tid < a.Lq) {
        const int64_t si = (b * a.stb + (qb0 + tid) * a.stq) * a.H + h;
        mv = a.st_max[si]; iv = a.st_inv[si]; dvv = gr.Dsum[si];
      }
      typename F::Frag kf[F::NKS], vf[F::NKS];
      if constexpr (GM == 1) {
#pragma unroll
        for (int ks = 0; ks < F::NKS; ++ks) { kf[ks] = kf1[ks]; vf[ks] = vf1[ks]; }
      } else {
        load_dfrag<T, D>(K + key * a.sp, lg, kok, kf);
        load_dfrag<T, D>(V + key * a.sp, lg, kok, vf);
      }
      __syncthreads();
      stQ.store(sQ, sQt, tid);
      stO.store(sO, sOt, tid);
      if (BM != BIAS_NONE && bi == 0) stB.store(sB, tid);
      if (tid < KB) { sM[tid] = mv; sI[tid] = iv; sD[tid] = dvv; }
      __syncthreads();
      f32x4 P[4], DS[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        typename F::Frag qf[F::NKS], of[F::NKS];
        load_dfrag<T, D>(sQ + (16 * t + lr) * F::DP, lg, true, qf);
        load_dfrag<T, D>(sO + (16 * t + lr) * F::DP, lg, true, of);
        const f32x4 sv = mfma_d<T, D>(qf, kf);
        const f32x4 dp = mfma_d<T, D>(of, vf);
        const f32x4 bv = BM != BIAS_NONE ? *(const f32x4*)(sB + kl * BP + 16 * t + 4 * lg)
                                         : f32x4{0.f, 0.f, 0.f, 0.f};
        const f32x4 m4 = *(const f32x4*)(sM + 16 * t + 4 * lg);
        const f32x4 i4 = *(const f32x4*)(sI + 16 * t + 4 * lg);
        const f32x4 d4 = *(const f32x4*)(sD + 16 * t + 4 * lg);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float x = fmaf(sv[i], scale_log2, bv[i]);
          x = krep ? xrep : x;
          const float p = exp2_hw(x - m4[i]) * i4[i];
          P[t][i] = p;
          // a masked key's logit is a constant: no logit gradient (its
          // probability still weighs V in wholly masked rows)
          DS[t][i] = krep ? 0.f : p * (dp[i] - d4[i]);
        }
      }
#pragma unroll
      for (int dt = 0; dt < F::NDT; ++dt) {
        const int dr = 16 * dt + lr;
        dv[bi][dt] = contract64<T, D>(sOt + dr * F::TP, true, P, lg, dv[bi][dt]);
        dk[bi][dt] = contract64<T, D>(sQt + dr * F::TP, true, DS, lg, dk[bi][dt]);
      }
      if constexpr (!F::BF) {
        // the logit gradients for the dQ pass, keys-major ([b][h][k][q]): a
        // lane's four consecutive queries of tile t as one 16-byte store, a
        // wave's store 64 contiguous bytes of each of its 16 keys' rows; the
        // last, partial query tile stores element by element
        if (gr.ds && kok) {
          float* drow = gr.ds + ((b * a.H + h) * a.Lk + key) * a.Lq + qb0 + 4 * lg;
          if (qb0 + KB <= a.Lq) {
#pragma unroll
            for (int t = 0; t < 4; ++t) *(f32x4*)(drow + 16 * t) = DS[t];
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (qb0 + 16 * t + 4 * lg + i < a.Lq) drow[16 * t + i] = DS[t][i];
          }
        }
      }
    }
  }
  if (!kok) return;
#pragma unroll
  for (int bi = 0; bi < GM; ++bi) {
    const int64_t b = b0 + bi;
    if (b >= b1) break;
    T* DK = (T*)gr.dk + b * gr.dsb + key * gr.dsp + h * D;
    T* DV = (T*)gr.dv + b * gr.dsb + key * gr.dsp + h * D;
#pragma unroll
    for (int dt = 0; dt < F::NDT; ++dt) {
      const int d0 = 16 * dt + 4 * lg;
      if (d0 < D) {
        store4<T>(DK + d0, dk[bi][dt] * scale);
        store4<T>(DV + d0, dv[bi][dt]);
      }
    }
  }
}

// ============================================================== backward: dQ from stored logit gradients (FP32)
// The FP32 backward keeps the logit gradients dS that the dK/dV kernel forms
// and takes dQ = dS K / sqrt(c) and the bias-gradient partials from them, so
// that the logits and dP, two of the three FP32 products of
// attn_bwd_dq_kernel, are formed once per backward instead of twice.  Same
// workgroups (64 queries of one head), batch groups and partial layout as
// attn_bwd_dq_kernel; the dS tile (keys-major, as the dK/dV kernel stores it)
// comes in as 16-byte vectors and through LDS to the lanes' query columns.
template <int D>
__global__ __launch_bounds__(256) void attn_bwd_dq_ds_kernel(AttnCore a, AttnGrad gr, float scale) {
  using T = float;
  using F = DF<T, D>;
  constexpr int GM = DqGroup<T, D>::GM;
  constexpr int SP = KB + 4;   // LDS pitch of the dS tile (keys x queries)
  __shared__ __attribute__((aligned(16))) T sKt[F::DR * F::TP];
  __shared__ __attribute__((aligned(16))) float sDs[KB * SP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const WgCoord wg = xcd_coord();
  const int h = wg.y;
  const int64_t grp = wg.z;
  const int64_t b0 = grp * gr.group;
  const int64_t b1 = b0 + gr.group < a.nbatch ? b0 + gr.group : a.nbatch;
  const int64_t q0 = (int64_t)wg.x * 64;
  const int64_t qi = q0 + wave * 16 + lr;
  const bool qok = qi < a.Lq;
  const bool dbias = gr.dbias_part != nullptr;
  float* dbp = dbias ? gr.dbias_part + (grp * a.H + h) * a.Lq * a.Lk : nullptr;
  // the thread's four 16-byte pieces of a dS tile: key row tr + 16 u, queries tc..tc+3
  const int tr = tid >> 4, tc = (tid & 15) * 4;
  const bool cok = q0 + tc + 3 < a.Lq;

  zero_pad_rows<T, D>(sKt, tid);
  f32x4 dq[GM][F::NDT];
#pragma unroll
  for (int bi = 0; bi < GM; ++bi)
#pragma unroll
    for (int dt = 0; dt < F::NDT; ++dt) dq[bi][dt] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int64_t kb0 = 0; kb0 < a.Lk; kb0 += KB) {
    f32x4 dbacc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) dbacc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int bi = 0; bi < GM; ++bi) {
      const int64_t b = b0 + bi;
      if (b >= b1) break;
      const T* K = (const T*)a.k + b * a.sb + h * D;
      RowsStage<T, D, true> stK;
      stK.load(K, a.sp, kb0, a.Lk, tid);
      // the dS tile (keys kb0.., queries q0..): zeros past either end
      const float* dsb = gr.ds + (b * a.H + h) * a.Lk * a.Lq;
      f32x4 piece[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t key = kb0 + tr + 16 * u;
        const float* src = dsb + (key < a.Lk ? key : 0) * a.Lq + q0 + tc;
        if (key < a.Lk && cok) {
          piece[u] = *(const f32x4*)src;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) piece[u][i] = key < a.Lk && q0 + tc + i < a.Lq ? src[i] : 0.f;
        }
      }
      __syncthreads();
      stK.store(nullptr, sKt, tid);
#pragma unroll
      for (int u = 0; u < 4; ++u) *(f32x4*)(sDs + (tr + 16 * u) * SP + tc) = piece[u];
      __syncthreads();
      // dS of query qi at keys kb0 + 16 t + 4 lg + i
      const int ql = wave * 16 + lr;
      f32x4 ds[4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) ds[t][i] = sDs[(16 * t + 4 * lg + i) * SP + ql];
#pragma unroll
      for (int t = 0; t < 4; ++t) dbacc[t] = dbacc[t] + ds[t];
#pragma unroll
      for (int dt = 0; dt < F::NDT; ++dt) {
        const int dr = 16 * dt + lr;
        dq[bi][dt] = contract64<T, D>(sKt + dr * F::TP, true, ds, lg, dq[bi][dt]);
      }
    }
    // this group's bias-gradient partial for the tile (layout: dbq, dbk)
    if (dbias && qok) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t key = kb0 + 16 * t + 4 * lg;
        const int64_t off = qi * gr.dbq + key * gr.dbk;
        if (gr.dbk == 1 && key + 3 < a.Lk && (off & 3) == 0) {
          *(f32x4*)(dbp + off) = dbacc[t];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (key + i < a.Lk) dbp[off + i * gr.dbk] = dbacc[t][i];
        }
      }
    }
  }
  if (!qok) return;
#pragma unroll
  for (int bi = 0; bi < GM; ++bi) {
    const int64_t b = b0 + bi;
    if (b >= b1) break;
    T* DQ = (T*)gr.dq + b * gr.dsb + qi * gr.dsp + h * D;
#pragma unroll
    for (int dt = 0; dt < F::NDT; ++dt) {
      const int d0 = 16 * dt + 4 * lg;
      if (d0 < D) store4<T>(DQ + d0, dq[bi][dt] * scale);
    }
  }
}

// ============================================================== launchers
static bool attn_shape_ok(const AttnCore& a) {
  if (!(a.D == 8 || a.D == 16 || a.D == 32 || a.D == 64)) {
    set_error("attention: head_dim %d not in {8,16,32,64}", a.D);
    return false;
  }
  if (a.Lq <= 0 || a.Lk <= 0 || a.nbatch <= 0 || a.H <= 0) {
    set_error("attention: empty problem");
    return false;
  }
  return true;
}

template <typename T, int D>
static std::string kname(const char* k) {
  return std::string(k) + "<" + tname<T>() + ", " + std::to_string(D) + ">";
}

// Bias tile layout of a launch whose tiles have rows [r_begin, r_begin + nrows)
// and columns [0, ncols) of a bias with strides (sr, sc): vector loads need
// 16-byte aligned vectors and whole 64-wide tiles along the unit stride.
static int bias_mode(const float* bias, int64_t bh, int64_t sr, int64_t sc, int64_t r_begin, int64_t nrows,
                     int64_t ncols) {
  if (!bias) return BIAS_NONE;
  const bool al = ((uintptr_t)bias % 16) == 0 && bh % 4 == 0;
  if (sc == 1 && al && sr % 4 == 0 && ncols % 64 == 0) return BIAS_ROWS;
  if (sr == 1 && al && sc % 4 == 0 && r_begin % 4 == 0 && nrows % 64 == 0) return BIAS_COLS;
  return BIAS_STRIDED;
}

#define EVO_BIAS_SWITCH(bm, KERNEL, ...)                \
  switch (bm) {                                         \
    case BIAS_NONE: KERNEL(BIAS_NONE, __VA_ARGS__); break;  \
    case BIAS_ROWS: KERNEL(BIAS_ROWS, __VA_ARGS__); break;  \
    case BIAS_COLS: KERNEL(BIAS_COLS, __VA_ARGS__); break;  \
    default: KERNEL(BIAS_STRIDED, __VA_ARGS__); break;  \
  }

// Resident-key forward (BF16): LDS bound for it (at least two workgroups per CU)
// and the workgroup count it aims for (four per CU).
constexpr int64_t kResLdsMax = 80 * 1024;
constexpr int64_t kResTargetWgs = 1024;

template <int D>
static bool launch_fwd_res(const Ctx& c, const AttnCore& a, int64_t nq, float sl2, double flops, double bytes) {
  int bm = BIAS_NONE;
  if (a.bias) {
    // unit stride along keys, 16-byte rows, and 32-bit byte offsets (buffer loads)
    const bool rows = a.bk == 1 && a.bq % 4 == 0 && a.bh % 4 == 0 && ((uintptr_t)a.bias % 16) == 0 &&
                      a.Lk % 4 == 0 && a.Lk >= 4 && (a.Lq + 128) * a.bq * 4 < (1LL << 31);
    if (!rows) return false;
    bm = BIAS_ROWS;
  }
  const ResLayout L = res_layout<D>(a.Lk);
  if (L.lkp / 64 > 64) return false;
  // two batches per workgroup (eight waves) when both fit in LDS: one bias
  // load then serves both
  // (head dim <= 32: the registers of two batches' state fit without spilling)
  const int nb = (D <= 32 && a.nbatch >= 2 && 2 * L.bytes <= kResLdsMax) ? 2 : 1;
  if (nb * L.bytes > kResLdsMax) return false;
  const int64_t ngroups = (a.nbatch + nb - 1) / nb;
  // queries per workgroup: the most (256, 128, 64) that still gives enough workgroups
  int qb = 64;
  for (int cand : {256, 128}) {
    if ((nq + cand - 1) / cand * a.H * ngroups * nb >= kResTargetWgs) { qb = cand; break; }
  }
  const dim3 grid((unsigned)((nq + qb - 1) / qb), (unsigned)a.H, (unsigned)ngroups);
  static const std::string nm = kname<bf16, D>("attn_fwd_res_kernel");
  const size_t lds = (size_t)(nb * L.bytes);
#define EVO_RES(BMV, NBV)                                                                                    \
  EVO_LAUNCH(nm.c_str(), flops, bytes, (attn_fwd_res_kernel<D, BMV, NBV>), grid, dim3(256 * NBV), lds, c.stream, \
             a, sl2, qb)
  if constexpr (D <= 32) {
    if (nb == 2) {
      if (bm == BIAS_NONE) EVO_RES(BIAS_NONE, 2);
      else EVO_RES(BIAS_ROWS, 2);
      return true;
    }
  }
  {
    if (bm == BIAS_NONE) EVO_RES(BIAS_NONE, 1);
    else EVO_RES(BIAS_ROWS, 1);
  }
#undef EVO_RES
  return true;
}

template <typename T, int D>
static void launch_fwd(const Ctx& c, const AttnCore& a) {
  static const std::string nm = kname<T, D>("attn_fwd_kernel");
  const int64_t nq = a.q_count < 0 ? a.Lq : a.q_count;
  const float sl2 = kLog2e / sqrtf((float)D);
  const double bh = (double)a.nbatch * a.H;
  const double flops = 4.0 * bh * nq * a.Lk * D;
  const double bytes = bh * ((double)nq * D * 4 + (double)a.Lk * D * 2) * sizeof(T) +
                       (a.bias ? (double)a.H * nq * a.Lk * 4.0 : 0.0) + bh * nq * 8.0;
  if constexpr (std::is_same<T, bf16>::value) {
    if (launch_fwd_res<D>(c, a, nq, sl2, flops, bytes)) return;
  }
  const int bm = bias_mode(a.bias, a.bh, a.bq, a.bk, a.q_begin, nq, a.Lk);
  dim3 grid((unsigned)((nq + 63) / 64), (unsigned)a.H, (unsigned)a.nbatch);
#define EVO_FWD(BMV, _) \
  EVO_LAUNCH(nm.c_str(), flops, bytes, (attn_fwd_kernel<T, D, BMV>), grid, dim3(256), 0, c.stream, a, sl2)
  EVO_BIAS_SWITCH(bm, EVO_FWD, 0)
#undef EVO_FWD
}

template <typename T>
evo_status_t attn_fwd(const Ctx& c, const AttnCore& a) {
  if (c.dry) return EVO_OK;
  if (!attn_shape_ok(a)) return EVO_ESHAPE;
  switch (a.D) {
    case 8: launch_fwd<T, 8>(c, a); break;
    case 16: launch_fwd<T, 16>(c, a); break;
    case 32: launch_fwd<T, 32>(c, a); break;
    default: launch_fwd<T, 64>(c, a); break;
  }
  return check_launch("attn_fwd");
}

template <typename T>
int64_t attn_bwd_groups(const AttnCore& a) {
  // about 1024 workgroups, and at most the batches one workgroup keeps in registers
  const int64_t qblocks = (a.Lq + 63) / 64;
  int64_t target = (1024 + qblocks * a.H - 1) / (qblocks * a.H);
  if (target < 1) target = 1;
  if (target > a.nbatch) target = a.nbatch;
  int64_t group = (a.nbatch + target - 1) / target;
  // at most the group of the dQ kernel instance for this head dim
  const int64_t gmax = a.D == 8    ? DqGroup<T, 8>::GM
                       : a.D == 16 ? DqGroup<T, 16>::GM
                       : a.D == 32 ? DqGroup<T, 32>::GM
                                   : DqGroup<T, 64>::GM;
  if (group > gmax) group = gmax;
  return (a.nbatch + group - 1) / group;
}

template <typename T, int D>
static evo_status_t launch_bwd(const Ctx& c, const AttnCore& a, AttnGrad g) {
  const float sl2 = kLog2e / sqrtf((float)D);
  const float sc = 1.0f / sqrtf((float)D);
  const int64_t ngroups = attn_bwd_groups<T>(a);
  g.group = (a.nbatch + ngroups - 1) / ngroups;
  constexpr int gm = DqGroup<T, D>::GM;
  EVO_CHECK_ARG(g.group <= gm, EVO_EINVAL, "attention backward: group of %lld batches > %d", (long long)g.group, gm);
  const size_t lds = 0;
  static const std::string n1 = kname<T, D>("attn_bwd_dq_kernel");
  static const std::string n2 = kname<T, D>("attn_bwd_dkdv_kernel");
  const double bh = (double)a.nbatch * a.H, ll = (double)a.Lq * a.Lk;
  // algorithmic products: dP and dQ here, dK and dV in the second kernel
  const double f1 = 4.0 * bh * ll * D, f2 = 4.0 * bh * ll * D;
  const double b1 = bh * ((double)a.Lq * D * 3 + (double)a.Lk * D * 2) * sizeof(T) + bh * a.Lq * 12.0 +
                    (g.dbias_part ? (double)ngroups * a.H * ll * 4.0 + a.H * ll * 4.0 : 0.0);
  const double b2 = bh * ((double)a.Lq * D * 2 + (double)a.Lk * D * 4) * sizeof(T) + bh * a.Lq * 12.0 +
                    (a.bias ? a.H * ll * 4.0 : 0.0);
  dim3 g1((unsigned)((a.Lq + 63) / 64), (unsigned)a.H, (unsigned)ngroups);
  // bias tiles: queries x keys in the dQ kernel, keys x queries in the dK/dV kernel
  const int bm1 = bias_mode(a.bias, a.bh, a.bq, a.bk, 0, a.Lq, a.Lk);
  const int bm2 = bias_mode(a.bias, a.bh, a.bk, a.bq, 0, a.Lk, a.Lq);
  // batches per dK/dV workgroup: the bias tile is shared across them (one batch when there is no bias)
  int32_t kgroup = a.bias ? DkvGroup<D>::GM : 1;
  const int64_t kblocks = (a.Lk + 63) / 64;
  while (kgroup > 1 && kblocks * a.H * ((a.nbatch + kgroup - 1) / kgroup) < 512) kgroup /= 2;
  dim3 g2((unsigned)kblocks, (unsigned)a.H, (unsigned)((a.nbatch + kgroup - 1) / kgroup));
  auto dkdv = [&](double flops, double bytes) -> evo_status_t {
#define EVO_DKDV(BMV, _)                                                                                        \
  EVO_LAUNCH(n2.c_str(), flops, bytes, (attn_bwd_dkdv_kernel<T, D, BMV>), g2, dim3(256), 0, c.stream, a, g, sl2, \
             sc, kgroup)
    EVO_BIAS_SWITCH(bm2, EVO_DKDV, 0)
#undef EVO_DKDV
    return check_launch("attn_bwd_dkdv");
  };
  if constexpr (sizeof(T) == 4) {
    if (g.ds) {
      // dK, dV and the stored dS (dP formed here only), then dQ and the bias partials from dS
      static const std::string n3 = kname<T, D>("attn_bwd_dq_ds_kernel");
      const double sbytes = bh * ll * 4.0;
      EVO_TRY(dkdv(f2 + 0.5 * f1, b2 + sbytes));
      const double b3 = bh * ((double)a.Lk * D * 4 + (double)a.Lq * D * 4) + sbytes +
                        (g.dbias_part ? (double)ngroups * a.H * ll * 4.0 : 0.0);
      EVO_LAUNCH(n3.c_str(), 0.5 * f1, b3, (attn_bwd_dq_ds_kernel<D>), g1, dim3(256), 0, c.stream, a, g, sc);
      return check_launch("attn_bwd_dq_ds");
    }
  }
#define EVO_DQ(BMV, _) \
  EVO_LAUNCH(n1.c_str(), f1, b1, (attn_bwd_dq_kernel<T, D, BMV>), g1, dim3(256), lds, c.stream, a, g, sl2, sc)
  EVO_BIAS_SWITCH(bm1, EVO_DQ, 0)
#undef EVO_DQ
  EVO_TRY(check_launch("attn_bwd_dq"));
  return dkdv(f2, b2);
}

template <typename T>
int64_t attn_bwd_ds_elems(const AttnCore& a) {
  // FP32 only (in BF16 the recomputed products are cheap and the stored FP32
  // dS would double the kernels' memory traffic); up to 2 GiB of dS, and
  // queries in whole 16-byte vectors
  if (sizeof(T) != 4 || a.Lq % 4 != 0) return 0;
  const int64_t n = a.nbatch * a.H * a.Lq * a.Lk;
  return n * 4 <= (int64_t)1 << 31 ? n : 0;
}
template int64_t attn_bwd_ds_elems<float>(const AttnCore&);
template int64_t attn_bwd_ds_elems<bf16>(const AttnCore&);

template int64_t attn_bwd_groups<float>(const AttnCore&);
template int64_t attn_bwd_groups<bf16>(const AttnCore&);

template <typename T>
evo_status_t attn_bwd(const Ctx& c, const AttnCore& a, const AttnGrad& g) {
  if (c.dry) return EVO_OK;
  if (!attn_shape_ok(a)) return EVO_ESHAPE;
  switch (a.D) {
    case 8: return launch_bwd<T, 8>(c, a, g);
    case 16: return launch_bwd<T, 16>(c, a, g);
    case 32: return launch_bwd<T, 32>(c, a, g);
    default: return launch_bwd<T, 64>(c, a, g);
  }
}

template evo_status_t attn_fwd<float>(const Ctx&, const AttnCore&);
template evo_status_t attn_fwd<bf16>(const Ctx&, const AttnCore&);
template evo_status_t attn_bwd<float>(const Ctx&, const AttnCore&, const AttnGrad&);
template evo_status_t attn_bwd<bf16>(const Ctx&, const AttnCore&, const AttnGrad&);

}  // namespace evo
