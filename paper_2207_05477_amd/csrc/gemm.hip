// Generic MFMA GEMM (gfx950): BF16 via v_mfma_f32_16x16x32_bf16, FP32 via
// v_mfma_f32_16x16x4_f32, FP32 accumulation, 256 threads (4 wave64s) per
// workgroup, double-buffered LDS tiles with a register prefetch of the next
// k-tile, fused elementwise epilogue.
#include <algorithm>
#include <string>

#include "gemm.h"

#include <type_traits>

namespace evo {

template <typename T> struct GemmTraits;
template <> struct GemmTraits<bf16> { static constexpr int BK = 64; static constexpr int VEC = 8; };
template <> struct GemmTraits<float> { static constexpr int BK = 32; static constexpr int VEC = 4; };
// VEC elements make one 16-byte group; a BK-wide LDS row holds 8 groups.

EVO_DEV int64_t addr2(int64_t r, int64_t lo, int64_t hi, int shift) {
  return shift < 0 ? r * lo : (r >> shift) * hi + (r & ((1LL << shift) - 1)) * lo;
}

// LDS tile [rows][BK]: row r starts at r * LDK elements (one group of padding);
// its 16-byte groups are XOR-permuted by (r >> 3) & 7, so that the transposing
// stores of row-contiguous operands (eight rows per lane) and the fragment
// reads of the MFMA loop both spread over the banks.
EVO_DEV int swz(int r) { return (r >> 3) & 7; }

template <int NB> struct Chunk;
template <> struct Chunk<2> { typedef uint16_t type; };
template <> struct Chunk<4> { typedef uint32_t type; };
template <> struct Chunk<8> { typedef uint2 type; };
template <> struct Chunk<16> { typedef uint4 type; };

// One operand tile (BROWS rows x BK reduction indices), global -> registers -> LDS.
// k-contiguous operands keep two register slots, so that the global loads of a
// tile are issued two k-tiles ahead of its use; the transposing loader keeps
// one (its registers are dearer).  k-contiguous operands move as 16-byte vectors
// along k.  Row-contiguous operands (rows contiguous, k strided) are read as
// 16-byte vectors of VEC rows at KB consecutive k, transposed in registers and
// stored as KB-element runs along k.  `ks`: plain k addressing (k_shift < 0),
// the per-tile offset is a constant step.  KC: the operand is k-contiguous.
template <typename T, int BROWS, bool KC>
struct TileLoader {
  static constexpr int BK = GemmTraits<T>::BK;
  static constexpr int VEC = GemmTraits<T>::VEC;
  static constexpr int LDK = BK + VEC;
  // k-contiguous layout
  static constexpr int NV = BROWS * BK / VEC;
  static constexpr int PASSES = (NV + 255) / 256;
  // row-contiguous layout
  static constexpr int KB0 = BROWS * BK / (VEC * 256);
  static constexpr int KB = KB0 < 1 ? 1 : (KB0 > VEC ? VEC : KB0);
  static constexpr int RB = BROWS / VEC;
  static constexpr int NBLK = RB * (BK / KB);
  static constexpr int NR = KC ? PASSES : KB;
  static constexpr int SLOTS = KC ? 2 : 1;
  static_assert(NBLK <= 256, "one transposed block per thread");

  uint4 regs[SLOTS][NR];
  const T* ptr[PASSES];
  int kk_[PASSES];
  int lds_[PASSES];
  bool ok[PASSES];
  bool ks, rfull;

  EVO_DEV void init(const GemmOperand& op, const T* base, int64_t rows_total, int64_t row0, int64_t kbeg,
                    int tid) {
    ks = op.k_shift < 0;
    rfull = row0 + BROWS <= rows_total && (KC ? NV % 256 == 0 : NBLK == 256);
    if constexpr (KC) {
#pragma unroll
      for (int p = 0; p < PASSES; ++p) {
        const int v = tid + 256 * p;
        const int r = v >> 3, g = v & 7;
        kk_[p] = g * VEC;
        ok[p] = (v < NV) && (row0 + r < rows_total);
        const int64_t roff = ok[p] ? addr2(row0 + r, op.r_lo, op.r_hi, op.r_shift) : 0;
        ptr[p] = base + roff + (ks ? kbeg + kk_[p] : 0);
        lds_[p] = r * LDK + VEC * (g ^ swz(r));
      }
    } else {
      const int rb = tid % RB, kb = tid / RB;
      const int r0 = rb * VEC;
      kk_[0] = kb * KB;
      ok[0] = (tid < NBLK) && (row0 + r0 < rows_total);
      const int64_t roff = ok[0] ? addr2(row0 + r0, 1, op.r_hi, op.r_shift) : 0;
      ptr[0] = base + roff + (ks ? (kbeg + kk_[0]) * op.k_lo : 0);
      lds_[0] = r0;
    }
  }
  // k0: first reduction index of the tile; kt_off = k0 - kbeg
  template <int S>
  EVO_DEV void load(const GemmOperand& op, int64_t k0, int64_t kt_off, int64_t kend) {
    const bool full = k0 + BK <= kend;   // uniform: no reduction index of the tile is out of range
    if constexpr (KC) {
      if (ks && full && rfull) {
#pragma unroll
        for (int p = 0; p < PASSES; ++p) regs[S][p] = *(const uint4*)(ptr[p] + kt_off);
      } else {
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
          const int64_t gk = k0 + kk_[p];
          if (ok[p] && gk < kend) {
            const T* a = ks ? ptr[p] + kt_off : ptr[p] + addr2(gk, 1, op.k_hi, op.k_shift);
            regs[S][p] = *(const uint4*)a;
          } else {
            regs[S][p] = make_uint4(0, 0, 0, 0);
          }
        }
      }
    } else {
      if (ks && full && rfull) {
        const T* a = ptr[0] + kt_off * op.k_lo;
#pragma unroll
        for (int q = 0; q < KB; ++q) regs[S][q] = *(const uint4*)(a + q * op.k_lo);
      } else {
#pragma unroll
        for (int q = 0; q < KB; ++q) {
          const int64_t gk = k0 + kk_[0] + q;
          if (ok[0] && gk < kend) {
            const T* a = ks ? ptr[0] + (kt_off + q) * op.k_lo : ptr[0] + addr2(gk, op.k_lo, op.k_hi, op.k_shift);
            regs[S][q] = *(const uint4*)a;
          } else {
            regs[S][q] = make_uint4(0, 0, 0, 0);
          }
        }
      }
    }
  }
  template <int S>
  EVO_DEV void store(T* lds, int tid) {
    if constexpr (KC) {
#pragma unroll
      for (int p = 0; p < PASSES; ++p)
        if (tid + 256 * p < NV) *(uint4*)(lds + lds_[p]) = regs[S][p];
    } else {
      if (tid >= NBLK) return;
      typedef typename Chunk<KB * sizeof(T)>::type C;
      const int r0 = lds_[0], k0 = kk_[0];
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        const int r = r0 + i;
        union { C c; T e[KB]; } u;
#pragma unroll
        for (int q = 0; q < KB; ++q) u.e[q] = ((const T*)&regs[S][q])[i];
        *(C*)(lds + r * LDK + VEC * ((k0 / VEC) ^ swz(r)) + (k0 % VEC)) = u.c;
      }
    }
  }
};

// Epilogue value of output element (m, n) before the store (see GemmEpilogue).
template <typename T>
EVO_DEV float epi_value(const GemmEpilogue& e, int64_t zo, int64_t off, int64_t m, int64_t n, float acc) {
  float v = e.alpha * acc;
  if (e.bias) v += e.bias[n];
  if (e.scale) v *= e.scale[scale_row(e, m) * e.sm_ld + (n >> e.sn_shift) * e.sn_ld];
  if (e.act == ACT_RELU) v = fmaxf(v, 0.0f);
  else if (e.act == ACT_SIGMOID && n >= e.act_n0) v = sigmoidf_(v);
  // auxiliary inputs: own plain strides, or the output's addressing when the m-stride is < 0
  const int64_t roff = e.r_m < 0 ? off : zo + m * e.r_m + n * e.r_n;
  if (e.relu_ref) {
    float r = to_f32(((const T*)e.relu_ref)[roff]);
    v = r > 0.0f ? v : 0.0f;
  }
  if (e.gate) {
    const int64_t goff = e.g_m < 0 ? off : zo + m * e.g_m + n * e.g_n;
    v *= e.gate_f32 ? ((const float*)e.gate)[goff] : to_f32(((const T*)e.gate)[goff]);
  }
  if (e.resid) v += e.resid_f32 ? ((const float*)e.resid)[roff] : to_f32(((const T*)e.resid)[roff]);
  return v;
}

template <typename T>
EVO_DEV void epi_store1(const GemmEpilogue& e, int64_t off, float v) {
  if (e.out_f32) {
    float* o = (float*)e.out + off;
    *o = e.accumulate ? (*o + v) : v;
  } else {
    ((T*)e.out)[off] = from_f32<T>(v);
  }
}

// Four consecutive outputs n..n+3 of row m (contiguous, 4-aligned when vec4).
template <typename T>
EVO_DEV void epi_store4(const GemmEpilogue& e, int z, int64_t m, int64_t n, int64_t N, f32x4 acc, bool vec4) {
  const int64_t zo = (int64_t)z * e.batch;
  if (vec4 && n + 3 < N) {
    const int64_t off = zo + addr2(m, e.m_lo, e.m_hi, e.m_shift) + addr2(n, 1, e.n_hi, e.n_shift);
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = epi_value<T>(e, zo, off + r, m, n + r, acc[r]);
    if (e.out_f32) {
      f32x4* o = (f32x4*)((float*)e.out + off);
      f32x4 w = f32x4{v[0], v[1], v[2], v[3]};
      if (e.accumulate) w += *o;
      *o = w;
    } else {
      typedef __attribute__((__vector_size__(4 * sizeof(T)))) T tx4;
      tx4 w;
#pragma unroll
      for (int r = 0; r < 4; ++r) w[r] = from_f32<T>(v[r]);
      *(tx4*)((T*)e.out + off) = w;
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (n + r >= N) break;
    const int64_t off = zo + addr2(m, e.m_lo, e.m_hi, e.m_shift) + addr2(n + r, e.n_lo, e.n_hi, e.n_shift);
    epi_store1<T>(e, off, epi_value<T>(e, zo, off, m, n + r, acc[r]));
  }
}

// Epilogue over an accumulator tile in LDS for plain strides: the output and
// every auxiliary input are addressed as base + m * ld + n with unit n-stride,
// 4-aligned, so values move as 4-element vectors.  (The host sets `fast` only
// when that holds.)  Each thread owns one 8-column slice of the tile and walks
// its rows; offsets are 32-bit relative to per-tile bases.
template <typename T, int BM, int BN, int ELD>
EVO_DEV void epi_tile_fast(const GemmEpilogue& e, int z, int64_t m0, int64_t n0, int64_t M, int64_t N,
                           const float* et, int tid) {
  typedef __attribute__((__vector_size__(4 * sizeof(T)))) T tx4;
  constexpr int CPR = BN / 8;             // 8-column slices per row
  constexpr int RPP = 256 / CPR;          // rows per pass
  const int cs = tid % CPR, r0 = tid / CPR;
  const int nl = cs * 8;
  const int64_t zo = (int64_t)z * e.batch;
  const int ld = (int)e.m_lo;
  const int rld = e.r_m < 0 ? ld : (int)e.r_m;
  const int gld = e.g_m < 0 ? ld : (int)e.g_m;
  const int64_t obase = zo + m0 * e.m_lo + n0 + nl;
  const int64_t rbase = e.r_m < 0 ? obase : zo + m0 * e.r_m + n0 + nl;
  const int64_t gbase = e.g_m < 0 ? obase : zo + m0 * e.g_m + n0 + nl;
  const int ml_lim = (int)(M - m0 < BM ? M - m0 : BM);
  const int nvalid = (int)(N - n0 - nl < 8 ? N - n0 - nl : 8);
  if (nvalid <= 0) return;
  float* outf = (float*)e.out + obase;
  T* outt = (T*)e.out + obase;
  const float* rf = e.resid_f32 ? (const float*)e.resid + rbase : nullptr;
  const T* rt = e.resid && !e.resid_f32 ? (const T*)e.resid + rbase : nullptr;
  const T* rr = e.relu_ref ? (const T*)e.relu_ref + rbase : nullptr;
  const float* gf = e.gate && e.gate_f32 ? (const float*)e.gate + gbase : nullptr;
  const T* gt = e.gate && !e.gate_f32 ? (const T*)e.gate + gbase : nullptr;
  f32x4 b0 = f32x4{0.f, 0.f, 0.f, 0.f}, b1 = b0;
  if (e.bias && nvalid == 8) {
    b0 = *(const f32x4*)(e.bias + n0 + nl);
    b1 = *(const f32x4*)(e.bias + n0 + nl + 4);
  }
  const int sig0 = e.act == ACT_SIGMOID ? (int)(e.act_n0 - n0 - nl) : 1 << 30;   // first sigmoid column
  for (int ml = r0; ml < ml_lim; ml += RPP) {
    f32x4 v0 = *(const f32x4*)(et + ml * ELD + nl);
    f32x4 v1 = *(const f32x4*)(et + ml * ELD + nl + 4);
    if (nvalid < 8) {
      // ragged right edge of the output
      const float a8[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
      for (int r = 0; r < nvalid; ++r) {
        const int64_t off = obase + (int64_t)ml * ld + r;
        epi_store1<T>(e, off, epi_value<T>(e, zo, off, m0 + ml, n0 + nl + r, a8[r]));
      }
      continue;
    }
    v0 *= e.alpha;
    v1 *= e.alpha;
    v0 += b0;
    v1 += b1;
    if (e.act == ACT_RELU) {
#pragma unroll
      for (int r = 0; r < 4; ++r) { v0[r] = fmaxf(v0[r], 0.0f); v1[r] = fmaxf(v1[r], 0.0f); }
    } else if (sig0 < 8) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r >= sig0) v0[r] = sigmoidf_(v0[r]);
        if (r + 4 >= sig0) v1[r] = sigmoidf_(v1[r]);
      }
    }
    const int ro = ml * rld;
    if (rr) {
      const tx4 q0 = *(const tx4*)(rr + ro), q1 = *(const tx4*)(rr + ro + 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v0[r] = to_f32(q0[r]) > 0.0f ? v0[r] : 0.0f;
        v1[r] = to_f32(q1[r]) > 0.0f ? v1[r] : 0.0f;
      }
    }
    if (gf) {
      const int go = ml * gld;
      v0 *= *(const f32x4*)(gf + go);
      v1 *= *(const f32x4*)(gf + go + 4);
    } else if (gt) {
      const int go = ml * gld;
      const tx4 q0 = *(const tx4*)(gt + go), q1 = *(const tx4*)(gt + go + 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) { v0[r] *= to_f32(q0[r]); v1[r] *= to_f32(q1[r]); }
    }
    if (rf) {
      v0 += *(const f32x4*)(rf + ro);
      v1 += *(const f32x4*)(rf + ro + 4);
    } else if (rt) {
      const tx4 q0 = *(const tx4*)(rt + ro), q1 = *(const tx4*)(rt + ro + 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) { v0[r] += to_f32(q0[r]); v1[r] += to_f32(q1[r]); }
    }
    const int oo = ml * ld;
    if (e.out_f32) {
      f32x4* o = (f32x4*)(outf + oo);
      if (e.accumulate) { v0 += o[0]; v1 += o[1]; }
      o[0] = v0;
      o[1] = v1;
    } else {
      tx4 w0, w1;
#pragma unroll
      for (int r = 0; r < 4; ++r) { w0[r] = from_f32<T>(v0[r]); w1[r] = from_f32<T>(v1[r]); }
      *(tx4*)(outt + oo) = w0;
      *(tx4*)(outt + oo + 4) = w1;
    }
  }
}

// The MFMA is issued with the B fragment first, so that each lane's four
// accumulator rows are four consecutive n of one m.  The accumulator tile then
// goes through LDS (FP32) and the epilogue walks it row by row: 4-element
// vectors, whole output rows per group of lanes.
template <typename T, int BM, int BN, int WAVES_M, int WAVES_N, bool KCA, bool KCB>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g, int32_t ntn, int32_t flags) {
  constexpr int BK = GemmTraits<T>::BK;
  constexpr int VEC = GemmTraits<T>::VEC;
  constexpr int LDK = BK + VEC;
  constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int ELD = BN + 4;                                   // epilogue tile pitch (floats)
  constexpr int MAIN_BYTES = 2 * (BM + BN) * LDK * (int)sizeof(T);
  constexpr int EPI_BYTES = BM * ELD * 4;
  static_assert(WAVES_M * WAVES_N == 4, "4 waves");
  static_assert(TM >= 1 && TN >= 1, "wave tile");
  __shared__ __attribute__((aligned(16))) char smem[MAIN_BYTES > EPI_BYTES ? MAIN_BYTES : EPI_BYTES];
  T (*lds)[(BM + BN) * LDK] = (T (*)[(BM + BN) * LDK])smem;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  // XCD-aware order (see xcd_order): each XCD gets a contiguous run of tiles,
  // so shared row panels stay in its L2
  const int tile = xcd_order(blockIdx.x, gridDim.x);
  const int64_t m0 = (int64_t)(tile / ntn) * BM;
  const int64_t n0 = (int64_t)(tile % ntn) * BN;
  const int z = blockIdx.z;

  const T* Ap = (const T*)g.A.ptr;
  const T* Bp = (const T*)g.B.ptr;
  int64_t kbeg = 0, kend = g.K;
  if (g.split_k > 1) {
    int64_t per = ((g.K + g.split_k - 1) / g.split_k + BK - 1) / BK * BK;
    kbeg = (int64_t)z * per;
    kend = kbeg + per < g.K ? kbeg + per : g.K;
  } else {
    Ap += (int64_t)z * g.A.batch;
    Bp += (int64_t)z * g.B.batch;
  }

  TileLoader<T, BM, KCA> la;
  TileLoader<T, BN, KCB> lb;
  la.init(g.A, Ap, g.M, m0, kbeg, tid);
  lb.init(g.B, Bp, g.N, n0, kbeg, tid);

  f32x4 acc[TN][TM];
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int i = 0; i < TM; ++i) acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nk = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;
  if (nk > 0) {
    la.template load<0>(g.A, kbeg, 0, kend);
    lb.template load<0>(g.B, kbeg, 0, kend);
  }
  if (nk > 1) {
    if constexpr (KCA) la.template load<1>(g.A, kbeg + BK, BK, kend);
    if constexpr (KCB) lb.template load<1>(g.B, kbeg + BK, BK, kend);
  }
  if (nk > 0) {
    la.template store<0>(lds[0], tid);
    lb.template store<0>(lds[0] + BM * LDK, tid);
  }
  __syncthreads();

  const int lr = lane & 15, lg = lane >> 4;
  // per-fragment LDS row offsets and swizzles
  int arow[TM], asw[TM], brow[TN], bsw[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int r = wm * WM + i * 16 + lr;
    arow[i] = r * LDK;
    asw[i] = swz(r);
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int r = wn * WN + j * 16 + lr;
    brow[j] = BM * LDK + r * LDK;
    bsw[j] = swz(r);
  }

  auto compute = [&](const T* s) {
#pragma unroll
    for (int kq = 0; kq < 2; ++kq) {   // two k-steps of four groups per tile
      const int grp = kq * 4 + lg;
      if constexpr (sizeof(T) == 2) {
        bf16x8 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const bf16x8*)(s + arow[i] + VEC * (grp ^ asw[i]));
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = *(const bf16x8*)(s + brow[j] + VEC * (grp ^ bsw[j]));
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int i = 0; i < TM; ++i) acc[j][i] = mfma_bf16(bfr[j], af[i], acc[j][i]);
      } else {
        f32x4 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const f32x4*)(s + arow[i] + VEC * (grp ^ asw[i]));
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = *(const f32x4*)(s + brow[j] + VEC * (grp ^ bsw[j]));
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int i = 0; i < TM; ++i) acc[j][i] = mfma_f32(bfr[j][t], af[i][t], acc[j][i]);
      }
    }
  };

  // Tile kt sits in LDS buffer kt & 1.  A two-slot (k-contiguous) loader has
  // tile kt + 1 waiting in slot (kt + 1) & 1 and fetches tile kt + 2 into slot
  // kt & 1 (freed when tile kt went to LDS); a one-slot loader fetches tile
  // kt + 1 at the start of the iteration.  Only loads and stores branch on the
  // slot, so the register slots stay compile-time.
#define EVO_ADVANCE(L, OP, KCX)                                                  \
  do {                                                                           \
    if constexpr (KCX) {                                                         \
      if (kt + 2 < nk) {                                                         \
        const int64_t off = (int64_t)(kt + 2) * BK;                              \
        if (cur == 0) L.template load<0>(OP, kbeg + off, off, kend);             \
        else L.template load<1>(OP, kbeg + off, off, kend);                      \
      }                                                                          \
    } else if (kt + 1 < nk) {                                                    \
      const int64_t off = (int64_t)(kt + 1) * BK;                                \
      L.template load<0>(OP, kbeg + off, off, kend);                             \
    }                                                                            \
  } while (0)
#define EVO_COMMIT(L, DST, KCX)                                                  \
  do {                                                                           \
    if (kt + 1 < nk) {                                                           \
      if constexpr (KCX) {                                                       \
        if (cur == 0) L.template store<1>(DST, tid);                             \
        else L.template store<0>(DST, tid);                                      \
      } else {                                                                   \
        L.template store<0>(DST, tid);                                           \
      }                                                                          \
    }                                                                            \
  } while (0)
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    EVO_ADVANCE(la, g.A, KCA);
    EVO_ADVANCE(lb, g.B, KCB);
    compute(lds[cur]);
    EVO_COMMIT(la, lds[cur ^ 1], KCA);
    EVO_COMMIT(lb, lds[cur ^ 1] + BM * LDK, KCB);
    __syncthreads();
  }
#undef EVO_ADVANCE
#undef EVO_COMMIT

  // the last loop iteration ended with a barrier: the operand tiles are dead
  float* et = (float*)smem;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
      *(f32x4*)(et + (wm * WM + i * 16 + lr) * ELD + wn * WN + j * 16 + lg * 4) = acc[j][i];
  __syncthreads();
  if (flags & 2) {
    epi_tile_fast<T, BM, BN, ELD>(g.epi, z, m0, n0, g.M, g.N, et, tid);
    return;
  }
  constexpr int CPR = BN / 4;   // 4-element chunks per row
  for (int c = tid; c < BM * CPR; c += 256) {
    const int ml = c / CPR, nl = (c % CPR) * 4;
    const int64_t m = m0 + ml, n = n0 + nl;
    if (m < g.M && n < g.N) epi_store4<T>(g.epi, z, m, n, g.N, *(const f32x4*)(et + ml * ELD + nl), (flags & 1) != 0);
  }
}

// ============================================================== plain-stride kernel
// The common case: operands whose k-tile advance is a constant step (plain k,
// or two-level k whose low block divides the tile), rows at fixed offsets,
// 4-aligned outputs.  Loads and stores go through buffer resources with 32-bit
// offsets (the k-tile step is a scalar offset), rows beyond the problem are
// clamped to the last row (their products only feed discarded outputs),
// reduction indices beyond the range read as zero, and out-of-range output
// elements get an offset past the resource's extent, which the hardware drops.
typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4;
typedef __attribute__((__vector_size__(2 * sizeof(int)))) int i32x2;
constexpr int kBufFlags = 0x00020000;   // raw 32-bit buffer, gfx9 family
constexpr uint32_t kOOB = 0x80000000u;  // an offset beyond every extent

struct PlainInfo {
  uint32_t ext_a, ext_b;       // bytes of one A / B slice
  int32_t ldo;                 // output row stride (elements)
  uint32_t ext_o;              // bytes of one output slice
  int32_t ldr, ldg;            // resid/relu_ref and gate row strides (elements)
  uint32_t ext_r, ext_g;
};

EVO_DEV __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, kBufFlags);
}

template <typename T, int BROWS, bool KC>
struct PlainLoader {
  static constexpr int BK = GemmTraits<T>::BK;
  static constexpr int VEC = GemmTraits<T>::VEC;
  static constexpr int LDK = BK + VEC;
  static constexpr int NV = BROWS * BK / VEC;
  static constexpr int PASSES = (NV + 255) / 256;
  static constexpr int KB0 = BROWS * BK / (VEC * 256);
  static constexpr int KB = KB0 < 1 ? 1 : (KB0 > VEC ? VEC : KB0);
  static constexpr int RB = BROWS / VEC;
  static constexpr int NBLK = RB * (BK / KB);
  static constexpr int NR = KC ? PASSES : KB;

  __amdgpu_buffer_rsrc_t rs;
  i32x4 regs[1][NR];
  uint32_t voff[PASSES];
  int kk_[PASSES];
  int lds_[PASSES];
  uint32_t step;     // bytes per k-tile
  uint32_t krow;     // bytes between consecutive k (row-contiguous)

  EVO_DEV static int a32(int r, int lo, int hi, int shift) {
    return shift < 0 ? r * lo : (r >> shift) * hi + (r & ((1 << shift) - 1)) * lo;
  }
  EVO_DEV void init(const void* base, uint32_t ext, const GemmOperand& op, int rows, int row0, int kbeg,
                    int tid) {
    rs = rsrc(base, ext);
    const int rlo = (int)op.r_lo, rhi = (int)op.r_hi, klo = (int)op.k_lo, khi = (int)op.k_hi;
    // per k-tile step: BK along plain k, BK >> k_shift low blocks along two-level k
    step = (uint32_t)((op.k_shift < 0 ? BK * klo : (BK >> op.k_shift) * khi) * (int)sizeof(T));
    if constexpr (KC) {
#pragma unroll
      for (int p = 0; p < PASSES; ++p) {
        const int v = tid + 256 * p;
        const int r = v >> 3, g = v & 7;
        kk_[p] = g * VEC;
        int gr = row0 + r;
        gr = gr < rows ? gr : rows - 1;
        voff[p] = (v < NV) ? (uint32_t)((a32(gr, rlo, rhi, op.r_shift) + a32(kbeg + kk_[p], klo, khi, op.k_shift)) *
                                        (int)sizeof(T))
                           : kOOB;
        lds_[p] = r * LDK + VEC * (g ^ swz(r));
      }
    } else {
      krow = (uint32_t)(klo * (int)sizeof(T));
      const int rb = tid % RB, kb = tid / RB;
      int r0 = row0 + rb * VEC;
      r0 = r0 < rows ? r0 : rows - VEC;
      kk_[0] = kb * KB;
      voff[0] = tid < NBLK ? (uint32_t)((a32(kbeg + kk_[0], klo, khi, op.k_shift) + a32(r0, rlo, rhi, op.r_shift)) *
                                        (int)sizeof(T))
                           : kOOB;
      lds_[0] = rb * VEC;
    }
  }
  // Tile kt into register slot S.  The slot must be a compile-time constant and
  // nothing may inspect the loaded values before store(): the loads then stay
  // in flight until the LDS store that consumes them.
  template <int S>
  EVO_DEV void load(int kt) {
    const uint32_t so = (uint32_t)kt * step;
    if constexpr (KC) {
#pragma unroll
      for (int p = 0; p < PASSES; ++p) regs[S][p] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff[p], so, 0);
    } else {
#pragma unroll
      for (int q = 0; q < KB; ++q)
        regs[S][q] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff[0] + q * krow, so, 0);
    }
  }
  // Adds slot S's values to the thread's column sums (row-contiguous layout:
  // VEC consecutive rows r0.. at KB reduction indices), with the tail-tile
  // indices at krem and beyond counted as zeros, as store() writes them.
  template <int S>
  EVO_DEV void colsum_acc(float* cs, int tid, int krem) const {
    if constexpr (!KC) {
      if (tid >= NBLK) return;
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        if (krem < BK && kk_[0] + q >= krem) continue;
        const T* e = (const T*)&regs[S][q];
#pragma unroll
        for (int i = 0; i < VEC; ++i) cs[i] += to_f32(e[i]);
      }
    }
  }
  // Slot S to LDS; `krem` = reduction indices left from the tile start: on a
  // tail tile (krem < BK) the indices beyond it are stored as zeros.
  template <int S>
  EVO_DEV void store(T* lds, int tid, int krem) {
    if constexpr (KC) {
#pragma unroll
      for (int p = 0; p < PASSES; ++p) {
        i32x4 v = regs[S][p];
        if (krem < BK && kk_[p] >= krem) v = i32x4{0, 0, 0, 0};
        if (tid + 256 * p < NV) *(i32x4*)(lds + lds_[p]) = v;
      }
    } else {
      if (tid >= NBLK) return;
      typedef typename Chunk<KB * sizeof(T)>::type C;
      const int r0 = lds_[0], k0 = kk_[0];
      i32x4 v[KB];
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        v[q] = regs[S][q];
        if (krem < BK && k0 + q >= krem) v[q] = i32x4{0, 0, 0, 0};
      }
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        const int r = r0 + i;
        union { C c; T e[KB]; } u;
#pragma unroll
        for (int q = 0; q < KB; ++q) u.e[q] = ((const T*)&v[q])[i];
        *(C*)(lds + r * LDK + VEC * ((k0 / VEC) ^ swz(r)) + (k0 % VEC)) = u.c;
      }
    }
  }
};

template <typename T>
EVO_DEV f32x4 load4(__amdgpu_buffer_rsrc_t r, uint32_t off, bool f32) {
  if (f32) {
    const i32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return f32x4{__int_as_float(q[0]), __int_as_float(q[1]), __int_as_float(q[2]), __int_as_float(q[3])};
  }
  if constexpr (sizeof(T) == 2) {
    const i32x2 q = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    const T* e = (const T*)&q;
    return f32x4{to_f32(e[0]), to_f32(e[1]), to_f32(e[2]), to_f32(e[3])};
  } else {
    const i32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return f32x4{__int_as_float(q[0]), __int_as_float(q[1]), __int_as_float(q[2]), __int_as_float(q[3])};
  }
}

// LDS buffers of the plain kernel: with both operands k-contiguous (the
// stores are plain vector copies) one buffer and two barriers per k-step, so
// that three workgroups fit on a CU; with a transposing operand two buffers.
template <bool KCA, bool KCB> struct PlainPipe {
  static constexpr int NBUF = (KCA && KCB) ? 1 : 2;
  static constexpr int WAVES_PER_EU = (KCA && KCB) ? 3 : 1;   // 1: no request
};

template <typename T, int BM, int BN, int WAVES_M, int WAVES_N, bool KCA, bool KCB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PlainPipe<KCA, KCB>::WAVES_PER_EU)))
void gemm_plain_kernel(GemmArgs g, PlainInfo pi, int32_t ntn) {
  constexpr int BK = GemmTraits<T>::BK;
  constexpr int VEC = GemmTraits<T>::VEC;
  constexpr int LDK = BK + VEC;
  constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(WAVES_M * WAVES_N == 4, "4 waves");
  constexpr int NBUF = PlainPipe<KCA, KCB>::NBUF;
  __shared__ __attribute__((aligned(16))) T lds[NBUF][(BM + BN) * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  // XCD-aware order over (tile, batch or k-slice): workgroups are dealt
  // round-robin over the 8 XCDs in linear launch order; each XCD gets a
  // contiguous run of (tile, z), tile fastest, so the tiles sharing a row or
  // column panel of one problem meet in one L2.
  const int ntiles = gridDim.x;
  const int lin = xcd_order(blockIdx.x + ntiles * blockIdx.z, ntiles * gridDim.z);
  const int tile = lin % ntiles;
  // grouped order: bands of 8 row blocks, column blocks outer within a band,
  // so consecutive tiles share a column panel and a band's row panels are
  // reused across all columns while they are still in L2
  constexpr int GRP = 8;
  const int ntm = ntiles / ntn;
  const int band = tile / (GRP * ntn), first = band * GRP;
  const int gs = ntm - first < GRP ? ntm - first : GRP;
  const int tib = tile - band * GRP * ntn;
  const int m0 = (first + tib % gs) * BM;
  const int n0 = (tib / gs) * BN;
  const int z = lin / ntiles;
  const int M = (int)g.M, N = (int)g.N;

  const T* Ap = (const T*)g.A.ptr;
  const T* Bp = (const T*)g.B.ptr;
  int kbeg = 0, kend = (int)g.K;
  if (g.split_k > 1) {
    const int per = (((int)g.K + g.split_k - 1) / g.split_k + BK - 1) / BK * BK;
    kbeg = z * per;
    kend = kbeg + per < (int)g.K ? kbeg + per : (int)g.K;
  } else {
    Ap += (int64_t)z * g.A.batch;
    Bp += (int64_t)z * g.B.batch;
  }
  PlainLoader<T, BM, KCA> la;
  PlainLoader<T, BN, KCB> lb;
  la.init(Ap, pi.ext_a, g.A, M, m0, kbeg, tid);
  lb.init(Bp, pi.ext_b, g.B, N, n0, kbeg, tid);

  f32x4 acc[TN][TM];
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int i = 0; i < TM; ++i) acc[j][i] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  const int kspan = kend - kbeg;
  // column sums of B (workgroups of the first row block only)
  const bool csum = !KCB && g.colsum != nullptr && m0 == 0;
  float cs[VEC];
#pragma unroll
  for (int i = 0; i < VEC; ++i) cs[i] = 0.f;
  if (nk > 0) {
    la.template load<0>(0);
    lb.template load<0>(0);
    la.template store<0>(lds[0], tid, kspan);
    lb.template store<0>(lds[0] + BM * LDK, tid, kspan);
    if (csum) lb.template colsum_acc<0>(cs, tid, kspan);
  }
  if (nk > 1) {
    la.template load<0>(1);
    lb.template load<0>(1);
  }
  __syncthreads();

  const int lr = lane & 15, lg = lane >> 4;
  int arow[TM], asw[TM], brow[TN], bsw[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int r = wm * WM + i * 16 + lr;
    arow[i] = r * LDK;
    asw[i] = swz(r);
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int r = wn * WN + j * 16 + lr;
    brow[j] = BM * LDK + r * LDK;
    bsw[j] = swz(r);
  }
  auto compute = [&](const T* s) {
#pragma unroll
    for (int kq = 0; kq < 2; ++kq) {
      const int grp = kq * 4 + lg;
      if constexpr (sizeof(T) == 2) {
        bf16x8 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const bf16x8*)(s + arow[i] + VEC * (grp ^ asw[i]));
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = *(const bf16x8*)(s + brow[j] + VEC * (grp ^ bsw[j]));
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int i = 0; i < TM; ++i) acc[j][i] = mfma_bf16(bfr[j], af[i], acc[j][i]);
      } else {
        f32x4 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const f32x4*)(s + arow[i] + VEC * (grp ^ asw[i]));
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = *(const f32x4*)(s + brow[j] + VEC * (grp ^ bsw[j]));
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int i = 0; i < TM; ++i) acc[j][i] = mfma_f32(bfr[j][t], af[i][t], acc[j][i]);
      }
    }
  };
  if constexpr (NBUF == 1) {
    // One buffer: the products of tile kt, a barrier, the store of tile kt + 1
    // (loaded during the products) and the loads of tile kt + 2, a barrier.
    for (int kt = 0; kt < nk; ++kt) {
      compute(lds[0]);
      if (kt + 1 < nk) {
        __syncthreads();
        const int krem = kspan - (kt + 1) * BK;
        la.template store<0>(lds[0], tid, krem);
        lb.template store<0>(lds[0] + BM * LDK, tid, krem);
        if (csum) lb.template colsum_acc<0>(cs, tid, krem);
        if (kt + 2 < nk) {
          la.template load<0>(kt + 2);
          lb.template load<0>(kt + 2);
        }
        __syncthreads();
      }
    }
  } else {
    // Two buffers, tile kt in buffer kt & 1.  A step first stores tile kt + 1
    // (its loads were issued a whole step earlier) into the other buffer, then
    // issues the loads of tile kt + 2 into the freed registers, then runs the
    // products of tile kt; one barrier ends the step.
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      if (kt + 1 < nk) {
        T* dst = lds[cur ^ 1];
        const int krem = kspan - (kt + 1) * BK;
        la.template store<0>(dst, tid, krem);
        lb.template store<0>(dst + BM * LDK, tid, krem);
        if (csum) lb.template colsum_acc<0>(cs, tid, krem);
        if (kt + 2 < nk) {
          la.template load<0>(kt + 2);
          lb.template load<0>(kt + 2);
        }
      }
      compute(lds[cur]);
      __syncthreads();
    }
  }

  if (csum) {
    // threads of one column block (tid % RB) hold partial sums over their k
    // offsets (tid / RB): summed through the idle LDS in a fixed order
    using LB = PlainLoader<T, BN, KCB>;
    float* red = (float*)&lds[0][0];
    __syncthreads();
    if (tid < LB::NBLK) {
      const int rb = tid % LB::RB, kb = tid / LB::RB;
#pragma unroll
      for (int i = 0; i < VEC; ++i) red[kb * BN + rb * VEC + i] = cs[i];
    }
    __syncthreads();
    if (tid < BN && n0 + tid < N) {
      float t = 0.f;
      for (int kb = 0; kb < LB::NBLK / LB::RB; ++kb) t += red[kb * BN + tid];
      g.colsum[(int64_t)z * N + n0 + tid] = t;
    }
    __syncthreads();
  }
  // epilogue straight from the accumulators: lane holds n..n+3 of row m
  const GemmEpilogue& e = g.epi;
  const int64_t zo = (int64_t)z * e.batch;
  const bool of32 = e.out_f32 != 0;
  const size_t osz = of32 ? 4 : sizeof(T);
  const __amdgpu_buffer_rsrc_t ro = rsrc((const char*)e.out + zo * osz, pi.ext_o);
  const size_t rsz = e.resid_f32 ? 4 : sizeof(T);
  const size_t gsz = e.gate_f32 ? 4 : sizeof(T);
  __amdgpu_buffer_rsrc_t rr = ro, rg = ro, rrl = ro;
  if (e.resid) rr = rsrc((const char*)e.resid + zo * rsz, pi.ext_r);
  if (e.relu_ref) rrl = rsrc((const char*)e.relu_ref + zo * sizeof(T), pi.ext_r);
  if (e.gate) rg = rsrc((const char*)e.gate + zo * gsz, pi.ext_g);
  const float alpha = e.alpha;
  const int mlo = (int)e.m_lo, mhi = (int)e.m_hi, nhi = (int)e.n_hi;
  // BF16 outputs with plain rows go out through LDS as whole 16-byte row
  // chunks: a lane's own 8-byte pieces (a quarter of a 128-byte line per store)
  // were measured to double the bytes written to HBM.
  constexpr int TPO = BN + 8;   // LDS row pitch of the staged output tile (elements)
  static_assert(sizeof(T) != 2 || BM * TPO <= (BM + BN) * LDK, "staged output tile fits the operand LDS");
  // (two-level layouts too: a 16-byte chunk of 8 columns stays contiguous when
  // the column blocks hold a multiple of 8, and rows start 16-byte aligned)
  const bool stage = sizeof(T) == 2 && !of32 && (N & 7) == 0 && (mlo & 7) == 0 &&
                     (e.m_shift < 0 || (mhi & 7) == 0) && (e.n_shift < 0 || (e.n_shift >= 3 && (nhi & 7) == 0)) &&
                     ((((uintptr_t)e.out) + (uintptr_t)zo * osz) & 15) == 0;
  T* sto = &lds[0][0];
  if (stage) __syncthreads();   // the operand tiles are no longer read
  // row and column offsets of the lane's outputs, once per row / column block
  int mrow[TM], moff[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    mrow[i] = m0 + wm * WM + i * 16 + lr;
    moff[i] = PlainLoader<T, BM, KCA>::a32(mrow[i], mlo, mhi, e.m_shift);
  }
  int ncol[TN], noff[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    ncol[j] = n0 + wn * WN + j * 16 + lg * 4;
    noff[j] = PlainLoader<T, BM, KCA>::a32(ncol[j], 1, nhi, e.n_shift);
  }
  // The epilogue runs one feature at a time over all of the lane's outputs,
  // each behind one uniform test, in the order of GemmEpilogue; the outputs
  // stay in the accumulators.  (Out-of-range elements load zeros through the
  // buffer resources and are dropped at the store.)
  auto inb = [&](int i, int j) { return ncol[j] < N && mrow[i] < M; };
  if (alpha != 1.0f) {
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int i = 0; i < TM; ++i) acc[j][i] = acc[j][i] * alpha;
  }
  if (e.bias) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const f32x4 bj = ncol[j] < N ? *(const f32x4*)(e.bias + ncol[j]) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < TM; ++i) acc[j][i] = acc[j][i] + bj;
    }
  }
  if (e.scale) {
    if (e.sn_shift >= 2) {   // n is a multiple of 4: the lane's 4 columns share one entry
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int64_t sr = scale_row(e, mrow[i]) * e.sm_ld;
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[j][i] *= inb(i, j) ? e.scale[sr + (ncol[j] >> e.sn_shift) * e.sn_ld] : 0.f;
      }
    } else {
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int64_t sr = scale_row(e, mrow[i]) * e.sm_ld;
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[j][i][r] *= inb(i, j) ? e.scale[sr + ((ncol[j] + r) >> e.sn_shift) * e.sn_ld] : 0.f;
      }
    }
  }
  if (e.act == ACT_RELU) {
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[j][i][r] = fmaxf(acc[j][i][r], 0.0f);
  } else if (e.act == ACT_SIGMOID) {
    // columns from act_n0 on (a lane's four columns share the test when act_n0 is a multiple of 4)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      if (ncol[j] >= e.act_n0 && (e.act_n0 & 3) == 0) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[j][i][r] = sigmoidf_(acc[j][i][r]);
      } else if (ncol[j] + 3 >= e.act_n0) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (ncol[j] + r >= e.act_n0) acc[j][i][r] = sigmoidf_(acc[j][i][r]);
      }
    }
  }
  // auxiliary element offsets: the output's addressing (m-stride < 0) or plain rows
  auto aux_off = [&](int i, int j, int64_t sm, int ld) -> uint32_t {
    return (uint32_t)(sm < 0 ? moff[i] + noff[j] : mrow[i] * ld + ncol[j]);
  };
  if (e.relu_ref) {
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const f32x4 q = load4<T>(rrl, inb(i, j) ? aux_off(i, j, e.r_m, pi.ldr) * (uint32_t)sizeof(T) : kOOB, false);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[j][i][r] = q[r] > 0.0f ? acc[j][i][r] : 0.0f;
      }
  }
  // (one loop per element type of the auxiliary input, so that the loads carry no test)
#define EVO_AUX_PASS(COND, RS, SM, LD, ESZ, F32, OP)                                                   \
  if (COND) {                                                                                       \
    _Pragma("unroll") for (int j = 0; j < TN; ++j)                                                  \
    _Pragma("unroll") for (int i = 0; i < TM; ++i)                                                  \
      acc[j][i] OP load4<T>(RS, inb(i, j) ? aux_off(i, j, SM, LD) * (uint32_t)(ESZ) : kOOB, F32);    \
  }
  if (e.gate) {
    EVO_AUX_PASS(e.gate_f32 != 0, rg, e.g_m, pi.ldg, 4, true, *=)
    else EVO_AUX_PASS(true, rg, e.g_m, pi.ldg, sizeof(T), false, *=)
  }
  if (e.resid) {
    EVO_AUX_PASS(e.resid_f32 != 0, rr, e.r_m, pi.ldr, 4, true, +=)
    else EVO_AUX_PASS(true, rr, e.r_m, pi.ldr, sizeof(T), false, +=)
  }
#undef EVO_AUX_PASS
  // stores: rows outer, column blocks inner, so that the two halves of a row's
  // 128-byte line (FP32 outputs) are written back to back
  if (of32) {
    const bool accu = e.accumulate != 0;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const uint32_t oo = inb(i, j) ? (uint32_t)(moff[i] + noff[j]) * 4u : kOOB;
        f32x4 v = acc[j][i];
        if (accu) v += load4<T>(ro, oo, true);
        const i32x4 w = i32x4{__float_as_int(v[0]), __float_as_int(v[1]), __float_as_int(v[2]), __float_as_int(v[3])};
        __builtin_amdgcn_raw_buffer_store_b128(w, ro, oo, 0, 0);
      }
  } else if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        union { i32x2 q; T e4[4]; } u;
#pragma unroll
        for (int r = 0; r < 4; ++r) u.e4[r] = from_f32<T>(acc[j][i][r]);
        if (stage) {
          *(i32x2*)(sto + (wm * WM + i * 16 + lr) * TPO + wn * WN + j * 16 + lg * 4) = u.q;
        } else {
          const uint32_t oo = inb(i, j) ? (uint32_t)(moff[i] + noff[j]) * 2u : kOOB;
          __builtin_amdgcn_raw_buffer_store_b64(u.q, ro, oo, 0, 0);
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const uint32_t oo = inb(i, j) ? (uint32_t)(moff[i] + noff[j]) * (uint32_t)osz : kOOB;
        const f32x4 v = acc[j][i];
        const i32x4 w = i32x4{__float_as_int(v[0]), __float_as_int(v[1]), __float_as_int(v[2]), __float_as_int(v[3])};
        __builtin_amdgcn_raw_buffer_store_b128(w, ro, oo, 0, 0);
      }
  }
  if constexpr (sizeof(T) == 2) {
    if (stage) {
      __syncthreads();
      constexpr int CPR = BN / 8;   // 16-byte chunks per tile row
      for (int c2 = tid; c2 < BM * CPR; c2 += 256) {
        const int r = c2 / CPR, cl = (c2 - r * CPR) * 8;
        const int m = m0 + r, n = n0 + cl;
        const int mo = PlainLoader<T, BM, KCA>::a32(m, mlo, mhi, e.m_shift);
        const int no = PlainLoader<T, BM, KCA>::a32(n, 1, nhi, e.n_shift);
        const uint32_t off = (m < M && n < N) ? (uint32_t)(mo + no) * 2u : kOOB;
        __builtin_amdgcn_raw_buffer_store_b128(*(const i32x4*)(sto + r * TPO + cl), ro, off, 0, 2);
      }
    }
  }
}

static bool pow2_ok(int32_t shift, int vec) {
  return shift < 0 || (shift < 40 && ((1LL << shift) % vec) == 0);
}

static bool operand_ok(const GemmOperand& o, int64_t rows, int vec, const char* name) {
  if (!o.ptr) { set_error("gemm: operand %s is null", name); return false; }
  if (((uintptr_t)o.ptr) % 16) { set_error("gemm: operand %s not 16-byte aligned", name); return false; }
  if (o.k_contig) {
    if (o.k_lo != 1 || o.r_lo % vec || o.r_hi % vec || o.k_hi % vec || o.batch % vec ||
        !pow2_ok(o.k_shift, vec)) {
      set_error("gemm: operand %s strides do not allow %d-wide loads along k", name, vec);
      return false;
    }
  } else {
    if (o.r_lo != 1 || o.k_lo % vec || o.k_hi % vec || o.r_hi % vec || o.batch % vec ||
        rows % vec || !pow2_ok(o.r_shift, vec)) {
      set_error("gemm: operand %s strides do not allow %d-wide loads along rows", name, vec);
      return false;
    }
  }
  return true;
}

// Largest offset addr2(x) over x < n (two-level addressing need not be monotonic).
static int64_t max_off(int64_t n, int64_t lo, int64_t hi, int32_t shift) {
  if (n <= 0) return 0;
  if (shift < 0) return (n - 1) * lo;
  const int64_t mask = (1LL << shift) - 1, top = (n - 1) >> shift;
  int64_t m = top * hi + ((n - 1) & mask) * lo;
  if (top > 0) m = std::max(m, (top - 1) * hi + mask * lo);
  return m;
}

// Plain-kernel eligibility (see gemm_plain_kernel) and the extents of its buffers.
template <typename T>
static bool plain_info(const GemmArgs& g, PlainInfo& pi) {
  constexpr int BK = GemmTraits<T>::BK, VEC = GemmTraits<T>::VEC;
  const int64_t lim = (1LL << 31) - 4096;
  const int64_t sz = sizeof(T);
  auto op = [&](const GemmOperand& o, int64_t rows, uint32_t& ext) {
    // k: plain, or two-level with a low block that divides the k-tile and holds a load vector
    if (o.k_shift >= 0 && (o.k_shift > 30 || (1LL << o.k_shift) < VEC || BK % (1LL << o.k_shift))) return false;
    if (o.r_shift > 30) return false;
    const int64_t e = (max_off(rows, o.r_lo, o.r_hi, o.r_shift) + max_off(g.K, o.k_lo, o.k_hi, o.k_shift) + 1) * sz;
    if (e <= 0 || e > lim || o.r_lo > lim || o.r_hi > lim || o.k_lo > lim || o.k_hi > lim) return false;
    ext = (uint32_t)e;
    return true;
  };
  if (g.K <= 0 || !op(g.A, g.M, pi.ext_a) || !op(g.B, g.N, pi.ext_b)) return false;
  const GemmEpilogue& e = g.epi;
  const int64_t osz = e.out_f32 ? 4 : sz;
  if (e.n_lo != 1 || g.N % 4 || (e.n_shift >= 0 && (e.n_shift < 2 || e.n_hi % 4)) || e.m_lo % 4 ||
      (e.m_shift >= 0 && e.m_hi % 4) || e.m_lo <= 0 || e.m_shift > 30 || e.n_shift > 30)
    return false;
  if ((g.split_k > 1 || g.batch > 1) && e.batch % 4) return false;
  if (((uintptr_t)e.out) % (4 * osz) || (e.bias && ((uintptr_t)e.bias) % 16)) return false;
  const int64_t out_max = max_off(g.M, e.m_lo, e.m_hi, e.m_shift) + max_off(g.N, 1, e.n_hi, e.n_shift);
  auto ext_of = [&](int64_t maxoff, int64_t esz, uint32_t& ext) {
    const int64_t x = (maxoff + 1) * esz;
    if (x > lim) return false;
    ext = (uint32_t)x;
    return true;
  };
  if (!ext_of(out_max, osz, pi.ext_o) || e.m_lo > lim || e.m_hi > lim || e.n_hi > lim) return false;
  pi.ldo = (int32_t)e.m_lo;
  auto aux = [&](const void* p, int64_t sm, int64_t sn, int64_t esz, int32_t& ld, uint32_t& ext) {
    ld = pi.ldo;
    ext = pi.ext_o;
    if (!p) return true;
    if (((uintptr_t)p) % (4 * esz)) return false;
    if (sm < 0) return ext_of(out_max, esz, ext);
    if (sn != 1 || sm % 4 || sm > lim) return false;
    ld = (int32_t)sm;
    return ext_of((g.M - 1) * sm + g.N - 1, esz, ext);
  };
  const void* rp = e.resid ? e.resid : e.relu_ref;
  if (e.resid && e.relu_ref && e.resid_f32) return false;   // one stride/extent serves both: same element size
  const int64_t rsz = e.resid ? (e.resid_f32 ? 4 : sz) : sz;
  if (!aux(rp, e.r_m, e.r_n, rsz, pi.ldr, pi.ext_r)) return false;
  if (!aux(e.gate, e.g_m, e.g_n, e.gate_f32 ? 4 : sz, pi.ldg, pi.ext_g)) return false;
  return true;
}

template <typename T, int BM, int BN, int WMW, int WNW>
static void launch(const Ctx& ctx, const GemmArgs& g) {
  // profiler names spell the kernel instantiation (as a trace shows it)
  static const std::string shape = std::string(tname<T>()) + ", " + std::to_string(BM) + ", " + std::to_string(BN) + ", " +
                                   std::to_string(WMW) + ", " + std::to_string(WNW);
  static const std::string names[2][4] = {
      {"gemm_kernel<" + shape + ", false, false>", "gemm_kernel<" + shape + ", false, true>",
       "gemm_kernel<" + shape + ", true, false>", "gemm_kernel<" + shape + ", true, true>"},
      {"gemm_plain_kernel<" + shape + ", false, false>", "gemm_plain_kernel<" + shape + ", false, true>",
       "gemm_plain_kernel<" + shape + ", true, false>", "gemm_plain_kernel<" + shape + ", true, true>"}};
  const int64_t ntn = (g.N + BN - 1) / BN, ntm = (g.M + BM - 1) / BM;
  dim3 grid((unsigned)(ntn * ntm), 1, (unsigned)(g.split_k > 1 ? g.split_k : g.batch));
  // four consecutive n of one m form one aligned vector of the output
  const GemmEpilogue& e = g.epi;
  const size_t osz = e.out_f32 ? 4 : sizeof(T);
  const bool vec4 = e.n_lo == 1 && (e.n_shift < 0 || e.n_shift >= 2) && (e.n_shift < 0 || e.n_hi % 4 == 0) &&
                    (e.m_shift < 0 ? e.m_lo % 4 == 0 : (e.m_lo % 4 == 0 && e.m_hi % 4 == 0)) &&
                    e.batch % 4 == 0 && ((uintptr_t)e.out) % (4 * osz) == 0;
  const double nb = g.split_k > 1 ? 1.0 : (double)g.batch;
  const double nout = g.split_k > 1 ? (double)g.split_k : (double)g.batch;
  const double mn = (double)g.M * g.N;
  const double flops = 2.0 * mn * g.K * nb;
  double bytes = ((double)g.M * g.K + (double)g.N * g.K) * sizeof(T) * nb +
                 mn * nout * (g.epi.out_f32 ? 4.0 : sizeof(T)) * (g.epi.accumulate ? 2.0 : 1.0);
  if (g.epi.resid) bytes += mn * nb * (g.epi.resid_f32 ? 4.0 : (double)sizeof(T));
  if (g.epi.gate) bytes += mn * nb * (g.epi.gate_f32 ? 4.0 : (double)sizeof(T));
  if (g.epi.relu_ref) bytes += mn * nb * sizeof(T);
  // plain strides everywhere, 4-aligned: vector epilogue without index arithmetic
  auto al16 = [](const void* p) { return ((uintptr_t)p) % 16 == 0; };
  const size_t tsz = sizeof(T);
  auto aux_ok = [&](const void* p, int64_t sm, int64_t sn, bool f32) {
    if (!p) return true;
    if (((uintptr_t)p) % (4 * (f32 ? 4 : tsz))) return false;
    return sm < 0 || (sn == 1 && sm % 4 == 0);
  };
  const int64_t lim = 1 << 24;   // 32-bit in-tile offsets
  const bool fast = vec4 && e.m_shift < 0 && e.n_shift < 0 && !e.scale && (!e.bias || al16(e.bias)) &&
                    e.m_lo < lim && e.r_m < lim && e.g_m < lim &&
                    aux_ok(e.resid, e.r_m, e.r_n, e.resid_f32 != 0) &&
                    aux_ok(e.relu_ref, e.r_m, e.r_n, false) && aux_ok(e.gate, e.g_m, e.g_n, e.gate_f32 != 0);
  const int32_t nt = (int32_t)ntn, v4 = (vec4 ? 1 : 0) | (fast ? 2 : 0);
  PlainInfo pi;
  const bool plain = plain_info<T>(g, pi);
  const char* nm = names[plain ? 1 : 0][(g.A.k_contig ? 2 : 0) + (g.B.k_contig ? 1 : 0)].c_str();
  if (plain) {
    if (g.A.k_contig && g.B.k_contig)
      EVO_LAUNCH(nm, flops, bytes, (gemm_plain_kernel<T, BM, BN, WMW, WNW, true, true>), grid, dim3(256), 0, ctx.stream, g, pi, nt);
    else if (g.A.k_contig)
      EVO_LAUNCH(nm, flops, bytes, (gemm_plain_kernel<T, BM, BN, WMW, WNW, true, false>), grid, dim3(256), 0, ctx.stream, g, pi, nt);
    else if (g.B.k_contig)
      EVO_LAUNCH(nm, flops, bytes, (gemm_plain_kernel<T, BM, BN, WMW, WNW, false, true>), grid, dim3(256), 0, ctx.stream, g, pi, nt);
    else
      EVO_LAUNCH(nm, flops, bytes, (gemm_plain_kernel<T, BM, BN, WMW, WNW, false, false>), grid, dim3(256), 0, ctx.stream, g, pi, nt);
    return;
  }
  if (g.A.k_contig && g.B.k_contig)
    EVO_LAUNCH(nm, flops, bytes, (gemm_kernel<T, BM, BN, WMW, WNW, true, true>), grid, dim3(256), 0, ctx.stream, g, nt, v4);
  else if (g.A.k_contig)
    EVO_LAUNCH(nm, flops, bytes, (gemm_kernel<T, BM, BN, WMW, WNW, true, false>), grid, dim3(256), 0, ctx.stream, g, nt, v4);
  else if (g.B.k_contig)
    EVO_LAUNCH(nm, flops, bytes, (gemm_kernel<T, BM, BN, WMW, WNW, false, true>), grid, dim3(256), 0, ctx.stream, g, nt, v4);
  else
    EVO_LAUNCH(nm, flops, bytes, (gemm_kernel<T, BM, BN, WMW, WNW, false, false>), grid, dim3(256), 0, ctx.stream, g, nt, v4);
}

template <typename T>
evo_status_t gemm(const Ctx& ctx, const GemmArgs& g) {
  if (ctx.dry) return EVO_OK;
  if (g.M <= 0 || g.N <= 0) return EVO_OK;
  constexpr int VEC = GemmTraits<T>::VEC;
  if ((g.A.k_contig || g.B.k_contig) && g.K % VEC) {
    set_error("gemm: K=%lld not a multiple of %d for loads along k", (long long)g.K, VEC);
    return EVO_ESHAPE;
  }
  if (!operand_ok(g.A, g.M, VEC, "A") || !operand_ok(g.B, g.N, VEC, "B")) return EVO_ESHAPE;
  if (!g.epi.out) { set_error("gemm: null output"); return EVO_EINVAL; }
  if (g.split_k > 1 && !g.epi.out_f32) { set_error("gemm: split-K needs FP32 partials"); return EVO_EINVAL; }
  if (g.colsum) {
    PlainInfo pi;
    if (g.B.k_contig || !plain_info<T>(g, pi)) {
      set_error("gemm: column sums need plain operand layouts with B row-contiguous");
      return EVO_EINVAL;
    }
  }
  if (g.big_tiles && g.M > 16) launch<T, 128, 128, 2, 2>(ctx, g);
  else if (g.M <= 16) launch<T, 16, 128, 1, 4>(ctx, g);
  else if (g.N <= 64 || g.M * g.N <= (int64_t)128 * 128 * 128) launch<T, 64, 64, 2, 2>(ctx, g);
  // 128 x 64 tiles also for wide outputs when both operands are contiguous
  // along k, in BF16 (twice the workgroups of the short-K projections, which are
  // bound by memory latency: measured 9 % faster per launch at K = 128-256) and
  // in FP32 at K <= 128 (3-6 % faster there, slower at K >= 256); a transposing
  // operand keeps 128 x 128
  else if (g.N <= 128 || (g.A.k_contig && g.B.k_contig && (sizeof(T) == 2 || g.K <= 128)))
    launch<T, 128, 64, 2, 2>(ctx, g);
  else launch<T, 128, 128, 2, 2>(ctx, g);
  return check_launch("gemm");
}

template evo_status_t gemm<float>(const Ctx&, const GemmArgs&);
template evo_status_t gemm<bf16>(const Ctx&, const GemmArgs&);

}  // namespace evo
