// Generic MFMA GEMM (gfx950): BF16 via v_mfma_f32_16x16x32_bf16, FP32 via
// v_mfma_f32_16x16x4_f32, FP32 accumulation, 256 threads (4 wave64s) per
// workgroup, double-buffered LDS tiles with a register prefetch of the next
// k-tile, fused elementwise epilogue.
#include <string>

#include "gemm.h"

namespace evo {

template <typename T> struct GemmTraits;
template <> struct GemmTraits<bf16> { static constexpr int BK = 64; static constexpr int VEC = 8; };
template <> struct GemmTraits<float> { static constexpr int BK = 32; static constexpr int VEC = 4; };

EVO_DEV int64_t addr2(int64_t r, int64_t lo, int64_t hi, int shift) {
  return shift < 0 ? r * lo : (r >> shift) * hi + (r & ((1LL << shift) - 1)) * lo;
}

// One operand tile of BROWS rows x BK reduction indices, global -> registers -> LDS.
template <typename T, int BROWS>
struct TileLoader {
  static constexpr int BK = GemmTraits<T>::BK;
  static constexpr int VEC = GemmTraits<T>::VEC;
  static constexpr int NV = BROWS * BK / VEC;
  static constexpr int PASSES = (NV + 255) / 256;
  uint4 regs[PASSES];
  int64_t rowoff[PASSES];
  int r_[PASSES], k_[PASSES];
  bool ok[PASSES];

  EVO_DEV void init(const GemmOperand& op, int64_t rows_total, int64_t row0, int tid) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      int v = tid + 256 * p;
      int r, k;
      if (op.k_contig) { r = v / (BK / VEC); k = (v % (BK / VEC)) * VEC; }
      else             { k = v / (BROWS / VEC); r = (v % (BROWS / VEC)) * VEC; }
      r_[p] = r; k_[p] = k;
      int64_t gr = row0 + r;
      ok[p] = (v < NV) && (gr < rows_total);
      rowoff[p] = ok[p] ? addr2(gr, op.r_lo, op.r_hi, op.r_shift) : 0;
    }
  }
  EVO_DEV void load(const GemmOperand& op, const T* base, int64_t k0, int64_t kend) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      int64_t gk = k0 + k_[p];
      if (ok[p] && gk < kend) {
        int64_t off = rowoff[p] + addr2(gk, op.k_lo, op.k_hi, op.k_shift);
        regs[p] = *(const uint4*)(base + off);
      } else {
        regs[p] = make_uint4(0, 0, 0, 0);
      }
    }
  }
  template <int LDK>
  EVO_DEV void store(const GemmOperand& op, T* lds, int tid) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      int v = tid + 256 * p;
      if (v >= NV) continue;
      if (op.k_contig) {
        *(uint4*)(lds + r_[p] * LDK + k_[p]) = regs[p];
      } else {
        const T* e = (const T*)&regs[p];
#pragma unroll
        for (int i = 0; i < VEC; ++i) lds[(r_[p] + i) * LDK + k_[p]] = e[i];
      }
    }
  }
};

template <typename T>
EVO_DEV void epilogue_apply(const GemmEpilogue& e, int z, int64_t m, int64_t n, float acc) {
  float v = e.alpha * acc;
  if (e.bias) v += e.bias[n];
  if (e.scale) v *= e.scale[(m >> e.sm_shift) * e.sm_ld + (n >> e.sn_shift) * e.sn_ld];
  if (e.act == ACT_RELU) v = fmaxf(v, 0.0f);
  else if (e.act == ACT_SIGMOID && n >= e.act_n0) v = sigmoidf_(v);
  const int64_t zo = (int64_t)z * e.batch;
  int64_t off = zo + addr2(m, e.m_lo, e.m_hi, e.m_shift) + addr2(n, e.n_lo, e.n_hi, e.n_shift);
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
  if (e.out_f32) {
    float* o = (float*)e.out + off;
    *o = e.accumulate ? (*o + v) : v;
  } else {
    ((T*)e.out)[off] = from_f32<T>(v);
  }
}

template <typename T, int BM, int BN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  constexpr int BK = GemmTraits<T>::BK;
  constexpr int LDK = BK + 16 / (int)sizeof(T);      // padded LDS row pitch (elements)
  constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  constexpr int TM = WM / 16, TN = WN / 16;
  static_assert(WAVES_M * WAVES_N == 4, "4 waves");
  static_assert(TM >= 1 && TN >= 1, "wave tile");
  __shared__ __attribute__((aligned(16))) T lds[2][(BM + BN) * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t n0 = (int64_t)blockIdx.x * BN;
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

  TileLoader<T, BM> la;
  TileLoader<T, BN> lb;
  la.init(g.A, g.M, m0, tid);
  lb.init(g.B, g.N, n0, tid);

  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nk = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;
  if (nk > 0) {
    la.load(g.A, Ap, kbeg, kend);
    lb.load(g.B, Bp, kbeg, kend);
    la.template store<LDK>(g.A, lds[0], tid);
    lb.template store<LDK>(g.B, lds[0] + BM * LDK, tid);
  }
  __syncthreads();

  const int lr = lane & 15, lg = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      la.load(g.A, Ap, kbeg + (int64_t)(kt + 1) * BK, kend);
      lb.load(g.B, Bp, kbeg + (int64_t)(kt + 1) * BK, kend);
    }
    const T* sA = lds[cur] + (wm * WM + lr) * LDK;
    const T* sB = lds[cur] + BM * LDK + (wn * WN + lr) * LDK;
    if constexpr (sizeof(T) == 2) {
#pragma unroll
      for (int ks = 0; ks < BK / 32; ++ks) {
        bf16x8 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const bf16x8*)(sA + i * 16 * LDK + ks * 32 + lg * 8);
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = *(const bf16x8*)(sB + j * 16 * LDK + ks * 32 + lg * 8);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = mfma_bf16(af[i], bfr[j], acc[i][j]);
      }
    } else {
#pragma unroll
      for (int kq = 0; kq < BK / 16; ++kq) {
        f32x4 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const f32x4*)(sA + i * 16 * LDK + kq * 16 + lg * 4);
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = *(const f32x4*)(sB + j * 16 * LDK + kq * 16 + lg * 4);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = mfma_f32(af[i][t], bfr[j][t], acc[i][j]);
      }
    }
    if (kt + 1 < nk) {
      la.template store<LDK>(g.A, lds[cur ^ 1], tid);
      lb.template store<LDK>(g.B, lds[cur ^ 1] + BM * LDK, tid);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t n = n0 + wn * WN + j * 16 + lr;
      if (n >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * WM + i * 16 + lg * 4 + r;
        if (m < g.M) epilogue_apply<T>(g.epi, z, m, n, acc[i][j][r]);
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

template <typename T, int BM, int BN, int WMW, int WNW>
static void launch(const Ctx& ctx, const GemmArgs& g) {
  static const std::string nm = std::string("gemm_kernel<") + tname<T>() + ", " + std::to_string(BM) +
                                ", " + std::to_string(BN) + ", " + std::to_string(WMW) + ", " +
                                std::to_string(WNW) + ">";
  dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM),
            (unsigned)(g.split_k > 1 ? g.split_k : g.batch));
  const double nb = g.split_k > 1 ? 1.0 : (double)g.batch;
  const double nout = g.split_k > 1 ? (double)g.split_k : (double)g.batch;
  const double mn = (double)g.M * g.N;
  const double flops = 2.0 * mn * g.K * nb;
  double bytes = ((double)g.M * g.K + (double)g.N * g.K) * sizeof(T) * nb +
                 mn * nout * (g.epi.out_f32 ? 4.0 : sizeof(T)) * (g.epi.accumulate ? 2.0 : 1.0);
  if (g.epi.resid) bytes += mn * nb * (g.epi.resid_f32 ? 4.0 : (double)sizeof(T));
  if (g.epi.gate) bytes += mn * nb * (g.epi.gate_f32 ? 4.0 : (double)sizeof(T));
  if (g.epi.relu_ref) bytes += mn * nb * sizeof(T);
  EVO_LAUNCH(nm.c_str(), flops, bytes, (gemm_kernel<T, BM, BN, WMW, WNW>), grid, dim3(256), 0, ctx.stream, g);
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
  if (g.M <= 16) launch<T, 16, 128, 1, 4>(ctx, g);
  else if (g.N <= 64 || g.M * g.N <= (int64_t)128 * 128 * 128) launch<T, 64, 64, 2, 2>(ctx, g);
  else if (g.N <= 128) launch<T, 128, 64, 2, 2>(ctx, g);
  else launch<T, 128, 128, 2, 2>(ctx, g);
  return check_launch("gemm");
}

template evo_status_t gemm<float>(const Ctx&, const GemmArgs&);
template evo_status_t gemm<bf16>(const Ctx&, const GemmArgs&);

}  // namespace evo
