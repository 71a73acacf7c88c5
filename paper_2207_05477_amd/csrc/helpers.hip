// Helpers shared by the ops: weight-gradient GEMMs (deterministic split-K),
// the small-N pair-bias projection and its backward, segmented column sums.
#include <stdarg.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ops.h"

namespace evo {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char* last_error() { return g_err; }

evo_status_t check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return EVO_EHIP;
  }
  return EVO_OK;
}

// ============================================================== launch profiler
namespace {
struct ProfSlot {
  const char* name;
  hipEvent_t a, b;
  double flops, bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfSlot> g_slots;
std::vector<hipEvent_t> g_pool;
hipEvent_t pool_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

thread_local std::vector<const char*> g_tags;
bool g_prof_detail = false;
std::vector<std::string> g_names;   // "kernel@tag/tag" names of the slots (detail mode)

ProfTag::ProfTag(const char* tag) { g_tags.push_back(tag); }
ProfTag::~ProfTag() { g_tags.pop_back(); }

int prof_begin(const char* name, hipStream_t s, double flops, double bytes) {
  if (!g_prof_on) return -1;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (g_prof_detail) {
    std::string key = std::string(name) + "@";
    for (size_t i = 0; i < g_tags.size(); ++i) key += (i ? "/" : "") + std::string(g_tags[i]);
    g_names.push_back(key);
    name = nullptr;
  }
  ProfSlot sl{name, pool_event(), pool_event(), flops, bytes};
  if (!sl.a || !sl.b) return -1;
  hipEventRecord(sl.a, s);
  g_slots.push_back(sl);
  return (int)g_slots.size() - 1;
}

void prof_end(int slot, hipStream_t s) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  hipEventRecord(g_slots[slot].b, s);
}

// ============================================================== weight gradients
template <typename T>
evo_status_t wgrad_segments(const Ctx& c, Arena& ws, const T* X, int64_t ldx, const T* dY, int64_t ldy,
                            int64_t rows, int64_t M, int nseg, const int* seg_off, const int* seg_n,
                            float* const* dW, float* const* dB) {
  // the span covers every segment (null outputs included): a size query with
  // null gradient pointers carves the same scratch as a real call
  int lo = 1 << 30, hi = 0;
  for (int s = 0; s < nseg; ++s) {
    lo = seg_off[s] < lo ? seg_off[s] : lo;
    hi = seg_off[s] + seg_n[s] > hi ? seg_off[s] + seg_n[s] : hi;
  }
  if (hi <= lo) return EVO_OK;
  const int64_t N = hi - lo;
  // BF16: 128 x 128 tiles split for about 256 workgroups (at least 1024 rows
  // per slice) when both extents allow; else 64 x 64 tiles for about 1024
  // (measured faster for FP32, whose k-tiles are half as deep).  FP32 at four
  // workgroups per CU: the FP32 weight-gradient GEMMs of a C1 step took 1.84 ms
  // split for 512 workgroups, 1.67 ms for 1024 (the partial sums they add cost
  // 0.03 ms more); BF16 split for 512 gained nothing measurable
  // (BF16 outputs of at most 256 x 256 on 64 x 64 tiles too: 28-30 -> 15-20 us
  // per C1 launch; the larger ones measured slower there)
  const bool big = sizeof(T) == 2 && M >= 128 && N >= 128 && M * N > 256 * 256;
  const int64_t tm = big ? 128 : 64;
  const int64_t tiles = ((M + tm - 1) / tm) * ((N + tm - 1) / tm);
  const int64_t target = big ? 256 : 1024;
  auto split_of = [&](int64_t r) {
    int64_t sp = (target + tiles - 1) / tiles;
    const int64_t mx = r / (big ? 1024 : 256) > 0 ? r / (big ? 1024 : 256) : 1;
    if (sp > mx) sp = mx;
    return sp < 1 ? (int64_t)1 : sp;
  };
  // Operands past 2 GiB (the plain GEMM kernel, which also takes the column
  // sums, addresses them with 32-bit buffer offsets): row chunks that fit, each
  // with slices of its own in the partial buffers, all reduced together.
  const int64_t lim = (1LL << 31) - 4096;
  const int64_t ldm = ldx > ldy ? ldx : ldy;
  int64_t crow = rows;
  if ((rows + 1) * ldm * (int64_t)sizeof(T) > lim) crow = (lim / ((int64_t)sizeof(T) * ldm) - 1) / 256 * 256;
  if (crow < 1) { set_error("wgrad: rows of %lld elements too long", (long long)ldm); return EVO_ESHAPE; }
  const int64_t nch = (rows + crow - 1) / crow;
  int64_t split = 0;
  for (int64_t ch = 0; ch < nch; ++ch) split += split_of(rows - ch * crow < crow ? rows - ch * crow : crow);
  const bool direct = split == 1 && nseg == 1;
  float* part = direct ? nullptr : ws.take_n<float>((size_t)split * M * N);
  // bias gradients: the column sums of dY, taken by the GEMM from the dY tiles
  // it loads anyway (one FP32 row per slice), then reduced like dW
  float* cpart = dB ? ws.take_n<float>((size_t)split * N) : nullptr;
  if (c.dry) return EVO_OK;
  bool any = false, anyb = false;
  for (int s = 0; s < nseg; ++s) {
    any = any || dW[s];
    anyb = anyb || (dB && dB[s]);
  }
  if (!any && !anyb) return EVO_OK;
  if (direct && !dW[0]) {
    set_error("wgrad: a bias gradient without its weight gradient");
    return EVO_EINVAL;
  }
  int64_t s0 = 0;
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int64_t r0 = ch * crow, r = rows - r0 < crow ? rows - r0 : crow, sp = split_of(r);
    GemmArgs g;
    g.M = M; g.N = N; g.K = r;
    g.split_k = (int)sp;
    g.big_tiles = big ? 1 : 0;
    g.A = op_colmajor(X + r0 * ldx, ldx);
    g.B = op_colmajor(dY + r0 * ldy + lo, ldy);
    g.colsum = anyb ? cpart + s0 * N : nullptr;
    if (direct) {   // single slice, single segment: accumulate straight into dW
      g.epi = epi_rowmajor(dW[0], N, true);
      g.epi.accumulate = 1;
    } else {
      g.epi = epi_rowmajor(part + s0 * M * N, N, true);
      g.epi.batch = M * N;
    }
    EVO_TRY(gemm<T>(c, g));
    s0 += sp;
  }
  if (anyb) {
    RedSegs rb;
    rb.nseg = nseg;
    for (int s = 0; s < nseg; ++s) { rb.off[s] = seg_off[s] - lo; rb.n[s] = seg_n[s]; rb.out[s] = dB[s]; }
    EVO_TRY(reduce_segments(c, cpart, split, 1, N, rb, true));
  }
  if (direct || !any) return EVO_OK;
  RedSegs rs;
  rs.nseg = nseg;
  for (int s = 0; s < nseg; ++s) { rs.off[s] = seg_off[s] - lo; rs.n[s] = seg_n[s]; rs.out[s] = dW[s]; }
  return reduce_segments(c, part, split, M, N, rs, true);
}

template <typename T>
evo_status_t wgrad(const Ctx& c, Arena& ws, const T* X, int64_t ldx, const T* dY, int64_t ldy,
                   int64_t rows, int64_t M, int64_t N, float* dW, float* const* dB) {
  const int off = 0, n = (int)N;
  return wgrad_segments<T>(c, ws, X, ldx, dY, ldy, rows, M, 1, &off, &n, &dW, dB);
}

// ============================================================== pair-bias projection
template <typename T>
__global__ __launch_bounds__(256) void rowproj_kernel(const T* __restrict__ x, int64_t rows, int C,
                                                      const float* __restrict__ W, int H,
                                                      float* __restrict__ out) {
  extern __shared__ float sW[];  // [C][H]
  for (int e = threadIdx.x; e < C * H; e += 256) sW[e] = W[e];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= rows) return;
  float acc[16];
#pragma unroll
  for (int h = 0; h < 16; ++h) acc[h] = 0.f;
  const T* xr = x + row * C;
  for (int cc = 0; cc < C; ++cc) {
    const float v = to_f32(xr[cc]);
#pragma unroll
    for (int h = 0; h < 16; ++h)
      if (h < H) acc[h] += v * sW[cc * H + h];
  }
#pragma unroll
  for (int h = 0; h < 16; ++h)
    if (h < H) out[(int64_t)h * rows + row] = acc[h];
}

template <typename T>
evo_status_t rowproj(const Ctx& c, const T* x, int64_t rows, int C, const float* W, int H, float* out) {
  if (c.dry || rows == 0) return EVO_OK;
  if (H > 16) { set_error("pair bias: %d heads > 16", H); return EVO_ESHAPE; }
  EVO_LAUNCH(EVO_KNAME("rowproj_kernel", T), 2.0 * (double)rows * C * H, (double)rows * C * sizeof(T) + (double)H * rows * 4.0, (rowproj_kernel<T>), dim3((unsigned)((rows + 255) / 256)), dim3(256),
                     (size_t)C * H * sizeof(float), c.stream, x, rows, C, W, H, out);
  return check_launch("rowproj");
}

// dx[row][c] (+)= sum_h dout[h][row] W[c][h]: a block owns 32 rows; dout for
// them and W sit in LDS; each lane produces 4 consecutive channels of a row.
__global__ __launch_bounds__(256) void rowproj_dx_kernel(int64_t rows, int C, const float* __restrict__ W,
                                                         int H, const float* __restrict__ dout,
                                                         float* dx, int accumulate) {
  extern __shared__ float sm[];          // W [C][H], then dout [H][32]
  float* sW = sm;
  float* sd = sm + C * H;
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int nrow = rows - r0 < 32 ? (int)(rows - r0) : 32;
  for (int e = tid; e < C * H; e += 256) sW[e] = W[e];
  for (int e = tid; e < 32 * H; e += 256) {
    const int h = e >> 5, rr = e & 31;
    sd[e] = rr < nrow ? dout[(int64_t)h * rows + r0 + rr] : 0.f;
  }
  __syncthreads();
  const int cpr = C >> 2;                // lanes per row
  for (int e = tid; e < 32 * cpr; e += 256) {
    const int rr = e / cpr, c0 = (e - rr * cpr) * 4;
    if (rr >= nrow) continue;
    f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int h = 0; h < H; ++h) {
      const float d = sd[h * 32 + rr];
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] += d * sW[(c0 + k) * H + h];
    }
    f32x4* o = (f32x4*)(dx + (r0 + rr) * C + c0);
    if (accumulate) s += *o;
    *o = s;
  }
}

// partial dW over 256-row blocks: part[blk][C*H]; the block's dout rows are
// staged in LDS, each thread owns one channel and a quarter of the rows.
template <typename T>
__global__ __launch_bounds__(256) void rowproj_dw_kernel(const T* __restrict__ x, int64_t rows, int C,
                                                         int H, const float* __restrict__ dout,
                                                         float* __restrict__ part) {
  __shared__ float sd[16 * 256];
  __shared__ float red[256 * 17];
  const int tid = threadIdx.x;
  const int per = 256 / C;            // row subsets (C divides 256)
  const int cc = tid % C, rs = tid / C;
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int nrow = rows - r0 < 256 ? (int)(rows - r0) : 256;
  for (int e = tid; e < H * 256; e += 256) {
    const int h = e >> 8, rr = e & 255;
    sd[e] = rr < nrow ? dout[(int64_t)h * rows + r0 + rr] : 0.f;
  }
  __syncthreads();
  float acc[16];
#pragma unroll
  for (int h = 0; h < 16; ++h) acc[h] = 0.f;
  for (int rr = rs; rr < nrow; rr += per) {
    const float v = to_f32(x[(r0 + rr) * C + cc]);
#pragma unroll
    for (int h = 0; h < 16; ++h)
      if (h < H) acc[h] += v * sd[h * 256 + rr];
  }
#pragma unroll
  for (int h = 0; h < 16; ++h) red[tid * 17 + h] = acc[h];
  __syncthreads();
  for (int e = tid; e < C * H; e += 256) {
    const int c2 = e / H, h = e - c2 * H;
    float s = 0.f;
    for (int q = 0; q < per; ++q) s += red[(q * C + c2) * 17 + h];
    part[(int64_t)blockIdx.x * C * H + e] = s;
  }
}

// Vectorised backward (C % 8 == 0, C <= 512, H <= HM): LPR = C / 8 lanes per
// row, each owning 8 channels (16-byte accesses).  A block owns RB rows; their
// dout values are staged in LDS as [row][HM] (coalesced loads along the rows),
// so a lane reads a row's HM values with vector broadcasts.  A lane's global
// loads of several rows are issued together before they are used.
constexpr int RPV_RB = 256;   // rows per block of the weight-gradient kernel
constexpr int RPX_RB = 64;    // rows per block of the input-gradient kernel
template <int HM, int RB>
EVO_DEV void stage_dout_rows(const float* dout, int64_t rows, int64_t r0, int H, float* sd, int tid) {
  for (int e = tid; e < HM * RB; e += 256) {
    const int h = e / RB, rr = e - h * RB;
    sd[rr * HM + h] = (h < H && r0 + rr < rows) ? dout[(int64_t)h * rows + r0 + rr] : 0.f;
  }
}

// dx[row][c] (+)= sum_h dout[h][row] W[c][h]; the lane's W slice stays in registers.
template <int LPR, int HM>
__global__ __launch_bounds__(256) void rowproj_dx_vec_kernel(int64_t rows, int C, const float* __restrict__ W,
                                                             int H, const float* __restrict__ dout, float* dx,
                                                             int accumulate) {
  __shared__ __attribute__((aligned(16))) float sd[RPX_RB * HM];
  constexpr int RPI = 256 / LPR, NR = RPX_RB / RPI;   // rows per block iteration, rows per lane
  const int tid = threadIdx.x, l = tid & (LPR - 1);
  const int c0 = l * 8;
  const bool cok = c0 < C;
  const int64_t r0 = (int64_t)blockIdx.x * RPX_RB;
  stage_dout_rows<HM, RPX_RB>(dout, rows, r0, H, sd, tid);
  // W staged once per block as [c][HM] (coalesced), the lane's slice read back as vectors
  __shared__ __attribute__((aligned(16))) float sw[8 * LPR * HM];
  for (int e = tid; e < 8 * LPR * HM; e += 256) {
    const int cc = e / HM, h = e - cc * HM;
    sw[e] = (cc < C && h < H) ? W[cc * H + h] : 0.f;
  }
  float prev[NR][8];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int64_t row = r0 + tid / LPR + j * RPI;
    if (accumulate && cok && row < rows) ld8(dx + row * C + c0, prev[j]);
    else
#pragma unroll
      for (int i = 0; i < 8; ++i) prev[j][i] = 0.f;
  }
  __syncthreads();
  float w[8][HM];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int h = 0; h < HM; h += 4) {
      const f32x4 q = *(const f32x4*)(sw + (c0 + i) * HM + h);
      w[i][h] = q[0]; w[i][h + 1] = q[1]; w[i][h + 2] = q[2]; w[i][h + 3] = q[3];
    }
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int rr = tid / LPR + j * RPI;
    const int64_t row = r0 + rr;
    if (row >= rows || !cok) continue;
    float d[HM];
#pragma unroll
    for (int h = 0; h < HM; h += 4) {
      const f32x4 q = *(const f32x4*)(sd + rr * HM + h);
      d[h] = q[0]; d[h + 1] = q[1]; d[h + 2] = q[2]; d[h + 3] = q[3];
    }
    float o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float t = 0.f;
#pragma unroll
      for (int h = 0; h < HM; ++h) t += d[h] * w[i][h];
      o[i] = t + prev[j][i];
    }
    st8(dx + row * C + c0, o);
  }
}

// part[blk][c * H + h] = sum over the block's rows of x[row][c] dout[h][row]:
// per-lane sums over the rows it visits, then the lanes sharing channels are
// combined by xor shuffles (within a wave) and through LDS (across the 4
// waves), in a fixed order.
template <typename T, int LPR, int HM>
__global__ __launch_bounds__(256) void rowproj_dw_vec_kernel(const T* __restrict__ x, int64_t rows, int C, int H,
                                                             const float* __restrict__ dout,
                                                             float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) float sd[RPV_RB * HM];
  __shared__ float red[4][8 * LPR * HM];
  constexpr int RPI = 256 / LPR;
  const int tid = threadIdx.x, l = tid & (LPR - 1), wave = tid >> 6;
  const int c0 = l * 8;
  const bool cok = c0 < C;
  const int64_t r0 = (int64_t)blockIdx.x * RPV_RB;
  stage_dout_rows<HM, RPV_RB>(dout, rows, r0, H, sd, tid);
  __syncthreads();
  float acc[8][HM];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int h = 0; h < HM; ++h) acc[i][h] = 0.f;
  // rows in batches of NB per lane, loads first; rows past the end read the
  // last row (in range) and meet dout = 0 staged for them
  constexpr int NR = RPV_RB / RPI, NB = NR < 4 ? NR : 4;
  if (cok) {
    for (int j0 = 0; j0 < NR; j0 += NB) {
      float v[NB][8];
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        int64_t row = r0 + tid / LPR + (j0 + jj) * RPI;
        row = row < rows ? row : rows - 1;
        ld8(x + row * C + c0, v[jj]);
      }
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        const int rr = tid / LPR + (j0 + jj) * RPI;
        float d[HM];
#pragma unroll
        for (int h = 0; h < HM; h += 4) {
          const f32x4 q = *(const f32x4*)(sd + rr * HM + h);
          d[h] = q[0]; d[h + 1] = q[1]; d[h + 2] = q[2]; d[h + 3] = q[3];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int h = 0; h < HM; ++h) acc[i][h] += v[jj][i] * d[h];
      }
    }
  }
  // lanes l, l + LPR, ... of a wave hold the same channels
#pragma unroll
  for (int o = LPR; o < 64; o <<= 1)
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int h = 0; h < HM; ++h) acc[i][h] += __shfl_xor(acc[i][h], o, 64);
  if ((tid & 63) < LPR)
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int h = 0; h < HM; ++h) red[wave][(c0 + i) * HM + h] = acc[i][h];
  __syncthreads();
  for (int e = tid; e < C * H; e += 256) {
    const int cc = e / H, h = e - cc * H;
    const int k = cc * HM + h;
    part[(int64_t)blockIdx.x * C * H + e] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
  }
}

template <typename T, int LPR, int HM>
static void rowproj_bwd_vec_launch(const Ctx& c, const T* x, int64_t rows, int C, const float* W, int H,
                                   const float* dout, float* dx, bool accumulate, float* part, int64_t nblk) {
  if (dx)
    EVO_LAUNCH("rowproj_dx_vec_kernel", 2.0 * (double)rows * C * H, (double)rows * C * (accumulate ? 8.0 : 4.0) + (double)H * rows * 4.0, (rowproj_dx_vec_kernel<LPR, HM>), dim3((unsigned)((rows + RPX_RB - 1) / RPX_RB)), dim3(256), 0, c.stream,
               rows, C, W, H, dout, dx, accumulate ? 1 : 0);
  EVO_LAUNCH(EVO_KNAME("rowproj_dw_vec_kernel", T), 2.0 * (double)rows * C * H, (double)rows * C * sizeof(T) + (double)H * rows * 4.0, (rowproj_dw_vec_kernel<T, LPR, HM>), dim3((unsigned)nblk), dim3(256), 0, c.stream,
             x, rows, C, H, dout, part);
}

template <typename T>
evo_status_t rowproj_bwd(const Ctx& c, Arena& ws, const T* x, int64_t rows, int C, const float* W,
                         int H, const float* dout, float* dx, bool accumulate, float* dW) {
  const int64_t nblk = (rows + 255) / 256;
  float* part = ws.take_n<float>((size_t)nblk * C * H);
  if (c.dry || rows == 0) return EVO_OK;
  if (C % 8 == 0 && C <= 256 && H <= 8 && aligned16(x) && (!dx || aligned16(dx))) {
    switch (C / 8 <= 4 ? 4 : C / 8 <= 8 ? 8 : C / 8 <= 16 ? 16 : 32) {
#define EVO_RPV(L)                                                                                    \
  case L:                                                                                             \
    if (H <= 4) rowproj_bwd_vec_launch<T, L, 4>(c, x, rows, C, W, H, dout, dx, accumulate, part, nblk); \
    else rowproj_bwd_vec_launch<T, L, 8>(c, x, rows, C, W, H, dout, dx, accumulate, part, nblk);        \
    break;
      EVO_RPV(4) EVO_RPV(8) EVO_RPV(16) EVO_RPV(32)
#undef EVO_RPV
      default: break;
    }
    EVO_TRY(check_launch("rowproj_bwd"));
    RedSegs rs;
    rs.nseg = 1; rs.off[0] = 0; rs.n[0] = C * H; rs.out[0] = dW;
    return reduce_segments(c, part, nblk, 1, (int64_t)C * H, rs, true);
  }
  if (H > 16 || C > 256 || 256 % C) { set_error("pair bias bwd: unsupported C=%d H=%d", C, H); return EVO_ESHAPE; }
  if (dx) {
    const int64_t n = rows * C;
    (void)n;
    if (C % 4 || ((uintptr_t)dx) % 16) { set_error("pair bias bwd: C=%d not a multiple of 4", C); return EVO_ESHAPE; }
    const size_t lds = ((size_t)C * H + 32 * (size_t)H) * sizeof(float);
    EVO_LAUNCH("rowproj_dx_kernel", 2.0 * (double)rows * C * H, (double)rows * C * (accumulate ? 8.0 : 4.0) + (double)H * rows * 4.0, rowproj_dx_kernel, dim3((unsigned)((rows + 31) / 32)), dim3(256), lds, c.stream,
                       rows, C, W, H, dout, dx, accumulate ? 1 : 0);
    EVO_TRY(check_launch("rowproj_dx"));
  }
  EVO_LAUNCH(EVO_KNAME("rowproj_dw_kernel", T), 2.0 * (double)rows * C * H, (double)rows * C * sizeof(T) + (double)H * rows * 4.0, (rowproj_dw_kernel<T>), dim3((unsigned)nblk), dim3(256), 0, c.stream, x, rows, C, H,
                     dout, part);
  EVO_TRY(check_launch("rowproj_dw"));
  RedSegs rs;
  rs.nseg = 1; rs.off[0] = 0; rs.n[0] = C * H; rs.out[0] = dW;
  return reduce_segments(c, part, nblk, 1, (int64_t)C * H, rs, true);
}

// ============================================================== segmented column sums
#define EVO_INST_H(T)                                                                              \
  template evo_status_t wgrad<T>(const Ctx&, Arena&, const T*, int64_t, const T*, int64_t, int64_t, \
                                 int64_t, int64_t, float*, float* const*);                         \
  template evo_status_t wgrad_segments<T>(const Ctx&, Arena&, const T*, int64_t, const T*, int64_t, \
                                          int64_t, int64_t, int, const int*, const int*,            \
                                          float* const*, float* const*);                           \
  template evo_status_t rowproj<T>(const Ctx&, const T*, int64_t, int, const float*, int, float*); \
  template evo_status_t rowproj_bwd<T>(const Ctx&, Arena&, const T*, int64_t, int, const float*,   \
                                       int, const float*, float*, bool, float*);                   \

EVO_INST_H(float)
EVO_INST_H(bf16)

}  // namespace evo

extern "C" void evo_profile_begin(void) {
  std::lock_guard<std::mutex> lk(evo::g_prof_mu);
  for (auto& sl : evo::g_slots) { evo::g_pool.push_back(sl.a); evo::g_pool.push_back(sl.b); }
  evo::g_slots.clear();
  evo::g_names.clear();
  evo::g_prof_on = true;
}

extern "C" void evo_profile_set_detail(int32_t detail) {
  std::lock_guard<std::mutex> lk(evo::g_prof_mu);
  evo::g_prof_detail = detail != 0;
}

extern "C" int32_t evo_profile_end(evo_kernel_stat_t* rec, int32_t max_records) {
  std::lock_guard<std::mutex> lk(evo::g_prof_mu);
  evo::g_prof_on = false;
  struct Agg { int64_t n = 0; double ms = 0, flops = 0, bytes = 0; };
  std::map<std::string, Agg> agg;
  size_t ni = 0;
  for (auto& sl : evo::g_slots) {
    if (hipEventSynchronize(sl.b) != hipSuccess) { evo::set_error("profile: event wait failed"); return -1; }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sl.a, sl.b) != hipSuccess) { evo::set_error("profile: elapsed failed"); return -1; }
    Agg& a = agg[sl.name ? std::string(sl.name) : evo::g_names[ni++]];
    a.n += 1; a.ms += ms; a.flops += sl.flops; a.bytes += sl.bytes;
  }
  int32_t k = 0;
  for (auto& kv : agg) {
    if (k >= max_records) break;
    evo_kernel_stat_t& r = rec[k++];
    memset(&r, 0, sizeof(r));
    strncpy(r.name, kv.first.c_str(), sizeof(r.name) - 1);
    r.launches = kv.second.n; r.total_ms = kv.second.ms; r.flops = kv.second.flops; r.bytes = kv.second.bytes;
  }
  return k;
}
