// Optimizer step over fused parameter buffers (paper, Section "Tensor
// Fusion": every parameter, its gradient and the Adam moments live in a few
// large flat tensors, so each optimizer stage is a handful of launches instead
// of one per parameter tensor).
//
// Stages, all HBM-bound streaming kernels over FP32 vectors of n elements:
//   global norm   sqnorm_partial_kernel: FP64 partial sums of g^2, one per
//                 workgroup (grid-stride, at most OPT_MAX_PARTS workgroups);
//   clip          clip_scale_kernel: every workgroup sums the partials in one
//                 fixed order (so all agree bit for bit), scale =
//                 max_norm / max(norm, max_norm), g *= scale;
//   Adam          adam_kernel: m, v, p updated in one pass; with clip partials
//                 given, the clip scale is formed in the prologue and applied
//                 to g in registers (the clipped gradient is never written);
//                 with an EMA buffer given, the EMA of the new parameters is
//                 updated in the same pass.
// The fused step is therefore two launches: the norm partials and one pass of
// clip + Adam + EMA.  Deterministic: no atomics, fixed reduction orders.
#include <mutex>

#include "ops.h"

namespace evo {

constexpr int OPT_THREADS = 256;
constexpr int OPT_MAX_PARTS = 1024;        // partial sums of the global norm
constexpr int OPT_MAX_BLOCKS = 4096;       // workgroups of the elementwise passes

// Workgroups of the norm pass: one per 16 float4 per thread, at most OPT_MAX_PARTS.
static int norm_parts(int64_t n) {
  const int64_t per = (int64_t)OPT_THREADS * 4 * 16;
  const int64_t p = (n + per - 1) / per;
  return (int)(p < 1 ? 1 : (p > OPT_MAX_PARTS ? OPT_MAX_PARTS : p));
}
static int elem_blocks(int64_t n) {
  const int64_t b = (n / 4 + OPT_THREADS - 1) / OPT_THREADS;
  return (int)(b < 1 ? 1 : (b > OPT_MAX_BLOCKS ? OPT_MAX_BLOCKS : b));
}

EVO_DEV double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of v over the workgroup (fixed order: wave tree, then waves in order);
// every thread receives the result.
EVO_DEV double block_sum_f64(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum_f64(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < OPT_THREADS / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(OPT_THREADS) void sqnorm_partial_kernel(const float* g, int64_t n, double* part) {
  __shared__ double red[OPT_THREADS / 64];
  double acc = 0.0;
  const int64_t n4 = n >> 2, stride = (int64_t)gridDim.x * OPT_THREADS;
  const f32x4* g4 = (const f32x4*)g;
  for (int64_t i = (int64_t)blockIdx.x * OPT_THREADS + threadIdx.x; i < n4; i += stride) {
    const f32x4 v = g4[i];
    acc += (double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2] + (double)v[3] * v[3];
  }
  for (int64_t i = (n4 << 2) + (int64_t)blockIdx.x * OPT_THREADS + threadIdx.x; i < n; i += stride)
    acc += (double)g[i] * g[i];
  acc = block_sum_f64(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Global norm from the partials (same order in every workgroup) and the clip
// factor max_norm / max(norm, max_norm).
EVO_DEV float clip_factor(const double* part, int nparts, float max_norm, double* red, double* norm_out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += OPT_THREADS) acc += part[i];
  const double norm = sqrt(block_sum_f64(acc, red));
  *norm_out = norm;
  return (float)((double)max_norm / (norm > (double)max_norm ? norm : (double)max_norm));
}

__global__ __launch_bounds__(OPT_THREADS) void clip_scale_kernel(float* g, int64_t n, const double* part, int nparts,
                                                                 float max_norm, float* norm_out) {
  __shared__ double red[OPT_THREADS / 64];
  double norm = 0.0;
  const float s = clip_factor(part, nparts, max_norm, red, &norm);
  if (blockIdx.x == 0 && threadIdx.x == 0 && norm_out) *norm_out = (float)norm;
  if (s >= 1.0f) return;
  const int64_t n4 = n >> 2, stride = (int64_t)gridDim.x * OPT_THREADS;
  f32x4* g4 = (f32x4*)g;
  for (int64_t i = (int64_t)blockIdx.x * OPT_THREADS + threadIdx.x; i < n4; i += stride) g4[i] = g4[i] * s;
  for (int64_t i = (n4 << 2) + (int64_t)blockIdx.x * OPT_THREADS + threadIdx.x; i < n; i += stride) g[i] *= s;
}

__global__ __launch_bounds__(OPT_THREADS) void norm_finalize_kernel(const double* part, int nparts, float* norm_out) {
  __shared__ double red[OPT_THREADS / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += OPT_THREADS) acc += part[i];
  const double norm = sqrt(block_sum_f64(acc, red));
  if (threadIdx.x == 0) *norm_out = (float)norm;
}

struct AdamArgs {
  float lr, beta1, beta2, eps;
  float omb1, omb2;           // 1 - beta, formed on the host in double
  float inv_bc1, inv_bc2;     // 1 / (1 - beta^step), formed on the host in double
  float ema_decay, ema_omd;   // decay and 1 - decay
  float max_norm;
  const double* part;         // clip partials (NULL: no clipping)
  int nparts;
  float* norm_out;            // global norm (NULL: not reported)
};

EVO_DEV void adam_elem(const AdamArgs& a, float s, float& p, float g, float& m, float& v) {
  g *= s;
  m = a.beta1 * m + a.omb1 * g;
  v = a.beta2 * v + a.omb2 * (g * g);
  const float mhat = m * a.inv_bc1, vhat = v * a.inv_bc2;
  p -= a.lr * mhat / (sqrtf(vhat) + a.eps);
}

__global__ __launch_bounds__(OPT_THREADS) void adam_kernel(float* p, const float* g, float* m, float* v, float* ema,
                                                           int64_t n, AdamArgs a) {
  __shared__ double red[OPT_THREADS / 64];
  float s = 1.0f;
  if (a.part) {
    double norm = 0.0;
    s = clip_factor(a.part, a.nparts, a.max_norm, red, &norm);
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.norm_out) *a.norm_out = (float)norm;
  }
  const float d = a.ema_decay, d1 = a.ema_omd;
  const int64_t n4 = n >> 2, stride = (int64_t)gridDim.x * OPT_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * OPT_THREADS + threadIdx.x; i < n4; i += stride) {
    f32x4 pv = ((f32x4*)p)[i], mv = ((f32x4*)m)[i], vv = ((f32x4*)v)[i];
    const f32x4 gv = ((const f32x4*)g)[i];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float pj = pv[j], mj = mv[j], vj = vv[j];
      adam_elem(a, s, pj, gv[j], mj, vj);
      pv[j] = pj; mv[j] = mj; vv[j] = vj;
    }
    ((f32x4*)p)[i] = pv;
    ((f32x4*)m)[i] = mv;
    ((f32x4*)v)[i] = vv;
    if (ema) {
      f32x4 ev = ((f32x4*)ema)[i];
#pragma unroll
      for (int j = 0; j < 4; ++j) ev[j] = d * ev[j] + d1 * pv[j];
      ((f32x4*)ema)[i] = ev;
    }
  }
  for (int64_t i = (n4 << 2) + (int64_t)blockIdx.x * OPT_THREADS + threadIdx.x; i < n; i += stride) {
    float pv = p[i], mv = m[i], vv = v[i];
    adam_elem(a, s, pv, g[i], mv, vv);
    p[i] = pv;
    m[i] = mv;
    v[i] = vv;
    if (ema) ema[i] = d * ema[i] + d1 * pv;
  }
}

__global__ __launch_bounds__(OPT_THREADS) void ema_kernel(float* ema, const float* p, int64_t n, float decay,
                                                          float d1) {
  const int64_t n4 = n >> 2, stride = (int64_t)gridDim.x * OPT_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * OPT_THREADS + threadIdx.x; i < n4; i += stride) {
    const f32x4 pv = ((const f32x4*)p)[i];
    f32x4 ev = ((f32x4*)ema)[i];
    ev = ev * decay + pv * d1;
    ((f32x4*)ema)[i] = ev;
  }
  for (int64_t i = (n4 << 2) + (int64_t)blockIdx.x * OPT_THREADS + threadIdx.x; i < n; i += stride)
    ema[i] = decay * ema[i] + d1 * p[i];
}

// ---------------------------------------------------------------- host side
static evo_status_t launch_norm(hipStream_t st, const float* g, int64_t n, double* part, int nparts) {
  EVO_LAUNCH("sqnorm_partial_kernel", 2.0 * (double)n, (double)n * 4, sqnorm_partial_kernel, dim3(nparts),
             dim3(OPT_THREADS), 0, st, g, n, part);
  return check_launch("global norm");
}

static AdamArgs adam_args(const evo_optim_desc_t& d) {
  AdamArgs a;
  a.lr = (float)d.lr; a.beta1 = (float)d.beta1; a.beta2 = (float)d.beta2; a.eps = (float)d.eps;
  a.omb1 = (float)(1.0 - d.beta1); a.omb2 = (float)(1.0 - d.beta2);
  a.inv_bc1 = (float)(1.0 / (1.0 - pow(d.beta1, (double)d.step)));
  a.inv_bc2 = (float)(1.0 / (1.0 - pow(d.beta2, (double)d.step)));
  a.ema_decay = (float)d.ema_decay; a.ema_omd = (float)(1.0 - d.ema_decay);
  a.max_norm = (float)d.max_norm;
  a.part = nullptr;
  a.nparts = 0;
  a.norm_out = nullptr;
  return a;
}

static evo_status_t optim_step(hipStream_t st, const evo_optim_desc_t& d, float* p, const float* g, float* m,
                               float* v, float* ema, int64_t n, float* norm_out, double* part) {
  AdamArgs a = adam_args(d);
  if (d.max_norm > 0.0) {
    const int np = norm_parts(n);
    EVO_TRY(launch_norm(st, g, n, part, np));
    a.part = part;
    a.nparts = np;
    a.norm_out = norm_out;
  }
  const double bytes = (double)n * 4 * (ema ? 9 : 7);
  EVO_LAUNCH("adam_kernel", 0.0, bytes, adam_kernel, dim3(elem_blocks(n)), dim3(OPT_THREADS), 0, st, p, g, m, v,
             ema, n, a);
  return check_launch("adam");
}

static evo_status_t check_optim_desc(const evo_optim_desc_t* d) {
  EVO_CHECK_ARG(d, EVO_EINVAL, "optimizer: null descriptor");
  EVO_CHECK_ARG(d->step >= 1, EVO_EINVAL, "optimizer: step %lld must be >= 1", (long long)d->step);
  EVO_CHECK_ARG(d->beta1 >= 0.0 && d->beta1 < 1.0 && d->beta2 >= 0.0 && d->beta2 < 1.0, EVO_EINVAL,
                "optimizer: betas must lie in [0, 1)");
  EVO_CHECK_ARG(d->eps > 0.0, EVO_EINVAL, "optimizer: eps must be positive");
  EVO_CHECK_ARG(d->ema_decay >= 0.0 && d->ema_decay <= 1.0, EVO_EINVAL, "optimizer: EMA decay outside [0, 1]");
  return EVO_OK;
}

static evo_status_t vec_ptrs_ok(std::initializer_list<const void*> req, std::initializer_list<const void*> opt,
                                bool empty = false) {
  for (const void* q : req) {
    EVO_CHECK_ARG(empty || q != nullptr, EVO_EINVAL, "optimizer: required pointer is null");
    EVO_CHECK_ARG(aligned16(q), EVO_EINVAL, "optimizer: pointer %p is not 16-byte aligned", q);
  }
  for (const void* q : opt) EVO_CHECK_ARG(aligned16(q), EVO_EINVAL, "optimizer: pointer %p is not 16-byte aligned", q);
  return EVO_OK;
}

// ---------------------------------------------------------------- no-allocation variant
// Scratch of evo_optimizer_step_noalloc: the global norm's partial sums, one
// static array per device (OPT_MAX_PARTS doubles = 8 KiB, whatever n).  Host
// code never passes the array's name to a kernel: its device address is
// taken once per device with hipGetSymbolAddress and kept here.
static __device__ __align__(256) double scratch[OPT_MAX_PARTS];

constexpr int OPT_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[OPT_MAX_DEVICES];

static evo_status_t scratch_address(double** out) {
  int dev = 0;
  EVO_CHECK_ARG(hipGetDevice(&dev) == hipSuccess, EVO_EHIP, "optimizer: no HIP device");
  EVO_CHECK_ARG(dev >= 0 && dev < OPT_MAX_DEVICES, EVO_EHIP, "optimizer: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    EVO_CHECK_ARG(e == hipSuccess && ptr, EVO_EHIP, "optimizer: hipGetSymbolAddress(scratch): %s",
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = (double*)g_scratch_ptr[dev];
  return EVO_OK;
}

evo_status_t check_device();

}  // namespace evo

using namespace evo;

extern "C" {

size_t evo_optim_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return (size_t)norm_parts(n) * sizeof(double);
}

evo_status_t evo_grad_global_norm(const float* grads, int64_t n, float* norm_out, void* ws, size_t ws_bytes,
                                  void* stream) {
  EVO_CHECK_ARG(n >= 0, EVO_ESHAPE, "optimizer: negative length");
  EVO_TRY(vec_ptrs_ok({grads}, {}, n == 0));
  EVO_TRY(vec_ptrs_ok({norm_out}, {}));
  const int np = norm_parts(n);
  EVO_CHECK_ARG(ws && ws_bytes >= (size_t)np * sizeof(double), EVO_EWORKSPACE,
                "optimizer: workspace of %zu bytes needed", (size_t)np * sizeof(double));
  EVO_TRY(vec_ptrs_ok({ws}, {}));
  EVO_TRY(check_device());
  hipStream_t st = (hipStream_t)stream;
  double* part = (double*)ws;
  EVO_TRY(launch_norm(st, grads, n, part, np));
  EVO_LAUNCH("norm_finalize_kernel", 0.0, (double)np * 8, norm_finalize_kernel, dim3(1), dim3(OPT_THREADS), 0, st,
             part, np, norm_out);
  return check_launch("global norm");
}

evo_status_t evo_clip_by_global_norm(float* grads, int64_t n, double max_norm, float* norm_out, void* ws,
                                     size_t ws_bytes, void* stream) {
  EVO_CHECK_ARG(n >= 0, EVO_ESHAPE, "optimizer: negative length");
  EVO_CHECK_ARG(max_norm > 0.0, EVO_EINVAL, "optimizer: max_norm must be positive");
  EVO_TRY(vec_ptrs_ok({grads}, {norm_out}, n == 0));
  const int np = norm_parts(n);
  EVO_CHECK_ARG(ws && ws_bytes >= (size_t)np * sizeof(double), EVO_EWORKSPACE,
                "optimizer: workspace of %zu bytes needed", (size_t)np * sizeof(double));
  EVO_TRY(vec_ptrs_ok({ws}, {}));
  EVO_TRY(check_device());
  hipStream_t st = (hipStream_t)stream;
  double* part = (double*)ws;
  EVO_TRY(launch_norm(st, grads, n, part, np));
  EVO_LAUNCH("clip_scale_kernel", 0.0, (double)n * 8, clip_scale_kernel, dim3(elem_blocks(n)), dim3(OPT_THREADS),
             0, st, grads, n, part, np, (float)max_norm, norm_out);
  return check_launch("clip");
}

evo_status_t evo_adam_step(const evo_optim_desc_t* d, float* params, const float* grads, float* m, float* v,
                           int64_t n, void* stream) {
  EVO_TRY(check_optim_desc(d));
  EVO_CHECK_ARG(n >= 0, EVO_ESHAPE, "optimizer: negative length");
  EVO_TRY(vec_ptrs_ok({params, grads, m, v}, {}, n == 0));
  EVO_TRY(check_device());
  evo_optim_desc_t dd = *d;
  dd.max_norm = 0.0;
  return optim_step((hipStream_t)stream, dd, params, grads, m, v, nullptr, n, nullptr, nullptr);
}

evo_status_t evo_ema_update(float* ema, const float* params, int64_t n, double decay, void* stream) {
  EVO_CHECK_ARG(n >= 0, EVO_ESHAPE, "optimizer: negative length");
  EVO_CHECK_ARG(decay >= 0.0 && decay <= 1.0, EVO_EINVAL, "optimizer: EMA decay outside [0, 1]");
  EVO_TRY(vec_ptrs_ok({ema, params}, {}, n == 0));
  EVO_TRY(check_device());
  EVO_LAUNCH("ema_kernel", 0.0, (double)n * 12, ema_kernel, dim3(elem_blocks(n)), dim3(OPT_THREADS), 0,
             (hipStream_t)stream, ema, params, n, (float)decay, (float)(1.0 - decay));
  return check_launch("ema");
}

evo_status_t evo_optimizer_step(const evo_optim_desc_t* d, float* params, const float* grads, float* m, float* v,
                                float* ema, int64_t n, float* norm_out, void* ws, size_t ws_bytes, void* stream) {
  EVO_TRY(check_optim_desc(d));
  EVO_CHECK_ARG(n >= 0, EVO_ESHAPE, "optimizer: negative length");
  EVO_TRY(vec_ptrs_ok({params, grads, m, v}, {ema, norm_out}, n == 0));
  double* part = nullptr;
  if (d->max_norm > 0.0) {
    const size_t need = (size_t)norm_parts(n) * sizeof(double);
    EVO_CHECK_ARG(ws && ws_bytes >= need, EVO_EWORKSPACE, "optimizer: workspace of %zu bytes needed", need);
    EVO_TRY(vec_ptrs_ok({ws}, {}));
    part = (double*)ws;
  }
  EVO_TRY(check_device());
  return optim_step((hipStream_t)stream, *d, params, grads, m, v, ema, n, norm_out, part);
}

evo_status_t evo_optimizer_step_noalloc(const evo_optim_desc_t* d, float* params, const float* grads, float* m,
                                        float* v, float* ema, int64_t n, float* norm_out, void* stream) {
  EVO_TRY(check_optim_desc(d));
  EVO_CHECK_ARG(n >= 0, EVO_ESHAPE, "optimizer: negative length");
  EVO_TRY(vec_ptrs_ok({params, grads, m, v}, {ema, norm_out}, n == 0));
  // the norm's partial sums live in the static scratch (at most OPT_MAX_PARTS of them)
  EVO_CHECK_ARG(norm_parts(n) <= OPT_MAX_PARTS, EVO_ESHAPE,
                "optimizer: %d norm partials exceed the static scratch of %d", norm_parts(n), OPT_MAX_PARTS);
  EVO_TRY(check_device());
  double* part = nullptr;
  if (d->max_norm > 0.0) EVO_TRY(scratch_address(&part));
  return optim_step((hipStream_t)stream, *d, params, grads, m, v, ema, n, norm_out, part);
}

}  // extern "C"
