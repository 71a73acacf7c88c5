// Shared device/host helpers for the gfx950 Evoformer kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#include <string>

#include "evo.h"

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2;

#define EVO_DEV __device__ __forceinline__

// ---------------------------------------------------------------- conversions
EVO_DEV float to_f32(float x) { return x; }
EVO_DEV float to_f32(bf16 x) { return (float)x; }
template <typename T> EVO_DEV T from_f32(float x);
template <> EVO_DEV float from_f32<float>(float x) { return x; }
template <> EVO_DEV bf16 from_f32<bf16>(float x) { return (bf16)x; }  // round to nearest even

EVO_DEV float sigmoidf_(float x) { return 1.0f / (1.0f + __expf(-x)); }

// ---------------------------------------------------------------- 8-wide vector access
// p must be 16-byte aligned (32-byte for float is not required: two 16-byte accesses).
EVO_DEV void ld8(const float* p, float v[8]) {
  const f32x4 a = *(const f32x4*)p, b = *(const f32x4*)(p + 4);
#pragma unroll
  for (int i = 0; i < 4; ++i) { v[i] = a[i]; v[4 + i] = b[i]; }
}
EVO_DEV void ld8(const bf16* p, float v[8]) {
  const bf16x8 a = *(const bf16x8*)p;
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = (float)a[i];
}
EVO_DEV void st8(float* p, const float v[8]) {
  f32x4 a, b;
#pragma unroll
  for (int i = 0; i < 4; ++i) { a[i] = v[i]; b[i] = v[4 + i]; }
  *(f32x4*)p = a;
  *(f32x4*)(p + 4) = b;
}
EVO_DEV void st8(bf16* p, const float v[8]) {
  bf16x8 a;
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = (bf16)v[i];
  *(bf16x8*)p = a;
}
// 4 consecutive values (8-byte aligned for BF16, 16-byte for float).
template <typename T>
EVO_DEV void store4(T* dst, f32x4 v) {
  if constexpr (sizeof(T) == 2) {
    *(bf16x4*)dst = bf16x4{(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
  } else {
    *(f32x4*)dst = v;
  }
}
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// ---------------------------------------------------------------- wave reductions (wave64)
// Lane exchanges on the VALU, no LDS round trips: DPP within 16-lane rows
// (quad permutations for partners l ^ 1 and l ^ 2, half-row mirror l ^ 7 and
// row mirror l ^ 15 of an 8- / 16-lane group, each landing in the other half of
// the group once the halves hold their own totals), and the gfx950 row swaps
// across rows (v_permlane16_swap: rows 0 <-> 1 and 2 <-> 3; v_permlane32_swap:
// the two halves of the wave).  Each step combines a lane's value with its
// partner's, a op b on one side and b op a on the other, so that with a
// commutative op every lane of a group ends with the same bits.
namespace dppc {
constexpr int XOR1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int XOR2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int HALF_MIRROR = 0x141;
constexpr int MIRROR = 0x140;
}  // namespace dppc
template <int CTRL> EVO_DEV float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// op over aligned groups of G lanes (G a power of two <= 64); every lane of a
// group gets the result.
template <int G, typename Op> EVO_DEV float group_reduce(float v, Op op) {
  static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "group size");
  if constexpr (G >= 2) v = op(v, dpp_f32<dppc::XOR1>(v));
  if constexpr (G >= 4) v = op(v, dpp_f32<dppc::XOR2>(v));
  if constexpr (G >= 8) v = op(v, dpp_f32<dppc::HALF_MIRROR>(v));
  if constexpr (G >= 16) v = op(v, dpp_f32<dppc::MIRROR>(v));
  if constexpr (G >= 32) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = op(__uint_as_float(p[0]), __uint_as_float(p[1]));
  }
  if constexpr (G >= 64) {
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = op(__uint_as_float(p[0]), __uint_as_float(p[1]));
  }
  return v;
}
struct AddOp { EVO_DEV float operator()(float a, float b) const { return a + b; } };
struct MaxOp { EVO_DEV float operator()(float a, float b) const { return fmaxf(a, b); } };
template <int G> EVO_DEV float group_sum(float v) { return group_reduce<G>(v, AddOp()); }
EVO_DEV float wave_sum(float v) { return group_reduce<64>(v, AddOp()); }
EVO_DEV float wave_max(float v) { return group_reduce<64>(v, MaxOp()); }

// ---------------------------------------------------------------- XCD-aware order
// Workgroups are dealt round-robin over the 8 XCDs (each with its own L2) in
// linear launch order: workgroup l runs on XCD l % 8.  xcd_order(l, n) maps
// the launch index to a logical index so that each XCD receives one
// contiguous run of logical indices (XCD x gets ceil or floor of n / 8 of
// them, in order); a bijection on [0, n) for any n.
EVO_DEV int xcd_order(int l, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = l & 7, i = l >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// ---------------------------------------------------------------- MFMA wrappers
// 16x16 output tiles for both precisions.  Lane l of a wave holds output rows
// 4*(l/16)+i (i = 0..3) of column l%16.  An operand fragment of lane l holds
// row (A) / column (B) l%16 at a lane-group-dependent set of k indices; the two
// operands of one product must use the same k set, any bijection works.
EVO_DEV f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
EVO_DEV f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- host side
namespace evo {

void set_error(const char* fmt, ...);

#define EVO_CHECK_ARG(cond, code, ...)      \
  do {                                      \
    if (!(cond)) {                          \
      ::evo::set_error(__VA_ARGS__);        \
      return (code);                        \
    }                                       \
  } while (0)

#define EVO_TRY(expr)                       \
  do {                                      \
    evo_status_t _s = (expr);               \
    if (_s != EVO_OK) return _s;            \
  } while (0)

evo_status_t check_launch(const char* what);

// Launch profiler (see evo_profile_begin): slot handle or -1 when disabled.
int prof_begin(const char* name, hipStream_t s, double flops, double bytes);
void prof_end(int slot, hipStream_t s);
// Sub-operation tag attached to the launches made while it is alive (detail mode).
// Tags nest: a launch is keyed by the chain of live tags, outermost first.
struct ProfTag {
  explicit ProfTag(const char* tag);
  ~ProfTag();
};

#define EVO_LAUNCH(name, flops, bytes, kernel, grid, block, lds, stream, ...)        \
  do {                                                                             \
    const int _ps = ::evo::prof_begin(name, stream, flops, bytes);                 \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);             \
    ::evo::prof_end(_ps, stream);                                                  \
  } while (0)

// Per-instantiation kernel name "lit<T>" for the profiler.
#define EVO_KNAME(lit, T)                                                                  \
  ([]() -> const char* {                                                                   \
    static const std::string s_ = std::string(lit) + "<" + ::evo::tname<T>() + ">";       \
    return s_.c_str();                                                                     \
  }())

template <typename T> inline const char* tname();
template <> inline const char* tname<float>() { return "float"; }
template <> inline const char* tname<__bf16>() { return "__bf16"; }

// Bump allocator over a caller-owned workspace.  In dry mode it only counts
// bytes, so one code path both sizes and carves the workspace.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  bool dry = false;
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = dry ? nullptr : (void*)(base + off);
    off += bytes;
    return p;
  }
  template <typename T> T* take_n(size_t n) { return (T*)take(n * sizeof(T)); }
  bool overflow() const { return !dry && off > cap; }
};

struct RedQueue;
struct PackCache;
struct Ctx {
  hipStream_t stream = nullptr;
  bool dry = false;      // size only: allocate from the arenas, launch nothing
  // When set, parameter-gradient reductions are queued here and run as one
  // batched launch by flush_reductions (see misc.h).
  RedQueue* defer = nullptr;
  // When set, parameter groups already packed for this call (see misc.h).
  const PackCache* packed = nullptr;
};

inline size_t dtype_bytes(int dt) { return dt == EVO_BF16 ? 2 : 4; }

}  // namespace evo
