// LayerNorm, reductions, parameter packing and the elementwise glue kernels.
#pragma once
#include "common.h"

#include <initializer_list>

namespace evo {

// y = LayerNorm(x) over the last axis (rows x C, row pitch C), FP32 statistics.
template <typename TI, typename TO = TI>
evo_status_t ln_fwd(const Ctx& c, const TI* x, int64_t rows, int C, const float* g, const float* b,
                    float eps, TO* y, float* mean, float* rstd);
// Same with row r of x at x + ((r >> rshift) * rhi + (r & (2^rshift - 1)) * C)
// (a chunk of rows of a larger matrix); y is dense.
template <typename TI, typename TO = TI>
evo_status_t ln_fwd_rows(const Ctx& c, const TI* x, int64_t rows, int C, int rshift, int64_t rhi,
                         const float* g, const float* b, float eps, TO* y, float* mean, float* rstd);
// out[h][row] = out_scale * sum_c LayerNorm(x)[row][c] W[c][h] without storing the
// LayerNorm output (the LayerNorm output is rounded to TO first, as a stored one
// would be).  tr_n > 0 (rows = tr_n^2): row a * tr_n + b goes to out[h][b][a].
template <typename TI, typename TO = TI>
evo_status_t ln_rowproj(const Ctx& c, const TI* x, int64_t rows, int C, const float* g, const float* b,
                        float eps, const float* W, int H, float* out, float out_scale = 1.f, int64_t tr_n = 0);
// Channel-major input x[C][P] (compute type) -> y[P][C].
template <typename T>
evo_status_t ln_fwd_cm(const Ctx& c, const T* x, int64_t P, int C, const float* g, const float* b,
                       float eps, T* y, float* mean, float* rstd);
// dx = base + LayerNorm_backward(dy): base = resid (may alias dx) when given, else dx itself
// when accumulate, else 0.  dgamma/dbeta partial sums go to part[nblk][2*C].
template <typename T>
evo_status_t ln_bwd(const Ctx& c, const T* x, const float* mean, const float* rstd, const float* g,
                    const float* dy, int64_t rows, int C, const T* resid, bool accumulate, T* dx,
                    float* part, int* nblk);
int64_t ln_bwd_partials(int64_t rows);
// Channel-major x[C][P] (compute type), dy[P][C] -> dx[C][P].
template <typename T>
evo_status_t ln_bwd_cm(const Ctx& c, const T* x, const float* mean, const float* rstd, const float* g,
                       const float* dy, int64_t P, int C, T* dx, float* part, int* nblk);
int64_t ln_bwd_cm_partials(int64_t P);

// out[j] (+)= sum_i part[i * ld + j], i < n, j < C (fixed order).
evo_status_t reduce_partials(const Ctx& c, const float* part, int64_t n, int64_t C, int64_t ld,
                             float* out, bool accumulate);
// Segmented reduction in one launch.  part is [n][M][ld]; segment s covers
// columns [off_s, off_s + n_s) and accumulates (or stores)
//   out_s[m * n_s + j] (+)= sum_{i<n} part[(i * M + m) * ld + off_s + j]
// in a fixed order.  Up to 8 segments; null outputs are skipped.
struct RedSegs {
  int32_t nseg = 0;
  int32_t off[8];
  int32_t n[8];
  float* out[8];
};
evo_status_t reduce_segments(const Ctx& c, const float* part, int64_t n, int64_t M, int64_t ld,
                             const RedSegs& segs, bool accumulate);
// With c.defer set, an accumulating reduce_segments is queued instead of
// launched: the queue holds the partial-buffer pointer, so the buffer must stay
// untouched until flush_reductions runs the queued reductions, all in one
// launch (outputs of queued reductions must not overlap).  Parameter gradients
// of a backward op use this: their partials live in the op's scratch and
// nothing in the op reads the gradients.
struct RedJob {
  const float* part;
  int64_t n, M, ld;
  RedSegs segs;
};
constexpr int RED_MAX_JOBS = 12;
struct RedQueue {
  int njobs = 0;
  RedJob jobs[RED_MAX_JOBS];
};
evo_status_t flush_reductions(const Ctx& c, RedQueue& q);
// Runs f(ctx) with its parameter-gradient reductions deferred to one launch at
// the end (a fresh queue: reductions queued by an enclosing scope are not
// touched and those of f are all run before it returns).
template <typename F>
evo_status_t with_batched_reductions(const Ctx& c, F&& f) {
  if (c.dry) return f(c);
  RedQueue q;
  Ctx cq = c;
  cq.defer = &q;
  EVO_TRY(f(cq));
  return flush_reductions(c, q);
}
// Two outputs from one [n][2C] partial buffer (LayerNorm gamma / beta).
evo_status_t reduce_partials2(const Ctx& c, const float* part, int64_t n, int C, float* out_a,
                              float* out_b);
// Parameter packing: up to 5 FP32 segments W_i[K][n_i] concatenated along n.
struct PackSeg { const float* w; const float* bias; int32_t n; };
struct PackArgs {
  PackSeg seg[5];
  int32_t nseg = 0;
  int32_t K = 0;
  void* dst_t = nullptr;   // [sum n][K], kernel type   (forward B operand)
  void* dst = nullptr;     // [K][sum n], kernel type   (backward B operand)
  float* bias = nullptr;   // [sum n] FP32 (missing segment biases are 0)
};
// Groups packed ahead of the operations that use them (a block packs the
// parameters of all its sub-operations in one pass at the start of a call).
// find() matches a request by its segments (weights, widths and, when the
// request wants the bias row, the segment biases) and by the layouts it asks
// for, and points the request's destinations at the packed copies.
struct PackCache {
  static constexpr int MAX = 40;
  int n = 0;
  PackArgs e[MAX];
  bool find(PackArgs& a) const;
};
// Packs the groups in `list` (any number, in launches of a few groups each);
// with c.packed set, groups found there are taken from it and not packed: the
// caller then reads the destinations back from the PackArgs.
template <typename T>
evo_status_t pack_params(const Ctx& c, std::initializer_list<PackArgs*> list);
template <typename T>
evo_status_t pack_groups(const Ctx& c, PackArgs* const* g, int n);

template <typename T>
evo_status_t fill_zero(const Ctx& c, T* p, int64_t n);
template <typename T>
evo_status_t copy_elems(const Ctx& c, const T* src, T* dst, int64_t n);
// dst = src converted (round to nearest even when narrowing).
template <typename TI, typename TO>
evo_status_t convert_elems(const Ctx& c, const TI* src, TO* dst, int64_t n);

// Attention gate backward. Per row r and head h (c = head_dim):
//   dctx = dgo * g; dgpre = dgo * o * g (1 - g); D[r*H+h] = sum_d dctx * o
// go/o/g/dgo have row pitches; dctx written with pitch ld_dctx, dgpre with ld_dg.  dgo is FP32.
template <typename T>
evo_status_t gate_bwd(const Ctx& c, int64_t rows, int H, int hd, const float* dgo, int64_t ld_dgo,
                      const float* o, int64_t ld_o, const T* g, int64_t ld_g, T* dctx,
                      int64_t ld_dctx, T* dgpre, int64_t ld_dg, float* D);

// Triangle multiplication projections, forward: raw[p][4*ch + cz] (ap | ag | bp | bg | g, compute type)
// -> a[c][p], b[c][p] (channel-major, masked, gated), and, when g is not null,
// a copy of the output-gate columns in FP32, g[p][cz] (the projection's
// epilogue has already applied their sigmoid).  a and b have channel stride
// ld_ab (>= P; pointers may be offset into larger tensors).
template <typename T>
evo_status_t trimul_proj(const Ctx& c, int64_t P, int ch, int cz, const T* raw, const float* mask,
                         T* a, T* b, int64_t ld_ab, float* g);
// Backward: FP32 da, db channel-major -> draw[p][4*ch] columns of ap, ag, bp, bg.
template <typename T>
evo_status_t trimul_proj_bwd(const Ctx& c, int64_t P, int ch, int cz, const T* raw,
                             const float* mask, const float* da, const float* db, T* draw);
// Output gate backward: dt = dz * g;  draw[p][4ch + n] = dz * t * g (1 - g)  (t FP32, g in
// the compute type at g[p * ld_g + n]).
template <typename T, typename X = T>
evo_status_t trimul_gate_bwd(const Ctx& c, int64_t P, int ch, int cz, const X* dz, const float* t,
                             const T* g, int64_t ld_g, T* dt, T* draw);

// Outer-product-mean input gradients from split-K partials:
//   dab[s][i][off + p] = mask[s][i] * sum_k part[k][s][i][p]   (part FP32 [nsplit][S][R][ch],
// dab rows [R][2 ch], mask NULL: ones; ch a multiple of 4).
template <typename T>
evo_status_t opm_dab_reduce(const Ctx& c, const float* part, int nsplit, int64_t S, int64_t R, int ch,
                            const float* mask, T* dab, int off);
// scale[i*R + j] = 1 / (eps + sum_s mask[s,i] mask[s,j])  (mask NULL: all ones).
evo_status_t opm_norm(const Ctx& c, const float* mask, int64_t S, int64_t R, float eps, float* scale);

}  // namespace evo
