/*
 * evo.h -- C ABI of the MI355X (gfx950) Evoformer block library (libevo.so).
 *
 * One Evoformer block of AlphaFold2 as re-implemented in HelixFold
 * (arXiv 2207.05477): gated self-attention with pair bias along MSA rows,
 * along MSA columns (or the global column attention of the extra-MSA stack)
 * and around the starting and ending node of the pair representation; the
 * triangle multiplicative updates; the outer product mean; the transitions.
 * Forward and backward, FP32 or BF16 activations.
 *
 * Layout (paper, Section "Dynamic Axial Parallelism"): the MSA representation
 * is [N_seq, N_res, C_m] and the pair representation [N_res, N_res, C_z], one
 * protein per call (mini-batch 1 per device, Section "Hyperparameter
 * setting"), channel-last, dense row-major.
 *
 * Conventions shared by every entry point
 *  - Return: evo_status_t.  On any error nothing has been enqueued; the
 *    message is available from evo_last_error() (thread-local).
 *  - Pointers: device pointers owned by the caller, unless stated.  The
 *    library never allocates device memory; scratch comes from the caller's
 *    workspace (ws, ws_bytes), sized by the matching *_workspace_bytes query.
 *    Every device pointer must be 16-byte aligned.
 *  - dtype: activations (x, pair, out, d_out, d_x, saved) are evo_dtype_t
 *    (FP32 or BF16).  Parameters and parameter gradients are always FP32.
 *    Masks are FP32 arrays of 0/1; NULL means all ones.
 *  - Asynchrony: work is enqueued on `stream` (a hipStream_t; NULL = default
 *    stream) with no host synchronisation; device faults surface at the
 *    caller's next synchronisation.
 *  - Forward computes out = x + f(x); out may alias x.
 *  - Backward writes d_x = d_out + J_f(x)^T d_out (d_x may alias d_out).
 *    Cross-input gradients (d_pair, d_m of the outer product mean) and all
 *    parameter gradients are ACCUMULATED (+=) into caller-initialised FP32 /
 *    activation buffers.
 *  - Determinism: no floating-point atomics; results are bitwise
 *    reproducible run to run for equal inputs and launch configuration.
 *  - Masked attention keys: the logit of a masked key is replaced by a large
 *    negative constant, so a partially masked row gives masked keys zero
 *    weight and a fully masked row averages all keys uniformly; no gradient
 *    flows through masked logits.
 */
#ifndef EVO_H_
#define EVO_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EVO_OK = 0,
  EVO_EINVAL = 1,       /* null / misaligned pointer, bad enum value */
  EVO_ESHAPE = 2,       /* unsupported sizes (e.g. head_dim not in {8,16,32,64}) */
  EVO_EWORKSPACE = 3,   /* workspace too small */
  EVO_EHIP = 4,         /* HIP runtime / launch error */
  EVO_EUNSUPPORTED = 5  /* device is not gfx950 */
} evo_status_t;

typedef enum { EVO_F32 = 0, EVO_BF16 = 1 } evo_dtype_t;

typedef enum { EVO_PHASE_FWD = 0, EVO_PHASE_BWD = 1 } evo_phase_t;

/* ------------------------------------------------------------------ attention
 * Gated multi-head self-attention (paper, Section "Fused Gated
 * Self-Attention" and its gated-attention figure: row-wise and column-wise
 * attention, gating before the output projection, a pair-derived
 * "nonbatched_bias" added to the logits):
 *   y = LayerNorm(x); q,k,v = y W_{q,k,v} (no bias); g = sigmoid(y W_g + b_g)
 *   o = g * softmax(q k^T / sqrt(head_dim) + bias (+ key mask)) v
 *   out = x + o W_o + b_o
 * kinds (x = [n_outer, n_inner, c_in], mask = [n_outer, n_inner]):
 *   ROW        MSA rows: for each s, queries/keys along residues;
 *              bias b_ij = LayerNorm_z(pair_ij) W_bias, pair = [n_inner, n_inner, c_pair];
 *              key mask mask[s, j].
 *   COL        MSA columns: for each residue i, queries/keys along s; no bias;
 *              key mask mask[t, i].
 *   COL_GLOBAL extra-MSA global column attention: one masked-mean query per
 *              (i, head), w_k, w_v are [c_in, head_dim] shared by all heads;
 *              mean over s uses global_eps.
 *   TRI_START  triangle attention around the starting node (x = z, square):
 *              o_ij = sum_k softmax_k(q_ij.k_ik/sqrt(c) + b_jk) v_ik, key mask mask[i, k];
 *              bias b_jk = y_jk W_bias (same LayerNorm as q, k, v).
 *   TRI_END    around the ending node: o_ij = sum_k softmax_k(q_ij.k_kj/sqrt(c) + b_ki) v_kj,
 *              key mask mask[k, j].
 */
typedef enum {
  EVO_ATTN_ROW = 0,
  EVO_ATTN_COL = 1,
  EVO_ATTN_COL_GLOBAL = 2,
  EVO_ATTN_TRI_START = 3,
  EVO_ATTN_TRI_END = 4
} evo_attn_kind_t;

typedef struct {
  int32_t kind;       /* evo_attn_kind_t */
  int32_t dtype;      /* evo_dtype_t */
  int64_t n_outer;    /* S for MSA kinds, N_res for TRI kinds */
  int64_t n_inner;    /* N_res */
  int64_t c_in;       /* channels of x */
  int64_t c_pair;     /* ROW: channels of pair; otherwise ignored */
  int32_t heads;
  int32_t head_dim;   /* 8, 16, 32 or 64 */
  float ln_eps;
  float global_eps;   /* COL_GLOBAL only */
  int64_t chunk;      /* TRI kinds, forward without saved: batch rows per chunk (0 = all); a
                         power of two dividing n_inner: starting node chunks rows i, ending node
                         columns j */
} evo_attn_desc_t;

/* Parameter (or parameter-gradient) pointers, FP32, Linear weights [fan_in, fan_out]. */
typedef struct {
  float *ln_g, *ln_b;         /* [c_in] */
  float *ln_z_g, *ln_z_b;     /* ROW: [c_pair]; else NULL */
  float *w_q;                 /* [c_in, H*c] */
  float *w_k, *w_v;           /* [c_in, H*c]; COL_GLOBAL: [c_in, c] */
  float *w_bias;              /* ROW: [c_pair, H]; TRI: [c_in, H]; else NULL */
  float *w_g, *b_g;           /* [c_in, H*c], [H*c] */
  float *w_o, *b_o;           /* [H*c, c_in], [c_in] */
} evo_attn_w_t;

size_t evo_attn_workspace_bytes(const evo_attn_desc_t* desc, int32_t phase);
/* Bytes of the buffer that evo_attn_fwd fills for evo_attn_bwd (0 if unsupported). */
size_t evo_attn_saved_bytes(const evo_attn_desc_t* desc);

/* out = x + Attn(x[, pair]).  saved: NULL for inference, else a buffer of
 * evo_attn_saved_bytes(desc) that evo_attn_bwd consumes. */
evo_status_t evo_attn_fwd(const evo_attn_desc_t* desc, const evo_attn_w_t* w,
                          const void* x, const void* pair, const float* mask,
                          void* out, void* saved, void* ws, size_t ws_bytes, void* stream);

/* d_x = d_out + J^T d_out; ROW: d_pair += J_pair^T d_out; d_w += parameter gradients.
 * x, pair, mask and w must be those of the forward that filled `saved`. */
evo_status_t evo_attn_bwd(const evo_attn_desc_t* desc, const evo_attn_w_t* w,
                          const void* x, const void* pair, const float* mask,
                          const void* saved, const void* d_out, void* d_x, void* d_pair,
                          const evo_attn_w_t* d_w, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ transition
 * The MSA and pair transitions of the two stacks of a block (paper, Section
 * "Branch Parallelism": the MSA stack and the pair stack each end in one; the
 * operator is AlphaFold2's, which the paper follows, Section "Hyperparameter
 * setting"):
 *   out = x + ReLU(LayerNorm(x) W_1 + b_1) W_2 + b_2,  hidden = factor * c;  x = [rows, c]
 *   (rows = N_seq * N_res for the MSA transition, N_res^2 for the pair transition).
 * Errors: EVO_ESHAPE unless c is a positive multiple of 8 at most 512 and factor >= 1. */
typedef struct {
  int32_t dtype;
  int64_t rows, c, factor;
  float ln_eps;
} evo_trans_desc_t;

typedef struct { float *ln_g, *ln_b, *w_1, *b_1, *w_2, *b_2; } evo_trans_w_t;

size_t evo_transition_workspace_bytes(const evo_trans_desc_t* desc, int32_t phase);
size_t evo_transition_saved_bytes(const evo_trans_desc_t* desc);
evo_status_t evo_transition_fwd(const evo_trans_desc_t* desc, const evo_trans_w_t* w,
                                const void* x, void* out, void* saved,
                                void* ws, size_t ws_bytes, void* stream);
evo_status_t evo_transition_bwd(const evo_trans_desc_t* desc, const evo_trans_w_t* w,
                                const void* x, const void* saved, const void* d_out, void* d_x,
                                const evo_trans_w_t* d_w, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ outer product mean
 * The only MSA-to-pair link of a block (paper, Section "Branch Parallelism"):
 *   y = LayerNorm(m); a = mask * (y W_a + b_a); b = mask * (y W_b + b_b)   [S, R, c_h]
 *   O_ij = sum_s a_si (outer) b_sj, flattened p*c_h + q;  n_ij = sum_s mask_si mask_sj
 *   z_out = z_in + (O_ij / (opm_eps + n_ij)) W_o + b_o
 */
typedef struct {
  int32_t dtype;
  int64_t n_seq, n_res, c_m, c_hidden, c_z;
  float ln_eps, opm_eps;
  int64_t chunk;      /* forward without saved: output rows i per chunk (0 = all) */
} evo_opm_desc_t;

typedef struct { float *ln_g, *ln_b, *w_a, *b_a, *w_b, *b_b, *w_o, *b_o; } evo_opm_w_t;

size_t opm_workspace_bytes(const evo_opm_desc_t* desc, int32_t phase);
size_t opm_saved_bytes(const evo_opm_desc_t* desc);
/* z_out = z_in + OPM(m); z_out may alias z_in. */
evo_status_t opm_fwd(const evo_opm_desc_t* desc, const evo_opm_w_t* w, const void* m,
                     const float* msa_mask, const void* z_in, void* z_out, void* saved,
                     void* ws, size_t ws_bytes, void* stream);
/* d_m += J_m^T dz_out (the pair gradient passes through unchanged); d_w += ... */
evo_status_t opm_bwd(const evo_opm_desc_t* desc, const evo_opm_w_t* w, const void* m,
                     const float* msa_mask, const void* saved, const void* dz_out, void* d_m,
                     const evo_opm_w_t* d_w, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ triangle multiplication
 * The triangle multiplicative updates of the pair stack, outgoing and incoming edges (paper,
 * Section "Branch Parallelism": the pair stack of a block, run on its own device under BP; the
 * operator is AlphaFold2's, Section "Hyperparameter setting"):
 *   y = LayerNorm(z); a = P * sigmoid(y W_ag + b_ag) * (y W_ap + b_ap); b likewise;
 *   g = sigmoid(y W_g + b_g)
 *   OUT: x_ij = sum_k a_ik b_jk      IN: x_ij = sum_k a_ki b_kj
 *   z_out = z + g * (LayerNorm_out(x) W_o + b_o);   P = pair mask [R, R]
 */
typedef enum { EVO_TRI_OUT = 0, EVO_TRI_IN = 1 } evo_tri_dir_t;

typedef struct {
  int32_t dtype;
  int32_t dir;        /* evo_tri_dir_t */
  int64_t n_res, c_z, c_hidden;
  float ln_eps;
  int64_t chunk;      /* forward without saved: output rows i per chunk (0 = all); a power of
                         two dividing n_res */
} evo_trimul_desc_t;

typedef struct {
  float *ln_g, *ln_b;
  float *w_ap, *b_ap, *w_ag, *b_ag, *w_bp, *b_bp, *w_bg, *b_bg;   /* [c_z, c_h], [c_h] */
  float *w_g, *b_g;                                               /* [c_z, c_z], [c_z] */
  float *ln_out_g, *ln_out_b;                                     /* [c_h] */
  float *w_o, *b_o;                                               /* [c_h, c_z], [c_z] */
} evo_trimul_w_t;

size_t tri_mul_workspace_bytes(const evo_trimul_desc_t* desc, int32_t phase);
size_t tri_mul_saved_bytes(const evo_trimul_desc_t* desc);
evo_status_t tri_mul_fwd(const evo_trimul_desc_t* desc, const evo_trimul_w_t* w,
                         const void* z, const float* pair_mask, void* z_out, void* saved,
                         void* ws, size_t ws_bytes, void* stream);
evo_status_t tri_mul_bwd(const evo_trimul_desc_t* desc, const evo_trimul_w_t* w,
                         const void* z, const float* pair_mask, const void* saved,
                         const void* dz_out, void* dz, const evo_trimul_w_t* d_w,
                         void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ Evoformer block
 * m <- m + RowAttn(m, z); m <- m + ColAttn(m) (ColGlobalAttn if extra_msa);
 * m <- m + Transition(m); z <- z + OPM(m); z <- z + TriMulOut(z);
 * z <- z + TriMulIn(z); z <- z + TriAttnStart(z); z <- z + TriAttnEnd(z);
 * z <- z + Transition(z).   Dropout is the identity.
 * The block is the activation-checkpoint boundary (paper, Section "Recompute"):
 * the forward saves nothing and the backward recomputes the forward into the
 * workspace before running the backward ops in reverse order.
 */
typedef struct {
  int32_t dtype;
  int32_t extra_msa;          /* 1: column attention is COL_GLOBAL */
  int64_t n_seq, n_res, c_m, c_z;
  int32_t msa_heads, msa_head_dim, tri_heads, tri_head_dim;
  int64_t tri_mul_hidden, opm_hidden, transition_factor;
  int64_t chunk;              /* forward only: row chunk of the outer product mean, triangle
                                 multiplication and triangle attention (0 = none; else a power
                                 of two dividing n_res).  Chunked results equal unchunked ones
                                 (paper, Section "Subbatch VS DAP": the split axis is
                                 independent). */
  float ln_eps, opm_eps, global_eps;
  int32_t opm_first;          /* 1: the outer product mean runs first, on the block's input m, and
                                 both branches read z + OPM(m): the MSA stack and the pair stack are
                                 then independent, as Branch Parallelism needs (paper, Section
                                 "Branch Parallelism"); 0: AlphaFold2's order above */
  int32_t dropout;            /* 1: training dropout of the residual updates (AlphaFold2's settings,
                                 paper Section "Hyperparameter setting"): row attention at
                                 drop_row_attn with one multiplier per (residue, channel) shared along
                                 the MSA rows; the triangle multiplications and starting-node attention
                                 at drop_tri_mul / drop_tri_att shared along the first residue axis;
                                 ending-node attention shared along the second.  Multipliers are 0 or
                                 1 / (1 - rate), from Philox4x32-10 with key drop_seed, counter
                                 (element, sub-op number [row 0, tri-mul out 4, in 5, attention start
                                 6, end 7], drop_offset low, high words); a stack gives block l the
                                 offset drop_offset + l.  Forward and backward of one step must pass
                                 the same values.  Not with chunk. */
  float drop_row_attn, drop_tri_mul, drop_tri_att;   /* rates in [0, 1) */
  uint64_t drop_seed, drop_offset;
} evo_block_desc_t;

typedef struct {
  evo_attn_w_t row_attn, col_attn;
  evo_trans_w_t msa_trans;
  evo_opm_w_t opm;
  evo_trimul_w_t tri_mul_out, tri_mul_in;
  evo_attn_w_t tri_att_start, tri_att_end;
  evo_trans_w_t pair_trans;
} evo_block_w_t;

size_t evoformer_block_workspace_bytes(const evo_block_desc_t* desc, int32_t phase);
/* m_out/z_out may alias m/z. */
evo_status_t evoformer_block_fwd(const evo_block_desc_t* desc, const evo_block_w_t* w,
                                 const void* m, const void* z, const float* msa_mask,
                                 const float* pair_mask, void* m_out, void* z_out,
                                 void* ws, size_t ws_bytes, void* stream);
/* dm = dm_out + J_m^T(...), dz likewise, d_w += parameter gradients of the block.
 * dm/dz may alias dm_out/dz_out. */
evo_status_t evoformer_block_bwd(const evo_block_desc_t* desc, const evo_block_w_t* w,
                                 const void* m, const void* z, const float* msa_mask,
                                 const float* pair_mask, const void* dm_out, const void* dz_out,
                                 void* dm, void* dz, const evo_block_w_t* d_w,
                                 void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ block without its checkpoint
 * The same block for callers with memory to spare (paper, Section "Recompute":
 * recomputation trades one more forward per block for the memory of the
 * block's intermediates; at N_seq=128, N_res=256 they are a few GB of the
 * 288 GB of HBM).  evoformer_block_fwd_save computes the forward of
 * evoformer_block_fwd and keeps the block's state in `saved`: the dropout
 * multipliers, the packed parameters, the activations between sub-operations
 * (with BF16, also the FP32 copies of m and z the block computes in) and every
 * sub-operation's saved tensors (evoformer_block_saved_bytes(desc)
 * bytes, 16-byte aligned, owned by the caller; 0 for an invalid or chunked
 * desc).  evoformer_block_bwd_saved is evoformer_block_bwd without the
 * recomputation: it reads `saved` as the forward left it (the same desc, w,
 * m, z and masks; `saved` unchanged in between) and gives bit-identical
 * results.  Here m_out / z_out must not alias m / z (the backward reads them).
 * Workspaces: evoformer_block_save_workspace_bytes(desc, EVO_PHASE_FWD) for the
 * forward, (desc, EVO_PHASE_BWD) for the backward.  chunk must be 0.
 */
size_t evoformer_block_saved_bytes(const evo_block_desc_t* desc);
size_t evoformer_block_save_workspace_bytes(const evo_block_desc_t* desc, int32_t phase);
evo_status_t evoformer_block_fwd_save(const evo_block_desc_t* desc, const evo_block_w_t* w,
                                      const void* m, const void* z, const float* msa_mask,
                                      const float* pair_mask, void* m_out, void* z_out,
                                      void* saved, size_t saved_bytes,
                                      void* ws, size_t ws_bytes, void* stream);
evo_status_t evoformer_block_bwd_saved(const evo_block_desc_t* desc, const evo_block_w_t* w,
                                       const void* m, const void* z, const float* msa_mask,
                                       const float* pair_mask, const void* saved,
                                       const void* dm_out, const void* dz_out, void* dm, void* dz,
                                       const evo_block_w_t* d_w, void* ws, size_t ws_bytes,
                                       void* stream);

/* ------------------------------------------------------------------ template pair stack block
 * One block of AlphaFold2's template pair stack, which the paper's initial-training
 * forward includes (its template embedding): the pair-stack operators on one
 * template's pair features t [N_res, N_res, c_t], in the order
 *   t <- t + TriAttnStart(t); t <- t + TriAttnEnd(t); t <- t + TriMulOut(t);
 *   t <- t + TriMulIn(t); t <- t + Transition(t).
 * Templates are independent: the caller runs every template through the same
 * blocks; template_index enters the dropout counter (sub-op number | index << 8).
 * Like the Evoformer block it is a checkpoint boundary (forward saves nothing).
 */
typedef struct {
  int32_t dtype;
  int64_t n_res, c_t;
  int32_t tri_heads, tri_head_dim;
  int64_t tri_mul_hidden, transition_factor;
  int64_t chunk;              /* forward only, as in evo_block_desc_t */
  float ln_eps;
  int32_t dropout;            /* as in evo_block_desc_t (no row attention here) */
  int32_t template_index;     /* 0 .. 2^24 - 1 */
  float drop_tri_mul, drop_tri_att;
  uint64_t drop_seed, drop_offset;
} evo_template_desc_t;

typedef struct {
  evo_attn_w_t tri_att_start, tri_att_end;
  evo_trimul_w_t tri_mul_out, tri_mul_in;
  evo_trans_w_t pair_trans;
} evo_template_w_t;

size_t template_pair_block_workspace_bytes(const evo_template_desc_t* desc, int32_t phase);
/* t_out may alias t. */
evo_status_t template_pair_block_fwd(const evo_template_desc_t* desc, const evo_template_w_t* w,
                                     const void* t, const float* pair_mask, void* t_out,
                                     void* ws, size_t ws_bytes, void* stream);
/* dt = dt_out + J^T dt_out (dt may alias dt_out); d_w += parameter gradients. */
evo_status_t template_pair_block_bwd(const evo_template_desc_t* desc, const evo_template_w_t* w,
                                     const void* t, const float* pair_mask, const void* dt_out, void* dt,
                                     const evo_template_w_t* d_w, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ optimizer step
 * The optimizer stages over fused (flat) FP32 buffers of n elements: the
 * parameters, their gradients, the Adam moments m and v, and the exponential
 * moving average of the parameters (paper, Section "Tensor Fusion" and its
 * table of kernel launches per stage: gradient clipping by global norm, Adam,
 * EMA; update rules as in AlphaFold2, Section "Hyperparameter setting"):
 *   clip   norm = sqrt(sum_i g_i^2);  g <- g * max_norm / max(norm, max_norm)
 *   Adam   m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
 *          p <- p - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 *   EMA    e <- decay e + (1 - decay) p
 * All buffers are caller-owned device pointers, 16-byte aligned, n >= 0
 * elements each (n = 0: buffers may be NULL; launches touch nothing).  The norm is
 * accumulated in FP64 in a fixed order (deterministic).  The workspace holds
 * the norm's partial sums: evo_optim_workspace_bytes(n) bytes, 16-byte
 * aligned, contents undefined on entry and after the call.
 */
typedef struct {
  double lr, beta1, beta2, eps;  /* Adam; 0 <= beta < 1, eps > 0 */
  double max_norm;               /* clip threshold; <= 0: no clipping */
  double ema_decay;              /* in [0, 1]; used only when an EMA buffer is given */
  int64_t step;                  /* Adam step counter, from 1 */
} evo_optim_desc_t;
/* The hyperparameters are double so that 1 - beta, 1 - decay and the bias
 * corrections are formed exactly on the host; the kernels compute in FP32. */

size_t evo_optim_workspace_bytes(int64_t n);
/* *norm_out (device) = ||grads||_2.  2 launches. */
evo_status_t evo_grad_global_norm(const float* grads, int64_t n, float* norm_out, void* ws, size_t ws_bytes,
                                  void* stream);
/* grads scaled in place to global norm at most max_norm (> 0); *norm_out (device, may
 * be NULL) = the norm before clipping.  2 launches. */
evo_status_t evo_clip_by_global_norm(float* grads, int64_t n, double max_norm, float* norm_out, void* ws,
                                     size_t ws_bytes, void* stream);
/* One Adam update of params, m, v in place (desc->max_norm ignored).  1 launch. */
evo_status_t evo_adam_step(const evo_optim_desc_t* desc, float* params, const float* grads, float* m,
                           float* v, int64_t n, void* stream);
/* ema updated in place from params.  1 launch. */
evo_status_t evo_ema_update(float* ema, const float* params, int64_t n, double decay, void* stream);
/* The whole step: clip (when desc->max_norm > 0; the clipped gradient is applied in
 * registers, grads is not modified), Adam, and the EMA of the updated parameters
 * when ema is not NULL.  *norm_out (may be NULL) = the gradient norm before clipping.
 * 2 launches with clipping, 1 without (then ws may be NULL). */
evo_status_t evo_optimizer_step(const evo_optim_desc_t* desc, float* params, const float* grads, float* m,
                                float* v, float* ema, int64_t n, float* norm_out, void* ws, size_t ws_bytes,
                                void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight training loops, harnesses that forbid hipMalloc): evo_optimizer_step
 * without a workspace.  The norm's partial sums go to a static device array of
 * the library (1024 doubles = 8 KiB per GPU, held until the process ends); the
 * partial count is min(1024, ceil(n / 16384)), so every n fits, and a count
 * above the array would be rejected with EVO_ESHAPE.  The call allocates
 * nothing.  Every call on one GPU shares that array: calls that overlap on one
 * GPU (other streams, other threads) race.  Its contents before a call do not
 * matter (the partials are written before they are read). */
evo_status_t evo_optimizer_step_noalloc(const evo_optim_desc_t* desc, float* params, const float* grads,
                                        float* m, float* v, float* ema, int64_t n, float* norm_out,
                                        void* stream);

/* ------------------------------------------------------------------ launch profiler
 * Optional per-launch timing for roofline reports.  Between evo_profile_begin
 * and evo_profile_end every kernel the library enqueues is bracketed by two
 * HIP events recorded on the stream it is launched on.  evo_profile_end waits
 * for those events and returns one record per kernel instance (template
 * instantiation) with the launch count, the summed event durations and the
 * summed algorithmic FLOPs and bytes of its launches (the products and the
 * compulsory reads/writes the launch's own inputs and outputs imply).
 * Returns the number of records written (at most max_records), -1 on error.
 * Not thread-safe with respect to concurrent library calls.
 */
typedef struct {
  char name[120];
  int64_t launches;
  double total_ms;
  double flops;
  double bytes;
} evo_kernel_stat_t;

void evo_profile_begin(void);
int32_t evo_profile_end(evo_kernel_stat_t* records, int32_t max_records);
/* detail != 0: records are keyed "kernel@sub-operation" instead of by kernel
 * instance alone (for a per-sub-operation breakdown). */
void evo_profile_set_detail(int32_t detail);

/* ------------------------------------------------------------------ misc */
const char* evo_version(void);
const char* evo_last_error(void);
/* EVO_OK if the current HIP device is gfx950, EVO_EUNSUPPORTED otherwise. */
evo_status_t evo_device_check(void);

#ifdef __cplusplus
}
#endif
#endif /* EVO_H_ */
