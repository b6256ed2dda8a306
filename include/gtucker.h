/*
 * gtucker.h -- C ABI of the groupwise Tucker channel-compression library for MI355X (gfx950).
 *
 * The library fits the groupwise Tucker model of OFDM massive-MIMO channel tensors and
 * evaluates per-subcarrier SINR directly from the compressed form (Zhang, Zhu & Zhang,
 * "Compressing MIMO Channel Submatrices with Tucker Decomposition", Sections 3.2 and 3.3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Complex data is interleaved (re, im) single precision ("c64", 8 bytes per element),
 *    the layout of a torch.complex64 tensor, and real outputs are float32; a plan created
 *    with dtype GT_C128 takes double precision instead (16 bytes, torch.complex128, float64
 *    outputs) on the calls that provide it (see gt_dtype).
 *  - Every data pointer is device memory owned by the caller.  The library never allocates
 *    device memory: scratch lives in a caller-allocated workspace whose size comes from
 *    gt_plan_workspace_bytes and which gt_workspace_init must fill once before use.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as void*; NULL is
 *    the default stream).  Host-detectable errors return synchronously and launch nothing.
 *    Numerical conditions found on the device are OR-ed into a per-channel int32 status
 *    word (GT_DEV_*); the caller clears it and reads it after synchronising.
 *  - No C++ exception crosses this boundary.  All functions are thread-compatible: a plan
 *    is immutable after creation (apart from the side streams its first fit makes, under a
 *    lock) and may be shared; a workspace must not be used by two calls that run
 *    concurrently, and one plan's fits must not overlap.
 *
 * Per-channel layouts (row-major; each channel's block starts at the offsets given by
 * gt_plan_offsets, in elements):
 *    X     [nsc][nr][nt]      channel tensor: H_s is the s-th nr x nt slice
 *    A     [nr][m]            mode-1 factor, orthonormal columns
 *    B     [nt][n]            mode-2 factor in matrix form: H_s ~ A Ht_s B^H
 *    C     [nsc][p]           row s of the group factor C_g of the group holding s;
 *                             entries q >= p_g are zero
 *    G     [groups][p][m][n]  core of each group, slice q is G_g[q]; slices q >= p_g zero
 *    Ht    [nsc][m][n]        compressed channel Ht_s = sum_q C[s,q] G_g[q]
 *    SINR  [n_snr][total_subcarriers][ns_max] float32, linear; the subcarriers of channel c
 *          start at offsets.sc; streams r >= ns of that channel are written as 0
 *  Groups: g(s) = s / group_size; the last group may be short; p_g = min(p, group size).
 */
#ifndef GTUCKER_H
#define GTUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GT_OK = 0,
  GT_ERR_ARG = 1,         /* null pointer, bad enum, bad count */
  GT_ERR_SHAPE = 2,       /* non-positive or unsupported dimension */
  GT_ERR_RANK = 3,        /* rank larger than its dimension, ns > min(m, n), p > group size */
  GT_ERR_WORKSPACE = 4,   /* workspace missing or smaller than gt_plan_workspace_bytes */
  GT_ERR_UNSUPPORTED = 5, /* operation or option not provided */
  GT_ERR_HIP = 6,         /* a HIP runtime call or kernel launch failed */
  GT_ERR_NO_DEVICE = 7    /* no usable GPU */
} gt_status;

/* device status bits, OR-ed per channel */
#define GT_DEV_NONFINITE 1u      /* a non-finite value entered an eigensolver or the SINR chain */
#define GT_DEV_EIG_SWEEPS 2u     /* an eigensolver stopped at its sweep cap before converging */
#define GT_DEV_CHOLESKY 4u       /* the MMSE covariance lost positive definiteness */
#define GT_DEV_ZERO_STREAM 8u    /* sigma_r <= 1e-3 sigma_1 (FP32) for a requested stream: SINR_r := 0 */

/* Element type of a plan's complex buffers.
 *   GT_C64   interleaved FP32 (re, im), 8 bytes; real outputs (SINR, its gradient input) are
 *            float32.  Every call is provided.
 *   GT_C128  interleaved FP64 (re, im), 16 bytes; SINR outputs and grad_sinr are float64.
 *            Provided for gt_sinr_eval, gt_sinr_eval_full and gt_sinr_eval_backward, which then
 *            run the whole SVD / MMSE / SINR chain and its adjoint in FP64 on the GPU (for
 *            validation and finite-difference gradient checks of the differentiation form, not
 *            for throughput); the fit, reconstruction, their adjoints and the autotuner return
 *            GT_ERR_UNSUPPORTED on such a plan.  sigma2 stays a float array. */
typedef enum { GT_C64 = 0, GT_C128 = 1 } gt_dtype;

/* Contraction precision of the fit's mode-n products H_s B and C_g^H H_s (the tensor-times-
 * matrix contractions of the A- and B-steps).  BF16 and FP16 round both operands to 16 bits;
 * SPLIT_BF16 writes each operand as hi + lo (two BF16 numbers) and sums the products hi hi,
 * hi lo and lo hi.  Products always accumulate in FP32; the Grams, eigensolves, cores and
 * the SINR chain stay in FP32.  The 16-bit forms need every nt to be a multiple of 4 (K steps
 * of 8 reals); gt_tucker_fit returns GT_ERR_UNSUPPORTED otherwise. */
typedef enum { GT_TTM_FP32 = 0, GT_TTM_BF16 = 1, GT_TTM_FP16 = 2, GT_TTM_SPLIT_BF16 = 3 } gt_ttm_prec;

#define GT_FIT_WARM_START 1u  /* A, B, C are read as the starting factors; the HOSVD step is skipped */

/* One channel tensor and its compression shape (paper notation M=nr, N=nt, (m, n, p)). */
typedef struct {
  int32_t nr, nt, nsc;   /* receive antennas, transmit antennas, subcarriers */
  int32_t group_size;    /* subcarriers per group */
  int32_t m, n, p;       /* Tucker ranks: 1<=m<=nr, 1<=n<=nt, 1<=p<=group_size */
  int32_t ns;            /* SVD-precoded streams evaluated by the SINR calls, 1<=ns<=min(m,n) */
  /* Factor sharing and the multi-cell system (equation "three matrix factorization"):
   * channels with the same nonzero a_id share the mode-1 factor A (the channels of one UE from
   * every BS), channels with the same nonzero b_id share the mode-2 factor B (every UE's channel
   * from one BS); 0 gives the channel a factor of its own.  Sharing channels must agree on
   * (nr, m) for A and (nt, n) for B.  For gt_sinr_eval_system, a_id labels the UE and b_id the BS
   * of every channel, and serving = 1 marks each UE's link to the BS that serves it (one per
   * UE). */
  int32_t a_id, b_id, serving;
} gt_channel_desc;

/* Element offsets of one channel inside packed batch buffers. */
typedef struct {
  int64_t x, a, b, c, g, ht;  /* complex elements */
  int64_t sc;                 /* first subcarrier of the channel in the SINR layout */
  int32_t n_groups;
  int32_t reserved;
} gt_offsets;

typedef struct {
  int32_t iters;       /* alternating sweeps S, >= 0 */
  int32_t ttm_prec;    /* gt_ttm_prec (GT_TTM_FP32 on a GT_C128 plan) */
  int32_t eig_fp64;    /* 1: Gram eigensolves in FP64 (on the FP32-accumulated Grams) */
  uint32_t flags;      /* GT_FIT_* */
  int32_t dtype;       /* gt_dtype of the plan's buffers (0 = GT_C64) */
} gt_fit_options;

typedef struct gt_plan gt_plan;

/* Validates the descriptors and builds an immutable host plan (sizes, offsets, device
 * tables, workspace layout).  Errors: GT_ERR_ARG (null, n_channels<1), GT_ERR_SHAPE (a
 * dimension out of range: nr<=16, nt<=256, group_size<=32, nsc>=1), GT_ERR_RANK (rank or
 * ns out of range), GT_ERR_UNSUPPORTED (an option not provided, such as 16-bit contractions on
 * a GT_C128 plan).  `opt` may be NULL (all options zero).  On success *out owns the
 * plan until gt_plan_destroy.  Pure host code: needs no GPU. */
gt_status gt_plan_create(const gt_channel_desc* descs, int32_t n_channels,
                         const gt_fit_options* opt, gt_plan** out);
void gt_plan_destroy(gt_plan* plan);

/* Offsets of channel `channel` (0 <= channel < n_channels).  Pure host code. */
gt_status gt_plan_offsets(const gt_plan* plan, int32_t channel, gt_offsets* out);
/* Total element counts of the packed buffers (x, a, b, c, g, ht in complex elements; sc in
 * subcarriers; n_groups summed) and the largest ns over the batch.  Pure host code. */
gt_status gt_plan_totals(const gt_plan* plan, gt_offsets* totals, int32_t* ns_max);
/* Workspace bytes every device call of this plan needs.  Pure host code. */
gt_status gt_plan_workspace_bytes(const gt_plan* plan, size_t* bytes);

/* Writes the plan's device tables into the workspace (an asynchronous host-to-device copy
 * from memory the plan owns).  Call once per workspace before any other device call. */
gt_status gt_workspace_init(const gt_plan* plan, void* ws, size_t ws_bytes, void* stream);

/* Groupwise Tucker compression (Algorithm "Groupwise Tucker compression algorithm" with the
 * HOSVD initialisation of Section 3.2; factor updates of equations "update A/B/C"; core of
 * equation "kernel").  Inputs: X.  Outputs: A, B, C, G.  obj_trace (device, double, may be
 * NULL) receives per channel 1 + 3*iters values of the objective f of equation "MT_origin"
 * after the initialisation and after each half-step, layout [n_channels][1 + 3*iters].
 * dev_status: [n_channels] int32 device words (may be NULL).  With GT_FIT_WARM_START the
 * initial A, B, C are read from the output buffers.  GT_ERR_UNSUPPORTED: a 16-bit ttm_prec
 * with some nt not a multiple of 4 (see gt_ttm_prec).  A batch of 8 or more channels that
 * runs the fused per-group passes spreads parts of each sweep over up to three side streams
 * of its own (made on the plan's first fit, default priority), forked from and joined back
 * into `stream` by events, so the call stays ordered on `stream` and can be captured in a
 * graph; a channel's results do not depend on the batch it is fitted in.  A plan whose channels
 * share factors (nonzero a_id or b_id) fits all of them together, without side streams, and
 * returns GT_ERR_UNSUPPORTED for a non-NULL obj_trace. */
gt_status gt_tucker_fit(const gt_plan* plan, const void* X, void* A, void* B, void* C, void* G,
                        double* obj_trace, int32_t* dev_status, void* ws, size_t ws_bytes,
                        void* stream);

/* Reconstruction from the compressed form (equation "compressed matrix SINR reduction" and
 * the matrix factorisation of equation "three matrix factorization"): Ht_s = sum_q C[s,q]
 * G_g[q] and Xhat_s = A Ht_s B^H.  Either output may be NULL. */
gt_status gt_tucker_reconstruct(const gt_plan* plan, const void* A, const void* B, const void* C,
                                const void* G, void* Ht, void* Xhat, void* ws, size_t ws_bytes,
                                void* stream);

/* Per-subcarrier SINR from the compressed form (Section 3.3): Ht_s from (C, G); SVD precoder
 * (equation "precoding matrix"); covariance, MMSE filter and per-stream SINR (equations
 * "covariance matrix", "MMSE receive filter", "s_r^ij", "SINR formula") on the m x m
 * compressed covariance; with Ns < m the FP32 row kernels form the same filter through the
 * push-through identity W = HV (HV^H HV + sigma2 I_Ns)^{-1}, an Ns x Ns Cholesky solve.
 * sigma2: host array of n_snr noise variances, each > 0 and finite (1 <= n_snr <= 16); any
 * other value is GT_ERR_ARG before a launch.
 * Output layout as above: float32 on a GT_C64 plan, float64 on a GT_C128 plan. */
gt_status gt_sinr_eval(const gt_plan* plan, const void* C, const void* G, const float* sigma2,
                       int32_t n_snr, void* sinr, int32_t* dev_status, void* ws, size_t ws_bytes,
                       void* stream);

/* Interference seen by each UE in gt_sinr_eval_system (equation "signal receiving"):
 *   GT_INTERF_NONE   its own link only;
 *   GT_INTERF_PAPER  its own link and, from every other BS k, the transmission to the first UE
 *                    of cell k (the UE with the lowest a_id among those BS k serves): inter-cell
 *                    interference only, the protocol of the paper's experiments (Section 4);
 *   GT_INTERF_ALL    every transmission of every BS to every other UE (intra- and inter-cell). */
#define GT_INTERF_NONE 0
#define GT_INTERF_PAPER 1
#define GT_INTERF_ALL 2

/* Per-subcarrier SINR of every UE of a multi-cell system from the compressed channels
 * (Sections 2.2 and 3.3: equations "covariance matrix", "compressed pre", "Cov", "reduced
 * inversion of interference matrix", "MMSE receive filter", "s_r^ij", "SINR formula").  The
 * plan's channels are the links (UE a_id, BS b_id) of the system (see gt_channel_desc); every
 * UE needs a channel from every BS whose transmissions it sees under `mode`, and all channels
 * the same nsc and ns, with m <= 8 and ns <= 4.  Each serving link's precoder (the first ns
 * right singular vectors of its compressed channel, equation "precoding matrix") is formed
 * first, in the workspace; then, for UE u served by BS i, Q~ = sum over the transmissions t
 * (BS k with the precoder V~_v of UE v) of (Ht_{u,k} V~_v)(Ht_{u,k} V~_v)^H + s2 I_m and the
 * MMSE chain on it.  The UE's SINR is written at its serving channel's subcarriers (layout of
 * gt_sinr_eval); the other channels' entries are written as 0.  GT_ERR_ARG: not a complete
 * system or a bad mode; GT_ERR_UNSUPPORTED: shapes outside the limits above, or a GT_C128 plan. */
gt_status gt_sinr_eval_system(const gt_plan* plan, const void* C, const void* G, const float* sigma2,
                              int32_t n_snr, int32_t mode, void* sinr, int32_t* dev_status, void* ws,
                              size_t ws_bytes, void* stream);

/* Channel matrices at general coefficient vectors (Section 2.2, equations "channel submatrices"
 * and "channel submatrices, tensor"; Section 3.3, equation "compressed matrix SINR reduction").
 * Mode 3 of X holds P path / delay submatrices H_s (nsc = P), and the channel at a time or
 * frequency point t is their combination by a row u_t of P complex weights: the row c*(t) of
 * the tensor form (pass u_t = c(t) to combine with the unconjugated coefficients of the
 * submatrix equation instead).  For every channel and each of its n_pts rows:
 *   gt_combine_full:        H(t)  = sum_s u_t[s] H_s                          (nr x nt)
 *   gt_combine_compressed:  Ht(t) = G x3 (u_t C) = sum_g sum_q w_g,q(t) G_g[q],
 *                           w_g,q(t) = sum_{s in group g} u_t[s] C[s,q]       (m x n)
 * with H(t) ~ A Ht(t) B^H.  u_t = e_s gives H_s and the Ht_s of gt_tucker_reconstruct.
 * Layouts, complex row-major, channels packed in order:
 *   U   [n_pts][nsc] per channel, channel c at n_pts * offsets.sc;
 *   H   [n_pts][nr][nt] per channel, channel c at n_pts * (sum of nr nt over channels < c);
 *   Ht  [n_pts][m][n] per channel, channel c at n_pts * (sum of m n over channels < c).
 * These are the X layouts of a plan with the descriptors (nr, nt, nsc = n_pts) or
 * (nr = m, nt = n, nsc = n_pts) and the same ns, so gt_sinr_eval_full on such a plan gives the
 * SINR of every combined channel (the compressed SINR of Section 3.3 is the same chain on
 * Ht(t)).  GT_ERR_ARG: null pointer or n_pts outside 1..2^20; GT_ERR_UNSUPPORTED: a GT_C128
 * plan. */
gt_status gt_combine_full(const gt_plan* plan, const void* X, const void* U, int32_t n_pts, void* H,
                          void* ws, size_t ws_bytes, void* stream);
gt_status gt_combine_compressed(const gt_plan* plan, const void* C, const void* G, const void* U,
                                int32_t n_pts, void* Ht, void* ws, size_t ws_bytes, void* stream);

/* The same chain on the uncompressed channel H_s (nr x nt) read from X (Section 2.2). */
gt_status gt_sinr_eval_full(const gt_plan* plan, const void* X, const float* sigma2, int32_t n_snr,
                            void* sinr, int32_t* dev_status, void* ws, size_t ws_bytes,
                            void* stream);

/* Adjoint of gt_sinr_eval: given grad_sinr (dl/dSINR, same layout and real type as the SINR
 * output), writes grad_C and grad_G (layouts of C and G, overwritten) as dl/dRe + i dl/dIm.
 * The SVD and the Cholesky factor are recomputed, not stored. */
gt_status gt_sinr_eval_backward(const gt_plan* plan, const void* C, const void* G,
                                const float* sigma2, int32_t n_snr, const void* grad_sinr,
                                void* grad_C, void* grad_G, int32_t* dev_status, void* ws,
                                size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gt_sinr_eval_backward without a workspace.  Its
 * scratch -- the plan's device tables and the per-subcarrier dl/dHt -- lives in a static
 * device array of 64 MiB that every GPU the library runs on holds from the first call on it
 * until the process ends; the call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).  The tables are copied into the array from memory the plan owns
 * (asynchronously on `stream`) at every call; dl/dHt needs no clearing.  A plan whose tables
 * and dl/dHt need more than 64 MiB (for example 20 or more 8 x 64 x 3276 channels at ranks
 * (8, 16, 12)) is refused with GT_ERR_WORKSPACE before anything is launched.  All calls on one
 * GPU share that GPU's array and it keeps the last call's contents: calls that overlap on one
 * GPU (on different streams or from different threads) race.  Arguments, outputs and errors
 * are otherwise those of gt_sinr_eval_backward. */
gt_status gt_sinr_eval_backward_static(const gt_plan* plan, const void* C, const void* G,
                                       const float* sigma2, int32_t n_snr, const void* grad_sinr,
                                       void* grad_C, void* grad_G, int32_t* dev_status,
                                       void* stream);

/* Adjoint of gt_tucker_reconstruct.  grad_Ht or grad_Xhat may be NULL (treated as zero).
 * Writes grad_A, grad_B, grad_C, grad_G (overwritten). */
gt_status gt_tucker_reconstruct_backward(const gt_plan* plan, const void* A, const void* B,
                                         const void* C, const void* G, const void* grad_Ht,
                                         const void* grad_Xhat, void* grad_A, void* grad_B,
                                         void* grad_C, void* grad_G, void* ws, size_t ws_bytes,
                                         void* stream);

/* Autotuner of the fit's pass variants on a plan's own shapes and data.  Each tunable choice
 * is timed in turn over short fits of X (HIP events, the other choices held at their current
 * values) and the fastest is kept in the plan for its later fits:
 *   bstep  B-step pass: 0 matrix-core kernel, 1 the same with the next group's operands
 *          prefetched during the current group's Gram, 2 the older matrix-core kernel;
 *   tpass  T pass: 0 matrix cores, 1 vector ALU;
 *   split  fits of 8 or more channels split into parts on concurrent streams: 0 off, 1 the
 *          B-step pass over the whole batch and the rest of each sweep per part, 2 every part
 *          runs whole sweeps on its own stream (pipelined: one part's matrix-core passes
 *          overlap another's eigensolves).  The results are the same in every mode.
 * Each configuration is timed as the faster of two fits of min(iters, 8) sweeps after an
 * untimed one, and a choice replaces the current one only when it is more than 2 % faster.
 * Choices that do not apply to the plan (no fused passes, 16-bit contractions for the
 * prefetching variant) keep 0 and are not timed.  A, B, C, G receive the last probe's fit
 * and are otherwise scratch.  Synchronises the stream and is not capturable: call it before
 * capturing the fits in a graph.  `out` (may be NULL) receives the choices and the probe
 * time of the kept configuration in ms. */
typedef struct {
  int32_t bstep, tpass, split;
  float probe_ms;
} gt_tune_result;
gt_status gt_plan_autotune(gt_plan* plan, const void* X, void* A, void* B, void* C, void* G,
                           void* ws, size_t ws_bytes, void* stream, gt_tune_result* out);
/* Sets the choices directly (for instance ones an earlier autotune stored for the same
 * shapes).  GT_ERR_ARG for a value out of range; GT_ERR_UNSUPPORTED for bstep or tpass other
 * than 0 on a plan with 16-bit contractions (those variants are FP32-only).  Pure host code.
 * gt_plan_autotune and gt_plan_set_tuning change the plan: they must not run concurrently
 * with any other call on the same plan. */
gt_status gt_plan_set_tuning(gt_plan* plan, int32_t bstep, int32_t tpass, int32_t split);

/* The fit is an argmax over eigenvectors and is not differentiated: always returns
 * GT_ERR_UNSUPPORTED. */
gt_status gt_tucker_fit_backward(const gt_plan* plan);

/* Static description of a status code. */
const char* gt_status_string(gt_status s);
/* Text of the last HIP error seen by this thread (empty if none). */
const char* gt_last_error_detail(void);

/* Kernel timing.  When enabled, every kernel the library launches is bracketed by HIP
 * events on its stream; gt_profile_query synchronises those events and returns the summed
 * duration and launch count of the kernels whose base name (identifier without template
 * arguments) equals `name`, or starts with it when `name` ends in '*'. */
gt_status gt_profile_enable(int32_t on);
gt_status gt_profile_reset(void);
gt_status gt_profile_query(const char* name, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* GTUCKER_H */
