/*
 * ftm.h -- C ABI of the MI355X (gfx950) FFT-based block lower-triangular
 * Toeplitz matvec ("FFTMatvec", arXiv 2508.10202).
 *
 * The operator is the block lower-triangular Toeplitz matrix F of
 * Section 2.3, eq. (ShiftInvariance): Nt x Nt blocks, each Nd x Nm, fixed by
 * its first block column F_0 .. F_{Nt-1} (0-based lag; the paper's
 * F_{11} .. F_{Nt,1}).  d = F m is  d_i = sum_{j<=i} F_{i-j} m_j  and the
 * adjoint m = F^T d is  m_j = sum_{i>=j} F_{i-j}^T d_i.
 *
 * Both are computed by the five phases of Section 2.4: (1) zero pad every
 * time series to L = 2 Nt, (2) batched real FFT over time, (3) per-frequency
 * complex matrix-vector product with the precomputed spectrum
 * Fhat_k (k = 0 .. Nt) of the zero-padded first block column (the conjugate
 * transpose for the adjoint), (4) inverse FFT, (5) drop the padding.
 * Each phase runs in its own precision (Section 3.2); inputs and outputs are
 * always float64.
 *
 * Memory and streams
 *   - Every array argument named as "device" is a pointer into device memory
 *     of the current HIP device (e.g. a torch.Tensor data_ptr()); the caller
 *     owns it.  The library never frees caller memory.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work on it and return without synchronising; outputs are
 *     valid once the stream has been synchronised.
 *   - The library owns the spectra, twiddle tables and workspaces it
 *     allocates; ftm_destroy_operator releases them.
 *   - ftm_matvec / ftm_rmatvec use the operator's own workspace: concurrent
 *     calls on one operator must then be on one stream.  ftm_apply takes a
 *     workspace from the caller, so calls with different workspaces may run
 *     concurrently on different streams; so do the serving API's batches.
 *   - The configuration setters (ftm_set_precision, ftm_set_rhs_mode,
 *     ftm_set_gemm_crossover, ftm_set_tuning, ftm_profile_enable) may be
 *     called from any thread: each call copies the configuration it runs
 *     with, under the operator's lock, when it is made.
 *
 * Errors
 *   - Every entry point returns an ftm_status; nothing throws or aborts
 *     across the ABI.  Argument errors are detected before any work is
 *     enqueued.  HIP errors map to FTM_ERR_HIP.  ftm_last_error() returns a
 *     thread-local message for the last failure on the calling thread.
 */
#ifndef FTM_H
#define FTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ftm_status {
  FTM_OK = 0,
  FTM_ERR_INVALID = 1,     /* bad argument (null pointer, size <= 0, ...) */
  FTM_ERR_UNSUPPORTED = 2, /* valid request this build cannot serve        */
  FTM_ERR_OOM = 3,         /* device allocation failed                     */
  FTM_ERR_BUDGET = 4,      /* request exceeds the serving memory budget    */
  FTM_ERR_HIP = 5,         /* a HIP runtime call or a launch failed        */
  FTM_ERR_STATE = 6        /* object used in a state that does not allow it */
} ftm_status;

/* Storage precision of a phase.  FP16 and BF16 phases store their data in
 * that format and compute in float32 (accumulating in float32). */
typedef enum ftm_dtype { FTM_F64 = 0, FTM_F32 = 1, FTM_F16 = 2, FTM_BF16 = 3 } ftm_dtype;

/* Per-phase precision configuration of one direction, in execution order
 * (Section 3.2: set when the operator is created and changeable at run
 * time).  Phase i takes its input rounded to its own precision, computes in
 * it (float32 for FP16/BF16) and rounds its output to it.
 *   pad   -- phase 1, broadcast + zero padding (a memory phase)
 *   fft   -- phase 2, real FFT of the input series
 *   gemv  -- phase 3, storage precision of Fhat and of the product
 *   ifft  -- phase 4, inverse real FFT
 *   unpad -- phase 5, unpadding (a memory phase)
 *   accum -- accumulation type of phase 3: FTM_F64 or FTM_F32.  Must be
 *            FTM_F64 when gemv is FTM_F64 and FTM_F32 when gemv is
 *            FTM_F16 or FTM_BF16; either for FTM_F32. */
typedef struct ftm_precision {
  int32_t pad, fft, gemv, ifft, unpad, accum;
} ftm_precision;

typedef struct ftm_operator_s* ftm_operator;

/* Build the operator from its first block column (Section 2.4: only the first
 * block column is stored; its zero-padded FFT along time is computed once, in
 * float64, Section 3.2.1 "Initial state").
 *   F        device, float64, [Nt][Nd][Nm] row-major (lag, sensor, parameter).
 *            Only read during the call's stream work; may be freed after the
 *            stream is synchronised.
 *   fwd, adj precision of F and F^T matvecs; NULL means all-FP64.
 *   spectra  bit mask (1 << ftm_dtype) of extra Fhat storage copies to keep
 *            for later ftm_set_precision calls; the copies fwd/adj need are
 *            always kept.
 *   max_rhs  largest nrhs later passed to matvec/rmatvec (>= 1); sizes the
 *            workspace.
 * Limits: Nt in [1, 2048], Nd, Nm >= 1.  The pad length L is 2 Nt when 2 Nt
 * has no prime factor above 7, else the next even length that has none (any
 * L >= 2 Nt - 1 gives the same product); K = L / 2 + 1 frequencies are
 * kept (ftm_operator_info reports L).  FTM_ERR_UNSUPPORTED when that length
 * exceeds 4096. */
ftm_status ftm_setup_operator(ftm_operator* out, const double* F, int64_t Nt, int64_t Nd,
                              int64_t Nm, const ftm_precision* fwd, const ftm_precision* adj,
                              uint32_t spectra, int64_t max_rhs, void* stream);

/* ftm_setup_operator for F in another memory layout: element (t, r, c) of
 * the first block column is F[t * stride_t + r * stride_r + c * stride_c]
 * (strides in elements).  Solver-native layouts (Section 2.4: the first block
 * column comes from Nd adjoint PDE solves, e.g. time series stored contiguously
 * per sensor and parameter, [Nd][Nm][Nt] or [Nm][Nd][Nt]) are read directly by
 * the setup transform: no permuted copy of F is made (the permutation kernel
 * of Section 3.1 is folded into the transform's loads).  The spectrum equals
 * the one of the same F in the [Nt][Nd][Nm] layout, bitwise.
 * FTM_ERR_INVALID also when the strides let two elements overlap (in
 * increasing stride order each stride must be at least the span of the
 * smaller ones; strides of extent-1 dimensions are ignored). */
ftm_status ftm_setup_operator_strided(ftm_operator* out, const double* F, int64_t Nt, int64_t Nd, int64_t Nm,
                                      int64_t stride_t, int64_t stride_r, int64_t stride_c,
                                      const ftm_precision* fwd, const ftm_precision* adj, uint32_t spectra,
                                      int64_t max_rhs, void* stream);

/* Change the precision configuration (NULL leaves a direction unchanged).
 * Fails with FTM_ERR_UNSUPPORTED if the needed Fhat copy was not kept. */
ftm_status ftm_set_precision(ftm_operator op, const ftm_precision* fwd, const ftm_precision* adj);

/* d = F m for nrhs right-hand sides (Section 2.4, phases 1-5).
 *   m device float64 [nrhs][Nt][Nm];  d device float64 [nrhs][Nt][Nd].
 *   1 <= nrhs <= max_rhs.  m and d must not overlap. */
ftm_status ftm_matvec(ftm_operator op, const double* m, double* d, int64_t nrhs, void* stream);

/* m = F^T d for nrhs right-hand sides (Section 2.4: phase 3 uses the
 * conjugate transpose of each Fhat_k; inputs and outputs swap).
 *   d device float64 [nrhs][Nt][Nd];  m device float64 [nrhs][Nt][Nm]. */
ftm_status ftm_rmatvec(ftm_operator op, const double* d, double* m, int64_t nrhs, void* stream);

/* Bytes of device workspace one call of ftm_apply needs for nrhs right-hand
 * sides (1 <= nrhs <= 2^20) in the given direction at the operator's current
 * precision configuration: K * nrhs * (ldm * e_m + ldd * e_d), each part
 * rounded up to 256 bytes, where e_m and e_d are 16 for a transformed vector
 * stored in float64 (both neighbouring phases float64) and 8 otherwise, and
 * ldm, ldd are Nm and Nd rounded up to 8. */
ftm_status ftm_workspace_size(ftm_operator op, int32_t adjoint, int64_t nrhs, size_t* bytes);

/* y = F x (adjoint = 0) or y = F^T x (adjoint != 0) for nrhs right-hand
 * sides (1 <= nrhs <= 2^20, not limited by max_rhs), as ftm_matvec /
 * ftm_rmatvec but on a workspace the caller provides (Section 2.4: the
 * transformed vectors of phases 2-4 live there).
 *   x, y       device float64, [nrhs][Nt][Nm] / [nrhs][Nt][Nd] as for
 *              ftm_matvec (swapped for the adjoint); must not overlap.
 *   workspace  device memory of at least ftm_workspace_size(op, adjoint,
 *              nrhs) bytes, 256-byte aligned, not overlapping x or y; its
 *              contents on entry do not matter and are clobbered.  It is in
 *              use until the stream reaches the end of the call.
 * Calls with distinct workspaces may run concurrently on different streams.
 * FTM_ERR_INVALID: NULL pointers, nrhs out of range, a workspace that is too
 * small, misaligned or overlapping. */
ftm_status ftm_apply(ftm_operator op, int32_t adjoint, const double* x, double* y, int64_t nrhs, void* workspace,
                     size_t workspace_bytes, void* stream);

/* Data-space Hessian actions y = F Gamma F^T x with Gamma = I (the dense
 * data-space Hessian of the outer-loop problems in Section 3.2 takes
 * Nd * Nt of them; Section 2.3 applies F^* inside the MAP point): for each of
 * nrhs data vectors, the adjoint matvec into a float64 parameter-space
 * intermediate, then the forward matvec, each at its direction's precision
 * configuration (the many-right-hand-side path of ftm_set_rhs_mode applies to
 * both).
 *   x, y       device float64 [nrhs][Nt][Nd]; must not overlap.
 *   workspace  device memory of at least ftm_hessian_workspace_size(op, nrhs)
 *              bytes (nrhs * Nt * Nm * 8 for the intermediate, rounded up to
 *              256, plus the larger of the two directions'
 *              ftm_workspace_size), 256-byte aligned, not overlapping x or y;
 *              contents on entry do not matter.  The call allocates nothing.
 * 1 <= nrhs <= 2^20.  Calls with distinct workspaces may run concurrently on
 * different streams.  FTM_ERR_INVALID: NULL pointers, nrhs out of range, a
 * workspace that is too small, misaligned or overlapping. */
ftm_status ftm_hessian_workspace_size(ftm_operator op, int64_t nrhs, size_t* bytes);
ftm_status ftm_hessian_apply(ftm_operator op, const double* x, double* y, int64_t nrhs, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Round n values into storage format dtype exactly as every phase does
 * (round to nearest, ties to even; values beyond the format's range become
 * infinities, NaN stays NaN; Section 3.2 casts).  With from_f32 the values are
 * first rounded to float32 and the float32 path of the kernels is used (as in
 * phases that compute in float32).
 *   x, y  device float64 [n] (may be the same array).
 * FTM_ERR_INVALID: unknown dtype, n < 0, NULL pointers with n > 0. */
ftm_status ftm_round(int32_t dtype, int32_t from_f32, const double* x, double* y, int64_t n, void* stream);

/* Bytes of the library's static scratch workspace on each GPU (96 MiB: one
 * float64 vector at Nt=1000, Nd=100, Nm=5000 needs 81.8 MB). */
#define FTM_SCRATCH_BYTES ((size_t)96 << 20)

/* ftm_apply without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): the transformed vectors live in a static
 * FTM_SCRATCH_BYTES array of the library, one per GPU, which each GPU holds
 * from the first call on it until the process ends.  The call allocates
 * nothing (no hipMalloc, no events) and records no profiling events.
 *   x, y   as for ftm_apply.
 * All calls on one GPU share its scratch, and it keeps the last call's
 * contents (no call depends on them): calls that overlap on one GPU (on
 * different streams, or from different threads without ordering) race and
 * must not be issued.
 * FTM_ERR_UNSUPPORTED: the call needs more than FTM_SCRATCH_BYTES of
 * workspace (ftm_workspace_size); FTM_ERR_INVALID: as for ftm_apply. */
ftm_status ftm_apply_scratch(ftm_operator op, int32_t adjoint, const double* x, double* y, int64_t nrhs,
                             void* stream);

/* How phase 3 treats nrhs > 1 right-hand sides:
 *   FTM_RHS_AUTO  (default) a complex GEMM per frequency on the matrix cores
 *                 when nrhs >= the crossover (ftm_set_gemm_crossover,
 *                 ftm_set_tuning), else one matrix-vector product per
 *                 right-hand side.  The GEMM accumulates in float64 for
 *                 FP64 products and FP32 ones with accum FTM_F64, in float32
 *                 otherwise; a vector's result does not depend on the batch
 *                 around it.
 *   FTM_RHS_GEMV  always one matrix-vector product per right-hand side
 *   FTM_RHS_GEMM  the GEMM for every nrhs >= 2 */
typedef enum ftm_rhs_mode { FTM_RHS_AUTO = 0, FTM_RHS_GEMV = 1, FTM_RHS_GEMM = 2 } ftm_rhs_mode;
ftm_status ftm_set_rhs_mode(ftm_operator op, int32_t mode);

/* Smallest nrhs for which FTM_RHS_AUTO uses the GEMM (>= 2; default 2), for
 * both directions and every storage format (ftm_set_tuning sets it per
 * direction for the current configuration). */
ftm_status ftm_set_gemm_crossover(ftm_operator op, int64_t min_rhs);

/* Tolerance-driven precision (Section 3.2: the fastest configuration whose
 * error is within a tolerance set by the application, from the error-vs-time
 * Pareto front).  For one direction, every {FP64, FP32, FP16, BF16}
 * assignment to the five phases (and FP32 products with float64
 * accumulation) whose product format's spectrum copy the operator keeps, and
 * whose coarsest unit roundoff / 64 does not exceed the tolerance, runs on
 * the probe input; its relative L2 error against the all-FP64 result on the
 * same probe is measured, and those within the tolerance are timed (reps
 * runs each, one vector).  The fastest (ties: the smaller error) becomes the
 * direction's configuration; its error and time (ms) are returned.  The
 * all-FP64 configuration always qualifies.
 *   probe  device float64 [Nt][Nm] (forward) or [Nt][Nd] (adjoint): an input
 *          representative of the application's (the errors depend on it).
 * Needs the FP64 spectrum (the reference; FTM_ERR_UNSUPPORTED otherwise).
 * Allocates scratch for the call; synchronises the stream. */
ftm_status ftm_select_precision(ftm_operator op, int32_t adjoint, double tolerance, const double* probe, int32_t reps,
                                ftm_precision* chosen, double* rel_err, double* ms, void* stream);

/* Kernel and tile choices of one operator for its current precision
 * configuration (the entries are kept per direction and per storage or
 * compute format, so switching precision keeps each configuration's own).
 *   gemv_variant[d]   matrix-vector tile of direction d (0 forward, 1
 *                     adjoint): 0 .. 3, 0 the default
 *   fft_shape[d][i]   transform kernel of direction d, i = 0 the input
 *                     transform (phases 1-2), 1 the output one (4-5): 0 the
 *                     default (the larger tile unless it gives fewer than 4
 *                     tiles per CU or needs more than half of a CU's LDS,
 *                     then the smaller), 1 / 2 the fixed-plan
 *                     kernels' larger / smaller column tile (lengths that
 *                     have them: 128, 256, 400, 512, 1024, 2000; others run
 *                     the runtime-plan kernels whatever the value), 3 the
 *                     runtime-plan kernels
 *   gemm_tile[d]      right-hand sides per matrix-core GEMM tile: 0 (the
 *                     default, 64), 16, 32 or 64
 *   gemm_kind[d]      matrix-core instructions of an FP32-storage product with
 *                     float32 accumulation: 1 the FP32 MFMA, 2 the BF16 MFMA
 *                     on the three-term BF16 split of both operands (FP32
 *                     accuracy, fewer cycles; faster when the product is
 *                     compute bound), 0 the default (2 at 64-right-hand-
 *                     side tiles, for the adjoint only when Nd > 32; else
 *                     1); other storage formats ignore it
 *   gemm_min_rhs[d]   smallest nrhs for which FTM_RHS_AUTO runs the GEMM (>= 2)
 *   ms[d]             the matvec time (milliseconds) of the last autotune at
 *                     these choices, 0 if none (read only) */
typedef struct ftm_tuning {
  int32_t gemv_variant[2];
  int32_t fft_shape[2][2];
  int32_t gemm_tile[2];
  int32_t gemm_kind[2];
  int64_t gemm_min_rhs[2];
  double ms[2];
} ftm_tuning;

/* Autotuning (Section 3.1.1: tile parameters per precision, transition
 * points from measurements): for both directions at the operator's current
 * precision configuration, time the matrix-vector tile variants and the
 * transform kernels on one vector (reps timed runs each, scratch inputs) and
 * keep the fastest; for an FP32-storage product with float32 accumulation,
 * keep the faster GEMM instructions (gemm_kind 1 or 2) at 64 right-hand
 * sides; then set the GEMM crossover to the smallest batch of 2, 4, .., 32
 * right-hand sides for which the matrix-core product is no slower than one
 * matrix-vector product per vector (33 if none).  These probes allocate
 * inputs and workspace for 64 vectors.  Synchronises the stream.  ftm_get_tuning /
 * ftm_set_tuning read and set the choice (for a persistent tuning cache kept
 * by the caller).  Out-of-range values are FTM_ERR_INVALID. */
ftm_status ftm_autotune(ftm_operator op, int32_t reps, void* stream);
ftm_status ftm_get_tuning(ftm_operator op, ftm_tuning* out);
ftm_status ftm_set_tuning(ftm_operator op, const ftm_tuning* t);

/* HIP graph of one matvec with fixed buffers (x, y as for ftm_matvec or
 * ftm_rmatvec; adjoint != 0 selects F^T).  Launching replays the three
 * kernels with one call.  The graph uses the operator's workspace: replays
 * must not overlap other calls on the operator.  The graph is bound to the
 * operator's precision and tuning at capture time. */
typedef struct ftm_graph_s* ftm_graph;
ftm_status ftm_graph_create(ftm_graph* out, ftm_operator op, int32_t adjoint, const double* x, double* y,
                            int64_t nrhs);
ftm_status ftm_graph_launch(ftm_graph g, void* stream);
ftm_status ftm_graph_destroy(ftm_graph g);

/* Copy bins k0 .. k0+nk-1 of the stored spectrum in storage precision
 * `which` (widened to float64) to out: device float64 [nk][Nd][Nm][2]
 * (real, imaginary).  Fhat_k = sum_{t<Nt} F_t exp(-2 pi i k t / L). */
ftm_status ftm_get_spectrum(ftm_operator op, int32_t which, int64_t k0, int64_t nk, double* out,
                            void* stream);

/* Shape and memory facts: any pointer may be NULL.  device_bytes counts every
 * device allocation the operator holds (spectra, tables, workspace). */
ftm_status ftm_operator_info(ftm_operator op, int64_t* Nt, int64_t* Nd, int64_t* Nm, int64_t* L,
                             size_t* device_bytes);

/* Per-kernel timing (instrumentation).  While enabled, every matvec and
 * rmatvec records HIP events on its own stream around each of its three
 * kernels: 0 = pad + FFT (phases 1-2), 1 = product (phase 3),
 * 2 = inverse FFT + unpad (phases 4-5).  Events come from a pool the operator
 * owns; enabling costs one event record per kernel boundary. */
ftm_status ftm_profile_enable(ftm_operator op, int32_t enable);

/* Sum the recorded kernel times (waits for the recorded events).
 *   ms     host double[6]: ms[dir * 3 + kernel], dir 0 = forward, 1 = adjoint
 *   counts host int64_t[2]: number of recorded calls per direction
 *   reset  non-zero clears the record afterwards. */
ftm_status ftm_profile_read(ftm_operator op, double* ms, int64_t* counts, int32_t reset);

/* Release everything the operator owns.  The caller must make sure no work
 * using it is still pending.  NULL is accepted and ignored. */
ftm_status ftm_destroy_operator(ftm_operator op);

/* ---- serving ------------------------------------------------------------
 * Continuous batching of matvec requests against device-resident operators
 * (one GPU).  A worker thread owns n_slots HIP streams and one workspace
 * arena of workspace_budget bytes allocated at creation.  Whenever a slot is
 * free it admits the oldest queued request together with every later queued
 * request for the same operator and direction, up to max_batch_rhs
 * right-hand sides, as one multi-right-hand-side matvec -- provided the
 * batch's workspace fits in the unused part of the budget; otherwise the
 * queue head waits (first in, first out) until running batches release
 * workspace.  Batches on different slots overlap on the device.  Requests
 * that arrive while others run are admitted as slots and workspace free up.
 * Results are the same, within the precision configuration's tolerance, as
 * a lone ftm_matvec/ftm_rmatvec of the same input (bitwise when the product
 * takes the same path; see ftm_set_rhs_mode).
 * The operators' precision configuration is copied when a batch is
 * admitted; the batch is sized and runs with that copy.  A batch's workspace
 * is ftm_workspace_size of its operator, direction and total nrhs.  The
 * budget is used in 256-byte granules (rounded down).  A queued request that
 * no longer fits the whole budget at its operator's configuration when it
 * reaches the head of the queue fails (FTM_ERR_HIP from ftm_server_wait /
 * poll, with the reason in ftm_last_error) instead of waiting forever. */
typedef struct ftm_server_s* ftm_server;

typedef struct ftm_server_stats {
  uint64_t submitted, completed, failed;
  uint64_t batches;             /* launched batches */
  uint64_t rhs_launched;        /* right-hand sides over all batches */
  uint64_t coalesced_requests;  /* requests that shared a batch with others */
  uint64_t budget_waits;        /* times the queue head had to wait for workspace */
  int64_t max_inflight_requests, queued_requests;
  size_t peak_workspace_bytes, workspace_in_use_bytes;
} ftm_server_stats;

/* workspace_budget >= 4 KiB, 1 <= n_slots <= 16, 1 <= max_batch_rhs <= 4096.
 * Uses the current HIP device. */
ftm_status ftm_server_create(ftm_server* out, size_t workspace_budget, int32_t n_slots, int64_t max_batch_rhs);

/* Queue one request: adjoint = 0 computes y = F x (x [nrhs][Nt][Nm], y
 * [nrhs][Nt][Nd]), adjoint != 0 computes y = F^T x (x [nrhs][Nt][Nd], y
 * [nrhs][Nt][Nm]); device float64.  ready_event (a hipEvent_t, may be NULL)
 * is waited for on the device before x is read: record it on the stream that
 * produced x.  The caller keeps x, y and the event alive, and x and y
 * untouched, until the ticket completes.  FTM_ERR_BUDGET: the request alone
 * needs more workspace than the whole budget at the operator's current
 * configuration (it would never run). */
ftm_status ftm_server_submit(ftm_server s, ftm_operator op, int32_t adjoint, const double* x, double* y,
                             int64_t nrhs, void* ready_event, uint64_t* ticket);

/* done = 1 once the request's output is written and visible to the device;
 * latency_s (may be NULL) = completion time - submit time, seconds. */
ftm_status ftm_server_poll(ftm_server s, uint64_t ticket, int32_t* done, double* latency_s);

/* Block until the ticket completes (timeout_s <= 0: no limit). */
ftm_status ftm_server_wait(ftm_server s, uint64_t ticket, double* latency_s, double timeout_s);

/* Latencies of tickets first_ticket .. first_ticket+n-1 (NaN while pending). */
ftm_status ftm_server_latencies(ftm_server s, uint64_t first_ticket, int64_t n, double* out);

ftm_status ftm_server_get_stats(ftm_server s, ftm_server_stats* out);

/* Drain every queued and running request, then release the server. */
ftm_status ftm_server_destroy(ftm_server s);

/* ---- strided-batched matrix-vector product ------------------------------
 * The standalone form of the phase-3 product (Section 3.1.1): for b < batch,
 *   y_b = alpha op(A_b) x_b + beta y_b
 * with BLAS semantics -- A_b is m x n column-major (element (i, j) at
 * A[b * stride_a + i + j * lda], lda >= max(m, 1)), x_b and y_b are
 * contiguous (unit increment) at x + b * stride_x and y + b * stride_y.
 * op = FTM_OP_N: x_b has n entries and y_b m; op = FTM_OP_T (transpose) or
 * FTM_OP_C (conjugate transpose; the same as T for real types): x_b has m
 * entries and y_b n.  type selects float, double, complex float or complex
 * double (complex numbers interleaved re, im); alpha and beta point to one
 * host value of that type.  y_b is not read when beta is zero.  Tuned for
 * short-wide matrices (m <= n), where op = T / C tiles the columns of every
 * matrix across workgroups.  Pointers A, x, y are device memory that the
 * caller owns; the batch's y_b must not overlap A or x.  Enqueued on stream
 * (a hipStream_t, NULL = default stream); nothing is allocated.
 * FTM_ERR_INVALID: bad type or op, NULL pointers, m, n or batch < 1 (with
 * m, n, batch = 0 the call does nothing and returns FTM_OK), lda < m, m or
 * n >= 2^31, strides too small for the matrices/vectors they separate
 * (negative strides included), or more than 2^31 workgroups. */
typedef enum ftm_gemv_type { FTM_TYPE_S = 0, FTM_TYPE_D = 1, FTM_TYPE_C = 2, FTM_TYPE_Z = 3 } ftm_gemv_type;
typedef enum ftm_gemv_op { FTM_OP_N = 0, FTM_OP_T = 1, FTM_OP_C = 2 } ftm_gemv_op;
ftm_status ftm_sbgemv(int32_t type, int32_t op, int64_t m, int64_t n, const void* alpha, const void* A, int64_t lda,
                      int64_t stride_a, const void* x, int64_t stride_x, const void* beta, void* y, int64_t stride_y,
                      int64_t batch, void* stream);

const char* ftm_status_string(ftm_status s);
const char* ftm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FTM_H */
