/*
 * cdm.h -- C ABI of the MI355X (gfx950) coordinate-descent MU-MIMO library.
 *
 * The library runs the coordinate-descent (CD) detector of Algorithm 1 and the CD
 * precoder of Algorithm 2 of K. Li, O. Castaneda, C. Jeon, J. R. Cavallaro and
 * C. Studer, "Decentralized Coordinate-Descent Data Detection and Precoding for
 * Massive MU-MIMO" (arXiv 1902.08653), entirely in hand-written HIP kernels.
 *
 * General rules
 *   - Every entry point returns a cdm_status (0 = CDM_OK, negative = error) and
 *     never throws, aborts or exits.
 *   - Pointers named "device" are HIP device pointers the caller owns; the library
 *     never frees them.  Pointers named "host" are ordinary host memory.
 *   - Complex values are interleaved (re, im): CDM_C128 = two doubles (16 B),
 *     CDM_C64 = two floats (8 B).
 *   - The channel H is always passed in the uplink orientation of Sec. II-A:
 *     B x U (B antennas = rows, U users = columns), column-major with leading
 *     dimension ldh >= B, so user column h_u is contiguous.  The downlink channel
 *     of Sec. II-B is its conjugate transpose (reciprocity), so the same storage
 *     serves Algorithm 2.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Solves are
 *     asynchronous: they enqueue work and return; results and the cdm_info records
 *     are valid once the stream has been synchronised.  A plan owns its device
 *     workspace; concurrent solves on one plan race -- use one plan per stream.
 *   - Data-dependent conditions (a zero column, NaN/Inf, no convergence within
 *     T_max) are reported as bits in cdm_info.flags, not as errors.
 */
#ifndef CDM_H
#define CDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDM_ABI_VERSION 2

typedef enum cdm_status {
    CDM_OK = 0,
    CDM_EINVAL = -1,        /* NULL pointer or out-of-range scalar argument */
    CDM_ESHAPE = -2,        /* inconsistent sizes (B, U, C, ldh, nnz, batch) */
    CDM_EDTYPE = -3,        /* precision / problem / layout combination not supported */
    CDM_ENOMEM = -4,        /* device workspace allocation failed */
    CDM_EHIP = -5,          /* a HIP runtime call failed (message via cdm_last_error) */
    CDM_EINFEASIBLE = -6,   /* lambda = 0 with B_c < U (eq. (1) not strictly convex), or
                               a downlink cluster with B_c < U (eq. (2) infeasible) */
    CDM_ENOTIMPL = -7,      /* valid request that this build does not implement */
    CDM_ENODEV = -8         /* no gfx950 device is current */
} cdm_status;

/* Problem: Algorithm 1 (uplink L-MMSE detection, eq. (1)) or Algorithm 2 (downlink
 * ZF precoding, eq. (2)-(4)). */
typedef enum cdm_problem { CDM_UPLINK_LMMSE = 0, CDM_DOWNLINK_ZF = 1 } cdm_problem;

/* Arithmetic of the sweep.  CDM_MIXED_* keep H, y and x in FP64 (C128 storage)
 * and run the inner operator products from a low-precision copy of H (BF16,
 * FP8-e4m3, or the complex64 rounding) with an FP64 residual refinement outside
 * (see cdm_solve and cdm_solve_batched).  CDM_MIXED_C64 is for batched plans only. */
typedef enum cdm_precision {
    CDM_C128 = 0, CDM_C64 = 1, CDM_MIXED_BF16 = 2, CDM_MIXED_FP8 = 3, CDM_MIXED_C64 = 4,
    CDM_C16 = 5   /* complex FP16 (two halves, 4 B): cdm_detect_batch and cdm_precode_batch only */
} cdm_precision;

typedef enum cdm_layout { CDM_DENSE = 0, CDM_CSR = 1 } cdm_layout;

/* Engine selection: AUTO lets the plan choose from the shape: PANEL for a single instance
 * (C = 1) with B >= 256 and either U >= 128 or B * U >= 2^18, WG otherwise (several
 * clusters, narrow or small instances, the downlink).
 * WG    - one workgroup per instance (cluster), residual held in registers.
 * PANEL - one cooperative launch over all CUs for one single instance; columns are
 *         processed in panels of `panel` users whose coupling is resolved exactly
 *         (block form of the cyclic sweep, identical to U sequential updates). */
typedef enum cdm_engine { CDM_ENGINE_AUTO = 0, CDM_ENGINE_WG = 1, CDM_ENGINE_PANEL = 2 } cdm_engine;

/* Option bits for cdm_desc.flags. */
#define CDM_F_RESIDUAL 1    /* also compute the FP64 normal-equation residual into cdm_info.resid
                               (single solves: after the sweeps; batched: per instance, in the
                               same persistent launch) */
#define CDM_F_TIMING   2    /* record HIP events around each kernel stage of a solve (cdm_plan_timings) */
#define CDM_F_AUTOTUNE 4    /* cdm_create_batched: time the candidate workgroup shapes on a sample of the
                               batch's own shapes (synthetic values) and keep the fastest */
#define CDM_F_NO_LOOKAHEAD 8 /* panel engine: use the two-hop schedule (partials -> reducers -> all,
                               per panel) instead of the look-ahead schedule, whose exchange of panel
                               K+1's partials overlaps the wait for panel K's update (same deltas in
                               exact arithmetic; kept for comparison) */
#define CDM_F_DEEP_LOOKAHEAD 16 /* panel engine, complex128 with 64-column panels and at least three
                               panels: look two panels ahead (partials of panel K+3 formed after
                               panel K's update, with a distance-two correction at the reducers)
                               instead of one (panel K+2); same deltas in exact arithmetic.  Slower
                               than the default on the devices measured (each tile is read twice
                               per sweep, and the exchange loads wait behind that stream) */

typedef struct cdm_desc {
    int32_t problem;     /* cdm_problem */
    int32_t precision;   /* cdm_precision */
    int32_t layout;      /* cdm_layout */
    int32_t engine;      /* cdm_engine */
    int32_t B;           /* antennas = rows of H (sum of the cluster sizes), >= 1 */
    int32_t U;           /* users = columns of H, >= 1 */
    int32_t C;           /* antenna clusters (Sec. II-A), 1 <= C <= B; cluster c owns the
                            c-th block of consecutive rows: B/C rows each (then B % C == 0),
                            or Bc[c] rows if Bc is given */
    int32_t T_max;       /* sweep cap T_max of Algorithms 1 and 2, 1..100000 */
    double tol;          /* 0: run exactly T_max sweeps (the paper's mode); > 0: stop after
                            sweep t once sqrt(sum_u |delta_u|^2) <= tol * ||x^(t)||_2 */
    int64_t nnz;         /* CDM_CSR: number of stored entries of H (exactly rowptr[B]), else 0 */
    int32_t panel;       /* CDM_ENGINE_PANEL panel width (64 or 128); 0 = choose */
    int32_t flags;       /* CDM_F_* */
    const int32_t* Bc;   /* host, optional: C cluster sizes B_c >= 1 summing to B (uneven
                            clusters, Sec. II-A); NULL = C equal blocks.  Read by cdm_create
                            only (the plan keeps a copy).  Batched plans: must be NULL. */
} cdm_desc;

/* Per-instance (per-cluster) result record written to device memory by a solve.
 * flags bits: */
#define CDM_INFO_ZERO_COLUMN   1   /* ||h_u||^2 + lambda == 0 for some u: coordinate kept inactive */
#define CDM_INFO_NONFINITE     2   /* the returned x holds NaN or Inf */
#define CDM_INFO_NOT_CONVERGED 4   /* tol > 0 and T_max sweeps ran without meeting it */
#define CDM_INFO_TIMEOUT       8   /* a cross-workgroup wait gave up (should never happen) */
#define CDM_INFO_BAD_INPUT    16   /* CDM_CSR: rowptr/colidx malformed (rowptr[0] != 0, rowptr
                                      decreasing, rowptr[B] != nnz, a column index outside
                                      [0, U), or column indices not strictly increasing in a
                                      row); no entry was read through them: the solve ran
                                      Algorithm 1 on H = 0 (all columns empty) */
typedef struct cdm_info {
    int32_t sweeps;      /* sweeps performed */
    int32_t flags;       /* CDM_INFO_* */
    double rel_step;     /* sqrt(sum_u |delta_u|^2) / ||x||_2 of the last sweep */
    double resid;        /* ||H^H(y - Hx) - lambda x|| / ||H^H y|| in FP64 if CDM_F_RESIDUAL, else -1 */
    double reserved;     /* mixed precisions: inner low-precision sweeps performed; else 0 */
} cdm_info;              /* 32 bytes */

typedef struct cdm_plan cdm_plan;

/* ABI version of the loaded library (CDM_ABI_VERSION). */
int32_t cdm_version(void);

/* Static text for a status code. */
const char* cdm_status_string(int32_t status);

/* Text of the last HIP error seen by this thread (empty if none). */
const char* cdm_last_error(void);

/* Create a plan for single solves of the shape in *desc on the current device.
 * Validates the descriptor, picks the engine and tiles, and allocates the whole
 * device workspace, so that cdm_solve itself never allocates.
 * CDM_CSR plans (uplink, C = 1, CDM_C128 or CDM_C64): the sweep cuts the rows into
 * slices of about 1024 (at most 64 slices, one workgroup each, at most 4096 rows per
 * slice), so B <= 262144; the workspace holds the column-compressed copy and about
 * 4 B per stored entry more.
 * Errors: CDM_EINVAL, CDM_ESHAPE, CDM_EDTYPE, CDM_EINFEASIBLE (downlink with
 * B/C < U), CDM_ENOMEM, CDM_ENODEV.  *plan is set to NULL on error. */
int32_t cdm_create(const cdm_desc* desc, cdm_plan** plan);

/* Solve one instance (Algorithm 1 or 2, Sec. III / Sec. IV).
 *  H      device, CDM_DENSE: B x U column-major, leading dimension ldh >= B;
 *         CDM_CSR: the nnz stored values in CSR order (rows = antennas)
 *  ldh    CDM_DENSE: leading dimension in elements; CDM_CSR: ignored
 *  rowptr device int32[B+1] (CDM_CSR only, else NULL)
 *  colidx device int32[nnz], column indices strictly increasing within each row
 *         (CDM_CSR only, else NULL)
 *  rhs    device, uplink: y (B complex); downlink: s (U complex)
 *  N0, Ex uplink: lambda = N0/Ex >= 0 regularises eq. (1) (Algorithm 1 input);
 *         lambda == 0 requires B/C >= U
 *  rho    downlink: total power constraint rho (each cluster scales to
 *         rho/sqrt(C), Sec. IV-B); rho <= 0 skips the scaling
 *  x0     device, optional warm start (U complex, uplink only), NULL = x^(0) = 0
 *  lambda_c device, optional: C fusion weights (double) of Algorithm 1's output,
 *         x_hat = sum_c lambda_c x_c, used as given (uplink with C > 1 only; a weight
 *         of 0 drops cluster c, e.g. one whose data did not arrive).  NULL = the
 *         weights of Sec. III, lambda_c = sigma_c^-2 / sum_c' sigma_c'^-2 with
 *         sigma_c^2 = (N0/U) sum_u m_{u,c}; the common factor N0/U cancels, so they
 *         are s_c^-1 / sum_c' s_c'^-1 (s_c = sum_u m_{u,c}), defined for N0 = 0 too;
 *         a cluster without an active coordinate (s_c = 0) gets weight 0
 *  x      device output; uplink: the fused estimate x_hat (U complex);
 *         downlink: the stacked precoded vector [x_1; ...; x_C] (B complex)
 *  info   device cdm_info[C] (one record per cluster)
 *  stream hipStream_t
 * Mixed precisions run the outer FP64 refinement loop: residual r = y - H x in
 * FP64, inner CD sweeps on the correction problem from the low-precision copy of
 * H, x += d, until ||d|| <= tol ||x|| (tol > 0 required) or T_max outer steps.
 * Each outer step runs CDM_MIXED_INNER_SWEEPS_BF16 (BF16 copy) or
 * CDM_MIXED_INNER_SWEEPS_FP8 (FP8 copy) inner sweeps; the solve enqueues all T_max
 * outer steps, and those after convergence return at once, so keep T_max near the
 * expected count (a cap of S sweeps over the copy is T_max = ceil(S / inner sweeps)).
 * Errors: CDM_EINVAL (NULL pointer, lambda < 0, lambda_c given for a downlink or
 * C = 1 plan), CDM_ESHAPE (ldh < B), CDM_EINFEASIBLE (lambda = 0 and some B_c < U),
 * CDM_EHIP. */
/* Inner sweeps per outer refinement step of a single mixed-precision solve: set where
 * one more inner sweep stops paying for itself against one more outer step (two FP64
 * passes over H); the FP8 copy's rounding bounds the gain of an outer step sooner. */
#define CDM_MIXED_INNER_SWEEPS_BF16 12
#define CDM_MIXED_INNER_SWEEPS_FP8 5

int32_t cdm_solve(cdm_plan* plan, const void* H, int64_t ldh, const int32_t* rowptr,
                  const int32_t* colidx, const void* rhs, double N0, double Ex, double rho,
                  const void* x0, const double* lambda_c, void* x, void* info, void* stream);

/* Create a plan for a batch of independent uplink instances of uneven size
 * (Algorithm 1 with C = 1 per instance).  m, n: host int32[batch], rows (antennas)
 * and columns (users) of each instance, 1 <= n, 1 <= m <= 8192 (2048 for the mixed
 * precisions); the largest n must fit the per-instance LDS state (32 n B for
 * complex128, 16 n B for complex64, 40 n B mixed, at most about 150 KB).  Packing rule for
 * the solve: instance i's H is m_i x n_i column-major with ld = m_i starting at
 * element offset H_off[i] = sum_{k<i} m_k n_k of the packed H buffer; y_i starts at
 * y_off[i] = sum_{k<i} m_k and x_i at x_off[i] = sum_{k<i} n_k.  The plan fixes the
 * launch schedule (largest instances first) and the tiles per size bucket.
 * desc->precision: CDM_C128 or CDM_C64 (plain sweeps; T_max, tol as in cdm_desc), or
 * CDM_MIXED_C64 / CDM_MIXED_BF16: mixed-precision refinement per instance, with H, y
 * and x in complex128 (m <= 2048).  Outer step: r = y - H x and g = H^H r - lambda x
 * in FP64 (two streaming launches over the batch), then inner CD sweeps (Algorithm
 * 1's rule with bias g) on the correction d from the complex64 or BF16 copy of H in
 * FP32 (one persistent launch), then x += d.  The copy is written by the first
 * gradient pass (plan workspace: 8 or 4 B per element of the batch).  An instance is
 * done after the first inner sweep with ||d|| <= tol ||x + d|| (tol > 0 required); a
 * step's inner loop stops once its own sweep step is <= tau ||d|| (tau = 1e-5 for the
 * complex64 copy, 3e-2 for BF16) or after 64 sweeps.  The solve enqueues T_max outer
 * steps (keep it small, e.g. 8); finished instances skip the remaining ones.
 * cdm_info.sweeps then counts outer steps and cdm_info.reserved the inner sweeps.
 * Errors: CDM_EINVAL (tol <= 0 for a mixed precision), CDM_ESHAPE, CDM_ENOTIMPL
 * (CDM_MIXED_FP8, downlink, CSR), CDM_ENOMEM, CDM_ENODEV. */
int32_t cdm_create_batched(const cdm_desc* desc, int32_t batch, const int32_t* m,
                           const int32_t* n, cdm_plan** plan);

/* The packing offsets of a batched plan (host int64[batch] each; any may be NULL). */
int32_t cdm_batched_offsets(const cdm_plan* plan, int64_t* H_off, int64_t* y_off,
                            int64_t* x_off);

/* Solve every instance of a batched plan in one persistent launch.
 *  H, y   device, packed as described at cdm_create_batched
 *  x0     device optional packed warm starts (NULL = zero)
 *  x      device packed outputs; info device cdm_info[batch].
 * Enqueues kernels only (no allocation, no host synchronisation), so it may be
 * captured into a HIP graph. */
int32_t cdm_solve_batched(cdm_plan* plan, const void* H, const void* y, double N0, double Ex,
                          const void* x0, void* x, void* info, void* stream);

/* Sparse plans (CDM_CSR): the column-compressed form the solve walks, so that it
 * can be checked.  Transposes the CSR input (val, rowptr, colidx as in cdm_solve)
 * and copies the result to the caller's device buffers (any may be NULL):
 * colptr_out int32[U+1], rowidx_out int32[nnz], cval_out complex[nnz].  Within a
 * column, entries are ordered by increasing row (the form is unique).  Unlike the
 * solve, this call synchronises `stream` to report malformed CSR arrays (the
 * conditions of CDM_INFO_BAD_INPUT) as CDM_EINVAL; the outputs then hold the empty form.
 * Errors: CDM_EINVAL (not a CSR plan, NULL input, malformed rowptr/colidx), CDM_EHIP. */
int32_t cdm_csr_transpose(cdm_plan* plan, const void* val, const int32_t* rowptr, const int32_t* colidx,
                          int32_t* colptr_out, int32_t* rowidx_out, void* cval_out, void* stream);

/* Mixed-precision plans: the low-precision copy of H the inner sweeps read, so that it
 * can be checked.  Quantises H (complex128, ld >= B, device) and copies the planar
 * codes to re_out / im_out (device; B*U uint16 for CDM_MIXED_BF16, B*U uint8 for
 * CDM_MIXED_FP8, column-major with ld = B) and, for FP8, the ceil(U/128) block
 * scales to scale_out (device float).  Any output may be NULL.
 * Definitions: BF16 = nearest-even rounding to FP32, then nearest-even to the top
 * 16 bits; FP8 = OCP E4M3 of fl32(h / s_b), nearest with ties to the even code,
 * saturating at 448, with s_b = fl32(amax_b / 448) over the block's Re and Im parts
 * (1 for an all-zero block).
 * Errors: CDM_EINVAL (not a mixed plan, NULL H), CDM_ESHAPE, CDM_EHIP. */
int32_t cdm_quantized_copy(cdm_plan* plan, const void* H, int64_t ldh, void* re_out, void* im_out,
                           float* scale_out, void* stream);

/* FP64 stationarity check of eq. (1) for a dense uplink plan:
 * *out (device double) = ||H^H (y - H x) - lambda x|| / ||H^H y||, lambda = N0/Ex.
 * Uses the plan's workspace; same argument conventions as cdm_solve. */
int32_t cdm_residual(cdm_plan* plan, const void* H, int64_t ldh, const void* y, double N0,
                     double Ex, const void* x, double* out, void* stream);

/* Decentralized detection of a batch of small clustered problems: the shape of the
 * paper's throughput measurements (Sec. VI, Table I; Algorithm 1 with the fusion of
 * Sec. III).  S subcarriers; subcarrier s has the channel H_s (B x U, B = C * Bc, rows
 * = antennas in C clusters of Bc consecutive rows) shared by V received vectors
 * y_{s,v} (B each).  For every (s, v) each cluster c runs exactly T_max sweeps of
 * Algorithm 1 from x = 0 on its rows, and the estimates are fused:
 *   x_hat = sum_c lambda_c x_c,  lambda_c = sigma_c^-2 / sum_c' sigma_c'^-2,
 *   sigma_c^2 = (N0 / U) sum_u m_{u,c},  m_{u,c} = 1 / (||h_{u,c}||^2 + N0 / Ex).
 *  H  device, S blocks of B x U column-major (ld = B), block s at element s*B*U
 *  Y  device, S*V vectors of B, vector (s, v) at element (s*V + v)*B
 *  X  device output, S*V vectors of U, vector (s, v) at element (s*V + v)*U
 * Elements are complex in `precision`: CDM_C64 (FP32 arithmetic) or CDM_C16 (FP16
 * storage; residual updates and dot products in packed FP16, scalar rule in FP32).
 * The factor N0/U is common to every cluster and cancels from lambda_c, so the weights
 * are s_c^-1 / sum_c' s_c'^-1 with s_c = sum_u m_{u,c} (a cluster with s_c = 0 gets 0).
 * Limits: C in {1, 2, 4, 8}, 1 <= Bc <= 32, 1 <= U <= 16; N0 = 0 needs Bc >= U.
 * Enqueues one kernel; allocates nothing.  Errors: CDM_EINVAL (NULL pointer, N0 < 0,
 * Ex <= 0, T_max < 1), CDM_EDTYPE, CDM_ESHAPE, CDM_EINFEASIBLE (N0 = 0 with Bc < U),
 * CDM_EHIP. */
int32_t cdm_detect_batch(int32_t S, int32_t V, int32_t C, int32_t Bc, int32_t U, int32_t T_max,
                         int32_t precision, const void* H, const void* Y, double N0, double Ex,
                         void* X, void* stream);

/* Decentralized ZF precoding of the same batch shape (Algorithm 2, Sec. IV; the
 * downlink half of Table I).  For every (s, v) the symbols s_{s,v} (U) are broadcast
 * to the C clusters; cluster c runs exactly T_max sweeps of eq. (4) from x_c = 0 on
 * its rows of H_s (p_u = 1/||h_{u,c}||, a zero column stays inactive), then scales
 * x_c to norm rho_c = rho / sqrt(C) (rho <= 0: no scaling; x_c = 0 stays 0).
 *  H    device, as in cdm_detect_batch (uplink orientation; the downlink channel of
 *       cluster c is its block's conjugate transpose)
 *  Sym  device, S*V symbol vectors of U, vector (s, v) at element (s*V + v)*U
 *  X    device output, S*V stacked vectors [x_1; ...; x_C] of B, at element (s*V + v)*B
 * Precisions and limits as cdm_detect_batch; Bc >= U.  Enqueues one kernel; allocates
 * nothing.  Errors: CDM_EINVAL (NULL pointer, non-finite rho, T_max < 1), CDM_EDTYPE,
 * CDM_ESHAPE, CDM_EINFEASIBLE (Bc < U), CDM_EHIP. */
int32_t cdm_precode_batch(int32_t S, int32_t V, int32_t C, int32_t Bc, int32_t U, int32_t T_max,
                          int32_t precision, const void* H, const void* Sym, double rho, void* X,
                          void* stream);

/* Per-coordinate features of a batched plan's packed instances, for the
 * learned warm start (one row of 8 floats per user u of instance i, rows in the
 * packed x order): [Re z, Im z, |z|, ||h_u||^2, lambda, m_i/2048, n_i/m_i, 1] with
 * z = h_u^H y_i / (||h_u||^2 + lambda), the regularised matched filter of the
 * instance, accumulated in FP64.  F: device float[sum_i n_i][8].  Errors: CDM_EINVAL. */
int32_t cdm_batched_features(cdm_plan* plan, const void* H, const void* y, double N0, double Ex, float* F,
                             void* stream);

/* ---- warm-start network -------------------------------------------------------
 * A per-coordinate MLP nin -> h1 -> h2 -> nout with ReLU after the first two layers,
 * trained by the library's own kernels: BF16 operands on MFMA with FP32
 * accumulation, FP32 master weights, mean-squared-error loss, Adam.  Its output for
 * a feature row is a warm start (Re, Im) for the coordinate (cdm_solve_batched x0).
 * Parameters are one flat FP32 array: W1 (nin x h1, row-major), b1 (h1), W2, b2, W3, b3.
 * All row matrices are row-major; X: rows x nin, T and Y: rows x nout (device FP32).
 * Calls on one network are ordered by their stream and share its activation buffers.
 * Errors: CDM_EINVAL (NULL handle or operand, rows outside 1..max_rows, count not
 * the parameter count), CDM_ESHAPE (a width < 1), CDM_ENOMEM, CDM_EHIP. */
typedef struct cdm_mlp cdm_mlp;
int32_t cdm_mlp_create(int32_t nin, int32_t h1, int32_t h2, int32_t nout, int32_t max_rows, cdm_mlp** out);
int64_t cdm_mlp_param_count(const cdm_mlp* mlp);
/* host float[count] in / out; set also resets the Adam state */
int32_t cdm_mlp_set_weights(cdm_mlp* mlp, const float* params, int64_t count);
int32_t cdm_mlp_get_weights(const cdm_mlp* mlp, float* params, int64_t count);
/* Y (device, may be NULL) = network(X) */
int32_t cdm_mlp_forward(cdm_mlp* mlp, const float* X, int32_t rows, float* Y, void* stream);
/* gradients of mean((Y - T)^2) into grads (device float[count], may be NULL) and the
 * per-256-element partial sums of (Y - T)^2 into loss_parts (device, may be NULL) */
int32_t cdm_mlp_gradients(cdm_mlp* mlp, const float* X, const float* T, int32_t rows, float* grads,
                          float* loss_parts, void* stream);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a mini-batch */
int32_t cdm_mlp_train_step(cdm_mlp* mlp, const float* X, const float* T, int32_t rows, float lr, void* stream);
/* Warm start from feature rows: x0[k] = Y[k][0] + i Y[k][1] for k < rows (any count;
 * evaluated in chunks of max_rows), written as interleaved complex in `precision`
 * (CDM_C128 or CDM_C64) into device x0.  Needs nout == 2.  Errors: CDM_EINVAL. */
int32_t cdm_mlp_predict(cdm_mlp* mlp, const float* X, int64_t rows, void* x0, int32_t precision, void* stream);
int32_t cdm_mlp_destroy(cdm_mlp* mlp);

/* Human-readable description of the plan's engine, tiles and workspace
 * (NUL-terminated, truncated to len bytes). */
int32_t cdm_plan_describe(const cdm_plan* plan, char* buf, int32_t len);

/* Stage durations of the most recent solve of a plan created with CDM_F_TIMING, in
 * milliseconds, measured with HIP events on the solve's stream (call after the
 * stream has been synchronised).  out_ms: host double[n]; stages, in order:
 *   [0] preprocessing (column energies; panel Gram blocks and their inverses),
 *   [1] init (r = y or y - H x0),
 *   [2] the sweep kernel (all CD sweeps),
 *   [3] finalisation and the optional FP64 residual.
 * Returns the number of stages written (<= n) through *count.
 * Errors: CDM_EINVAL (no timing flag, NULL), CDM_EHIP. */
int32_t cdm_plan_timings(const cdm_plan* plan, double* out_ms, int32_t n, int32_t* count);

/* Measurement utility (not part of the method): a plain coalesced device-to-device
 * copy of `bytes` bytes (a multiple of 16) with the library's own kernel, used to
 * calibrate HBM byte counters against a known traffic volume.
 * src, dst: device, 16-byte aligned, non-overlapping. */
int32_t cdm_stream_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* Measurement utility (not part of the method): a read-only stream over `bytes` bytes (a
 * multiple of 16) with the library's own kernel, the achievable HBM read rate that the
 * read-dominated sweep kernels are compared with.  Every 16-byte word of src is read
 * once; out receives CDM_STREAM_READ_SLOTS partial XORs of 16 bytes each (every slot is
 * written), whose XOR is the XOR of all words of src.
 * src: device, 16-byte aligned.  out: device, CDM_STREAM_READ_SLOTS * 16 bytes,
 * caller-owned.  Errors: CDM_EINVAL (NULL, bytes < 0 or not a multiple of 16), CDM_EHIP. */
#define CDM_STREAM_READ_SLOTS 8192
int32_t cdm_stream_read(const void* src, int64_t bytes, void* out, void* stream);

/* ---- solve without allocation -------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The same solve as cdm_create +
 * cdm_solve + cdm_destroy for the per-cluster engine (one workgroup per cluster; the
 * same kernels, so the same bits), with no plan: every buffer beyond the caller's
 * inputs and outputs lives in one static device array of CDM_NOALLOC_SCRATCH_BYTES per
 * device, held from the first call on that device until the process ends.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine) and does not
 * synchronise.  All calls on one device share its array and its contents persist
 * between calls: calls whose executions overlap on one device (different streams,
 * threads, or an unsynchronised graph replay next to a direct call) race and give
 * wrong results; order them on one stream.
 * Arguments as cdm_create (desc, read by this call only) and cdm_solve (no rowptr /
 * colidx).  Limits: dense layout, CDM_C128 or CDM_C64, engine AUTO or WG, every cluster
 * within the per-cluster engine's rows (4096 complex128, 8192 complex64 per cluster),
 * C <= CDM_NOALLOC_MAX_CLUSTERS, and for an uplink with C > 1 the C x U local estimates
 * within the array (16 or 8 B each, CDM_NOALLOC_SCRATCH_BYTES - 8 KiB in all).
 * Errors: as cdm_create and cdm_solve; CDM_ESHAPE (message via cdm_last_error) for
 * sizes beyond the limits, CDM_EDTYPE for other layouts or precisions, CDM_ENOTIMPL for
 * the panel engine. */
#define CDM_NOALLOC_SCRATCH_BYTES (4u << 20)
#define CDM_NOALLOC_MAX_CLUSTERS 64
int32_t cdm_solve_noalloc(const cdm_desc* desc, const void* H, int64_t ldh, const void* rhs, double N0,
                          double Ex, double rho, const void* x0, const double* lambda_c, void* x, void* info,
                          void* stream);

/* Release the plan and its device workspace. NULL is accepted. */
int32_t cdm_destroy(cdm_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* CDM_H */
