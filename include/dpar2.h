/*
 * libdpar2 -- DPar2 (fast PARAFAC2 of irregular dense tensors) on one AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Jang & Kang, "DPar2: Fast and Scalable PARAFAC2 Decomposition for
 * Irregular Dense Tensors" (arXiv 2203.12798).
 *   - dpar2_compress   : the two-stage randomized-SVD compression of Sec. III-B
 *                        (Alg. 1 applied to every slice, Eq. 4; M = ||_k C_k B_k;
 *                        Alg. 1 applied to M, Eq. 5; F^(k) blocks, Eqs. 6-7).
 *   - dpar2_als_step   : the repeat loop of Alg. 3 (Eq. 8 Q-step, implicit Y_k of
 *                        Sec. III-D, Lemmas 1-3 for G^(1), G^(2), G^(3),
 *                        pseudoinverse updates of H, V, W, S_k = diag(W(k,:)),
 *                        the compressed error of Sec. III-E and its stop rule).
 *   - dpar2_fitness    : fitness of Sec. IV-A against the original slices, from
 *                        the compressed factors (no second pass over the slab).
 *   - dpar2_output_U   : U_k = A_k Z_k P_k^T H (last lines of Alg. 3).
 *   - dpar2_output_A   : the first-stage factors A_k of Eq. 4.
 *   - dpar2_decompose  : all of the above, Alg. 3 end to end.
 *   - dpar2_append     : the same after slices were appended to a decomposed
 *                        tensor (first stage of the new slices only).
 *
 * Conventions (all calls):
 *   - Pointers are DEVICE pointers unless marked (host).  The caller owns every
 *     buffer; the library never allocates or frees device memory.  All
 *     intermediate data lives in one caller-provided workspace whose size comes
 *     from dpar2_workspace_bytes(); compress, als_step, fitness, output_U and
 *     output_A of one decomposition must be given the same workspace.
 *   - Host-side state: per workspace the library keeps a small ring of pinned
 *     staging buffers for the schedule upload and the HIP graphs of captured
 *     iterations; dpar2_release(ws) frees them (dpar2_release_all for every
 *     workspace), after which the workspace may be freed or reused.
 *   - Work is enqueued on the caller's stream `stream` and is asynchronous;
 *     results are valid after the stream is synchronised.  Calls on different
 *     streams need different workspaces.  The only host<->device copies the
 *     library makes are the small schedule upload in dpar2_compress and the
 *     report read in dpar2_report_read.
 *   - Matrices are row-major.  Factor matrices are float64: H (R x R),
 *     V (J x R), W (K x R); S_k = diag(W(k,:)).
 *   - Irregular tensor {X_k}: slab of N = sum_k I_k rows, each of J values
 *     (float32, bfloat16 or fp8 e4m3, see dpar2_dtype), row-major; slice k is
 *     rows row_offsets[k] .. row_offsets[k+1]-1.
 *   - Errors: every call returns a dpar2_status.  Shape and argument errors are
 *     detected on the host before anything is enqueued.  HIP errors map to
 *     DPAR2_EHIP with the HIP message available from dpar2_last_error()
 *     (thread-local).  No call aborts or throws across the ABI.
 */
#ifndef LIBDPAR2_DPAR2_H
#define LIBDPAR2_DPAR2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* dpar2_stream_t;   /* = hipStream_t; NULL = default stream */

typedef enum {
  DPAR2_OK = 0,
  DPAR2_EINVAL = -1,     /* NULL pointer, bad option value, malformed row_offsets   */
  DPAR2_ESHAPE = -2,     /* rank / sketch width incompatible with K, J or some I_k  */
  DPAR2_ENUMERIC = -3,   /* the slab holds NaN or Inf (some ||X_k||^2 is not finite):
                            reported by dpar2_report_read / dpar2_decompose (rep) */
  DPAR2_ENOCONV = -4,    /* dpar2_decompose with a report and tol >= 0: the stop
                            rule did not fire within max_iter (results are valid) */
  DPAR2_EHIP = -5,       /* a HIP runtime call failed (see dpar2_last_error)        */
  DPAR2_EWORKSPACE = -6  /* workspace NULL, misaligned (256 B) or too small         */
} dpar2_status;

typedef enum {
  DPAR2_F32 = 0,         /* slab of float32 values                                  */
  DPAR2_BF16 = 1,        /* slab of bfloat16 bit patterns (uint16)                   */
  DPAR2_FP8_E4M3 = 2     /* slab of OCP fp8 e4m3fn bytes; value = decode(byte) *
                            slice_scale[k] in float32 (powers of two keep it exact)  */
  /* every dtype: J <= 16384; the whole-row slab pass covers J <= 256 (float32)
     or J <= 128 (bf16, fp8) at L <= 32, the 128-column-chunk pass the rest */
} dpar2_dtype;

/* Warning bits reported in dpar2_report.warn_bits (device-side, never fatal). */
/* dpar2_opts.flags: the iterations of dpar2_als_step / dpar2_decompose /
 * dpar2_decompose_batch (begin, n_steps iterations, end) are captured once
 * per workspace and step count into a HIP graph and replayed on later calls
 * (kernel arguments point into the workspace only, so a replay reads the
 * current factors, tolerances and trace through the descriptors).  This
 * flag launches them one by one instead.  Results are identical. */
#define DPAR2_FLAG_NO_GRAPH     0x1u
/* dpar2_opts.flags: the first stage's slab pass (Sec. III-B, Eq. 4) in
 * 128-column chunks (a sketch kernel that writes Y, then a projection kernel
 * per chunk) for any J <= 16384, not only above the whole-row limit (J > 256
 * for float32, > 128 for bf16 / fp8) or above L = 32.  Reads the slab twice
 * and needs about 1.6 (L <= 16), 3.1 (L <= 32) or 6.1 (L > 32) KiB per 64
 * rows of workspace for the digit planes of Y (dpar2_workspace_bytes accounts
 * for it).  Results agree with the whole-row pass to rounding;
 * dpar2_autotune_slab chooses between the two. */
#define DPAR2_FLAG_WIDE_SLAB    0x2u

/* dpar2_opts.flags: resumable bit for bit.  Every iteration ends in the state
 * a new dpar2_als_step call starts from (V written back as a J x R array and
 * W^T W, V^T V, E D^T V recomputed from the factors as at the start of a
 * call), so that n1 iterations followed by n2 more on the same workspace give
 * the same bits as n1 + n2 in one call.  Costs four more launches per
 * iteration.  Without the flag the two differ by rounding only. */
#define DPAR2_FLAG_DETERMINISTIC 0x4u

#define DPAR2_WARN_JACOBI_CAP   0x1u  /* a Jacobi eigen/SVD solve hit its sweep cap   */
#define DPAR2_WARN_RANK_DEFICIENT 0x2u /* a T_k had a (near) zero singular value      */
#define DPAR2_WARN_NONFINITE    0x4u  /* the slab holds NaN or Inf: the tensor's
                                         iteration is skipped (status ENUMERIC)      */

/* Irregular dense tensor {X_k}, k = 0..K-1, X_k in R^{I_k x J} (Sec. II-A). */
typedef struct {
  int64_t K;                        /* number of slices, >= 1                           */
  int64_t J;                        /* number of columns, >= 1                          */
  const int64_t* row_offsets;       /* device, K+1 entries: [0] = 0, non-decreasing      */
  const int64_t* row_offsets_host;  /* (host) the same K+1 values (validation, schedule) */
  const void* slab;                 /* device, N x J row-major, N = row_offsets[K]       */
  int32_t dtype;                    /* dpar2_dtype                                       */
  const float* slice_scale;         /* device, K per-slice scales (DPAR2_FP8_E4M3 only,
                                       else ignored)                                     */
} dpar2_tensor;

/* Parameters of Alg. 1 / Alg. 3. */
typedef struct {
  int32_t rank;        /* R: target rank of both stages and of PARAFAC2: 1..32, 40
                          or 50 (the rank sweep of Sec. IV-C goes to 50); the
                          warm start takes R <= 32                              */
  int32_t sketch;      /* L = R + s: columns of Omega_1 (first stage), R <= L, L in
                          1..32 or one of 40, 50, 60 (above 32 the slab pass is
                          always the 128-column-chunk pass), L <= J and L <=
                          every I_k                                                 */
  int32_t sketch2;     /* L2: columns of Omega_2 (second stage), R <= L2, L2 in
                          1..32 or one of 40, 50, 60, L2 <= J and L2 <= K R          */
  int32_t max_iter;    /* iterations of the repeat loop of Alg. 3, >= 0             */
  double tol;          /* stop when e_{t-1} - e_t < tol * e_{t-1}; tol < 0: never   */
  uint32_t flags;      /* DPAR2_FLAG_* bits, others must be 0                        */
  int32_t power_iters; /* q of Alg. 1 for the first stage, 0..4; each step is one more
                          pass over the slab with a per-slice sketch matrix (the
                          orthonormal right singular vectors of the previous B_k,
                          which spans X_k^T Q_k: the stabilised power iteration)   */
  int32_t item_rows;   /* rows per work item of the slab pass (the unit that Alg. 4's
                          longest-first scheduling hands to compute units): longer
                          slices are cut into near-equal pieces; 0 = 16384, else
                          64..65536 (dpar2_autotune_item_rows picks one)           */
} dpar2_opts;

/* Factor matrices (device, float64, row-major). */
typedef struct {
  double* H;           /* R x R */
  double* V;           /* J x R */
  double* W;           /* K x R, row k = diagonal of S_k */
} dpar2_factors;

/* Device views of the compressed representation held in the workspace after
 * dpar2_compress (Sec. III-B; the preprocessed data of Sec. III-G).  All
 * float64, row-major.  Valid until the workspace is reused. */
typedef struct {
  const double* Mt;      /* (K R) x J: row kR + r is column r of C_k B_k (M^T)      */
  const double* D;       /* J x R                                                    */
  const double* E;       /* R, diagonal of E                                         */
  const double* F;       /* (K R) x R; F^(k) = rows kR .. kR+R-1                     */
  const double* Phi;     /* K x L x R: A_k = (X_k Omega) Phi_k, Omega = Omega_1 (q = 0)
                            or the slice's power-step sketch matrix                   */
  const double* sigma;   /* K x R: first-stage singular values (diagonal of B_k)    */
  const double* xnorm2;  /* K: ||X_k||_F^2                                           */
} dpar2_compressed;

/* Host-side summary of a decomposition (filled by dpar2_report_read). */
typedef struct {
  int32_t iters;           /* iterations executed by the repeat loop          */
  int32_t converged;       /* 1 if the stop rule fired before max_iter        */
  double err_last;         /* e of the last iteration (Sec. III-E)             */
  double fit_compressed;   /* 1 - e / sum_k ||X_k||^2                          */
  double fit_true;         /* fitness of Sec. IV-A (after dpar2_fitness)       */
  double xnorm2;           /* sum_k ||X_k||_F^2                                */
  uint32_t warn_bits;      /* DPAR2_WARN_* bits                                */
} dpar2_report;

/* Bytes of device workspace needed for a decomposition of X with options o
 * (host only, pure; 0 on invalid arguments).  dpar2_workspace_size is the
 * same function under its earlier name. */
size_t dpar2_workspace_bytes(const dpar2_tensor* X, const dpar2_opts* o);
size_t dpar2_workspace_size(const dpar2_tensor* X, const dpar2_opts* o);

/* Sec. III-B, two-stage compression (Alg. 3, first loop and the two lines
 * after it).  omega1: device float32 J x L (Gaussian test matrix shared by all
 * slices); omega2: device float32 (K R) x L2 (second stage).  Leaves A_k (as a
 * recipe), M, D, E, F and sum ||X_k||^2 in the workspace.  The slab is read
 * 1 + opts.power_iters times.  For bf16 / fp8 slabs the sketch runs on the bf16
 * matrix cores with Omega rounded to bf16 (round to nearest even); for float32
 * slabs of J <= 128 it sums products of three-piece bf16 splits of X and Omega
 * (FP32-level error, Omega used as given).  The Gram Y^T Y and projection
 * Y^T X of the whole-row pass (J <= 256 float32, J <= 128 otherwise) are the
 * exact products of X and Y rounded to 22-bit fixed point per column of each
 * 64-row tile (relative to that tile column's largest magnitude: an entry
 * 2^22 times smaller than its tile column's maximum rounds to zero); the
 * 128-column-chunk pass forms them from float32 Y and X on the FP64 matrix
 * cores.  A NaN or Inf in the slab sets DPAR2_WARN_NONFINITE.  Resets the
 * iteration state and report held in the workspace. */
dpar2_status dpar2_compress(const dpar2_tensor* X, const dpar2_opts* o,
                            const float* omega1, const float* omega2,
                            void* ws, size_t ws_bytes, dpar2_stream_t stream);

/* Alg. 3, repeat loop: runs up to n_steps further iterations starting from the
 * factors in f (updated in place), stopping early by the rule of opts.tol
 * (checked on the device; later iterations become no-ops).  Requires a prior
 * dpar2_compress on the same workspace.  err_trace: device, n_steps doubles or
 * NULL; receives e_t for each executed iteration (untouched after a stop). */
dpar2_status dpar2_als_step(const dpar2_tensor* X, const dpar2_opts* o, dpar2_factors* f,
                            int32_t n_steps, double* err_trace,
                            void* ws, size_t ws_bytes, dpar2_stream_t stream);

/* Sec. IV-A fitness 1 - sum_k ||X_k - U_k S_k V^T||^2 / sum_k ||X_k||^2 with
 * U_k = A_k Z_k P_k^T H from the last Q-step, computed from the compressed
 * factors via A_k^T X_k = (C_k B_k)^T.  fit: device, 1 double. */
dpar2_status dpar2_fitness(const dpar2_tensor* X, const dpar2_opts* o, const dpar2_factors* f,
                           double* fit, void* ws, size_t ws_bytes, dpar2_stream_t stream);

/* Alg. 3 output U_k = A_k Z_k P_k^T H for all k: U device float64 N x R
 * (row i of slice k at row row_offsets[k] + i).  Reads the slab once more. */
dpar2_status dpar2_output_U(const dpar2_tensor* X, const dpar2_opts* o, const dpar2_factors* f,
                            double* U, void* ws, size_t ws_bytes, dpar2_stream_t stream);

/* Alg. 3 output A_k (Eq. 4, the column-orthonormal first-stage factor of
 * X_k, I_k x R) for all k: A device float64 N x R (row i of slice k at row
 * row_offsets[k] + i), after dpar2_compress.  Reads the slab once more
 * (A_k = Y_k Phi_k recomputed tile by tile; the workspace keeps only the
 * L x R recipe Phi_k). */
dpar2_status dpar2_output_A(const dpar2_tensor* X, const dpar2_opts* o, double* A,
                            void* ws, size_t ws_bytes, dpar2_stream_t stream);

/* Alg. 3 end to end: compress, iterate from the factors in `f` (in/out),
 * then the fitness (written into the workspace report) and, if U != NULL,
 * U_k.  rep (host) NULL: enqueue only, read the report later with
 * dpar2_report_read.  rep != NULL: synchronises the stream, fills *rep and
 * returns DPAR2_ENUMERIC if the slab held NaN or Inf, else DPAR2_ENOCONV if
 * tol >= 0 and the stop rule did not fire within max_iter (results valid),
 * else DPAR2_OK. */
dpar2_status dpar2_decompose(const dpar2_tensor* X, const dpar2_opts* o,
                             const float* omega1, const float* omega2,
                             dpar2_factors* f, double* U, dpar2_report* rep,
                             void* ws, size_t ws_bytes, dpar2_stream_t stream);

/* DPar2 on a tensor that grows by appended slices (the streaming setting
 * of Sec. VI).  The first stage of Sec. III-B factors each slice by itself
 * (Eq. 4), so an append runs it on the new slices only; the second stage
 * (Eq. 5) then runs again over the whole M = ||_k C_k B_k and Alg. 3 iterates
 * from the factors in `f`, as in dpar2_decompose.
 *   X       : the tensor after the append, K slices; slices 0..k_prev-1 are
 *             the ones the earlier call decomposed (same row offsets), slices
 *             k_prev..K-1 the new ones.  Only the new slices' rows are read
 *             (and every row once more if U != NULL).
 *   k_prev  : 1 <= k_prev < K.
 *   o       : the options of the earlier call (rank, sketch widths,
 *             power_iters, item_rows, flags and dtype must be the same).
 *   omega1  : the J x L Omega_1 of the earlier call (the new slices are
 *             sketched with it).
 *   omega2  : (K R) x L2, for all K slices (rows kR..kR+R-1: slice k).
 *   ws_prev : the workspace of the earlier dpar2_decompose or dpar2_append
 *             on slices 0..k_prev-1 (read only; its per-slice first-stage
 *             results are copied), ws_prev_bytes its size.
 *   f       : starting factors of all K slices (W: K x R) in, result out.
 *   U, rep  : as in dpar2_decompose; the warning bits of ws_prev's call
 *             carry over.
 *   ws      : workspace of dpar2_append_workspace_bytes(X, k_prev, o) bytes,
 *             not overlapping ws_prev.  Its first dpar2_workspace_bytes(X, o)
 *             bytes are then the workspace of a decomposition of all K
 *             slices: a later append passes it as ws_prev.
 * The result equals dpar2_decompose on the K slices from the same factors
 * (the per-slice arithmetic is the same).  Errors as in dpar2_decompose;
 * DPAR2_EINVAL also for k_prev out of range or overlapping workspaces,
 * DPAR2_EWORKSPACE for a ws_prev smaller than the earlier layout. */
size_t dpar2_append_workspace_bytes(const dpar2_tensor* X, int64_t k_prev, const dpar2_opts* o);
dpar2_status dpar2_append(const dpar2_tensor* X, int64_t k_prev, const dpar2_opts* o,
                          const float* omega1, const float* omega2,
                          const void* ws_prev, size_t ws_prev_bytes,
                          dpar2_factors* f, double* U, dpar2_report* rep,
                          void* ws, size_t ws_bytes, dpar2_stream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dpar2_decompose without a
 * workspace argument.  The workspace is a static device array of
 * DPAR2_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends (its address is looked up on the first call on a device).
 * The call allocates no device or pinned host memory and instantiates no
 * graph: the schedule tables reach the device as by-value kernel arguments
 * (at most 1 MiB of them, roughly 30k slices), the iterations are launched
 * one by one.  Decompositions whose workspace (dpar2_workspace_bytes) exceeds
 * the scratch, or whose tables exceed 1 MiB, are rejected with
 * DPAR2_EWORKSPACE before anything is enqueued.  Results equal
 * dpar2_decompose's bit for bit.  Every call on one GPU shares that GPU's
 * scratch (the previous call's contents stay; everything a call reads is
 * written by it first): calls that overlap on one GPU, on any streams or
 * threads, race and must be serialised by the caller.  rep as in
 * dpar2_decompose. */
#define DPAR2_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dpar2_status dpar2_decompose_noalloc(const dpar2_tensor* X, const dpar2_opts* o,
                                     const float* omega1, const float* omega2,
                                     dpar2_factors* f, double* U, dpar2_report* rep,
                                     dpar2_stream_t stream);

/* PARAFAC2-ALS on the uncompressed slices (Alg. 2, the iteration DPar2
 * accelerates; its accuracy reference): per iteration, Q_k = the polar
 * factor of X_k V S_k H^T, Y_k = Q_k^T X_k, then one CP-ALS sweep (H, V, W,
 * each a least-squares update with a pseudoinverse, H and V with unit
 * columns) on the R x J x K tensor {Y_k}, and the error
 * e = sum_k ||X_k - Q_k H S_k V^T||^2 with its stop rule.  Every iteration
 * reads the slab once (the first stage's slab kernel sketching with V:
 * X_k V and its exact Gram and projection); everything else is FP64.  Uses
 * opts.rank, max_iter, tol, item_rows and DPAR2_FLAG_WIDE_SLAB (sketch,
 * sketch2 and power_iters are ignored); needs I_k >= R and J >= R.
 * f: starting factors in, result out.  err_trace: device, max_iter doubles
 * or NULL.  U (device, N x R float64, or NULL) receives U_k = Q_k H of the
 * last iteration (one more slab pass).  rep (host) as in dpar2_decompose
 * (fit_true = fit_compressed = 1 - e / sum_k ||X_k||^2 of the last
 * iteration).  Workspace from dpar2_plain_workspace_bytes. */
size_t dpar2_plain_workspace_bytes(const dpar2_tensor* X, const dpar2_opts* o);
dpar2_status dpar2_als_plain(const dpar2_tensor* X, const dpar2_opts* o, dpar2_factors* f,
                             double* err_trace, double* U, dpar2_report* rep,
                             void* ws, size_t ws_bytes, dpar2_stream_t stream);

/* ---- Post-processing of the factors (Sec. IV-E, discovery) ----------------
 * Feature similarity: C (device, J x J float64) = the Pearson correlation
 * coefficients between the rows V(i,:) (device, J x R float64, row-major,
 * e.g. the V of a decomposition; R in 1..32, 40 or 50, else DPAR2_EINVAL); a
 * row of zero variance has no defined correlation and gets 0 in its row and
 * column. */
dpar2_status dpar2_feature_pcc(int64_t J, int32_t R, const double* V, double* C, dpar2_stream_t stream);

/* Slice similarity of Eq. 9: S (device, n x n float64) with
 * S[i][j] = exp(-gamma ||U_{idx[i]} - U_{idx[j]}||_F^2), U the N x R float64
 * output of dpar2_output_U (rows row_offsets[k] .. of slice k; X supplies
 * the offsets, device and host; R in 1..32, 40 or 50).  idx: device int32 n
 * slice indices and its
 * host copy; every listed slice must have the same number of rows (else
 * DPAR2_ESHAPE, checked on the host). */
dpar2_status dpar2_slice_similarity(const dpar2_tensor* X, int32_t R, const double* U, int32_t n,
                                    const int32_t* idx, const int32_t* idx_host, double gamma, double* S,
                                    dpar2_stream_t stream);

/* The k-nearest-neighbour ranking of Sec. IV-E: out (device, k int32) = the
 * indices of the k largest entries of v (device, n float64) in decreasing
 * order, entry `exclude` (the target; -1 for none) left out, ties to the
 * lower index, NaN below every number.  k <= the entries available. */
dpar2_status dpar2_top_k(const double* v, int32_t n, int32_t exclude, int32_t k, int32_t* out,
                         dpar2_stream_t stream);

/* Random walk with restart on the similarity graph (Eqs. 10-11): A = S
 * (device, n x n float64) with its diagonal taken as 0, A~ = A with each row
 * divided by its sum (a row summing to 0 stays 0), q = e_target; r (device,
 * n) starts at q and takes `iters` steps r <- (1 - c) A~^T r + c q (the
 * paper's c = 0.15, 100 steps).  work: device scratch of 3 n doubles. */
dpar2_status dpar2_rwr(const double* S, int32_t n, int32_t target, double c, int32_t iters, double* r,
                       double* work, dpar2_stream_t stream);

/* Fills *out (host struct) with device pointers into the workspace (host-only
 * pointer arithmetic; nothing is enqueued). */
dpar2_status dpar2_compressed_view(const dpar2_tensor* X, const dpar2_opts* o, const void* ws,
                                   size_t ws_bytes, dpar2_compressed* out);

/* Synchronises `stream` and copies the report held in the workspace to *rep
 * (host).  Returns DPAR2_ENUMERIC (report filled) if the slab held NaN or
 * Inf. */
dpar2_status dpar2_report_read(const dpar2_tensor* X, const dpar2_opts* o, const void* ws,
                               dpar2_report* rep, dpar2_stream_t stream);

/* Batched decomposition of n independent tensors (the throughput form of
 * Alg. 3 for many small tensors).  X[t], o[t] (host arrays of n) may differ
 * in everything; the library partitions the batch into groups of tensors that
 * share J, dtype, rank, sketch, sketch2, power_iters, max_iter and flags (in
 * order of first appearance), and runs each group through one set of
 * launches: one slab pass over the work items of all its tensors, one launch
 * per second-stage step and per iteration kernel, each tensor stopping by its
 * own tol; the groups run side by side on library-owned streams (default
 * priority) forked from and joined back into `stream` with events, so the
 * call stays ordered on `stream`.  omega1[t] (J_t x L_t) and omega2[t] ((K_t R_t) x L2_t) are host
 * arrays of device pointers; f[t] holds each tensor's initial factors and
 * receives the result.  Each tensor's result is bit-for-bit the result of
 * dpar2_decompose on that tensor alone (no U output here).  Workspace from
 * dpar2_batch_workspace_size (the groups' layouts end to end); reports from
 * dpar2_batch_report_read (rep: host array of n, in the caller's order;
 * returns DPAR2_ENUMERIC, all reports filled, if some tensor's slab held
 * NaN or Inf). */
size_t dpar2_batch_workspace_size(int32_t n, const dpar2_tensor* X, const dpar2_opts* o);
dpar2_status dpar2_decompose_batch(int32_t n, const dpar2_tensor* X, const dpar2_opts* o,
                                   const float* const* omega1, const float* const* omega2,
                                   dpar2_factors* f, void* ws, size_t ws_bytes,
                                   dpar2_stream_t stream);
dpar2_status dpar2_batch_report_read(int32_t n, const dpar2_tensor* X, const dpar2_opts* o,
                                     const void* ws, dpar2_report* rep, dpar2_stream_t stream);

/* Autotuner of the slab pass's work-item size for one tensor: times the
 * slab pass (first stage only, as dpar2_compress runs it) for each
 * candidate item_rows in cands (host array of n_cands values, each 0 or in
 * 64..65536) and writes the fastest to *best (host) and, if times_ms is not
 * NULL, the median of 3 timed launches of each (host, n_cands).  ws must be
 * large enough for every candidate (dpar2_workspace_size with the candidate
 * that cuts the most items).  Synchronises the stream; the workspace's
 * decomposition state is overwritten. */
dpar2_status dpar2_autotune_item_rows(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                                      const int32_t* cands, int32_t n_cands, void* ws, size_t ws_bytes,
                                      int32_t* best, float* times_ms, dpar2_stream_t stream);

/* Autotuner of the slab pass's tiling for one tensor (the batching form's
 * per-(J, L) choice): candidate c is the work-item size item_rows[c] (rows
 * per unit of Alg. 4's scheduling, 0 or 64..65536) with the whole-row pass
 * (wide[c] == 0) or the 128-column-chunk pass (wide[c] != 0, i.e.
 * DPAR2_FLAG_WIDE_SLAB; the only one above the whole-row limit).  Each is
 * timed as dpar2_autotune_item_rows does; *best (host) receives the index of
 * the fastest, times_ms (host, n_cands, or NULL) the medians.  ws must be
 * large enough for every candidate (dpar2_workspace_size of the options with
 * the flag set, if any candidate sets it).  Synchronises the stream; the
 * workspace's decomposition state is overwritten. */
dpar2_status dpar2_autotune_slab(const dpar2_tensor* X, const dpar2_opts* o, const float* omega1,
                                 const int32_t* item_rows, const int32_t* wide, int32_t n_cands, void* ws,
                                 size_t ws_bytes, int32_t* best, float* times_ms, dpar2_stream_t stream);

/* ---- Learned warm start ---------------------------------------------------
 * Not part of the paper: a set encoder proposes the starting H, V, W of the
 * iteration of Alg. 3 from the compressed representation of Sec. III-B.
 * Tokens: per slice the upper triangle (row-major, a <= b) of
 * R Phi_k / e_mean, Phi_k = (F^(k) E S)^T (F^(k) E S), S = diag of the signs
 * that make the largest-magnitude entry of each column of D positive,
 * e_mean = ||E||^2 / K; NF = R (R + 1) / 2 floats per token.  Network (FP32,
 * width DPAR2_WARM_WIDTH): Z1 = relu(W1 x + b1), Z2 = relu(W2 Z1 + b2) per
 * token, p = mean_k Z2; outputs H = WH p + bH (R x R), V~ = WV p + bV (R x R,
 * V in the basis D S), W(k, :) = Ww [Z2_k; p] + bw.  Parameters are one flat
 * float32 array of dpar2_warm_param_count(R) values, blocks in the order W1
 * (128 x NF), b1, W2 (128 x 128), b2, WH (R^2 x 128), bH, WV (R^2 x 128), bV,
 * Ww (R x 256), bw, each row-major. */
#define DPAR2_WARM_WIDTH 128

/* Number of float parameters for rank R (0 if R is outside 1..32). */
int64_t dpar2_warm_param_count(int32_t rank);

/* Tokens of a compressed tensor (after dpar2_compress on ws): tok device
 * float32 K x NF. */
dpar2_status dpar2_warm_features(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, size_t ws_bytes,
                                 float* tok, dpar2_stream_t stream);

/* Training targets from factors f (e.g. converged ones) of the same
 * tensor: the gauge is fixed by unit-norm columns of H and V (scale into W),
 * V~ = (D S)^T V with each column signed by its largest-magnitude entry,
 * each column of W signed to a non-negative sum (same flip on H), components
 * sorted by decreasing ||W(:, r)||.  tH = H^T H (R x R), tV = V~ (R x R),
 * tW = W / sqrt(e_mean / R) (K x R); device float32. */
dpar2_status dpar2_warm_targets(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, size_t ws_bytes,
                                const dpar2_factors* f, float* tH, float* tV, float* tW, dpar2_stream_t stream);

/* Starting factors from network outputs: H = pH, V = D S pV,
 * W = pW sqrt(e_mean / R) (pH, pV: R x R, pW: K x R, device float32). */
dpar2_status dpar2_warm_apply(const dpar2_tensor* X, const dpar2_opts* o, const void* ws, size_t ws_bytes,
                              const float* pH, const float* pV, const float* pW, dpar2_factors* f,
                              dpar2_stream_t stream);

/* Forward pass over n tensors at once.  tok_off: device and (host) copies of
 * n + 1 token offsets (tensor b owns tokens tok_off[b] .. tok_off[b+1]-1, at
 * least one); tok: device float32 (tok_off[n]) x NF; act: device scratch of
 * tok_off[n] x 4 x DPAR2_WARM_WIDTH floats (kept for the backward pass);
 * outputs pH, pV: n x R x R, pW: tok_off[n] x R. */
dpar2_status dpar2_warm_forward(int32_t rank, int32_t n, const int32_t* tok_off, const int32_t* tok_off_host,
                                const float* tok, const float* theta, float* act, float* pH, float* pV, float* pW,
                                dpar2_stream_t stream);

/* Backward pass after dpar2_warm_forward on the same arguments: loss
 * sum_b (||pH_b^T pH_b - tH_b||^2 / R^2 + ||pV_b - tV_b||^2 / R^2 +
 * ||pW_b - tW_b||^2 / (K_b R)); grad_part: device scratch n x P; grad (P)
 * receives the gradient summed over the n tensors (fixed order); loss: device
 * n x 3 (the three terms per tensor). */
dpar2_status dpar2_warm_backward(int32_t rank, int32_t n, const int32_t* tok_off, const int32_t* tok_off_host,
                                 const float* tok, const float* theta, float* act, const float* pH, const float* pV,
                                 const float* pW, const float* tH, const float* tV, const float* tW,
                                 float* grad_part, float* grad, float* loss, dpar2_stream_t stream);

/* One Adam step (Kingma & Ba, with bias correction; step counts from 1) on
 * theta with gradient grad * grad_scale; m, v: device moment buffers (P). */
dpar2_status dpar2_warm_adam(int32_t rank, float* theta, const float* grad, float* m, float* v, int32_t step,
                             float lr, float beta1, float beta2, float eps, float grad_scale,
                             dpar2_stream_t stream);

/* Kernel timing for measurement.  While enabled, every dpar2_compress records
 * a pair of HIP events around its slab pass (the first-stage kernel that reads
 * the slab) on the launch stream.  dpar2_profile_read waits for the recorded
 * events, returns the number of timed launches and their summed duration in
 * milliseconds (host pointers), and clears the record.  Process-wide. */
dpar2_status dpar2_profile_enable(int32_t on);
dpar2_status dpar2_profile_read(int32_t* launches, double* total_ms);

/* Frees the host-side state the library keeps for workspace ws (pinned
 * staging buffers of the schedule upload, graphs of captured iterations),
 * after waiting for the uploads out of that staging to finish.  Call it
 * before freeing or repurposing ws; a later call on ws rebuilds the state.
 * Unknown ws: no-op.  dpar2_release_all does it for every workspace and also
 * frees the batch stream pool. */
dpar2_status dpar2_release(const void* ws);
dpar2_status dpar2_release_all(void);

/* Static description of a status code. */
const char* dpar2_status_string(int32_t status);

/* Message of the last error on the calling thread ("" if none). */
const char* dpar2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LIBDPAR2_DPAR2_H */
