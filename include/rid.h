/*
 * rid.h - C ABI of the MI355X streaming randomized interpolative decomposition.
 *
 * The library computes, for a stream of snapshots a_1, a_2, ... (the columns of
 * an m x n matrix A that arrive one time step at a time and are discarded after
 * use, Sec. 1), the single-pass randomized ID A ~ A(:,J) P of Alg. 3:
 *
 *   per snapshot   s_j = Omega a_j, SS^T += s_j s_j^T, ||A_obs||_F^2 += ||a_j||^2
 *                  (eq. random_sketch; Alg. 3 steps 10-13);
 *   per t columns  sketched ridge leverage scores of the basis and of the new
 *                  columns (eq. sketch_ridge_leverage_score), the prune/fill of
 *                  the basis (Alg. 3 steps 16-27), the full-sketch coefficients
 *                  of Alg. 4 (eq. coeff_rID_fullsketch) and the NA-Hutch++ error
 *                  estimate of Alg. 8 (eqs. NAhutchPP_expansion and
 *                  NAhutchPP_2nd_term).
 *
 * Conventions shared by every entry point:
 *  - All matrices are column-major.  A batch of b snapshots is a device buffer
 *    holding b columns of m elements each, element stride 1, column stride
 *    ld >= m elements (a contiguous torch tensor of shape (b, m)).
 *  - "device" pointers are HIP device memory on the stream's device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library owns all stream state and never frees caller memory.
 *  - Every call that launches work enqueues it on the stream given to
 *    rid_init_stream (a hipStream_t passed as void*; NULL = the null stream).
 *    Only the getters (rid_select, rid_coefficients, rid_error_estimate,
 *    rid_get_info, rid_get_update, rid_debug_*) synchronise that stream.
 *  - A handle is not thread safe; distinct handles are independent.
 *  - Errors are reported by the return code, never by exceptions.  The first
 *    device error or non-finite input latches the handle into the FAILED
 *    state: afterwards only rid_get_info, rid_last_error and rid_destroy
 *    succeed (others return RID_ESTATE).
 *  - Snapshot indices are 0-based; an empty basis slot holds -1.
 */
#ifndef RID_H
#define RID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rid_status {
  RID_OK = 0,
  RID_EINVAL = 1,     /* invalid argument (null pointer, bad size or range) */
  RID_ENOMEM = 2,     /* device or host allocation failed */
  RID_EDEVICE = 3,    /* a HIP call or kernel launch failed */
  RID_ESTATE = 4,     /* call not valid in the handle's current state */
  RID_ECAPACITY = 5,  /* the push would exceed n_max observed columns */
  RID_ENUMERIC = 6,   /* non-finite input or numerical breakdown */
  RID_ENOTSUP = 7     /* configuration not supported by this build */
} rid_status;

/* Element type of the snapshots. */
typedef enum rid_dtype { RID_F32 = 0, RID_F64 = 1 } rid_dtype;

/* Arithmetic of the sketch contraction Omega * a_j.  Every form accumulates in
 * binary32 inside a row slab and in binary64 across slabs, except RID_SKETCH_F64
 * which is binary64 throughout.  RID_SKETCH_F64 needs RID_F64 data; the other
 * forms need RID_F32 data. */
typedef enum rid_sketch_prec {
  RID_SKETCH_F64 = 0,   /* binary64 test matrix and products */
  RID_SKETCH_F32 = 1,   /* binary32 test matrix and data, matrix cores */
  RID_SKETCH_BF16 = 2,  /* bfloat16-rounded test matrix and data, matrix cores */
  RID_SKETCH_FP8 = 3    /* e4m3 test matrix (scale 2^-6) and e4m3 data with one
                           power-of-two scale per 32 rows of each column,
                           scaled fp8 matrix cores */
} rid_sketch_prec;

/* Work split of the bf16 sketch (the results are the same up to the order
 * of binary32 sums within a slab).  NARROW: one workgroup per 256-column
 * tile holds every sketch row.  WIDE (bf16, 128 < l <= 320): two workgroups
 * per 512-column tile hold half of the rows each, so each Gaussian of the
 * test matrix serves twice as many columns, and the columns the two fetch
 * meet in L2.  A single stream uses NARROW under AUTO (faster on the
 * 19M-row channel stream: one 64 KB chunk in flight per workgroup instead of
 * two 32 KB ones); the batch tuner times both. */
typedef enum rid_sketch_tile { RID_TILE_AUTO = 0, RID_TILE_NARROW = 1, RID_TILE_WIDE = 2 } rid_sketch_tile;

/* Coefficients of each update (Alg. 3's coefficient steps, Sec. 3.2):
 * RID_COEFF_ALG4 computes Alg. 4 (full sketch least squares) only;
 * RID_COEFF_BEST4 computes Algs. 4, 5, 6 and 7 and keeps the one whose
 * NA-Hutch++ estimate (Alg. 8) is smallest (ties: the lowest algorithm).
 * Alg. 5 takes (Omega A_J)^T (Omega A_obs) / l as its approximation of
 * A_J^T A_obs; Alg. 6 fits the residual with the new basis columns (the
 * text's reading); Algs. 6 and 7 update the previous update's kept P and give
 * the columns observed since it Alg. 4's coefficients; Alg. 7's transform is
 * G^{-1} A_J^T A_{J_prev} from exact Grams. */
typedef enum rid_coeff_mode { RID_COEFF_ALG4 = 0, RID_COEFF_BEST4 = 1 } rid_coeff_mode;

/* Arithmetic of the basis Gram G = A_J^T A_J (Alg. 8's ||A_J P||_F^2 term and
 * the Grams of Algs. 5 and 7) for binary32 data.  EXACT: binary32 products are
 * exact in binary64 and summed in binary64 (binary64 matrix cores).  SPLIT:
 * each value is split exactly into three bfloat16 pieces, the six piece
 * products of order <= 2 are summed on the bfloat16 matrix cores in binary32
 * over 32 rows, two such sums added in binary32, then in binary64; elementwise
 * |G_ij - A_i^T A_j| <= (37 * 2^-24 + (m / 64 + 1024) * 2^-53) sum_r |a_ri| |a_rj|
 * for data of magnitude in [2^-100, 2^60] (or zero), so the NA-Hutch++
 * estimate moves by at most that factor times || |A_J| |P| ||_F^2.  AUTO: SPLIT
 * in RID_COEFF_ALG4 mode, EXACT in RID_COEFF_BEST4 mode (Algs. 5 and 7 solve
 * with G).  binary64 data always uses binary64 products (AUTO or EXACT). */
typedef enum rid_gram_mode { RID_GRAM_AUTO = 0, RID_GRAM_EXACT = 1, RID_GRAM_SPLIT = 2 } rid_gram_mode;

/* Push flags. */
#define RID_COPY   0u  /* copy the columns into the library's ring; the buffer
                          may be reused once prior work on the stream is done */
#define RID_BORROW 1u  /* keep pointers only; the buffer must stay valid and
                          unmodified until rid_get_info reports a
                          release_watermark past its last column */

/* Where rid_coefficients writes P. */
#define RID_HOST   0u
#define RID_DEVICE 1u

/* Stream configuration.  Fill it with rid_config_default, then set the sizes.
 * Parameters follow Alg. 3: l = k + p sketch rows, target rank k, basis size t
 * (the paper sets k = t), accuracy eps and failure probability delta of the
 * fill probability c (k ln k + k ln(1/delta)/eps) tau^D / t. */
typedef struct rid_config {
  int64_t m;              /* rows per snapshot, >= 1 */
  int32_t ell;            /* sketch rows l, 4 <= l <= 512 */
  int32_t k;              /* target rank, 1 <= k <= l */
  int32_t t;              /* basis size, 1 <= t <= min(l, 256) */
  int32_t data_dtype;     /* rid_dtype */
  int32_t sketch_prec;    /* rid_sketch_prec */
  uint64_t omega_seed;    /* seed of the Philox stream that defines Omega */
  uint64_t select_seed;   /* seed of the Philox stream of the prune/fill draws */
  double delta;           /* 0 < delta < 1 (default 0.05) */
  double eps;             /* eps > 0 (default 0.5) */
  double c_sample;        /* c > 0 (default 1) */
  double ridge_floor;     /* rho >= 0: lam >= rho F / k (default 1e-8) */
  int32_t hutch_n1;       /* rows of Omega_1 (0 = l/4) */
  int32_t hutch_n2;       /* rows of Omega_2 (0 = l/2); n1 + n2 < l */
  int32_t lookahead;      /* columns buffered before a sketch launch; 0 = auto */
  int32_t sketch_tile;    /* rid_sketch_tile (default RID_TILE_AUTO) */
  int64_t n_max;          /* capacity: maximum number of pushed columns */
  int32_t coeff_mode;     /* rid_coeff_mode (default RID_COEFF_ALG4); RID_COEFF_BEST4 needs
                             t <= 154 and a stream of its own (not a batch member) */
  int32_t gram_mode;      /* rid_gram_mode (default RID_GRAM_AUTO); SPLIT needs RID_F32 data and
                             RID_COEFF_ALG4 (RID_ENOTSUP with RID_COEFF_BEST4) */
} rid_config;

/* Error estimate of the last completed update (Alg. 8). */
typedef struct rid_error {
  double E2;        /* estimate of ||A_obs - A_J P||_F^2 (may be negative) */
  double E_abs;     /* sqrt(max(E2, 0)) */
  double rel;       /* E_abs / sqrt(F) (0 when F = 0) */
  double F;         /* ||A_obs||_F^2 */
  int64_t n_obs;    /* columns covered by P */
  int64_t update;   /* index of the update the estimate belongs to */
} rid_error;

/* Per-update record (all values as computed on the device). */
typedef struct rid_update {
  int64_t update;       /* 0-based update index u */
  int64_t n_obs;        /* observed columns when the update ran */
  int64_t count;        /* buffered columns the update scanned */
  double F;             /* ||A_obs||_F^2 */
  double sk2;           /* ||S_k||_F^2: sum of the top min(k,l) eigenvalues of SS^T */
  double lam;           /* ridge parameter lam = max(F (tr(SS^T) - sk2) / tr(SS^T) / k,
                           rho F / k) (tau uses SS^T + l*lam*I) */
  double E2, tr_est, gpp, term1, h, corr;  /* NA-Hutch++ terms (Alg. 8) */
  int32_t n_pruned;     /* slots emptied by the prune draws */
  int32_t n_filled;     /* slots filled from the buffer */
  int32_t n_occupied;   /* occupied slots after the update */
  int32_t flags;        /* RID_UPD_* bits */
} rid_update;

#define RID_UPD_SKIPPED       1  /* F = 0: selection skipped */
#define RID_UPD_RANK_DEFICIENT 2 /* Omega A_J numerically rank deficient */
#define RID_UPD_PINV_TRUNCATED 4 /* NA-Hutch++ K truncated to its numerical rank */

typedef struct rid_info {
  int64_t n_pushed;           /* columns pushed so far */
  int64_t n_sketched;         /* columns whose sketch has been enqueued */
  int64_t n_updates;          /* updates enqueued */
  int64_t release_watermark;  /* columns < this are no longer read (BORROW) */
  int32_t failed;             /* 1 when the handle is latched FAILED */
  int32_t finalized;          /* 1 after rid_finalize */
  int32_t last_status;        /* status that latched FAILED (RID_OK otherwise) */
  int32_t reserved0;
  int64_t device_bytes;       /* device memory held by the handle */
} rid_info;

typedef struct rid_stream rid_stream;

/* Fills *cfg with the defaults listed above (sizes zero).  Never fails on a
 * non-null pointer; returns RID_EINVAL for NULL. */
rid_status rid_config_default(rid_config* cfg);

/* Validates *cfg, allocates the stream state on the current HIP device and
 * returns the handle in *out.  stream: hipStream_t passed as void* (NULL = the
 * null stream).  Errors: RID_EINVAL (bad sizes, t > l, k > l, l < 4, m < 1,
 * dtype/precision mismatch), RID_ENOMEM, RID_EDEVICE. */
rid_status rid_init_stream(const rid_config* cfg, void* stream, rid_stream** out);

/* Pushes b snapshots: d_cols is a device buffer of b columns of m elements
 * (the data dtype), column stride ld >= m elements.  flags: RID_COPY or
 * RID_BORROW.  Asynchronous; may enqueue sketches and zero or more updates.
 * Alg. 3 steps 9-13 (and steps 14-32 whenever t columns are buffered).
 * Errors: RID_EINVAL, RID_ECAPACITY (n_pushed + b > n_max), RID_ESTATE
 * (finalized or failed), RID_EDEVICE. */
rid_status rid_push_snapshots(rid_stream* h, const void* d_cols, int64_t ld, int32_t b,
                              uint32_t flags);

/* Enqueues the sketch of every pushed column and every update whose t columns
 * are all pushed.  Asynchronous.  Errors: RID_ESTATE, RID_EDEVICE. */
rid_status rid_flush(rid_stream* h);

/* Ends the stream: flushes, then runs one last update over the partially filled
 * buffer when it is not empty, so that P covers every pushed column.
 * Asynchronous.  Errors: RID_ESTATE (already finalized or failed). */
rid_status rid_finalize(rid_stream* h);

/* Restarts the stream (no columns observed, empty basis) keeping its
 * allocations.  Asynchronous: the state is cleared in stream order after all
 * earlier work of the handle; the host waits only until the previous upload
 * of the column-pointer table has been copied.  Borrowed buffers of the
 * previous pass stay in use until that earlier work has run.  Errors:
 * RID_ESTATE (failed). */
rid_status rid_reset(rid_stream* h);

/* Copies the current index set J (slot order, -1 = empty) into the host array
 * J[0..cap), cap >= t, and stores t in *t_out.  Flushes and synchronises.
 * Errors: RID_EINVAL, RID_ESTATE (no update yet, or failed), RID_ENUMERIC. */
rid_status rid_select(rid_stream* h, int64_t* J, int32_t cap, int32_t* t_out);

/* Copies P (t x n_cols, binary64, column-major, rows in slot order, rows of
 * empty slots zero) of the last update into P with leading dimension ldp >= t
 * and at most cap_cols columns; *n_cols receives the number of columns P
 * covers.  where: RID_HOST (host pointer) or RID_DEVICE (device pointer).
 * Flushes and synchronises.  Alg. 4.  Errors: RID_EINVAL (ldp < t or
 * cap_cols < n_cols), RID_ESTATE, RID_ENUMERIC. */
rid_status rid_coefficients(rid_stream* h, double* P, int64_t ldp, int64_t cap_cols,
                            int64_t* n_cols, uint32_t where);

/* The NA-Hutch++ estimate of the last update (Alg. 8).  Flushes and
 * synchronises.  Errors: RID_EINVAL, RID_ESTATE, RID_ENUMERIC. */
rid_status rid_error_estimate(rid_stream* h, rid_error* e);

/* Writes d_out(:, 0:c) = A_J P(:, j0:j0+c) (m x c, data dtype, column stride
 * ld >= m, device memory).  Eq. eqn:id.  Asynchronous; the columns must be
 * covered by the last update.  Errors: RID_EINVAL (range outside the covered
 * columns, ld < m), RID_ESTATE. */
rid_status rid_reconstruct(rid_stream* h, int64_t j0, int32_t c, void* d_out, int64_t ld);

/* Counters and state of the handle.  Synchronises.  Never fails on a valid
 * handle (RID_EINVAL for NULL arguments). */
rid_status rid_get_info(rid_stream* h, rid_info* info);

/* Record of update u (0 <= u < n_updates) and, when non-null, the index set
 * after it (J_out[0..t)) and the scores it used (tau_C[0..t): scores of the
 * slots occupied before the update, NaN for empty slots; tau_D[0..count):
 * scores of the buffered columns).  Flushes and synchronises.  Errors:
 * RID_EINVAL (u out of range), RID_ESTATE. */
rid_status rid_get_update(rid_stream* h, int64_t u, rid_update* rec, int64_t* J_out,
                          double* tau_C, double* tau_D);

/* Frees every resource of the handle; valid in any state, synchronises. */
rid_status rid_destroy(rid_stream* h);

/* Static text for a status code. */
const char* rid_status_string(rid_status s);

/* Copies the last error message of the handle (or of the library when h is
 * NULL) into buf[0..n), NUL-terminated. */
rid_status rid_last_error(rid_stream* h, char* buf, size_t n);

/* ---- live timing --------------------------------------------------------- */

/* Device time of the work the handle enqueued since profiling was enabled,
 * measured with HIP events recorded on the handle's stream around each launch
 * group. */
typedef struct rid_profile {
  double sketch_ms;         /* sketch contraction kernels (eq. random_sketch) */
  int64_t sketch_launches;  /* number of sketch contraction launches */
  double sketch_bytes;      /* snapshot bytes those launches read (columns x m x size) */
  double reduce_ms;         /* slab reductions of the sketch */
  double update_ms;         /* per-update phases on the main stream (Alg. 3 steps 16-29) */
  int64_t updates;          /* updates timed */
  double gram_ms;           /* basis copy + Gram kernels inside the updates */
  double gram_bytes;        /* basis columns the Gram reads: every occupied column once per
                               update that brings new columns (columns x m x size) */
  double coeff_ms;          /* Alg. 4 and Alg. 8 phases, on the second stream: they run beside
                               later main-stream work (the next pass's sketch after a reset),
                               so their span is not additive with the other phases */
  double pool_copy_bytes;   /* new basis columns written into the pool (columns x m x size);
                               not part of the method's own traffic (single streams only) */
  int64_t gram_launches;    /* updates that brought new columns, each one Gram launch
                               (single streams only) */
} rid_profile;

/* on != 0 starts recording (and clears earlier records); on == 0 stops.
 * Errors: RID_EINVAL, RID_EDEVICE. */
rid_status rid_profile_enable(rid_stream* h, int32_t on);

/* Synchronises the stream and sums the recorded intervals into *p.
 * Errors: RID_EINVAL, RID_EDEVICE. */
rid_status rid_profile_read(rid_stream* h, rid_profile* p);

/* ---- inspection entry points used by the parity tests ------------------ */

/* The choice of update u in RID_COEFF_BEST4 mode: e2[q - 4] = the NA-Hutch++
 * estimate E^2 of Alg. q's coefficients (q = 4..7, host array of 4) and
 * *q_star = the algorithm kept.  Synchronises.  Errors: RID_EINVAL (null
 * arguments, u outside the enqueued updates), RID_ESTATE (another mode,
 * failed stream). */
rid_status rid_get_coeff_choice(rid_stream* h, int64_t u, double* e2, int32_t* q_star);

/* Sketch state: S (l x n_sketched, binary64) into the host array S with
 * leading dimension lds >= l and at most cap_cols columns, ||a_j||^2 into
 * colsq[0..n_sketched) (may be NULL) and the basis Gram G = A_J^T A_J (t x t)
 * into G (may be NULL).  Flushes and synchronises.  Errors: RID_EINVAL,
 * RID_ESTATE. */
rid_status rid_debug_state(rid_stream* h, double* S, int64_t lds, int64_t cap_cols,
                           int64_t* n_cols, double* colsq, double* G);

/* Writes Omega(0:ell, i0:i0+count) of the given seed into the device buffer
 * d_out (ell x count, column-major, column stride ld >= ell), evaluated the way
 * the sketch form `prec` evaluates it (binary32 for RID_SKETCH_F32 and
 * RID_SKETCH_BF16 and RID_SKETCH_FP8, binary64 for RID_SKETCH_F64; the element
 * type of d_out is float for the former and double for the latter;
 * RID_SKETCH_BF16 values are rounded to bfloat16 and RID_SKETCH_FP8 values are
 * e4m3(64 Omega) / 64, both widened back to float).  Alg. 3 step 2.
 * Asynchronous on `stream`.  Errors: RID_EINVAL, RID_EDEVICE. */
rid_status rid_omega_block(int32_t prec, uint64_t omega_seed, int32_t ell, int64_t i0,
                           int64_t count, void* d_out, int64_t ld, void* stream);

/* One-shot sketch of a block of b snapshots with no stream state (eq.
 * random_sketch and the column norms of Alg. 3 step 13): S = Omega A and
 * colsq[j] = ||a_j||^2, Omega the test matrix of omega_seed evaluated the way
 * the form sketch_prec evaluates it in a stream (RID_SKETCH_F64 takes binary64
 * data, the other forms binary32).
 *   d_cols       device, column-major m x b, column stride ld >= m elements;
 *                the pointer and ld * element size are multiples of 16 bytes
 *   d_S          device, l x b binary64, column-major, leading dimension l
 *   d_colsq      device, b binary64
 *   d_nonfinite  device int32 or NULL: set to 0, then to 1 if a column holds a
 *                non-finite value (its norm is then not finite)
 *   stream       hipStream_t as void* (NULL = the null stream)
 * The caller owns every buffer and keeps them valid until the work enqueued
 * on `stream` completes.  The rows of each column are summed in slabs whose
 * count depends only on (sketch_prec, ell, m, b): the count a stream uses for
 * a lookahead batch of b columns, lowered until the per-slab partial sketches
 * fit 128 MiB; the work space (column table, partial sketches and norms, at
 * most 128 MiB) is allocated stream-ordered (hipMallocAsync) and freed the
 * same way.  Errors (message via rid_last_error(NULL, ...)): RID_EINVAL
 * (unknown form, sizes, null pointers, alignment), RID_ECAPACITY (b columns
 * of m rows need more than 128 MiB of partial sketches even at the largest
 * slab: pass fewer columns), RID_ENOMEM, RID_EDEVICE. */
rid_status rid_sketch_columns(int32_t sketch_prec, uint64_t omega_seed, int32_t ell, int64_t m,
                              const void* d_cols, int64_t ld, int32_t b, double* d_S,
                              double* d_colsq, int32_t* d_nonfinite, void* stream);

/* rid_sketch_columns for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, slab geometry, kernels and results (bit for
 * bit), with the work space in a fixed 128 MiB array that the library holds
 * on every device it runs on until the process ends.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); on its first
 * call on a device it looks up that device's array address once.  It clears
 * what must start at zero (the non-finite flag) with a kernel, not a memset.
 * Every call on one device uses that device's array: calls whose work
 * overlaps on one device (other streams, other threads) race and must be
 * ordered by the caller.  Errors as rid_sketch_columns, with RID_ECAPACITY
 * when the work space of the call would pass 128 MiB; RID_EDEVICE if the
 * array's address cannot be found. */
rid_status rid_sketch_columns_noalloc(int32_t sketch_prec, uint64_t omega_seed, int32_t ell, int64_t m,
                                      const void* d_cols, int64_t ld, int32_t b, double* d_S,
                                      double* d_colsq, int32_t* d_nonfinite, void* stream);

/* ---------------------------------------------------------------------------
 * Batched streams.
 *
 * Many independent streams (fields, spatial blocks) of uneven m advanced
 * together on one device; not part of the paper, whose method handles one
 * stream.  Each member is an ordinary stream (Alg. 3 with Alg. 4 and Alg. 8,
 * its own configuration, seeds and results); the batch only changes how its
 * work is launched: per round, one persistent sketch launch whose workgroups
 * walk the (member, row slab, sketch rows, column tile) work items of every
 * member, one reduction launch, and each update kernel launched once for all
 * members with an update due.  The launches of a round are captured into one
 * HIP graph, updated in place from round to round.  The row slab of the
 * sketch (the tile height) is chosen by timing the candidates on the first
 * round's columns (sketch and reduction), once per batch shape in the
 * process; for bf16 members whose lookahead fills two 512-column tiles the
 * tuner also times both work splits of rid_sketch_tile.
 *
 * A member's results are bitwise independent of the other members.  They
 * equal those of a stand-alone stream with the same slab: the slab fixes the
 * order of the binary64 sums over slabs, so the sketch can differ from a
 * stand-alone stream's in the last bits.
 * ------------------------------------------------------------------------- */
typedef struct rid_batch rid_batch;

#define RID_BATCH_NO_GRAPH 1u  /* launch each round directly (no graph capture) */
#define RID_BATCH_NO_TUNE  2u  /* keep the default slab of 16384 rows */

typedef struct rid_batch_info {
  int32_t ns;                    /* members */
  int32_t failed;                /* 1 after a device error */
  int64_t rounds;                /* rounds run so far */
  int64_t graph_launches;        /* rounds launched as a graph */
  int64_t graph_instantiations;  /* executable graphs built */
  int64_t graph_updates;         /* rounds that updated the executable in place */
  int64_t slab_rows;             /* sketch rows per work item (tuned or default) */
  int32_t tuned;                 /* 1 once the slab has been chosen by timing */
  int32_t wide;                  /* 1 when some member uses RID_TILE_WIDE */
  double tune_ms;                /* device time spent timing candidates */
} rid_batch_info;

/* Creates ns member streams from cfgs[0..ns-1] (each validated as by
 * rid_init_stream; every member keeps its own sizes, precision and seeds).
 * All batch work runs on an internal stream that is ordered after the work
 * enqueued on `stream` before each batch call, and `stream` waits for it at
 * the end of each call.  flags: RID_BATCH_NO_GRAPH, RID_BATCH_NO_TUNE.
 * 1 <= ns <= 4096.  Errors: RID_EINVAL, RID_ENOMEM, RID_EDEVICE. */
rid_status rid_init_batch(int32_t ns, const rid_config* cfgs, void* stream, uint32_t flags,
                          rid_batch** out);

/* One push round: member i receives b[i] >= 0 snapshots, d_cols[i] a device
 * buffer of b[i] columns with column stride ld[i] >= m_i (as for
 * rid_push_snapshots; d_cols[i] may be NULL when b[i] = 0).  flags:
 * RID_COPY or RID_BORROW for every member of this call.  Full lookahead
 * batches are sketched and their updates enqueued; a member whose pending
 * columns fit in one lookahead batch waits for a later round or for
 * rid_finalize_batch.  Asynchronous.  Errors: RID_EINVAL, RID_ECAPACITY,
 * RID_ESTATE (batch failed or a member finalized), RID_EDEVICE. */
rid_status rid_push_batch(rid_batch* bt, const void* const* d_cols, const int64_t* ld, const int32_t* b,
                          uint32_t flags);

/* Sketches everything pending and runs every member's remaining updates,
 * the last one over its partial buffer (as rid_finalize).  Asynchronous. */
rid_status rid_finalize_batch(rid_batch* bt);

/* Returns every member to its state right after rid_init_batch (as
 * rid_reset); the chosen slab and the executable graph are kept. */
rid_status rid_reset_batch(rid_batch* bt);

/* Member i as a stream handle owned by the batch: valid for rid_select,
 * rid_coefficients, rid_error_estimate, rid_reconstruct (ordered before later
 * work on the batch's caller stream), rid_get_info, rid_get_update,
 * rid_debug_state and rid_last_error; rid_push_snapshots, rid_finalize,
 * rid_reset and rid_destroy on it return RID_ESTATE. */
rid_status rid_batch_stream(rid_batch* bt, int32_t i, rid_stream** out);

/* Counters of the batch (synchronises its internal stream). */
rid_status rid_batch_get_info(rid_batch* bt, rid_batch_info* info);

/* Candidate i (0-based, in the order timed) of the slab tuner: its slab
 * rows, work split (1 = RID_TILE_WIDE) and the faster of two timed runs of
 * the round's persistent sketch over one column tile per member, in ms (the
 * scan of a split stops at the first slab 15% slower than its best).  RID_EINVAL past the last candidate (none when
 * the shape was tuned earlier in the process or RID_BATCH_NO_TUNE is set). */
rid_status rid_batch_tune_result(rid_batch* bt, int32_t i, int64_t* slab_rows, int32_t* wide, double* ms);

/* Message of the batch's last error (or of the last failed creation when bt
 * is NULL). */
rid_status rid_batch_last_error(rid_batch* bt, char* buf, size_t n);

/* Timing of the batch's launches: while on, rounds run as direct launches
 * (no graph) with events around each, so the figures cover the same kernels
 * the graph runs.  rid_batch_profile_read sums them since the last enable:
 * sketch_ms / sketch_launches / sketch_bytes for the persistent sketch
 * launches (snapshot bytes they read), reduce_ms, update_ms (every update
 * kernel, Gram included), gram_ms, and in `updates` the number of rounds
 * timed; gram_bytes stays 0.  Both synchronise the batch's stream. */
rid_status rid_batch_profile_enable(rid_batch* bt, int32_t on);
rid_status rid_batch_profile_read(rid_batch* bt, rid_profile* p);

/* Waits for the batch's work and frees it with all its members. */
rid_status rid_destroy_batch(rid_batch* bt);

#ifdef __cplusplus
}
#endif

#endif /* RID_H */
