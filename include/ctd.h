/*
 * ctd.h — C ABI of the MI355X (gfx950) CTD library.
 *
 * CTD ("Compact Tensor Decomposition") approximates a sparse tensor X by a
 * mode-alpha LR decomposition X ~ C x_alpha (R U) whose factor R holds
 * actual, linearly independent mode-alpha fibers of X (Section 3 of the
 * paper).  CTD-S (Section 3.1, Algorithm 1) decomposes a static tensor;
 * CTD-D (Section 3.2, Algorithm 2) extends the factors with each arriving
 * time slice.  This library runs the data-parallel path of both on one GPU:
 * fiber keying, squared fiber norms, weighted sampling with replacement,
 * unique selection, the independence filter, the projection of X_(alpha)
 * onto span(R) and the Frobenius residual of Eq. 14.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Modes are 0-based: the paper's alpha = 1 is mode 0.
 *  - Tensors arrive as COO ("sparse-unordered" storage, Section 2.1): a
 *    device array of int32 indices laid out mode-major ([order][nnz]) and a
 *    device array of nnz values, float64 or float32.  Coordinates must be
 *    distinct and inside `dims`; values must be finite.
 *  - Columns of X_(alpha) are numbered column-major over the other modes in
 *    increasing mode order (fiber id f = sum_{m != alpha} i_m prod_{l<m,
 *    l != alpha} I_l), so a new last-mode (time) slice appends trailing
 *    columns.  The product of all mode lengths must stay below 2^62.
 *  - Every call is asynchronous on the stream given to ctd_create.  Inputs
 *    are borrowed: they must stay valid until the stream passes the call.
 *    Results live in the handle until the next decompose/update/destroy.
 *  - Arguments the host can check are checked at once (CTD_ERR_INVALID_ARG,
 *    CTD_ERR_STATE).  Errors found by kernels (index out of range,
 *    duplicate coordinate, non-finite value, zero norm) are latched on the
 *    device and returned by ctd_sync / ctd_get_result.  After any error the
 *    handle only accepts ctd_decompose, ctd_get_result, ctd_last_error and
 *    ctd_destroy.
 *  - Device allocations that fail return CTD_ERR_OOM with a message; the
 *    handle then accepts the same call again.  For testing those paths, the
 *    environment variable CTD_FAIL_ALLOC=k makes the k-th device allocation
 *    the library attempts after the value was set (or changed) fail as if
 *    the device were out of memory; the ones after it succeed.
 *  - Random draws are reproducible: draw j of a call uses Philox4x32-10
 *    (Salmon et al., SC'11) with key (seed mod 2^32, seed >> 32) and counter
 *    (j mod 2^32, j >> 32, step, tensor); step is 0 for ctd_decompose and t
 *    for the t-th ctd_update after it; tensor is 0.
 */
#ifndef CTD_H_
#define CTD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CTD_OK = 0,
  CTD_ERR_INVALID_ARG = 1,  /* bad scalar argument (mode, sample size, order, dims, dtype) */
  CTD_ERR_EMPTY = 2,        /* ||X||_F = 0: the column distribution of Algorithm 1 is undefined */
  CTD_ERR_INDEX_OOB = 3,    /* a coordinate lies outside dims */
  CTD_ERR_DUPLICATE = 4,    /* two nonzeros share a coordinate */
  CTD_ERR_NONFINITE = 5,    /* a value is NaN or infinite */
  CTD_ERR_OOM = 6,          /* device allocation failed */
  CTD_ERR_HIP = 7,          /* a HIP runtime call failed */
  CTD_ERR_STATE = 8,        /* call not valid in the handle's state (update before decompose, shape mismatch) */
  CTD_ERR_CAPACITY = 9      /* a size exceeds a documented limit of the library */
} ctd_status;

enum { CTD_F64 = 0, CTD_F32 = 1 };                 /* value dtype of a ctd_coo */
enum { CTD_PREC_FP64 = 0, CTD_PREC_MIXED = 1 };    /* arithmetic of the projection and of C */

/* A sparse tensor in COO form.  `dims` is a host array; `idx` and `val`
 * are device arrays owned by the caller. */
typedef struct {
  int32_t order;            /* N, 2 <= N <= 8 */
  const int64_t* dims;      /* host [order]: I_1 .. I_N, each >= 1 */
  int64_t nnz;              /* number of stored entries, 0 <= nnz < 2^31 */
  const int32_t* idx;       /* device [order * nnz]: idx[m * nnz + e] is the mode-m index of entry e */
  const void* val;          /* device [nnz], float64 or float32 per val_dtype */
  int32_t val_dtype;        /* CTD_F64 or CTD_F32 */
} ctd_coo;

typedef struct {
  int32_t precision;        /* CTD_PREC_FP64 (all float64) or CTD_PREC_MIXED (float32 projection;
                               the CTD-D C held and updated in float32) */
  double eps;               /* tolerance of Algorithm 1's independence test (the paper uses 1e-6) */
  int32_t want_C;           /* CTD-S: also write C_(alpha) = R^T X_(alpha) (dense s~ x n_f) */
  int32_t want_fiber_stats; /* also keep per-fiber ||x_f||^2 - ||P x_f||^2 */
  int32_t profile;          /* time the stages of each call with HIP events (see stage_ms) */
} ctd_options;

/* Stages timed when ctd_options.profile is set (milliseconds, device time
 * between HIP events recorded on the handle's stream). */
enum {
  CTD_STAGE_SORT = 0,       /* fiber keys and radix sort (matricization) */
  CTD_STAGE_SAMPLE = 1,     /* weights, prefix, draws, unique */
  CTD_STAGE_PANEL = 2,      /* dense panel of the candidates */
  CTD_STAGE_BASIS = 3,      /* independence filter and orthonormal basis */
  CTD_STAGE_PROJECT = 4,    /* projection of all nonzeros and the residual (Eq. 14) */
  CTD_STAGE_SPMM = 5,       /* the multi-nonzero fiber SpMM kernel alone (inside PROJECT) */
  CTD_STAGE_CORE = 6,       /* C: CTD-S core if want_C; CTD-D: the cross-term passes after the slices */
  CTD_STAGE_TOTAL = 7,
  CTD_N_STAGES = 8
};

/* Results of the last call.  Scalars are copies; pointers are device
 * memory owned by the handle (valid until the next decompose/update/destroy). */
typedef struct {
  int64_t s;                /* number of draws of the last call */
  int64_t s_unique;         /* s': unique drawn fibers */
  int64_t s_tilde;          /* accepted fibers held in R (CTD-D: all steps) */
  int64_t n_f;              /* non-empty fibers of the last input (CTD-D: of the slice) */
  int64_t n_rows;           /* I_alpha */
  int64_t step;             /* 0 after ctd_decompose, t after the t-th ctd_update */
  uint64_t weight_total;    /* W, total integer sampling weight of the last input */
  double norm2;             /* ||X||_F^2 (CTD-D: of all data seen) */
  double err2;              /* ||X - X~||_F^2, Eq. 14 numerator */
  double rel_err;           /* err2 / norm2, Eq. 14 */
  double slice_err2;        /* CTD-D: ||dX - P dX||_F^2 of the last slice */
  int32_t status;           /* latched device status (ctd_status) */
  float stage_ms[8];        /* per-stage device time of the last call if profiling, else 0 */
  /* device arrays */
  const uint64_t* draws;    /* [s] fiber ids in draw order */
  const uint64_t* unique;   /* [s'] ascending unique fiber ids */
  const int32_t* counts;    /* [s'] multiplicity of each unique fiber */
  const double* prob;       /* [s'] quantized sampling probability w/W */
  const double* scale;      /* [s'] duplicate-merge scale sqrt(k / (s p)) */
  const uint64_t* accepted; /* [s~] fiber ids kept in R, in order of acceptance */
  const double* Q;          /* [I_alpha x ldq] row-major orthonormal basis R L^{-T} */
  int64_t ldq;
  const double* Linv_t;     /* [s~ x ldx] row-major upper M with Q = R M: U = (R^T R)^{-1} = M M^T */
  int64_t ldx;
  const double* R;          /* [I_alpha x ldr] row-major kept fibers (the paper's R) */
  int64_t ldr;
  const void* C;            /* column-major C_(alpha), ldc rows per column: CTD-S n_f columns if
                               want_C; CTD-D one column per non-empty fiber seen (n_cols);
                               element type C_dtype */
  int64_t ldc;
  int64_t n_cols;           /* columns of C */
  const uint64_t* col_ids;  /* [n_cols] fiber id of each column of C */
  const uint64_t* fiber_ids;/* [n_f] ascending non-empty fiber ids of the last input */
  const double* fiber_resid;/* [n_f] ||x_f||^2 - ||P x_f||^2 if want_fiber_stats */
  int32_t C_dtype;          /* CTD_F64; CTD_F32 for the CTD-D C of a mixed-precision handle
                               (held and updated in float32) */
} ctd_result;

typedef struct ctd_handle ctd_handle;

/* Create a handle bound to a HIP stream (NULL = default stream).  Options may
 * be NULL (float64, eps 1e-6, no C).  Allocates device memory lazily.
 *
 * Where kernels have variants that compute identical values and differ only
 * in how work is spread (fibers per wave of the projection and of C's
 * columns), a per-process autotuner times every variant on the first call of
 * an input-size bucket and keeps the fastest; results never depend on the
 * choice.  If the environment variable CTD_TUNE_CACHE names a file, choices
 * are read from it at first use and appended to it when made. */
ctd_status ctd_create(ctd_handle** out, const ctd_options* opt, void* hip_stream);

/* CTD-S, Algorithm 1 (Section 3.1) on tensor X for mode `mode` with s draws
 * (1 <= s <= N_alpha, the REQUIRE clause of Algorithm 1) and Philox seed
 * `seed`.  Also starts a CTD-D stream whose time mode is the last mode. */
ctd_status ctd_decompose(ctd_handle* h, const ctd_coo* X, int32_t mode, int64_t s, uint64_t seed);

/* CTD-S from given draws instead of sampling (Lemma 2's "given R_0"):
 * `draws` is a host array of s fiber ids of X_(alpha), repeats allowed;
 * every id must name a non-empty fiber (else CTD_ERR_INVALID_ARG at sync). */
ctd_status ctd_decompose_given(ctd_handle* h, const ctd_coo* X, int32_t mode,
                               const uint64_t* draws, int64_t s);

/* CTD-D, Algorithm 2 (Section 3.2): one time slice dX whose dims equal the
 * stream's first N-1 dims with a last dim of 1, d draws (1 <= d <= dN_alpha).
 * Requires a prior ctd_decompose with want_C set and a non-time mode.  The
 * rows of C for the slice's kept fibers over the earlier columns (Eq. 13) are
 * written on a stream of the handle (default priority) beside the slice's
 * own columns and residual; the handle's stream waits for it before the call
 * returns, so later work on that stream sees all of C. */
ctd_status ctd_update(ctd_handle* h, const ctd_coo* slice, int64_t d);

/* CTD-D on B consecutive slices (Algorithm 2 applied B times in order): the
 * results equal B calls of ctd_update up to rounding.  `slices` is a host
 * array of B slice descriptors (each as for ctd_update; their device arrays
 * must stay valid until the stream passes the call).  Slice b draws with
 * Philox step word t + 1 + b.  The rows of C for the fibers the batch keeps
 * are formed after the batch: over the columns held before it in one pass
 * over C (the projector onto the grown span leaves the earlier
 * reconstructions unchanged, Eqs. 8-13), so C is streamed once per batch
 * instead of once per slice.  1 <= B <= CTD_MAX_BATCH. */
ctd_status ctd_update_batched(ctd_handle* h, const ctd_coo* slices, int32_t B, int64_t d);

/* Checkpoint of a CTD-D stream.  Algorithm 2 (Section 3.2) carries R, U and C
 * and the stream's error from each time step to the next; this call copies
 * that state (R, the orthonormal Q = R M and M with U = M M^T, the row
 * leverages, C, the fiber ids of R's and C's columns, the step t, the totals
 * of Eq. 14 and the handle's internal sizes) into the host buffer `host_buf`
 * of *bytes bytes, after waiting for the handle's stream.  On return *bytes
 * holds the size the state needs (about (2 I_alpha + n_cols) d~ values plus
 * the ids); host_buf == NULL only reports it (CTD_OK); a buffer smaller than
 * that returns CTD_ERR_CAPACITY and writes nothing.  The buffer is plain
 * bytes in the library's native layout (versioned header, then the arrays),
 * owned by the caller.  Needs a CTD-D stream: a ctd_decompose with want_C on
 * a non-time mode, with or without updates after it (else CTD_ERR_STATE). */
ctd_status ctd_save_state(ctd_handle* h, void* host_buf, size_t* bytes);

/* Resume a CTD-D stream from a checkpoint of ctd_save_state: the handle drops
 * any stream it held and continues the saved one, so later ctd_update calls
 * give the same draws, kept fibers and bits as on the handle that saved it.
 * The handle must have been created with the saved precision and eps and
 * with want_C (else CTD_ERR_STATE); a buffer that is not a complete state of
 * this library version returns CTD_ERR_INVALID_ARG.  The host buffer is read
 * before the call returns.  Afterwards ctd_get_result reports the stream's
 * step, kept fibers, factors, C and error; the per-input fields of the last
 * call before the save (draws, unique fibers, s, s', n_f) are empty. */
ctd_status ctd_load_state(ctd_handle* h, const void* host_buf, size_t bytes);

/* Many independent tensors in one call (the batched execution form of
 * CTD-S): tensor b of the host array Xs[0..B) gets Algorithm 1 with s[b]
 * draws in mode `mode`, its draws using Philox counter word tensor = b
 * (tensor 0 has the draws and kept fibers of ctd_decompose, its floating-point
 * results equal to rounding: how a launch splits its reductions depends on how
 * many tensors share it).  Tensors go in groups within a
 * workspace budget (128 GiB): the per-tensor stages run concurrently on internal
 * streams of default priority, and the independence filter and basis of a
 * whole group run as one sequence of launches on the handle's stream.  All
 * of it is ordered after the caller's earlier work on that stream, and later
 * work on it runs after all of them.
 * Per-tensor results are read with ctd_get_batch_result; the handle's own
 * CTD-S / CTD-D state is left as it was.  Host argument errors are returned
 * at once; device errors are latched per tensor.  A call with the same
 * tensors (pointers, shapes, nonzero counts), sizes, seed and mode as the
 * call just before it on the handle is captured as a HIP graph, and later
 * such calls replay it (same results, bit for bit; the inputs' current values
 * are read); the environment variable CTD_NO_GRAPH=1 turns this off.  The
 * graph is captured on, and replayed on, a stream of the handle that forks
 * from the caller's stream and joins it again, so any caller's stream works,
 * the legacy default stream included.  The caller's stream must not be
 * capturing when the call is made. */
ctd_status ctd_decompose_batched(ctd_handle* h, const ctd_coo* Xs, int32_t B, int32_t mode,
                                 const int64_t* s, uint64_t seed);

/* Wait for the stream and fill `out` with tensor b of the last batched call:
 * scalars and the index arrays (draws, unique, counts, prob, scale,
 * accepted; device memory owned by the handle until the next batched call).
 * Factor pointers are NULL.  Returns tensor b's latched device status. */
ctd_status ctd_get_batch_result(ctd_handle* h, int32_t b, ctd_result* out);

/* Number of ctd_decompose_batched calls on h whose work ran as a graph launch
 * (the capturing call and every replay); 0 for a null handle.  For tests and
 * diagnostics of the graph form; it does not synchronize. */
int64_t ctd_batch_graph_launches(const ctd_handle* h);

/* Attack candidates read off R (the online detection of the paper's
 * application section, Section 5).  The kept fibers, in order of acceptance,
 * are grouped by their coordinate in mode `group_mode` (the destination host
 * of a source x destination x time tensor decomposed along the source mode;
 * for the last mode of a CTD-D stream the time index counts the slices too);
 * the earliest kept fiber of a group represents it, and representatives
 * whose norm ||x_f|| is strictly above the mean norm of all representatives
 * are the candidates.  Writes up to `cap` candidate fiber ids and norms, in
 * order of acceptance, to the host arrays `fids` / `norms` (may be NULL when
 * cap == 0), the number of candidates to *n_out (it may exceed cap) and the
 * number of groups to *n_groups.  Needs the dense R of the last
 * ctd_decompose / ctd_update; waits for the handle's stream.  group_mode must
 * differ from the decomposition mode (CTD_ERR_INVALID_ARG); without a
 * decomposition CTD_ERR_STATE. */
ctd_status ctd_attack_candidates(ctd_handle* h, int32_t group_mode, uint64_t* fids, double* norms,
                                 int64_t cap, int64_t* n_out, int64_t* n_groups);

/* Memory usage of the factors (Eq. 15): (nnz(C) + nnz(U) + nnz(R)) / nnz(X),
 * X being all input held (CTD-D: the initial tensor and every slice).
 * nnz(R) and nnz(C) count the nonzero entries of the kept fibers and of C;
 * nnz(U) counts U = (R^T R)^{-1} structurally: kept fibers that share a row
 * are linked, U is block diagonal over the connected groups, and each group
 * of g fibers contributes g^2.  Needs C (want_C); waits for the stream. */
typedef struct {
  int64_t nnz_C, nnz_U, nnz_R, nnz_X;
  double usage;
} ctd_memory;
ctd_status ctd_memory_usage(ctd_handle* h, ctd_memory* out);

/* The factor C_(alpha) = R^T X_(alpha) of Algorithm 1 as a sparse matrix (the
 * sparse output of C whose nonzeros Eq. 15 counts).  R's columns are actual
 * fibers, so entry (a, f) can be nonzero only where kept fiber a and fiber f
 * share a row.  Compressed-column form over the n_f non-empty fibers of the
 * last ctd_decompose, in the order of the dense C (ascending fiber id): column
 * f holds its entries at [col_ptr[f], col_ptr[f + 1]) with row indices a (the
 * kept fiber's position in R's order) increasing; only entries whose computed
 * value is nonzero are stored, each summed over the fiber's nonzeros in fiber
 * order (deterministic).  col_ptr: device int64[n_f + 1], written always;
 * row_idx: device int32[cap] and vals: device float64[cap], written only when
 * nnz(C) <= cap (they may be NULL when cap == 0).  *nnz_out receives nnz(C)
 * in every case; nnz(C) > cap returns CTD_ERR_CAPACITY, so a caller can size
 * the arrays from a first call with cap = 0.  Needs the dense R of a CTD-S
 * handle after ctd_decompose (after ctd_update, CTD_ERR_STATE: the CTD-D C
 * is a projection, not R^T X) and s~ <= 8192 (else CTD_ERR_CAPACITY: one
 * column's accumulator lives in 64 KiB of LDS).  Waits for the handle's
 * stream; allocates and frees a workspace of (I_alpha + 1) int64 and nnz(R)
 * (int32, float64) pairs per call. */
ctd_status ctd_sparse_core(ctd_handle* h, int64_t* col_ptr, int32_t* row_idx, double* vals,
                        int64_t cap, int64_t* nnz_out);

/* The same as ctd_sparse_core, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): this call allocates and frees nothing.  Its workspace
 * (R's row pointers, (I_alpha + 1) int64; the scan's block sums; R's row
 * lists, nnz(R) (int32, float64) pairs; each part aligned to 256 bytes) lives
 * in a static device array of CTD_NOALLOC_SCRATCH_BYTES bytes that each GPU
 * the library runs on holds until the process ends.  Arguments, outputs,
 * the capacity protocol and the results are those of ctd_sparse_core;
 * a workspace beyond the scratch size returns CTD_ERR_CAPACITY before any
 * kernel touches it (I_alpha up to about 8M rows, nnz(R) up to about 5M at
 * small I_alpha).  Every call on one GPU shares that GPU's scratch and leaves
 * its contents behind (each call writes every workspace entry it reads before
 * reading it), so calls that overlap on one GPU, from several handles or
 * threads, race: the caller serializes them. */
ctd_status ctd_sparse_core_noalloc(ctd_handle* h, int64_t* col_ptr, int32_t* row_idx, double* vals,
                                int64_t cap, int64_t* nnz_out);

/* Wait for the stream and return the latched device status. */
ctd_status ctd_sync(ctd_handle* h);

/* Wait for the stream and fill `out` (see ctd_result). */
ctd_status ctd_get_result(ctd_handle* h, ctd_result* out);

/* Message for the last error on this handle ("" if none).  With h == NULL:
 * the message of this thread's last failed ctd_create, if it failed for a
 * runtime reason, else "null handle". */
const char* ctd_last_error(const ctd_handle* h);

void ctd_destroy(ctd_handle* h);

/* Limits of the library. */
#define CTD_MAX_ORDER 8
#define CTD_MAX_DRAWS 16384
#define CTD_MAX_BATCH 256
#define CTD_MAX_TENSORS 65536
#define CTD_NOALLOC_SCRATCH_BYTES (64u << 20)   /* per-GPU scratch of ctd_sparse_core_noalloc */

#ifdef __cplusplus
}
#endif
#endif /* CTD_H_ */
