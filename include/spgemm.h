/*
 * spgemm.h - C ABI of the MI355X (gfx950) local SpGEMM of the sparsity-aware
 * 1D algorithm (Hong & Buluc, "A sparsity-aware distributed-memory algorithm
 * for sparse-sparse matrix multiplication").
 *
 * One call sequence computes one 1D partition's local product
 *     C_i = A * B_i          (Sec. II: C = AB; Alg. 1, the local step)
 * with A (m x k), B_i (k x n_i) and C_i (m x n_i) in CSC:
 *
 *   spgemm_plan      H_i, Alg. 2 block selection, column map, gather of A~
 *   spgemm_symbolic  sparse flops per column, binning, nnz per column, scan
 *   spgemm_numeric   values of C_i (rows ascending inside every column)
 *   spgemm_backward  (dC*B_i^T) o pattern(A) and (A^T*dC) o pattern(B_i)
 *   spgemm_batched   numeric of many planned products as one DAG (or one hipGraph)
 *                    (spgemm_batch_create/run/destroy: the same with an explicit batch handle)
 *
 * Conventions for every entry point:
 *   - Matrices are CSC: colptr int64[ncols+1], rowidx int32[nnz] with row ids
 *     ascending and unique inside each column, vals float or double (the
 *     plan's dtype).  Unless a comment says "host", pointers are DEVICE
 *     pointers on the current HIP device.
 *   - The caller owns every buffer it passes in and keeps A, B_i and the
 *     given value arrays alive and unchanged until the plan is destroyed (or,
 *     for value arrays passed to spgemm_numeric, until the stream reaches the
 *     end of that call).  A plan owns its workspace and the gathered A~.
 *   - Work is enqueued on the plan's stream (a hipStream_t passed as void*,
 *     NULL = the null stream) and is asynchronous unless stated otherwise.
 *   - Every call returns SPGEMM_OK (0) or a negative status; nothing aborts
 *     or throws across the ABI.  spgemm_last_error() returns a message for
 *     the last failing call on the calling thread.
 *   - Sizes are int64; row and column ids are int32, so m, k and n_i must be
 *     below 2^31.
 */
#ifndef SPGEMM_MI355X_H
#define SPGEMM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SPGEMM_OK 0
#define SPGEMM_EINVAL (-1)       /* bad argument or malformed matrix */
#define SPGEMM_ENOMEM (-2)       /* device or host allocation failed / over limit */
#define SPGEMM_EHIP (-3)         /* a HIP runtime call failed (message has text) */
#define SPGEMM_EUNSUPPORTED (-4) /* valid request the library does not serve */
#define SPGEMM_ESTATE (-5)       /* call out of order (e.g. numeric before symbolic) */

typedef enum { SPGEMM_F32 = 0, SPGEMM_F64 = 1 } spgemm_dtype;

typedef struct {
    int64_t nrows;
    int64_t ncols;
    int64_t nnz;
    const int64_t *colptr; /* device, ncols+1, colptr[0] == 0, colptr[ncols] == nnz */
    const int32_t *rowidx; /* device, nnz */
    const void *vals;      /* device, nnz values of the plan's dtype (may be NULL
                              for a pattern-only plan; numeric then needs values) */
} spgemm_csc;

/*
 * Tuning knobs.  spgemm_default_tuning() fills the defaults; a NULL tuning
 * pointer means the defaults.  Thresholds only change which kernel computes
 * a column, never the result.
 */
typedef struct {
    int32_t tiny_max_flop;      /* columns with flop <= this (0..512) use one wave each */
    int32_t hash_max_flop;      /* symbolic LDS hash up to this flop (<= 4096), else bitmap */
    int32_t hash_max_nnz;       /* numeric LDS hash up to this nnz (<= 2048), else dense windows */
    int32_t dense_window;       /* most output rows one dense-bin pass holds in LDS
                                   (0 = as many as LDS allows, else a power of 2 >= 32) */
    int32_t validate;           /* 1: check the CSC invariants of A and B_i on the device */
    int32_t own_partition;      /* >= 0: B_i's own partition of A (local to the caller) ... */
    int32_t own_partition_whole;/* ... and 1 takes all of its nonzero columns into A~ (every
                                   group of it chosen) instead of applying the block rule of
                                   Alg. 2 to it as to the remote partitions; C_i is the same */
    int32_t medium_kernel;      /* medium numeric bins: 0 = choose by m, 1 = LDS hash and
                                   sort, 2 = LDS bitmap and rank */
    int32_t batch_streams;      /* batched: side streams that, with the caller's stream, the
                                   independent work of one depth (products, grouped
                                   launches) is spread over (0 = 4, at most 8) */
    int32_t batch_form;         /* batched: 0 = the stream DAG, where at each dependency
                                   depth the products of at most 4096 columns without dense
                                   columns share one launch per numeric bin and kernel (the
                                   others, and value gathers, run their own kernels on side
                                   streams); 1 = one persistent launch per run (products
                                   with tiny and hash columns only: SPGEMM_EUNSUPPORTED when
                                   a product has dense columns or tiny_max_flop > 256); 2 =
                                   the stream DAG with every product launching its own
                                   kernels */
    int32_t dense_first_flop;   /* dense output columns with at least this many products are
                                   handed out first (numeric bin 7), so the longest ones do
                                   not finish last; 0 = no such bin */
    int32_t reserved;           /* must be 0 */
    int64_t workspace_limit;    /* bytes of device workspace a plan may take; 0 = no limit */
} spgemm_tuning;

/* Plan statistics (host struct), filled by spgemm_plan_stats. */
typedef struct {
    int64_t m, k, n;        /* A is m x k, B_i is k x n */
    int64_t nnz_A, nnz_B;
    int64_t h_count;        /* |H_i|: rows of B_i holding an entry */
    int64_t nzc_A;          /* nonzero columns of A over all partitions */
    int64_t K;              /* groups formed by Alg. 2 over all partitions */
    int64_t M;              /* groups chosen (hit blocks, i.e. fetch messages) */
    int64_t kt;             /* columns of A~ */
    int64_t nnz_At;         /* stored entries of A~ */
    double cv_memA;         /* nnz_At / nnz_A: fetched share of A (Discussion) */
    int64_t flops;          /* sparse flops of A*B_i (-1 before symbolic) */
    int64_t nnz_C;          /* stored entries of C_i (-1 before symbolic) */
    int64_t sym_bins[8];    /* columns per symbolic bin: 0 empty, 1 tiny, 2..5 hash, 6 bitmap, 7 unused */
    int64_t num_bins[8];    /* columns per numeric bin: 0 empty, 1 tiny, 2..5 hash, 6 dense,
                               7 dense with at least dense_first_flop products */
} spgemm_stats;

typedef struct spgemm_plan_s *spgemm_plan_t;

/* Message for the last failing call on this thread ("" if none). */
const char *spgemm_last_error(void);

/* Library version string. */
const char *spgemm_version(void);

/*
 * Fills *t with the default tuning.  Environment variables override single
 * fields (decimal integers; unparsable values are ignored, ranges are
 * checked when a plan uses the tuning): SPGEMM_TINY_MAX_FLOP,
 * SPGEMM_HASH_MAX_FLOP, SPGEMM_HASH_MAX_NNZ, SPGEMM_DENSE_WINDOW, SPGEMM_DENSE_FIRST_FLOP,
 * SPGEMM_MEDIUM_KERNEL, SPGEMM_BATCH_STREAMS, SPGEMM_VALIDATE,
 * SPGEMM_WORKSPACE_LIMIT.  Returns SPGEMM_EINVAL for NULL.
 */
int spgemm_default_tuning(spgemm_tuning *t);

/*
 * spgemm_plan - the gather half of Alg. 1 for partition i.
 *
 *   A            m x k, all P column partitions of A (Alg. 1 Data: A_r is a
 *                column slice of A).  A->vals may be NULL for a pattern-only
 *                plan.
 *   Bi           k x n_i, the caller's column slice of B.
 *   dtype        value type of A, B_i and C_i.
 *   a_part_offsets  HOST int64[P+1]: partition r owns columns
 *                [offs[r], offs[r+1]) of A; offs[0] = 0, offs[P] = k,
 *                non-decreasing.
 *   P            number of partitions (>= 1).
 *   block_size   b >= 1: Alg. 2 cuts each partition's ordered nonzero
 *                column ids into consecutive groups of b (the last group may
 *                be shorter); a group holding any column named by H_i is
 *                fetched whole.
 *   tuning       NULL = defaults.
 *   stream       hipStream_t used by this and every later call on the plan.
 *   out          receives the plan handle (NULL on failure).
 *
 * Computes, on the device and asynchronously: H_i (rows of B_i that hold an
 * entry; notation table, Alg. 1), the group id of every nonzero column of A,
 * the chosen groups (Alg. 2), the selection and map of A's columns into A~
 * (an exclusive prefix over the selected columns, -1 for others) and copies
 * the selected columns' row ids and values into A~ (Alg. 1, fetch and build
 * A~).  Host-side checks cover dimensions, pointers and offsets; with
 * tuning->validate the CSC invariants of A and B_i are checked on the device
 * and the call synchronises the stream to report them (SPGEMM_EINVAL).
 */
int spgemm_plan(const spgemm_csc *A, const spgemm_csc *Bi, spgemm_dtype dtype,
                const int64_t *a_part_offsets, int32_t P, int64_t block_size,
                const spgemm_tuning *tuning, void *stream, spgemm_plan_t *out);

/* Re-targets later calls on the plan to another stream (NULL = null stream).
 * Work already enqueued on the old stream is ordered before the new
 * stream's later work (an event wait), and counts a pending symbolic phase
 * publishes are read first (which may wait for that phase).  EHIP on a
 * failed event call. */
int spgemm_plan_set_stream(spgemm_plan_t plan, void *stream);

/* Synchronises the plan's stream and fills *stats (host struct). */
int spgemm_plan_stats(spgemm_plan_t plan, spgemm_stats *stats);

/*
 * Copies plan internals to caller buffers (DEVICE pointers; any may be NULL):
 *   H         uint8[k]        H_i
 *   map       int32[k]        column of A -> column of A~, or -1
 *   At_colptr int64[kt+1]     A~ column pointers
 *   At_rowidx int32[nnz_At]   A~ row ids
 *   At_vals   dtype[nnz_At]   A~ values
 *   blocks    int64[2*M]      (first, last) column of each chosen group, in
 *                             partition then group order (Alg. 2's R)
 * Sizes come from spgemm_plan_stats.  Enqueued on the plan's stream.
 */
int spgemm_plan_export(spgemm_plan_t plan, uint8_t *H, int32_t *map, int64_t *At_colptr,
                       int32_t *At_rowidx, void *At_vals, int64_t *blocks);

/*
 * Copies the symbolic phase's per-column data (DEVICE pointers, may be NULL):
 *   flop     int64[n_i]  sparse flops of each column of C_i (Sec. III-B)
 *   sym_bin  int32[n_i]  symbolic bin of each column (see spgemm_stats)
 *   num_bin  int32[n_i]  numeric bin of each column
 * Valid after spgemm_symbolic; SPGEMM_ESTATE before.
 */
int spgemm_plan_export_bins(spgemm_plan_t plan, int64_t *flop, int32_t *sym_bin,
                            int32_t *num_bin);

/*
 * spgemm_symbolic - pattern size of C_i (Sec. III-A column-by-column formula).
 *
 *   C_colptr  int64[n_i+1], caller-allocated; receives C_i's column pointers.
 *   nnzC      HOST int64*; receives nnz(C_i).
 *
 * Uses the sparse flops and bins of every column (Sec. III-B) that the
 * plan computed, counts the distinct rows of every output column (a row is
 * stored whenever a product reaches it, even if values later cancel) and
 * scans the counts.  Waits on the host twice: for the bin sizes (first call
 * on a plan only) and for nnzC.  Both are written to pinned host memory by
 * the device (the bin sizes by the kernel after the flops pass; nnzC by the
 * scan as soon as it has the total, for n_i <= 8192 ahead of its other
 * writes), each behind a flag the host polls for a short while before it
 * falls back to a blocking synchronisation of the plan's stream.  C_colptr
 * is written by work enqueued on the plan's stream: later work on that
 * stream, or a synchronisation of it, sees it complete.
 */
int spgemm_symbolic(spgemm_plan_t plan, int64_t *C_colptr, int64_t *nnzC);

/*
 * spgemm_symbolic_noalloc - spgemm_symbolic for callers that cannot allocate
 * device or pinned memory once their plans exist (tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results, waits and
 * errors as spgemm_symbolic; it calls no allocator.  What the symbolic phase
 * keeps for the numeric phase (the sorted product order of every tiny
 * column, the row bitmap of every dense column) goes to a fixed array of
 * 64 MiB that the library holds on each device until the process ends,
 * instead of pooled blocks.  Limits and sharing:
 *   - SPGEMM_ENOMEM (with the byte count in spgemm_last_error) when the kept
 *     data exceed 64 MiB: 1 KiB per tiny column (every column of a B_i with
 *     at most 16384 columns) plus m/8 bytes per column with more flops than
 *     the largest symbolic hash bin (m <= 2^18; taller plans keep no
 *     bitmaps).  C_colptr is then undefined; the plan accepts a later
 *     spgemm_symbolic.
 *   - SPGEMM_ENOMEM for a plan of more than 2^18 rows with such columns
 *     until one spgemm_symbolic run on it has built its split table
 *     (4 * k * (ceil(m / 8192) + 1) bytes, kept by the plan).
 *   - The plan's device must be current (SPGEMM_EINVAL otherwise).
 *   - Every call on a device takes that device's array over: spgemm_numeric,
 *     spgemm_backward and spgemm_batch_create/spgemm_batched then fail with
 *     SPGEMM_ESTATE on a plan whose data an earlier call placed there, until
 *     it runs a symbolic phase again.  Calls on one device whose work
 *     overlaps in time (other streams, other threads) race on the array.
 */
int spgemm_symbolic_noalloc(spgemm_plan_t plan, int64_t *C_colptr, int64_t *nnzC);

/*
 * spgemm_numeric - values of C_i = A * B_i.
 *
 *   A_vals    dtype[nnz(A)] new values of A on the planned pattern, or NULL
 *             to use the values A~ holds (gathered by spgemm_plan, or by the
 *             last call that gathered new ones).  Non-NULL values are
 *             gathered into A~ first (values half of Alg. 1's fetch) - except
 *             when A~ holds every entry of A (every nonzero column chosen),
 *             where they are read in place and A~ keeps its values.
 *   Bi_vals   dtype[nnz(B_i)] or NULL for the values given to spgemm_plan.
 *   C_rowidx  int32[nnzC], caller-allocated; receives ascending row ids.
 *   C_vals    dtype[nnzC], caller-allocated.
 *
 * Requires spgemm_symbolic (SPGEMM_ESTATE otherwise) with the C_colptr it
 * filled still alive.  Can be re-run with new values on the same patterns.
 * Products are summed in an unspecified order, in FP64 for both dtypes (a
 * product of two FP32 values is exact in FP64); each FP32 entry is rounded
 * once, when written.
 */
int spgemm_numeric(spgemm_plan_t plan, const void *A_vals, const void *Bi_vals,
                   int32_t *C_rowidx, void *C_vals);

/*
 * spgemm_backward - gradients of L = <dC, A * B_i> on the stored entries:
 *   dA = (dC * B_i^T) o pattern(A)      dtype[nnz(A)] (zero where B_i's row is empty)
 *   dB = (A^T * dC) o pattern(B_i)      dtype[nnz(B_i)]
 *
 *   C_colptr/C_rowidx  C_i's pattern as produced by symbolic/numeric.
 *   A_vals/Bi_vals     values (NULL = the plan's).
 *   dC_vals            dtype[nnzC] upstream gradient on pattern(C_i).
 *   dA_vals/dB_vals    outputs; either may be NULL to skip it.
 * dB entries are each summed by one thread in a fixed order (bitwise
 * reproducible); dA entries receive their products through atomic adds, so
 * their summation order, and the last bits, may vary between calls.
 * Requires spgemm_symbolic.
 */
int spgemm_backward(spgemm_plan_t plan, const int64_t *C_colptr, const int32_t *C_rowidx,
                    const void *A_vals, const void *Bi_vals, const void *dC_vals,
                    void *dA_vals, void *dB_vals);

/* Frees the plan and returns its workspace to the library's pool.  NULL is OK. */
int spgemm_plan_destroy(spgemm_plan_t plan);

/* ---------------------------------------------------------------------------
 * Batched numeric (the Galerkin products of an AMG setup, Sec. II-C and
 * Sec. IV-B, and any set of independent products): the numeric phase of many
 * planned products of uneven sizes, optionally chained (the C of one product
 * is the A or B of a later one), enqueued as one dependency DAG and
 * optionally captured once into a hipGraph and replayed with new values in
 * the same buffers.
 * ------------------------------------------------------------------------- */
typedef struct {
    const void *A_vals;   /* dtype[nnz(A)]: new values of A, gathered into A~ before the
                             product (NULL = keep A~ as the plan gathered it) */
    const void *B_vals;   /* dtype[nnz(B)] or NULL = the plan's values of B_i */
    int32_t *C_rowidx;    /* int32[nnzC] of this product */
    void *C_vals;         /* dtype[nnzC] */
    int32_t dep_A;        /* index of an earlier product whose C is this A, or -1 */
    int32_t dep_B;        /* index of an earlier product whose C is this B, or -1 */
} spgemm_batch_io;

typedef struct spgemm_batch_s *spgemm_batch_t;

/*
 * spgemm_batched - the numeric phase of `count` planned products of one
 * dtype, as one launch DAG on `stream` (or one persistent launch, see
 * below):
 *   count    number of products (>= 1).
 *   plans    HOST array of `count` distinct plans that have all finished
 *            spgemm_symbolic.
 *   io       HOST array of `count` entries: per product the value inputs, the
 *            output buffers and the dependency indices (spgemm_batch_io).
 *            Dependencies point to lower indices; a product that reads
 *            another's C names it (dep_A/dep_B) and passes that C's value
 *            buffer as A_vals/B_vals.
 *   mode     0 enqueue the DAG's kernels directly;
 *            1 capture the DAG into a hipGraph, instantiate it and launch it;
 *            2 relaunch the graph captured by mode 1 for the same (plans, io)
 *              table (SPGEMM_ESTATE if there is none).
 *   stream   hipStream_t (NULL = null stream); side streams fork from it and
 *            join back, so every product has finished when `stream` reaches
 *            the end of the call.
 * The library keeps one batch per distinct (plans, io) table (built on first
 * use with the batch fields of plans[0]'s tuning: batch_streams and
 * batch_form (1: one persistent launch per run); that call
 * synchronises the plans' streams once) until one of its plans is
 * destroyed.  Runs of one table
 * must not overlap (they share the plans' A~ and scratch); work on the
 * plans' own streams is not ordered with the batch.  Errors: EINVAL (bad
 * table or mode, repeated plan), ESTATE (no symbolic, replay without
 * capture), EHIP.
 */
int spgemm_batched(int32_t count, const spgemm_plan_t *plans, const spgemm_batch_io *io,
                   int32_t mode, void *stream);

/*
 * The same batch with an explicit handle, for callers that choose its
 * tuning (batch_streams) or its lifetime: spgemm_batch_create validates the
 * table exactly as spgemm_batched does and synchronises the plans' streams
 * once; spgemm_batch_run takes spgemm_batched's mode and stream; the io
 * table is copied and the plans and buffers must outlive the batch.
 * With tuning.batch_form = 1 one run is ONE persistent launch: its
 * workgroups take the products' work items (value-gather tiles of A~,
 * numeric column groups) by an atomic ticket in dependency order and wait,
 * bounded in time, for the completion flags of the items they read; the
 * batch keeps a small control block (ticket, flags, error word) that the
 * launch puts back to 0, so runs and graph replays of one batch must not
 * overlap.  spgemm_batch_check then also reports (SPGEMM_EHIP) a run whose
 * dependency wait ran out of time (its outputs are not valid).
 * Errors of create: EINVAL, ESTATE, EUNSUPPORTED (batch_form = 1 and a
 * product with dense columns or tiny_max_flop > 256), EHIP.
 */
int spgemm_batch_create(int32_t count, const spgemm_plan_t *plans, const spgemm_batch_io *io,
                        const spgemm_tuning *tuning, spgemm_batch_t *out);

int spgemm_batch_run(spgemm_batch_t batch, int32_t mode, void *stream);

/* Side streams the batch uses, and kernels one run enqueues. */
int spgemm_batch_info(spgemm_batch_t batch, int64_t *streams, int64_t *launches);

/* Synchronises the device and returns SPGEMM_EHIP if a launch failed. */
int spgemm_batch_check(spgemm_batch_t batch);

int spgemm_batch_destroy(spgemm_batch_t batch);

/* ---------------------------------------------------------------------------
 * Outer-product form (Alg. 3): with the inner dimension split into row
 * blocks K_r of B, C = sum_r A(:, K_r) * B(K_r, :).  The two steps that move
 * data in Alg. 3 (row blocks of B to their owners; the partial results to
 * the owners of C for merging) are the two calls below; the partial
 * products and their sum run through spgemm_plan/symbolic/numeric.
 * ------------------------------------------------------------------------- */

/*
 * Row block B(r0:r1, :) of B (device CSC) with its global row ids, so that a
 * plan of A times it selects only columns r0..r1-1 of A.  Outputs (device,
 * caller-allocated): colptr_out int64[ncols+1]; rowidx_out int32 and vals_out
 * dtype with room for nnz(B) entries (the block's count ends up in
 * colptr_out[ncols]).  Asynchronous on `stream`.  Errors: EINVAL (NULL
 * arrays, 0 <= r0 <= r1 <= nrows violated), EHIP.
 */
int spgemm_row_block(const spgemm_csc *B, spgemm_dtype dtype, int64_t r0, int64_t r1,
                     int64_t *colptr_out, int32_t *rowidx_out, void *vals_out, void *stream);

/*
 * Stacks P partial results of one shape (m x n, host array of device CSCs)
 * side by side, stack = [C_0 ... C_{P-1}] (m x P*n: colptr int64[P*n+1],
 * row ids int32 and values dtype[sum of nnz]), and writes the selector
 * S = [I_n; ...; I_n] (P*n x n: colptr int64[n+1], row ids int32[P*n],
 * values dtype[P*n], all 1), so that stack * S = sum_r C_r.  All outputs are
 * device arrays the caller allocates.  Asynchronous on `stream`.  Errors:
 * EINVAL (P < 1, parts of different shapes, P*n >= 2^31, NULL arrays), EHIP.
 */
int spgemm_stack_parts(int32_t P, const spgemm_csc *parts, spgemm_dtype dtype,
                       int64_t *stack_colptr, int32_t *stack_rowidx, void *stack_vals,
                       int64_t *sel_colptr, int32_t *sel_rowidx, void *sel_vals, void *stream);

/* Releases every pooled device/host buffer not held by a live plan. */
int spgemm_pool_trim(void);

#ifdef __cplusplus
}
#endif

#endif /* SPGEMM_MI355X_H */
