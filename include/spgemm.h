/*
 * spgemm.h -- C ABI of libspgemm, a general sparse matrix-matrix
 * multiplication C = A*B on CSR matrices for AMD Instinct MI355X (gfx950).
 *
 * The method follows W. Liu and B. Vinter, "A Framework for General Sparse
 * Matrix-Matrix Multiplication on GPUs and Heterogeneous Processors"
 * (J. Parallel Distrib. Comput., extended version of IPDPS'14):
 *   stage 1  per-row upper bound u_i of nnz(c_i*) (Algorithm 2),
 *   stage 2  binning of the rows by u_i into 38 bins (Algorithm 3),
 *   stage 3  hybrid allocation of the temporary matrix C~ (u_i entries for
 *            short rows, 256 for long rows, progressive 2x growth beyond;
 *            long-row work that fits one tile writes to a place of its own
 *            instead, so that no work-group has to allocate) and the per-bin
 *            insert kernels (Section 3.1, "the third stage"),
 *   stage 4  arranging data: row pointers of C from the row sizes, then a
 *            copy of C~ into C (Section 3.1, "the fourth stage").
 * The output nnz is not known in advance (Section 3.1): analyze runs stages
 * 1-2 and sizes C~, compute runs stages 3-4 and allocates C through the
 * caller's allocator.
 *
 * Conventions for every entry point:
 *  - All matrix arrays are DEVICE pointers on the current HIP device.  Index
 *    arrays are int32; value arrays are binary32 or binary64 (spgemm_dtype).
 *    Inputs must have row_ptr[0] = 0, non-decreasing row_ptr and strictly
 *    increasing column indices inside each row (the paper assumes sorted
 *    columns, Section 2.3 footnote); with options.validate != 0 this is
 *    checked on the device and violations return SPGEMM_EINVAL.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    All device work is ordered on that stream.
 *  - Return value: SPGEMM_OK (0) or a negative spgemm_status.  On error no
 *    caller-owned memory is leaked or left half-written, and no C++
 *    exception crosses the boundary.
 *  - Memory: the library obtains device memory only through the caller's
 *    spgemm_alloc_fn / spgemm_free_fn (NULL pointers select the HIP
 *    stream-ordered allocator).  Inputs stay owned by the caller.  Plans own
 *    their scratch and release it in spgemm_plan_destroy.  Output arrays of C
 *    are allocated with alloc_fn and then belong to the caller.
 */
#ifndef SPGEMM_H
#define SPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPGEMM_OK = 0,
  SPGEMM_EINVAL = -1,    /* bad argument, shape or dtype mismatch, invalid CSR */
  SPGEMM_ENOMEM = -2,    /* alloc_fn returned NULL                              */
  SPGEMM_EOVERFLOW = -3, /* nnz(C) or another count does not fit the index type */
  SPGEMM_EHIP = -4,      /* HIP runtime error (spgemm_last_error has details)   */
  SPGEMM_ESTATE = -5     /* plan used with matrices other than those analyzed   */
} spgemm_status;

typedef enum { SPGEMM_F32 = 0, SPGEMM_F64 = 1 } spgemm_dtype;

/* A borrowed CSR view (the library never frees it).  rows x cols, nnz
 * entries: row_ptr[rows+1], col_idx[nnz], val[nnz] of `dtype`. */
typedef struct {
  int64_t rows, cols, nnz;
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const void *val;
  int32_t dtype;
} spgemm_csr;

/* An output CSR.  The three arrays are allocated by the library through the
 * caller's alloc_fn and owned by the caller afterwards. */
typedef struct {
  int64_t rows, cols, nnz;
  int32_t *row_ptr;
  int32_t *col_idx;
  void *val;
  int32_t dtype;
} spgemm_csr_out;

/* Device allocator: return `bytes` of device memory usable in stream order on
 * `stream`, or NULL on failure.  free_fn releases a pointer from alloc_fn. */
typedef void *(*spgemm_alloc_fn)(size_t bytes, void *ctx, void *stream);
typedef void (*spgemm_free_fn)(void *ptr, void *ctx, void *stream);

/* Tuning knobs.  spgemm_default_options() gives the paper's settings
 * (Algorithm 3 thresholds, 256-entry long-row slot, 2x growth).  None of
 * them changes the structure of C.  Every column is summed in the order of
 * Gustavson's algorithm (ascending j) except (a) long-row work that goes
 * through the level-1 merge method (work items or output column ranges of
 * more than 4096 entries, or seg < 0) and (b) with column windows, long
 * rows of more than 16384 products when B has at most 2048 (binary64) /
 * 4096 (binary32) columns, which are cut into product ranges: there
 * partial sums are added in a fixed order that may round differently. */
typedef struct {
  /* upper row sizes of: the single-size bins (group 3, default 32), then the
   * four range bins of group 4 (defaults 64, 128, 256, 512).  Rows above the
   * last edge form bin 37 (group 5).  Strictly increasing, edge[0] in
   * [1, 32], edge[4] <= 1024. */
  int32_t bin_edges[5];
  int32_t long_slot;    /* C~ entries reserved per long row (default 256)     */
  int32_t l1_cap;       /* level-1 (LDS) sequence entries of the long-row
                           kernel, 0 = automatic                              */
  int64_t seg;          /* max products per long-row work item (rows with
                           more are split across work-groups); 0 = automatic
                           (rows up to 1024 stay whole, longer ones are cut
                           into 512), < 0 = never split                      */
  int64_t pool_entries; /* initial long-row pool size in entries, 0 = auto   */
  int32_t validate;     /* nonzero: check the input CSR arrays on the device  */
  int32_t timing;       /* nonzero: record per-stage times into spgemm_info   */
  int32_t timing_mask;  /* with timing: 0 times every stage, else only the
                           stages whose bit (1 << SPGEMM_T_x) is set.  Every
                           timed stage adds two event records to the stream,
                           and spgemm_compute waits for the end of the last
                           timed stage before it returns                     */
  int32_t tiny_heap;    /* nonzero: rows of sizes 2..bin_edges[0] use the
                           paper's heap method (one thread per row, one
                           kernel per exact size) instead of the wavefront
                           ESC; duplicates are then added in heap order, so
                           values may round differently (plain path only)   */
  int32_t long_path;    /* method for long rows (bin 37):
                           0 = automatic (default): column windows when B
                             has at most 2048 (binary64) / 4096 (binary32)
                             columns -- every long row then sums into one
                             dense window of LDS -- else method 1;
                           1 = product segments and column ranges, with the
                             paper's merge method as fallback (also what
                             seg != 0 selects);
                           2 = column windows: each long row is cut into
                             windows of columns, sized by a symbolic pass
                             and written straight into C                     */
  int32_t long_direct;  /* merge method only: 0 = results of split long rows
                           go to a range buffer of u_i entries per row and
                           are copied into C (default, faster); 1 = a
                           counting pass sizes them first and they are
                           written straight into C (no range buffer: less
                           device memory, about 5% slower on workload 2)   */
  int32_t batch_shapes; /* batched form: 0 = the autotuner picks the tile-shape
                           set (default); 1..3 = shape set 0..2 fixed         */
  int32_t pad_;
} spgemm_options;

#define SPGEMM_NBINS 38
#define SPGEMM_NSTAGES 12

/* Per-stage timer slots of spgemm_info.stage_ms (options.timing != 0). */
enum {
  SPGEMM_T_UPPER = 0,   /* stage 1: upper bounds and scan                    */
  SPGEMM_T_BIN = 1,     /* stage 2: binning, C~ offsets                      */
  SPGEMM_T_TINY = 2,    /* stage 3: rows with u <= edge[0]                   */
  SPGEMM_T_MEDIUM = 3,  /* stage 3: rows in the four range bins              */
  SPGEMM_T_LONG = 4,    /* stage 3: long rows (all relaunch rounds); window
                           method: planning, partition and symbolic pass  */
  SPGEMM_T_SCAN = 5,    /* stage 4: row pointers of C                        */
  SPGEMM_T_COPY = 6,    /* stage 4: copy C~ into C                           */
  SPGEMM_T_BACKWARD = 7,/* backward kernels (not read back by compute)       */
  SPGEMM_T_LONG_WAVE = 8,    /* inside LONG: the one-wavefront segment kernel;
                                window method: the partition kernel          */
  SPGEMM_T_COMBINE = 9,      /* stage 3: column ranges of split long rows;
                                window method: the numeric pass into C       */
  SPGEMM_T_COMBINE_WAVE = 10,/* inside COMBINE: the one-wavefront range kernel;
                                window method: the numeric window kernel     */
  SPGEMM_T_LONG_SYM = 11     /* window method: the symbolic window kernel     */
};

typedef struct {
  int64_t m, k, n;
  int64_t flops;        /* 2 * sum(u_i) (Table 2 caption)                     */
  int64_t nnz_hat;      /* sum(u_i) = nnz of the expanded matrix             */
  int64_t nnz_tilde;    /* sum of C~ row sizes (Algorithm 3)                 */
  int64_t nnz_c;        /* nnz(C), after compute                             */
  int64_t max_u;
  int64_t bin_count[SPGEMM_NBINS];
  int64_t long_items;   /* long-row work items after splitting               */
  int64_t bytes_scratch;/* most device memory the plan held at once during
                           the latest call, as requested from the allocator:
                           analysis arrays, C~ with the long-row tables and
                           pool (compute), A's transposed pattern and the
                           staged products (backward); C itself excluded    */
  int64_t pool_entries; /* long-row pool capacity at the end of compute      */
  int64_t pool_used;    /* entries taken from the pool                       */
  int32_t realloc_rounds; /* pool exhaustions handled by relaunching         */
  int32_t reserved;
  float stage_ms[SPGEMM_NSTAGES]; /* 0 for stages that did not run        */
  float long_kernel_ms; /* summed duration of the long-row kernel launches   */
  int32_t long_launches;
} spgemm_info;

typedef struct spgemm_plan_s *spgemm_plan;

/* Fill `opt` with the defaults described above. */
void spgemm_default_options(spgemm_options *opt);

/* Human-readable text of a status code (static storage). */
const char *spgemm_strerror(int code);

/* Detail of the last SPGEMM_EHIP / SPGEMM_EINVAL raised in this thread. */
const char *spgemm_last_error(void);

/*
 * Stages 1-2 (Algorithms 2 and 3) plus the sizing of C~ (hybrid allocation,
 * Section 3.1).  Computes u_i for every row of C, bins the rows and reserves
 * the plan's scratch; synchronizes `stream` once to read back a small
 * summary (sums, bin counts).  A: m x k, B: k x n, same dtype.  The plan
 * remembers the pointers and sizes of A's and B's index arrays; later calls
 * must pass the same matrices (values may change).  `opt` may be NULL
 * (defaults); `info` may be NULL.  On success *plan is a new plan.
 */
int spgemm_analyze(const spgemm_csr *A, const spgemm_csr *B, const spgemm_options *opt,
                   spgemm_alloc_fn alloc_fn, spgemm_free_fn free_fn, void *ctx,
                   void *stream, spgemm_plan *plan, spgemm_info *info);

/*
 * Stages 3-4: computes every row of C into C~ (bin groups 1-5 with their
 * own kernels), sums the row sizes into C's row pointers, allocates C's
 * column and value arrays (exactly nnz(C) entries) with the plan's allocator
 * and copies C~ into C.  Synchronizes `stream` once to read nnz(C), plus once
 * more per exhaustion of the long-row pool (the pool then grows 2x and the
 * affected long rows resume from their checkpoints).  C receives rows = m,
 * cols = n, nnz, three owned arrays and A's dtype.  Entries of every row are
 * in ascending column order without duplicates; structural products that
 * cancel are kept.
 */
int spgemm_compute(spgemm_plan plan, const spgemm_csr *A, const spgemm_csr *B,
                   spgemm_csr_out *C, void *stream, spgemm_info *info);

/*
 * Gradient of L = <dC, A*B> for the values of A and B on their fixed
 * patterns: dA_ij = sum_k dC_ik b_jk over the stored b_jk (= (dC B^T) on
 * S(A)), dB_jk = sum_i a_ij dC_ik over the stored a_ij (= (A^T dC) on S(B)).
 * `C` must be the result of spgemm_compute for this plan, with C->val holding
 * dC (same pattern as C, A's dtype).  dA_val (nnz(A) entries) or dB_val
 * (nnz(B) entries) may be NULL to skip them.  Device pointers.  Fully
 * asynchronous on `stream`.
 */
int spgemm_backward(spgemm_plan plan, const spgemm_csr *A, const spgemm_csr *B,
                    const spgemm_csr *C, void *dA_val, void *dB_val, void *stream);

/*
 * spgemm_backward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight training loops, harnesses that forbid allocation.
 * Arguments, results and ordering as for spgemm_backward.  The scratch it
 * needs lives in a fixed device area of SPGEMM_STATIC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends; nothing is
 * allocated or freed.  With dB wanted, A's transposed pattern takes
 * 4 k + 8 (k + 1) + 8 nnz(A) bytes plus a scan area of about k / 128
 * entries (k = A's columns): SPGEMM_EINVAL when that exceeds the area.  The
 * products of the dB sums (nnz(hat C) values) are staged beside it when they
 * fit, else dB is summed without staging (the same products in the same
 * order, so the same values).  Every call on one GPU uses the same area:
 * calls that overlap on one GPU (other streams, other host threads) race and
 * must be ordered by the caller.
 */
#define SPGEMM_STATIC_SCRATCH_BYTES (64u << 20)
int spgemm_backward_static(spgemm_plan plan, const spgemm_csr *A, const spgemm_csr *B,
                           const spgemm_csr *C, void *dA_val, void *dB_val, void *stream);

/* Fill `info` with the plan's latest statistics. */
int spgemm_plan_info(spgemm_plan plan, spgemm_info *info);

/* Release the plan and its scratch (ordered on the plan's last stream). */
int spgemm_plan_destroy(spgemm_plan plan);

/*
 * C = A*B in one call (stages 1-4 of Section 3.1): spgemm_analyze, then
 * spgemm_compute, then spgemm_plan_destroy, without returning to the caller
 * in between.  Arguments, outputs, ownership and synchronisation as for those
 * three calls; `opt` and `info` may be NULL.  On failure no plan survives and
 * C is untouched.
 */
int spgemm_multiply(const spgemm_csr *A, const spgemm_csr *B, const spgemm_options *opt,
                    spgemm_alloc_fn alloc_fn, spgemm_free_fn free_fn, void *ctx, void *stream,
                    spgemm_csr_out *C, spgemm_info *info);

/* ------------------------------------------------------------------------
 * Batched products (extension beyond the paper): many independent
 * C_p = A_p * B_p of uneven sizes and mixed binary32/binary64 values,
 * computed by one HIP graph of one kernel launch per capacity class.
 */
typedef struct spgemm_batch_s *spgemm_batch;

typedef struct {
  int32_t count;        /* problems                                           */
  int32_t fallback;     /* problems recomputed with the plain path per run    */
  int32_t grid;         /* kernel launches in the graph (nonempty classes)    */
  int32_t shapes;       /* tile-shape set chosen by the autotuner: 0 = the
                           plain path's (G lanes, K products per lane) per
                           capacity, 1 = wider groups, 2 = narrower groups   */
  int64_t items;        /* work items (one work-group each)                   */
  int64_t flops;        /* sum of 2 * sum(u_i) over the problems              */
  int64_t nnz_c;        /* sum of nnz(C_p)                                    */
  int32_t bin_edges[5]; /* thresholds chosen by the autotuner                 */
  float tune_ms[12];    /* timed candidates (ms per run): threshold set t and
                           shape set k at [3 t + k]; 0 where not timed       */
  int64_t bytes_scratch;/* spgemm_batch_multiply: most device memory it held
                           at once besides the outputs (analysis arrays, C~,
                           items, a fallback problem's plain-path peak); 0
                           for a graph-replayed batch                        */
} spgemm_batch_stats;

/*
 * Analyze `count` problems (A[p], B[p]: borrowed CSR views that must stay
 * valid, with unchanged patterns, for the batch's lifetime; values may
 * change between runs), compute every C_p once, allocate the outputs with
 * alloc_fn, tune the bin thresholds (unless opt sets non-default ones) by
 * timing the batched kernel, and capture the graph.  Rows with more than
 * 1024 products (or n_p * 1024 >= 2^32) make their problem fall back to the
 * plain path inside spgemm_batch_run.  Synchronizes `stream`.
 */
int spgemm_batch_create(int32_t count, const spgemm_csr *A, const spgemm_csr *B,
                        const spgemm_options *opt, spgemm_alloc_fn alloc_fn,
                        spgemm_free_fn free_fn, void *ctx, void *stream, spgemm_batch *batch,
                        spgemm_batch_stats *stats);

/* Recompute every C_p (structure and values) by replaying the graph on
 * `stream`; asynchronous unless problems fall back to the plain path.  If C
 * is not NULL it receives `count` views of the outputs, which stay owned by
 * the batch: valid until spgemm_batch_destroy, except that a fallback
 * problem receives new arrays on every run (its previous ones are released
 * with free_fn, in stream order). */
int spgemm_batch_run(spgemm_batch batch, spgemm_csr_out *C, void *stream);

int spgemm_batch_stats_get(spgemm_batch batch, spgemm_batch_stats *stats);

/* Release the graph, the plans and the outputs. */
int spgemm_batch_destroy(spgemm_batch batch);

/*
 * One-shot batched products for problems seen once (no plan is kept):
 * every stage for all `count` problems at once.  Stage 1 (Algorithm 2)
 * runs over the concatenated entries and rows of every problem in single
 * launches; one read-back of the per-problem row counts of each capacity
 * class (2^c products, c = 0..10) sizes C~ with u_i entries per row (the
 * hybrid allocation of Section 3.1) and the class lists (stage 2,
 * Algorithm 3, with power-of-two bins); the wavefront ESC runs once per
 * class over the rows of every problem; a scan of the row sizes and a
 * second read-back size the outputs; one launch compacts every C_p
 * (stage 5).  Problems with a row above 1024 products, or with
 * n_p * 1024 >= 2^32, go through the plain path (spgemm_multiply) instead
 * and are counted in stats->fallback.
 *
 * opt: checked as for spgemm_analyze; batch_shapes picks the tile-shape set
 * (0 = set 0, the plain path's shapes; no autotuning here).  Outputs: C[p]
 * (count entries) describe C_p, whose three arrays all lie in one device
 * block from alloc_fn (hipMallocAsync when alloc_fn is NULL) returned in
 * *out_mem; the caller owns it and releases every C_p at once with free_fn
 * (hipFreeAsync).  *out_mem is NULL when count is 0 or on error (nothing
 * stays allocated then).  Every C_p equals spgemm_multiply's bit for bit
 * (same structure; each sum in the same (column, product index) order).
 * Synchronizes `stream` twice; the scratch is released in stream order
 * before returning.
 */
int spgemm_batch_multiply(int32_t count, const spgemm_csr *A, const spgemm_csr *B,
                          const spgemm_options *opt, spgemm_alloc_fn alloc_fn,
                          spgemm_free_fn free_fn, void *ctx, void *stream, spgemm_csr_out *C,
                          void **out_mem, spgemm_batch_stats *stats);

/*
 * Merge-algorithm microbenchmark (Section 3.2, Fig. 5): merge `pairs`
 * pairs of sorted sequences, each pair stored as 2l consecutive entries
 * (first sequence, then second, both ascending), into ascending order, in
 * LDS, with one of the five algorithms the paper compares.  Keys are 32-bit
 * unsigned; value_bytes = 0 (keys only), 4 or 8 (a value moves with each
 * key).  l is a power of two; `threads` (64..1024, a power of two) is the
 * work-group size, and a work-group merges max(2l, 2 threads) entries.
 * Ranking merge and merge path keep entries of the first sequence first
 * among equal keys; the networks may order equal keys either way.  Device
 * pointers; outputs must not overlap inputs.  Returns SPGEMM_EINVAL when the
 * tile does not fit in 160 KB of LDS or when merge path would hold more
 * than 32 outputs per thread.  Asynchronous on `stream`.
 */
enum {
  SPGEMM_MERGE_RANKING = 0,     /* ranking merge (out of place)              */
  SPGEMM_MERGE_PATH = 1,        /* merge path                                 */
  SPGEMM_MERGE_ODDEVEN = 2,     /* Batcher's odd-even merging network         */
  SPGEMM_MERGE_BITONIC = 3,     /* bitonic merging network                    */
  SPGEMM_MERGE_BITONIC_ADV = 4  /* bitonic, three stages per register pass    */
};
int spgemm_merge_pairs(int algorithm, int value_bytes, int64_t l, int64_t pairs, int threads,
                       const uint32_t *keys_in, const void *vals_in, uint32_t *keys_out,
                       void *vals_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPGEMM_H */
