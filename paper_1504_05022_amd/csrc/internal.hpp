// Internal declarations shared by the host orchestration (api.hip) and the
// kernel translation units: device-visible records and launcher entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spgemm.h"

namespace spg {

constexpr int NBINS = SPGEMM_NBINS;  // 38 bins in five groups (Algorithm 3)
constexpr int LONG_BIN = NBINS - 1;  // bin 37: group 5

// Bin thresholds: edge[0] is the largest single-size bin (group 3),
// edge[1..4] the upper ends of the four range bins of group 4.
struct BinEdges {
  int32_t e[5];
};

// Bin of a row with upper bound u (Algorithm 3, generalised thresholds).
__host__ __device__ inline int bin_of(int64_t u, const BinEdges &be) {
  if (u <= 0) return 0;
  if (u == 1) return 1;
  if (u <= be.e[0]) return static_cast<int>(u);
  if (u <= be.e[1]) return 33;
  if (u <= be.e[2]) return 34;
  if (u <= be.e[3]) return 35;
  if (u <= be.e[4]) return 36;
  return LONG_BIN;
}

// Written by the analyze kernels, read back once by the host.
struct Summary {
  int64_t sum_u;              // nnz of the expanded matrix, sum of u_i
  int64_t sum_h;              // nnz(C~)
  unsigned long long max_u;   // largest u_i
  int64_t bin_off[NBINS + 1]; // start of every bin's segment in the row list
  int64_t sum_u_long;         // sum of u_i over long rows (bin 37)
  int64_t sum_r_long;         // sum of min(u_i, n) over long rows
  int32_t err;                // nonzero: input validation failed
  int32_t pad;
};

// A long-row work item: products [p0, p1) of row `row` (positions in the
// row's expansion order: ascending j, then ascending k inside b_j*).
struct LongItem {
  int32_t row;
  int32_t part;  // index of this piece within its row (0 if unsplit)
  int64_t p0, p1;
};

// Checkpoint of a long-row work item (resumable after pool exhaustion).
struct LongState {
  int64_t pos;       // next product to process; L1 is empty at this point
  int64_t gcnt;      // entries in the global result block G
  int64_t gcap;      // capacity of G
  int32_t *gcol;     // G (pool block) or nullptr
  void *gval;
  int64_t scap;      // capacity of the spare block (previous G) or 0
  int32_t *scol;
  void *sval;
  int32_t status;    // 0 running/done, 1 failed (checkpointed)
  int32_t pad;
};

// Long-row result pool: blocks are carved with an atomic bump pointer.
struct Pool {
  int32_t *col;
  void *val;
  unsigned long long cap;     // entries
  unsigned long long top;     // next free entry (atomic)
  unsigned int fail_count;    // work items that failed to obtain a block
  unsigned int pad;
  unsigned long long used;    // entries handed out successfully
};

// Small block of device counters read back by compute.
struct ComputeStatus {
  int64_t nnz_c;
  unsigned int fail_count;
  unsigned int pad;
  unsigned long long pool_used;
};

// ----------------------------------------------------------------- scans

// Exclusive scan of v[0..n) into out[0..n], out[n] = total (int64).  Input
// is produced by one of the functors below.  `part` needs scan_part_len(n)
// int64 entries.
int64_t scan_part_len(int64_t n);

// w_e = nnz(b_{acol[e]*}), the per-entry term of Algorithm 2.
void scan_row_lengths(const int32_t *acol, const int32_t *brp, int64_t n, int64_t *out,
                      int64_t *part, hipStream_t s);
// Plain int64 arrays (hybrid row sizes, row nnz, histograms).
void scan_i64(const int64_t *v, int64_t n, int64_t *out, int64_t *part, hipStream_t s);
void scan_i32(const int32_t *v, int64_t n, int64_t *out, int64_t *part, hipStream_t s);

// ------------------------------------------------------------- analyze

void launch_validate(const int32_t *rp, const int32_t *ci, int64_t rows, int64_t cols,
                     int64_t nnz, Summary *sum, hipStream_t s);

// Stage 1 per row: u_i from the scanned row lengths, C~ row sizes, bin
// histograms per wavefront; zeroes nnz of empty rows.
void launch_row_stats(const int32_t *arp, const int64_t *P, int64_t m, int64_t ncols,
                      BinEdges be, int32_t long_slot, int64_t *u, int64_t *h, int32_t *hist,
                      int64_t nwaves, int64_t *rownnz, Summary *sum, hipStream_t s);
// Stable scatter of the rows into their bins.
void launch_bin_scatter(const int64_t *u, int64_t m, BinEdges be, const int64_t *hist_scan,
                        int64_t nwaves, int32_t *binlist, hipStream_t s);
void launch_summary(const int64_t *P, int64_t nnzA, const int64_t *cto, int64_t m,
                    const int64_t *hist_scan, int64_t nwaves, Summary *sum, hipStream_t s);

// ------------------------------------------------------------- compute

template <typename T> struct EscArgs {
  const int32_t *arp, *acol;
  const T *aval;
  const int32_t *brp, *bcol;
  const T *bval;
  const int64_t *P;       // scanned row lengths (Algorithm 2 partial sums)
  const int64_t *u;
  const int64_t *cto;     // C~ row offsets
  int32_t *ct_col;        // C~
  T *ct_val;
  int64_t *rownnz;
};

// Rows of one capacity class (u <= cap, cap a power of two <= 1024) with
// the wavefront-level expand-sort-compress kernel.
template <typename T>
int launch_esc(const EscArgs<T> &a, const int32_t *rows, int64_t nrows, int cap, int64_t ncols,
               hipStream_t s);

template <typename T> struct LongArgs {
  EscArgs<T> e;
  const LongItem *items;
  const int32_t *work;    // item ids to process
  LongState *state;
  Pool *pool;
  unsigned int *fail_list;
  int32_t long_slot;
  int32_t **rsrc_col;     // per row: where the long row's result lives
  T **rsrc_val;
};

template <typename T>
int launch_long(const LongArgs<T> &a, int64_t nwork, int64_t ncols, int l1cap, hipStream_t s);
int long_l1cap_default(int dtype_bytes);
void launch_long_init(const LongItem *items, LongState *state, int64_t n, hipStream_t s);
void launch_long_items(const int32_t *binlist, int64_t off, int64_t n, const int64_t *u,
                       LongItem *items, hipStream_t s);

template <typename T> struct CompactArgs {
  const int64_t *u;
  const int64_t *cto;
  const int32_t *ct_col;
  const T *ct_val;
  int32_t *const *rsrc_col;
  T *const *rsrc_val;
  const int64_t *rowoff;  // exclusive scan of rownnz, m+1
  int64_t long_min;       // rows with u > long_min take rsrc
  int32_t *c_rp;
  int32_t *c_col;
  T *c_val;
};
template <typename T> void launch_compact(const CompactArgs<T> &a, int64_t m, hipStream_t s);

void launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);

// ------------------------------------------------------------- backward
// A^T pattern (per column j of A: rows i ascending and entry positions)
void launch_transpose_pattern(const int32_t *arp, const int32_t *acol, int64_t m, int64_t k,
                              int64_t nnz, int32_t *cnt, int64_t *tptr, int32_t *trow,
                              int32_t *tpos, int64_t *part, hipStream_t s);
template <typename T>
void launch_grad_a(const int32_t *arp, const int32_t *acol, int64_t m, const int32_t *brp,
                   const int32_t *bcol, const T *bval, const int32_t *crp, const int32_t *ccol,
                   const T *dc, T *dA, hipStream_t s);
template <typename T>
void launch_grad_b(const int64_t *tptr, const int32_t *trow, const int32_t *tpos, const T *aval,
                   const int32_t *brp, const int32_t *bcol, int64_t kb, const int32_t *crp,
                   const int32_t *ccol, const T *dc, T *dB, hipStream_t s);
void launch_zero(void *p, size_t bytes, hipStream_t s);
void launch_status(const int64_t *rowoff, int64_t m, const Pool *pool, ComputeStatus *st,
                   hipStream_t s);

}  // namespace spg
