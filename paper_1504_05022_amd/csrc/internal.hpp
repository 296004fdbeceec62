// Internal declarations shared by the host orchestration (api.hip) and the
// kernel translation units: device-visible records and launcher entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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
  int64_t n_items;            // long-row work items
  int64_t n_pieces;           // long-row output pieces
  int64_t sum_u_multi;        // output space of the one-tile paths: u_i of split rows plus
                              // min(u_i, n) of one-item rows with u_i <= kOneShot
  int64_t n_split;            // range-start table entries (multi-item rows)
  int64_t pool_single;        // pool entries for final blocks of one-item rows above kOneShot
  int64_t sum_r_multi;        // sum of min(u_i, n) over multi-item rows
  int64_t spill_bound;        // sum of min(segment, n) over items that may spill L1
  int64_t w_items;            // window path: items
  int64_t w_segs;             // window path: partition segments
  int64_t w_table;            // window path: piece-start table entries
  int64_t w_partial;          // window path: partial entries
  int64_t w_dslots;           // window path: dense partial rows
  int64_t w_none;             // long rows without a window plan
  int32_t err;                // nonzero: input validation failed
  int32_t pad;
};

// Splitting of long rows (bin 37) into work items and output pieces.
//  * a row with u products is cut into nseg product segments of at most segp
//    consecutive products (expansion order); each segment is one work item
//    of the merge-method kernel and yields a sorted, duplicate-free partial;
//  * a row with one segment is finished by that item (one output piece);
//  * a row with several segments is finished by combine work-groups, one
//    per column range of width 2^shift (npiece ranges), each folding the
//    ranges of all partials in segment order into one output piece.
struct LongParams {
  int64_t segp;      // products per segment; < 0: never split
  int64_t single;    // rows with at most this many products stay one item
  int32_t maxs;      // at most this many segments per row (segp grows)
  int32_t cb;        // target entries per combine range
  int32_t minw_shift;
  int32_t maxw_shift;  // combine ranges are at most the level-1 capacity
};

__host__ __device__ inline int32_t ceil_log2_i64(int64_t x) {
  int32_t s = 0;
  while ((int64_t(1) << s) < x) ++s;
  return s;
}

__host__ __device__ inline void long_row_plan(int64_t u, int64_t n, const LongParams &lp,
                                              int64_t &segp, int32_t &nseg, int32_t &shift,
                                              int32_t &npiece) {
  if (lp.segp < 0 || u <= lp.segp || u <= lp.single) {
    segp = u > 0 ? u : 1;
    nseg = 1;
    shift = 0;
    npiece = 1;
    return;
  }
  segp = lp.segp;
  const int64_t need = (u + lp.maxs - 1) / lp.maxs;
  if (need > segp) segp = need;
  nseg = static_cast<int32_t>((u + segp - 1) / segp);
  if (nseg <= 1) {
    segp = u;
    nseg = 1;
    shift = 0;
    npiece = 1;
    return;
  }
  const int64_t w = (n * lp.cb + u - 1) / u;
  shift = ceil_log2_i64(w > 1 ? w : 1);
  if (shift < lp.minw_shift) shift = lp.minw_shift;
  if (shift > lp.maxw_shift) shift = lp.maxw_shift;
  npiece = static_cast<int32_t>((n + (int64_t(1) << shift) - 1) >> shift);
  if (npiece < 1) npiece = 1;
}

// ------------------------------------------------- window path (long rows)
// Column windows (long_path 2, and the default when B has at most a dense
// window of columns) compute each long row of C in windows of columns
// ("items").  A symbolic pass sizes every item first, so the numeric pass
// writes straight into C.  Three row plans:
//  * DIRECT DENSE: n <= the dense window (2048 binary64 / 4096 binary32
//    columns): the whole row is one window, a dense accumulator in LDS that
//    one wavefront updates in expansion order; rows above kWinSplit
//    products are cut into product ranges whose dense partial rows are
//    added in range order afterwards (a fixed order, not Gustavson's);
//  * DIRECT SPARSE: u <= kWinDirect: one item, products gathered straight
//    from the B rows, ordered by a counting sort in LDS and folded in
//    Gustavson's order by one wavefront;
//  * PARTITIONED: the row's products are cut into segments of kWinSeg,
//    each segment scatters its products stably (expansion order kept inside
//    every bucket) by column piece (2^shift columns) into a partial array
//    and records where every piece starts (a piece-start table); a piece
//    then gathers its share of every segment, in segment order, and is one
//    item, finished like a direct sparse row.  A piece with more products
//    than a wavefront stages goes to a work-group kernel, which sweeps it in
//    dense sub-windows.
constexpr int kWinStage = 1024;     // products staged in LDS per wavefront item
constexpr int kWinSeg = 512;        // products per partition segment
constexpr int kWinTarget = 512;     // expected products per piece
constexpr int kWinDirect = 1024;    // direct sparse rows: at most this many products
constexpr int kWinBitmapLog = 18;   // pieces are at most 2^18 columns wide
constexpr int kWinSplit = 16384;    // direct dense rows: products per item
constexpr int kWinMaxPieces = 1024; // pieces per partitioned row
constexpr int kWinBuckets = 512;    // buckets of the wavefront counting sort
constexpr int kWinBucketLog = 9;

enum { WIN_DS = 0, WIN_DD = 1, WIN_PT = 2, WIN_NONE = 3 };

// log2 of the dense window width: its accumulator (value per column) and
// counters fill the same LDS budget for both value types
__host__ __device__ inline int win_dense_log(int vbytes) { return vbytes == 8 ? 11 : 12; }

struct WinPlan {
  int32_t mode;    // WIN_DS, WIN_DD, WIN_PT, or WIN_NONE (no window plan)
  int32_t nitem;   // items of the row
  int32_t shift;   // WIN_PT: log2 of the piece width
  int32_t nseg;    // WIN_PT: segments
  int64_t table;   // WIN_PT: entries of the piece-start table, (nitem + 1) * nseg
  int64_t partial; // WIN_PT: partial entries (u)
  int64_t dslots;  // WIN_DD with several items: dense partial rows
};

__host__ __device__ inline WinPlan win_plan(int64_t u, int64_t n, int vbytes) {
  WinPlan p{};
  p.mode = WIN_NONE;
  if (u <= 0) return p;
  const int dl = win_dense_log(vbytes);
  if (n <= (int64_t(1) << dl)) {
    p.mode = WIN_DD;
    p.nitem = static_cast<int32_t>((u + kWinSplit - 1) / kWinSplit);
    p.dslots = p.nitem > 1 ? p.nitem : 0;
    return p;
  }
  if (u <= kWinDirect) {
    p.mode = WIN_DS;
    p.nitem = 1;
    return p;
  }
  // widest power of two that holds at most kWinTarget products on average
  const int64_t w = n * kWinTarget / u;
  int32_t sh = 0;
  while ((int64_t(2) << sh) <= w) ++sh;
  if (sh > kWinBitmapLog) sh = kWinBitmapLog;
  int64_t R = (n + (int64_t(1) << sh) - 1) >> sh;
  while (R > kWinMaxPieces && sh < kWinBitmapLog) {  // wider pieces, fewer of them
    ++sh;
    R = (n + (int64_t(1) << sh) - 1) >> sh;
  }
  if (R > kWinMaxPieces) return p;  // column space too wide for this plan
  p.mode = WIN_PT;
  p.nitem = static_cast<int32_t>(R);
  p.shift = sh;
  p.nseg = static_cast<int32_t>((u + kWinSeg - 1) / kWinSeg);
  p.table = static_cast<int64_t>(p.nseg) * (R + 1);
  p.partial = u;
  return p;
}

struct WinRow {
  int32_t row;
  int32_t mode;
  int32_t nitem;
  int32_t shift;
  int32_t nseg;
  int32_t pad;
  int64_t u;
  int64_t item0;   // first item
  int64_t seg0;    // WIN_PT: first segment
  int64_t pbase;   // WIN_PT: first partial entry
  int64_t tbase;   // WIN_PT: first piece-start table entry
  int64_t dslot0;  // WIN_DD with several items: first dense partial row
};

// An item (k-th of its row) or a segment (k-th of its row) of the window
// path; e0 is the entry of A holding the item's / segment's first product
// (direct dense product ranges and segments).
struct WinWork {
  int32_t wrow;
  int32_t k;
  int32_t e0;
  int32_t pad;
};

struct LongRow {
  int32_t row;
  int32_t nseg;
  int32_t npiece;
  int32_t shift;
  int64_t u;
  int64_t segp;
  int64_t item0;   // first work item
  int64_t piece0;  // first output piece
  int64_t pbase;   // offset of the row's partials (multi-segment rows)
  int64_t sbase;   // offset of the row's range-start table (multi-segment rows)
};

// A long-row work item: products [p0, p1) of row `row` (positions in the
// row's expansion order: ascending j, then ascending k inside b_j*).
struct LongItem {
  int32_t row;
  int32_t lrow;     // index in the long-row table
  int64_t p0, p1;
  int32_t e_first;  // entry of A's row containing product p0
  int32_t pad;
};

// Work the one-tile kernels leave to the general kernels.
struct LongCounters {
  unsigned int glong;  // items for the general kernel
  unsigned int gcomb;  // pieces for the general combine kernel
  unsigned int l1;     // items for the one-tile work-group kernel
  unsigned int l2;     // pieces for the second wavefront combine pass
  unsigned int l3;     // pieces for the one-tile work-group combine kernel
  unsigned int lw;     // items for the second wavefront pass
};

// Sorted, duplicate-free sequence in device memory.
struct Seq {
  int32_t *col;
  void *val;
  int64_t cnt;
};

// One output piece of a long row: `cnt` entries to be copied to C at
// row offset + (pieces of the same row before it).
struct Piece {
  int32_t *col;
  void *val;
  int64_t cnt;
  int32_t lrow;
  int32_t pad;
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
  unsigned int fail_count;    // phase-1 work items that failed to obtain a block
  unsigned int fail2;         // combine pieces that failed to obtain a block
  unsigned long long used;    // entries handed out successfully
};

// Small block of device counters read back by compute.
struct ComputeStatus {
  int64_t nnz_c;
  unsigned int fail_count;
  unsigned int fail2;
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
struct RowStatsArgs {
  const int32_t *arp;
  const int64_t *P;
  int64_t m, ncols;
  BinEdges be;
  int32_t long_slot;
  int32_t l1cap;
  int32_t vbytes;  // value size (window plan)
  LongParams lp;
  int64_t *u, *h;
  int32_t *hist;
  int64_t nwaves;
  int64_t *rownnz;
  int64_t *bpart;  // per-block partial sums, kBlockStats per block
};
// per block: max u, sum u (long), sum min(u,n) (long), items, pieces,
// sum u (multi), split entries, pool (single), sum min(u,n) (multi), spill,
// then the window plan: items, segments, table entries, partial entries,
// dense partial rows, rows without a window plan
constexpr int kBlockStats = 16;
void launch_row_stats(const RowStatsArgs &a, hipStream_t s);
// Stable scatter of the rows into their bins.
void launch_bin_scatter(const int64_t *u, int64_t m, BinEdges be, const int64_t *hist_scan,
                        int64_t nwaves, int32_t *binlist, hipStream_t s);
void launch_summary(const int64_t *P, int64_t nnzA, const int64_t *cto, int64_t m,
                    const int64_t *hist_scan, int64_t nwaves, const int64_t *bpart,
                    int64_t nblocks, Summary *sum, hipStream_t s);

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

// Rows of one exact size 2..32 with the paper's one-thread heap method
// (bin group 3); returns -1 for other sizes.
template <typename T>
int launch_heap(const EscArgs<T> &a, const int32_t *rows, int64_t nrows, int usz, hipStream_t s);

template <typename T> struct LongArgs {
  EscArgs<T> e;
  const LongRow *lrows;
  const LongItem *items;
  const int32_t *work;    // item ids to process (nullptr: all)
  LongState *state;
  Pool *pool;             // progressive blocks of the general kernels (spills, growth)
  unsigned int *fail_list;
  int32_t long_slot;
  Seq *partials;          // per item (multi-item rows)
  int32_t *pcol;          // partials of split rows / results of one-tile rows (at pbase)
  T *pval;
  int32_t *ocol;          // results of the pieces of split rows (at pbase + range start)
  T *oval;
  int32_t *split;         // range starts in every partial
  Piece *pieces;
  const int32_t *piece_lrow;
  LongState *cstate;      // checkpoints of the combine pieces
  unsigned int *fail_list2;
  LongCounters *cnt;      // lengths of the two lists below
  unsigned int *glist;    // items left to the general (multi-tile) kernel
  unsigned int *glist2;   // pieces left to the general combine kernel
  unsigned int *list1;    // items too large for one wavefront
  unsigned int *listw;    // items too large for the first wavefront pass
  unsigned int *list2;    // pieces too large for the first wavefront pass
  unsigned int *list3;    // pieces too large for one wavefront
  int64_t ncols;
  // direct output: the pieces of split rows go straight into C, at offsets
  // from a counting pass run before C is allocated (else to ocol / oval)
  int32_t direct;
  int32_t *c_col;
  T *c_val;
  const int64_t *rowoff;  // row offsets of C
  const int64_t *pscan;   // exclusive scan of the piece counts
};

// Whether every range of every split row is at most 2^kPieceCountLog
// columns wide, so that the counting pass can count its columns in a
// wavefront's LDS bitmap (the widest range belongs to the shortest split
// row).
constexpr int kPieceCountLog = 16;
bool long_direct_ok(const LongParams &lp, int64_t ncols);
// Distinct columns of every piece of a split row (one wavefront each,
// from phase 1's sorted segments), into pieces[pid].cnt.
template <typename T>
void launch_piece_count(const LongArgs<T> &a, int64_t npieces, hipStream_t s);

// Long-row table, work items and piece map (three launches).
void launch_long_table(const int32_t *binlist, int64_t off, int64_t nlong, const int64_t *u,
                       int64_t ncols, LongParams lp, LongRow *lrows, int64_t nitems,
                       LongItem *items, LongState *state, Seq *partials, int64_t npieces,
                       int32_t *piece_lrow, const int32_t *arp, const int64_t *P, int64_t *tmp,
                       hipStream_t s);
void launch_cstate_init(LongState *state, int64_t n, LongCounters *cnt, hipStream_t s);
int combine_maxs();
int combine_l1cap();
constexpr int kLongTile = 1024;
int64_t long_table_tmp_len(int64_t nlong);

template <typename T>
int launch_long(const LongArgs<T> &a, int64_t nwork, int l1cap, hipStream_t s);
// One-tile fast paths: items / pieces of at most kOneShot entries are sorted
// and folded in a single pass without the level-1 sequence.
constexpr int kOneShot = 4096;
template <typename T> void launch_long_oneshot(const LongArgs<T> &a, int64_t nitems, hipStream_t s);
// Wavefront paths: items / pieces of at most kWaveTile entries, one
// wavefront each; larger ones are listed for the one-tile work-group kernels,
// which then run over those lists.
constexpr int kWaveTile = 1024;
template <typename T> void launch_long_wave(const LongArgs<T> &a, int64_t nitems, hipStream_t s);
template <typename T>
void launch_long_wave_large(const LongArgs<T> &a, int64_t nitems, hipStream_t s);
template <typename T>
void launch_combine_wave(const LongArgs<T> &a, int64_t npieces, hipStream_t s);
template <typename T>
void launch_combine_wave_large(const LongArgs<T> &a, int64_t npieces, hipStream_t s);
template <typename T>
void launch_combine_oneshot(const LongArgs<T> &a, int64_t npieces, hipStream_t s);
template <typename T>
int launch_combine(const LongArgs<T> &a, int64_t npieces, hipStream_t s);
int long_l1cap_default(int dtype_bytes);
// Output sizes of the long rows from their pieces: piece scan -> rownnz.
void launch_long_rownnz(const LongRow *lrows, int64_t nlong, const int64_t *pscan,
                        int64_t *rownnz, hipStream_t s);
void scan_piece_counts(const Piece *pieces, int64_t n, int64_t *out, int64_t *part,
                       hipStream_t s);

// Window path for long rows (window.hip).  Planning: row records, the
// item and segment lists (bsum: 5 * ceil(nlong / 256) int64).
void win_plan_launch(const int32_t *lrows, int64_t nlong, const int64_t *u, int64_t n,
                     int vbytes, int64_t *bsum, WinRow *rows, WinWork *items, int64_t nitems,
                     WinWork *segs, int64_t nsegs, int32_t *slot_row, int64_t nslots,
                     const int32_t *arp, const int64_t *P, hipStream_t s);
// Partition segments of partitioned rows into piece buckets.
template <typename T>
void win_partition(const EscArgs<T> &e, const WinRow *rows, const WinWork *segs, int64_t nsegs,
                   uint16_t *table, uint32_t *pkey, T *pval, hipStream_t s);
// Symbolic pass: output count of every item (cnt), dense partial bitmaps;
// lists (list_ids, list_count: nitems + 1 entries) the items that the
// work-group kernels finish.
template <typename T>
void win_symbolic(const EscArgs<T> &e, int64_t n, const WinRow *rows, const WinWork *items,
                  int64_t nitems, const uint16_t *table, const uint32_t *pkey,
                  const int32_t *slot_row, int64_t nslots, uint32_t *list_ids,
                  uint32_t *list_count, uint32_t *dbits, int64_t *cnt, hipStream_t s);
// Long-row sizes from the scanned item counts.
void win_rownnz(const WinRow *rows, int64_t nlong, const int64_t *iscan, int64_t *rownnz,
                hipStream_t s);
// Numeric pass: every item written to its place in C.
template <typename T>
void win_numeric(const EscArgs<T> &e, int64_t n, const WinRow *rows, const WinWork *items,
                 int64_t nitems, const uint16_t *table, const uint32_t *pkey, const T *pval,
                 const int32_t *slot_row, int64_t nslots, uint32_t *list_ids,
                 uint32_t *list_count, const uint32_t *dbits, T *dacc, const int64_t *iscan,
                 const int64_t *rowoff, int32_t *c_col, T *c_val, hipStream_t s);

template <typename T> struct CompactArgs {
  const int64_t *u;
  const int64_t *cto;
  const int32_t *ct_col;
  const T *ct_val;
  const int64_t *rowoff;  // exclusive scan of rownnz, m+1
  int64_t long_min;       // rows with u > long_min are copied piece by piece
  const LongRow *lrows;
  const Piece *pieces;
  const int64_t *pscan;   // exclusive scan of the piece sizes
  int32_t *c_rp;
  int32_t *c_col;
  T *c_val;
};
template <typename T>
void launch_compact(const CompactArgs<T> &a, int64_t m, int64_t npieces, hipStream_t s);

void launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);

// ------------------------------------------------------------- backward
// A^T pattern (per column j of A: rows i ascending and entry positions)
void launch_transpose_pattern(const int32_t *arp, const int32_t *acol, int64_t m, int64_t k,
                              int64_t nnz, int32_t *cnt, int64_t *tptr, int32_t *trow,
                              int32_t *tpos, int64_t *part, hipStream_t s);
// Entry-parallel gradient: dA (nullable) and the products W (nullable,
// sum(u) entries) of the dB sums; then dB from W over A's transposed pattern.
template <typename T>
void launch_grad_entries(const int32_t *arp, const int32_t *acol, const T *aval, int64_t m,
                         int64_t nnz, const int64_t *P, const int32_t *brp, const int32_t *bcol,
                         const T *bval, int64_t n, const int32_t *crp, const int32_t *ccol,
                         const T *dc, T *dA, T *W, hipStream_t s);
template <typename T>
void launch_grad_b_sum(const int64_t *tptr, const int32_t *tpos, const int64_t *P,
                       const int32_t *brp, int64_t kb, const T *W, T *dB, hipStream_t s);
template <typename T>
void launch_grad_b(const int64_t *tptr, const int32_t *trow, const int32_t *tpos, const T *aval,
                   const int32_t *brp, const int32_t *bcol, int64_t kb, const int32_t *crp,
                   const int32_t *ccol, const T *dc, T *dB, hipStream_t s);
void launch_zero(void *p, size_t bytes, hipStream_t s);
void launch_set_pool(Pool *dst, Pool value, hipStream_t s);
void launch_status(const int64_t *rowoff, int64_t m, const Pool *pool, ComputeStatus *st,
                   hipStream_t s);

// Access to a plan's device arrays (defined with the plan in api.hip).
const int64_t *plan_rowoff(spgemm_plan p);
const int64_t *plan_scan(spgemm_plan p);
const int64_t *plan_upper(spgemm_plan p);
int64_t *plan_rownnz(spgemm_plan p);
const int32_t *plan_binlist(spgemm_plan p);
void set_last_error(const std::string &msg);
// input checks of spgemm_analyze (CSR shapes and dtypes; option ranges)
int check_problem(const spgemm_csr *A, const spgemm_csr *B);
int check_opts(const spgemm_options &o);

}  // namespace spg
