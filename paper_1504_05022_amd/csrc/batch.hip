// Batched SpGEMM: many independent products C_p = A_p * B_p of uneven sizes
// and mixed precision in one HIP graph of at most eleven kernel launches.
//
// batch_create analyzes every problem (stages 1-2, Algorithms 2 and 3),
// computes every C_p once with the plain path to fix its structure and
// row pointers, then builds one item list over all problems: every item is
// a group of rows of one problem from one bin (capacity class of the
// wavefront expand-sort-compress).  Items are grouped by class, and each
// class is one launch with one work-group per item, so every kernel holds
// only its own tile's registers and LDS.  An autotuner times the launches
// under a few bin-threshold sets and, for each, three tile-shape sets (lanes
// per row against products per lane of every capacity class) and keeps the
// fastest pair; its launches are captured in a graph.  batch_run replays the
// graph: every row is recomputed straight into its place in C_p, whose row
// offsets are known.
//
// Scope: every row of every problem must have at most 1024 products and
// 32-bit sort keys (n_p * 1024 < 2^32); other problems are recomputed with
// the plain path by batch_run (reported in spgemm_batch_stats).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <utility>
#include <string>
#include <vector>

#include "esc_body.hpp"
#include "stream_copy.hpp"

namespace spg {

struct BatchProblem {
  const int32_t *arp, *acol;
  const void *aval;
  const int32_t *brp, *bcol;
  const void *bval;
  const int64_t *P, *u, *rowoff;
  int32_t *ccol;
  void *cval;
  int64_t *rownnz;
  const int32_t *binlist;
  int32_t dtype;
  int32_t pad;
};

struct BatchItem {
  int32_t prob;
  int32_t cls;    // capacity class, index into kBatchClasses
  int64_t start;  // first row in the problem's bin list
  int32_t count;  // rows (at most the class's rows per work-group pass)
  int32_t pad;
};

// (G lanes per row, K products per lane) of every capacity class; the same
// shapes as the per-bin launches of the plain path.
constexpr int kBatchNumClasses = 11;
__host__ __device__ constexpr int batch_class_cap(int c) { return 1 << c; }

template <typename T>
DEVI EscArgs<T> esc_args_of(const BatchProblem &bp) {
  EscArgs<T> e;
  e.arp = bp.arp;
  e.acol = bp.acol;
  e.aval = static_cast<const T *>(bp.aval);
  e.brp = bp.brp;
  e.bcol = bp.bcol;
  e.bval = static_cast<const T *>(bp.bval);
  e.P = bp.P;
  e.u = bp.u;
  e.cto = bp.rowoff;  // rows land directly at their final place in C
  e.ct_col = bp.ccol;
  e.ct_val = static_cast<T *>(bp.cval);
  e.rownnz = bp.rownnz;
  return e;
}

// Tile shape (G lanes per row, K products per lane, G * K = capacity) of
// every capacity class in each of the shape sets the autotuner tries: the
// plain path's shapes, wider groups (more lanes, fewer products per lane:
// shorter sorts, more rows' latency in flight per lane) and narrower ones
// (up to 8 products per lane below the two largest classes: more rows per
// work-group).
constexpr int kBatchShapeSets = 3;
__host__ __device__ constexpr int batch_class_g(int set, int c) {
  constexpr int G[kBatchShapeSets][kBatchNumClasses] = {
      {1, 2, 4, 4, 4, 8, 16, 16, 32, 64, 64},
      {1, 2, 4, 8, 16, 16, 32, 32, 64, 64, 64},
      {1, 1, 1, 1, 2, 4, 8, 16, 32, 32, 64}};
  return G[set][c];
}

// One work-group per item of capacity class C under shape set SET: the rows
// of one problem's bin list, expanded, sorted and compressed straight into
// their places in C_p (binary32 and binary64 problems alike).  One launch
// per class over the items of every problem: each kernel is held only to
// its own tile's registers and LDS (a single kernel over all classes would
// be held to the largest tile's).
template <int SET, int C>
__global__ __launch_bounds__(ESC_NT) void k_batch_class(const BatchItem *items,
                                                        const BatchProblem *probs) {
  constexpr int G = batch_class_g(SET, C);
  constexpr int K = batch_class_cap(C) / G;
  __shared__ __align__(16) unsigned char lds[EscShape<double, G, K, uint32_t>::lds_bytes];
  const BatchItem it = items[blockIdx.x];
  const BatchProblem bp = probs[it.prob];
  const int32_t *rows = bp.binlist + it.start;
  if (bp.dtype == SPGEMM_F64)
    esc_rows<double, G, K, uint32_t>(esc_args_of<double>(bp), rows, 0, it.count, lds);
  else
    esc_rows<float, G, K, uint32_t>(esc_args_of<float>(bp), rows, 0, it.count, lds);
}

using BatchKernel = void (*)(const BatchItem *, const BatchProblem *);

template <int SET, int... C>
constexpr std::array<BatchKernel, sizeof...(C)> batch_kernels_of(std::integer_sequence<int, C...>) {
  return {{&k_batch_class<SET, C>...}};
}

// kernel of (shape set, class)
BatchKernel batch_kernel(int set, int c) {
  static const std::array<BatchKernel, kBatchNumClasses> k0 =
      batch_kernels_of<0>(std::make_integer_sequence<int, kBatchNumClasses>{});
  static const std::array<BatchKernel, kBatchNumClasses> k1 =
      batch_kernels_of<1>(std::make_integer_sequence<int, kBatchNumClasses>{});
  static const std::array<BatchKernel, kBatchNumClasses> k2 =
      batch_kernels_of<2>(std::make_integer_sequence<int, kBatchNumClasses>{});
  return set == 1 ? k1[c] : (set == 2 ? k2[c] : k0[c]);
}

// One launch per class over an item list grouped by ascending class (items
// of class c at [off[c], off[c+1])), the largest rows first (their
// work-groups run longest), one work-group per item.
void launch_classes(hipStream_t st, const BatchItem *ditems, const BatchProblem *dprob,
                    const int64_t (&off)[kBatchNumClasses + 1], int set) {
  for (int c = kBatchNumClasses - 1; c >= 0; --c) {
    const int64_t n = off[c + 1] - off[c];
    if (n > 0)
      hipLaunchKernelGGL(batch_kernel(set, c), dim3(static_cast<unsigned int>(n)), dim3(ESC_NT),
                         0, st, ditems + off[c], dprob);
  }
}


// ------------------------------------------------- one-shot batched product
//
// spgemm_batch_multiply runs every stage for many problems at once, without
// a plan: stage 1 (Algorithm 2) over the concatenated entries and rows of
// all problems, one read-back of the class counts, the hybrid allocation of
// C~ (every row gets u_i entries, Section 3.1), the wavefront ESC per
// capacity class, the scan of the row sizes and one compaction over all
// problems.  Problems are cut into tiles of entries or rows, so that a
// work-group never spans two problems.

constexpr int BM_NT = 256;
constexpr int BM_ENTRY_TILE = BM_NT * 16;       // entries of A_p per work-group
constexpr int BM_ROW_TILE = BM_NT;              // rows per work-group
constexpr int BM_NCLS = kBatchNumClasses + 1;   // capacity classes, then rows above 1024

struct BmProblem {
  const int32_t *arp, *acol, *brp;
  int64_t m, nnz;       // rows and entries of A_p
  int64_t eo, ro;       // the problem's first entry and first row in the concatenation
  int32_t *crp, *ccol;  // C_p (set before the compaction)
  void *cval;
  const void *tval;     // C~ values of the problem, indexed by C~ offsets
  int32_t dtype;
  int32_t batched;      // 0: computed by the plain path instead
};

struct BmTile {
  int32_t prob;
  int32_t pad;
  int64_t start;  // first entry or row of the tile in its problem
};

// capacity class of a row with u products: -1 for none, kBatchNumClasses
// above the largest class
__host__ __device__ inline int bm_class(int64_t u) {
  if (u <= 0) return -1;
  if (u > batch_class_cap(kBatchNumClasses - 1)) return kBatchNumClasses;
  int c = 0;
  while ((int64_t(1) << c) < u) ++c;
  return c;
}

// Stage 1, products of every entry: w[e] = nnz(b_{col(e)*}).
__global__ __launch_bounds__(BM_NT) void k_bm_entries(const BmTile *tiles, const BmProblem *probs,
                                                      int32_t *w) {
  const BmTile t = tiles[blockIdx.x];
  const BmProblem &q = probs[t.prob];
  const int32_t *acol = q.acol;
  const int32_t *brp = q.brp;
  const int64_t nnz = q.nnz;
  int32_t *wp = w + q.eo;
#pragma unroll
  for (int j = 0; j < BM_ENTRY_TILE / BM_NT; ++j) {
    const int64_t e = t.start + j * BM_NT + threadIdx.x;
    if (e < nnz) {
      const int32_t c = acol[e];
      wp[e] = brp[c + 1] - brp[c];
    }
  }
}

// Stage 1, rows: u_i from the entry scan P, rows of every capacity class
// and the sum of u_i counted per problem (one atomic per wavefront and
// class).  Rows without products get their final size, 0, here.
__global__ __launch_bounds__(BM_NT) void k_bm_rows(const BmTile *tiles, const BmProblem *probs,
                                                   const int64_t *P, int64_t *U, int64_t *RN,
                                                   unsigned long long *cnt,
                                                   unsigned long long *sumu) {
  const BmTile t = tiles[blockIdx.x];
  const BmProblem &q = probs[t.prob];
  const int64_t i = t.start + threadIdx.x;
  const bool valid = i < q.m;
  int64_t u = 0;
  if (valid) {
    u = P[q.eo + q.arp[i + 1]] - P[q.eo + q.arp[i]];
    U[q.ro + i] = u;
    if (u == 0) RN[q.ro + i] = 0;
  }
  const int c = valid ? bm_class(u) : -1;
  unsigned long long *cp = cnt + static_cast<int64_t>(t.prob) * BM_NCLS;
  for (int k = 0; k < BM_NCLS; ++k) {
    const unsigned long long mk = __ballot(c == k);
    if (mk != 0 && lane() == 0) atomicAdd(cp + k, static_cast<unsigned long long>(__popcll(mk)));
  }
  const long long tot = group_last<WAVE>(group_incl_sum<WAVE>(static_cast<long long>(u)));
  if (tot != 0 && lane() == 0) atomicAdd(sumu + t.prob, static_cast<unsigned long long>(tot));
}

// Stage 2: the rows of every batched problem into its class lists; cur
// holds the next free position of every (problem, class) list.  The order
// within a list does not matter (every row goes to its own place in C~).
__global__ __launch_bounds__(BM_NT) void k_bm_scatter(const BmTile *tiles, const BmProblem *probs,
                                                      const int64_t *U, unsigned long long *cur,
                                                      int32_t *list) {
  const BmTile t = tiles[blockIdx.x];
  const BmProblem &q = probs[t.prob];
  if (!q.batched) return;
  const int64_t i = t.start + threadIdx.x;
  const int c = i < q.m ? bm_class(U[q.ro + i]) : -1;
  unsigned long long *cp = cur + static_cast<int64_t>(t.prob) * BM_NCLS;
  const unsigned long long below = (1ull << lane()) - 1ull;
  for (int k = 0; k < kBatchNumClasses; ++k) {
    const unsigned long long mk = __ballot(c == k);
    if (mk == 0) continue;
    unsigned long long b = 0;
    if (lane() == 0) b = atomicAdd(cp + k, static_cast<unsigned long long>(__popcll(mk)));
    b = static_cast<unsigned long long>(__shfl(static_cast<long long>(b), 0, WAVE));
    if (c == k) list[b + __popcll(mk & below)] = static_cast<int32_t>(i);
  }
}

// Work items of list (problem, class) = blockIdx.x: rows [base + k * rpb,
// + rpb) of the class list from item io on (io < 0: no items); runs before
// k_bm_scatter advances the list cursors past the bases.
__global__ __launch_bounds__(BM_NT) void k_bm_items(const unsigned long long *cnt,
                                                    const unsigned long long *base,
                                                    const int64_t *io, int set,
                                                    BatchItem *items) {
  const int64_t k = blockIdx.x;
  const int64_t first = io[k];
  if (first < 0) return;
  const int c = static_cast<int>(k % BM_NCLS);
  const int rpb = ESC_NT / batch_class_g(set, c);
  const int64_t n = static_cast<int64_t>(cnt[k]);
  const int64_t b = static_cast<int64_t>(base[k]);
  for (int64_t j = threadIdx.x; j * rpb < n; j += BM_NT) {
    BatchItem it;
    it.prob = static_cast<int32_t>(k / BM_NCLS);
    it.cls = c;
    it.start = b + j * rpb;
    it.count = static_cast<int32_t>(min<int64_t>(rpb, n - j * rpb));
    it.pad = 0;
    items[first + j] = it;
  }
}

// nnz(C_p) boundaries: g[p] = RO at the problem's first row, g[count] = RO's total.
__global__ void k_bm_gather(const BmProblem *probs, int32_t count, const int64_t *RO, int64_t R,
                            int64_t *g) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < count) g[p] = RO[probs[p].ro];
  if (p == count) g[p] = RO[R];
}

template <typename T>
DEVI void bm_copy_rows(const BmProblem &q, const int32_t *tcol, const int64_t *CTO,
                       const int64_t *RO, const int64_t *RN, int64_t r0, int64_t end,
                       CopyTable<CP_ROWS> &tb) {
  const int64_t i = r0 + lane();
  int64_t n = 0, src = 0, o = 0;
  if (lane() < CP_ROWS && i < end) {
    const int64_t base = RO[q.ro];
    o = RO[q.ro + i] - base;
    q.crp[i] = static_cast<int32_t>(o);
    if (i == q.m - 1) q.crp[q.m] = static_cast<int32_t>(RO[q.ro + q.m] - base);
    n = RN[q.ro + i];
    src = CTO[q.ro + i];
  }
  wave_stream_copy<T, CP_ROWS>(n, tcol + src, static_cast<const T *>(q.tval) + src, o, q.ccol,
                               static_cast<T *>(q.cval), tb);
}

// Stage 5 for every batched problem: row pointers of C_p and its rows
// copied from C~, CP_ROWS rows per wavefront.
__global__ __launch_bounds__(CP_NT) void k_bm_compact(const BmTile *tiles, const BmProblem *probs,
                                                      const int32_t *tcol, const int64_t *CTO,
                                                      const int64_t *RO, const int64_t *RN) {
  __shared__ CopyTable<CP_ROWS> tabs[CP_NT / WAVE];
  const BmTile t = tiles[blockIdx.x];
  const BmProblem &q = probs[t.prob];
  if (!q.batched) return;
  if (q.m == 0) {
    if (threadIdx.x == 0) q.crp[0] = 0;
    return;
  }
  const int w = threadIdx.x / WAVE;
  const int64_t end = min(t.start + BM_ROW_TILE, q.m);
  for (int64_t r0 = t.start + w * CP_ROWS; r0 < end; r0 += (CP_NT / WAVE) * CP_ROWS) {
    if (q.dtype == SPGEMM_F64)
      bm_copy_rows<double>(q, tcol, CTO, RO, RN, r0, end, tabs[w]);
    else
      bm_copy_rows<float>(q, tcol, CTO, RO, RN, r0, end, tabs[w]);
  }
}

}  // namespace spg

// ------------------------------------------------------------- host side

using namespace spg;

namespace {

int bfail(int code, const std::string &msg) {
  set_last_error(msg);
  return code;
}

struct Candidate {
  int32_t edges[5];
  std::vector<spgemm_plan> plans;
  std::vector<BatchItem> items[kBatchShapeSets];  // per tile-shape set
  float ms[kBatchShapeSets] = {};
};

}  // namespace

struct spgemm_batch_s {
  int32_t count = 0;
  spgemm_options opt{};
  spgemm_alloc_fn af = nullptr;
  spgemm_free_fn ff = nullptr;
  void *ctx = nullptr;
  std::vector<const spgemm_csr *> A, B;
  std::vector<spgemm_csr> Ad, Bd;
  std::vector<spgemm_csr_out> C;
  std::vector<spgemm_plan> plans;  // winning candidate's plans (bin lists, P, u)
  std::vector<int32_t> fallback;   // problems recomputed with the plain path
  std::vector<int64_t *> rowoff;   // per problem, copied from the first compute
  void *dmem = nullptr;            // problems table + items
  void *doff = nullptr;            // row offsets of all problems
  int64_t nitems = 0;
  int shape_set = 0;  // tile shapes chosen by the autotuner
  int64_t cls_off[kBatchNumClasses + 1] = {};  // items of class c: [cls_off[c], cls_off[c+1])
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  spgemm_batch_stats stats{};
  hipStream_t stream = nullptr;

  void *get(size_t bytes, hipStream_t s) {
    bytes = (bytes + 255) & ~static_cast<size_t>(255);
    if (bytes == 0) bytes = 256;
    if (af) return af(bytes, ctx, reinterpret_cast<void *>(s));
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void put(void *p, hipStream_t s) {
    if (!p) return;
    if (ff)
      ff(p, ctx, reinterpret_cast<void *>(s));
    else
      (void)hipFreeAsync(p, s);
  }
};

namespace {

int class_of_cap(int64_t cap) {
  int c = 0;
  while ((int64_t(1) << c) < cap) ++c;
  return c;
}

// rows per work-group pass of each class (256 / G)
int class_rpb(int set, int c) { return ESC_NT / batch_class_g(set, c); }

// Work items of one analyzed problem (bins 1..36) under its thresholds and
// a tile-shape set.
void build_items(int32_t prob, const spgemm_info &I, const int32_t edges[5], int set,
                 std::vector<BatchItem> &out) {
  // bin segment starts from the per-bin counts (bins are stored in order)
  int64_t off[SPGEMM_NBINS + 1];
  off[0] = 0;
  for (int b = 0; b < SPGEMM_NBINS; ++b) off[b + 1] = off[b] + I.bin_count[b];
  auto emit = [&](int b_lo, int b_hi, int64_t cap) {
    const int c = class_of_cap(cap);
    const int rpb = class_rpb(set, c);
    for (int64_t r = off[b_lo]; r < off[b_hi + 1]; r += rpb) {
      BatchItem it;
      it.prob = prob;
      it.cls = c;
      it.start = r;
      it.count = static_cast<int32_t>(std::min<int64_t>(rpb, off[b_hi + 1] - r));
      it.pad = 0;
      out.push_back(it);
    }
  };
  int b = 1;
  while (b <= edges[0]) {
    int64_t cap = 1;
    while (cap < b) cap <<= 1;
    const int hi = static_cast<int>(std::min<int64_t>(cap, edges[0]));
    emit(b, hi, cap);
    b = hi + 1;
  }
  for (int g = 33; g <= 36; ++g) {
    int64_t cap = 1;
    while (cap < edges[g - 32]) cap <<= 1;
    emit(g, g, cap);
  }
}

void destroy_plans(std::vector<spgemm_plan> &v) {
  for (auto p : v) spgemm_plan_destroy(p);
  v.clear();
}

}  // namespace

extern "C" {

int spgemm_batch_create(int32_t count, const spgemm_csr *A, const spgemm_csr *B,
                        const spgemm_options *opt, spgemm_alloc_fn alloc_fn,
                        spgemm_free_fn free_fn, void *ctx, void *stream, spgemm_batch *out,
                        spgemm_batch_stats *stats) {
  if (!out) return bfail(SPGEMM_EINVAL, "batch is NULL");
  *out = nullptr;
  if (count < 0 || (count > 0 && (!A || !B)))
    return bfail(SPGEMM_EINVAL, "bad problem count or NULL arrays");
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return bfail(SPGEMM_EINVAL, "alloc_fn and free_fn must both be set or both be NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  spgemm_batch b = new (std::nothrow) spgemm_batch_s();
  if (!b) return bfail(SPGEMM_ENOMEM, "host allocation failed");
  b->count = count;
  spgemm_default_options(&b->opt);
  if (opt) b->opt = *opt;
  b->af = alloc_fn;
  b->ff = free_fn;
  b->ctx = ctx;
  b->stream = s;
  b->Ad.assign(A, A + count);
  b->Bd.assign(B, B + count);
  b->C.assign(count, spgemm_csr_out{});
  int rc = SPGEMM_OK;

  // candidate bin thresholds (group 4 ends at 1024: every row of a batched
  // problem stays in the wavefront kernel)
  static const int32_t kDefaultEdges[5] = {32, 64, 128, 256, 512};
  static const int32_t kCands[][5] = {{32, 64, 128, 256, 1024},
                                      {16, 64, 256, 512, 1024},
                                      {32, 128, 256, 512, 1024},
                                      {8, 32, 128, 512, 1024}};
  // the autotuner runs unless the caller fixed the thresholds; a fixed
  // tile-shape set is timed alone
  if (b->opt.batch_shapes < 0 || b->opt.batch_shapes > kBatchShapeSets) {
    spgemm_batch_destroy(b);
    return bfail(SPGEMM_EINVAL, "batch_shapes must be 0 (autotune) or 1..3");
  }
  const bool tune = std::memcmp(b->opt.bin_edges, kDefaultEdges, sizeof(kDefaultEdges)) == 0;
  const int ncand = tune ? 4 : 1;
  const int set_lo = b->opt.batch_shapes ? b->opt.batch_shapes - 1 : 0;
  const int set_hi = b->opt.batch_shapes ? b->opt.batch_shapes : kBatchShapeSets;
  std::vector<Candidate> cands(ncand);
  std::vector<char> batched(count, 1);
  std::vector<int64_t> m_of(count, 0);
  int64_t total_off = 0;
  for (int32_t p = 0; p < count; ++p) {
    m_of[p] = A[p].rows;
    total_off += A[p].rows + 1;
  }
  b->doff = b->get(static_cast<size_t>(std::max<int64_t>(total_off, 1)) * 8, s);
  if (!b->doff) {
    spgemm_batch_destroy(b);
    return bfail(SPGEMM_ENOMEM, "row offset allocation failed");
  }
  b->rowoff.assign(count, nullptr);
  {
    int64_t o = 0;
    for (int32_t p = 0; p < count; ++p) {
      b->rowoff[p] = static_cast<int64_t *>(b->doff) + o;
      o += m_of[p] + 1;
    }
  }

  for (int ci = 0; ci < ncand && rc == SPGEMM_OK; ++ci) {
    Candidate &cd = cands[ci];
    std::memcpy(cd.edges, tune ? kCands[ci] : b->opt.bin_edges, sizeof(cd.edges));
    spgemm_options o = b->opt;
    std::memcpy(o.bin_edges, cd.edges, sizeof(cd.edges));
    o.timing = 0;
    cd.plans.assign(count, nullptr);
    for (int32_t p = 0; p < count && rc == SPGEMM_OK; ++p) {
      spgemm_info I;
      rc = spgemm_analyze(&A[p], &B[p], &o, alloc_fn, free_fn, ctx, stream, &cd.plans[p], &I);
      if (rc != SPGEMM_OK) break;
      if (ci == 0) {
        // the structure of C_p, once, with the plain path
        rc = spgemm_compute(cd.plans[p], &A[p], &B[p], &b->C[p], stream, nullptr);
        if (rc != SPGEMM_OK) break;
        const bool keys32 = (static_cast<uint64_t>(B[p].cols) << 10) <= 0xffffffffull;
        if (I.bin_count[LONG_BIN] > 0 || !keys32 || I.max_u > 1024) batched[p] = 0;
        // row offsets of C_p (the exclusive scan compute left in the plan)
        hipError_t e = hipMemcpyAsync(b->rowoff[p], plan_rowoff(cd.plans[p]),
                                      static_cast<size_t>(m_of[p] + 1) * 8,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) rc = bfail(SPGEMM_EHIP, "row offset copy failed");
      }
      if (batched[p])
        for (int set = 0; set < kBatchShapeSets; ++set) build_items(p, I, cd.edges, set, cd.items[set]);
    }
    // items grouped by class (one launch each)
    for (auto &v : cd.items)
      std::stable_sort(v.begin(), v.end(),
                       [](const BatchItem &x, const BatchItem &y) { return x.cls < y.cls; });
  }
  if (rc != SPGEMM_OK) {
    for (auto &cd : cands) destroy_plans(cd.plans);
    spgemm_batch_destroy(b);
    return rc;
  }
  for (int32_t p = 0; p < count; ++p)
    if (!batched[p]) b->fallback.push_back(p);

  // device tables: problems and the largest item list
  size_t maxitems = 1;
  for (auto &cd : cands)
    for (auto &v : cd.items) maxitems = std::max(maxitems, v.size());
  const size_t oprob = 0;
  const size_t oitems = (sizeof(BatchProblem) * std::max(count, 1) + 255) & ~size_t(255);
  b->dmem = b->get(oitems + sizeof(BatchItem) * maxitems, s);
  if (!b->dmem) {
    for (auto &cd : cands) destroy_plans(cd.plans);
    spgemm_batch_destroy(b);
    return bfail(SPGEMM_ENOMEM, "batch table allocation failed");
  }
  BatchProblem *dprob = reinterpret_cast<BatchProblem *>(static_cast<char *>(b->dmem) + oprob);
  BatchItem *ditems = reinterpret_cast<BatchItem *>(static_cast<char *>(b->dmem) + oitems);

  // item ranges of every class in a list sorted by ascending class
  auto class_ranges = [](const std::vector<BatchItem> &v, int64_t (&off)[kBatchNumClasses + 1]) {
    int64_t k = 0;
    for (int c = 0; c <= kBatchNumClasses; ++c) {
      while (k < static_cast<int64_t>(v.size()) && v[k].cls < c) ++k;
      off[c] = k;
    }
  };
  auto upload = [&](Candidate &cd, int set) -> int {
    std::vector<BatchProblem> hp(count);
    for (int32_t p = 0; p < count; ++p) {
      BatchProblem &q = hp[p];
      q.arp = A[p].row_ptr;
      q.acol = A[p].col_idx;
      q.aval = A[p].val;
      q.brp = B[p].row_ptr;
      q.bcol = B[p].col_idx;
      q.bval = B[p].val;
      q.P = plan_scan(cd.plans[p]);
      q.u = plan_upper(cd.plans[p]);
      q.rowoff = b->rowoff[p];
      q.ccol = b->C[p].col_idx;
      q.cval = b->C[p].val;
      q.rownnz = plan_rownnz(cd.plans[p]);
      q.binlist = plan_binlist(cd.plans[p]);
      q.dtype = A[p].dtype;
      q.pad = 0;
    }
    if (count > 0 &&
        hipMemcpyAsync(dprob, hp.data(), sizeof(BatchProblem) * count, hipMemcpyHostToDevice,
                       s) != hipSuccess)
      return bfail(SPGEMM_EHIP, "problem table upload failed");
    if (!cd.items[set].empty() &&
        hipMemcpyAsync(ditems, cd.items[set].data(), sizeof(BatchItem) * cd.items[set].size(),
                       hipMemcpyHostToDevice, s) != hipSuccess)
      return bfail(SPGEMM_EHIP, "item list upload failed");
    if (hipStreamSynchronize(s) != hipSuccess) return bfail(SPGEMM_EHIP, "upload sync failed");
    return SPGEMM_OK;
  };
  auto enqueue = [&](hipStream_t st, const int64_t (&off)[kBatchNumClasses + 1], int set) {
    launch_classes(st, ditems, dprob, off, set);
  };

  // autotuner: time the class launches under every candidate threshold set
  // and tile-shape set
  int best = 0, best_set = set_lo;
  if (ncand > 1 || set_hi - set_lo > 1) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (int ci = 0; ci < ncand && rc == SPGEMM_OK; ++ci) {
      Candidate &cd = cands[ci];
      for (int set = set_lo; set < set_hi && rc == SPGEMM_OK; ++set) {
        if ((rc = upload(cd, set)) != SPGEMM_OK) break;
        int64_t off[kBatchNumClasses + 1];
        class_ranges(cd.items[set], off);
        enqueue(s, off, set);  // warm-up
        (void)hipEventRecord(e0, s);
        for (int rep = 0; rep < 3; ++rep) enqueue(s, off, set);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) rc = bfail(SPGEMM_EHIP, "autotune sync failed");
        (void)hipEventElapsedTime(&cd.ms[set], e0, e1);
        cd.ms[set] /= 3.f;
        if ((ci == 0 && set == set_lo) || cd.ms[set] < cands[best].ms[best_set]) {
          best = ci;
          best_set = set;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  if (rc == SPGEMM_OK) rc = upload(cands[best], best_set);
  if (rc != SPGEMM_OK) {
    for (auto &cd : cands) destroy_plans(cd.plans);
    spgemm_batch_destroy(b);
    return rc;
  }
  for (int ci = 0; ci < ncand; ++ci)
    if (ci != best) destroy_plans(cands[ci].plans);
  b->plans = cands[best].plans;
  b->nitems = static_cast<int64_t>(cands[best].items[best_set].size());
  class_ranges(cands[best].items[best_set], b->cls_off);
  b->shape_set = best_set;

  // the replayable graph: one kernel node per nonempty class (no graph when
  // every problem falls back to the plain path)
  hipStream_t cs = nullptr;
  hipError_t e = hipSuccess;
  if (b->nitems > 0) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess && cs) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess && cs) {
    enqueue(cs, b->cls_off, b->shape_set);
    e = hipStreamEndCapture(cs, &b->graph);
  }
  if (e == hipSuccess && cs) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    spgemm_batch_destroy(b);
    return bfail(SPGEMM_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
  }

  spgemm_batch_stats &st = b->stats;
  std::memset(&st, 0, sizeof(st));
  st.count = count;
  st.items = b->nitems;
  st.grid = 0;
  for (int c = 0; c < kBatchNumClasses; ++c) st.grid += b->cls_off[c + 1] > b->cls_off[c];
  st.fallback = static_cast<int32_t>(b->fallback.size());
  std::memcpy(st.bin_edges, cands[best].edges, sizeof(st.bin_edges));
  st.shapes = best_set;
  for (int ci = 0; ci < ncand && ci < 4; ++ci)
    for (int set = 0; set < kBatchShapeSets; ++set) st.tune_ms[ci * kBatchShapeSets + set] = cands[ci].ms[set];
  for (int32_t p = 0; p < count; ++p) {
    spgemm_info I;
    spgemm_plan_info(b->plans[p], &I);
    st.flops += I.flops;
    st.nnz_c += b->C[p].nnz;
  }
  if (stats) *stats = st;
  *out = b;
  return SPGEMM_OK;
}

int spgemm_batch_run(spgemm_batch b, spgemm_csr_out *C, void *stream) {
  if (!b) return bfail(SPGEMM_EINVAL, "batch is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = b->exec ? hipGraphLaunch(b->exec, s) : hipSuccess;
  if (e != hipSuccess) return bfail(SPGEMM_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
  for (int32_t p : b->fallback) {
    // recompute into a fresh output, then move it into the batch's slot
    spgemm_csr_out tmp{};
    int rc = spgemm_compute(b->plans[p], &b->Ad[p], &b->Bd[p], &tmp, stream, nullptr);
    if (rc != SPGEMM_OK) return rc;
    b->put(b->C[p].row_ptr, s);
    b->put(b->C[p].col_idx, s);
    b->put(b->C[p].val, s);
    b->C[p] = tmp;
  }
  if (C)
    for (int32_t p = 0; p < b->count; ++p) C[p] = b->C[p];
  return SPGEMM_OK;
}

int spgemm_batch_stats_get(spgemm_batch b, spgemm_batch_stats *st) {
  if (!b || !st) return bfail(SPGEMM_EINVAL, "NULL argument");
  *st = b->stats;
  return SPGEMM_OK;
}

int spgemm_batch_destroy(spgemm_batch b) {
  if (!b) return SPGEMM_OK;
  hipStream_t s = b->stream;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  destroy_plans(b->plans);
  for (auto &c : b->C) {
    b->put(c.row_ptr, s);
    b->put(c.col_idx, s);
    b->put(c.val, s);
  }
  b->put(b->dmem, s);
  b->put(b->doff, s);
  delete b;
  return SPGEMM_OK;
}

}  // extern "C"

namespace {

// Device memory of one spgemm_batch_multiply call, released on every exit
// unless kept.
struct BmMem {
  spgemm_alloc_fn af;
  spgemm_free_fn ff;
  void *ctx;
  hipStream_t s;
  std::vector<void *> held;
  void *get(size_t bytes) {
    bytes = (bytes + 255) & ~static_cast<size_t>(255);
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (af) {
      p = af(bytes, ctx, reinterpret_cast<void *>(s));
    } else if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (p) held.push_back(p);
    return p;
  }
  void put(void *p) {
    if (!p) return;
    if (ff)
      ff(p, ctx, reinterpret_cast<void *>(s));
    else
      (void)hipFreeAsync(p, s);
  }
  void keep(void *p) { held.erase(std::remove(held.begin(), held.end(), p), held.end()); }
  ~BmMem() {
    for (void *p : held) put(p);
  }
};

size_t round256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

}  // namespace

extern "C" {

int spgemm_batch_multiply(int32_t count, const spgemm_csr *A, const spgemm_csr *B,
                          const spgemm_options *opt, spgemm_alloc_fn alloc_fn,
                          spgemm_free_fn free_fn, void *ctx, void *stream, spgemm_csr_out *C,
                          void **out_mem, spgemm_batch_stats *stats) {
  if (!out_mem) return bfail(SPGEMM_EINVAL, "out_mem is NULL");
  *out_mem = nullptr;
  if (count < 0 || (count > 0 && (!A || !B || !C)))
    return bfail(SPGEMM_EINVAL, "bad problem count or NULL arrays");
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return bfail(SPGEMM_EINVAL, "alloc_fn and free_fn must both be set or both be NULL");
  spgemm_options o;
  spgemm_default_options(&o);
  if (opt) o = *opt;
  int rc = check_opts(o);
  if (rc != SPGEMM_OK) return rc;
  if (o.batch_shapes < 0 || o.batch_shapes > kBatchShapeSets)
    return bfail(SPGEMM_EINVAL, "batch_shapes must be 0 (default shapes) or 1..3");
  for (int32_t p = 0; p < count; ++p)
    if ((rc = check_problem(&A[p], &B[p])) != SPGEMM_OK) return rc;
  const int set = o.batch_shapes ? o.batch_shapes - 1 : 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  spgemm_batch_stats st;
  std::memset(&st, 0, sizeof(st));
  st.count = count;
  st.shapes = set;
  if (count == 0) {
    if (stats) *stats = st;
    return SPGEMM_OK;
  }
  BmMem mem{alloc_fn, free_fn, ctx, s, {}};

  // the concatenation: entries and rows of every problem in turn, in tiles
  std::vector<BmProblem> hp(count);
  std::vector<BmTile> etile, rtile;
  int64_t E = 0, R = 0;
  for (int32_t p = 0; p < count; ++p) {
    BmProblem &q = hp[p];
    std::memset(&q, 0, sizeof(q));
    q.arp = A[p].row_ptr;
    q.acol = A[p].col_idx;
    q.brp = B[p].row_ptr;
    q.m = A[p].rows;
    q.nnz = A[p].nnz;
    q.eo = E;
    q.ro = R;
    q.dtype = A[p].dtype;
    for (int64_t e = 0; e < q.nnz; e += BM_ENTRY_TILE) etile.push_back(BmTile{p, 0, e});
    for (int64_t r = 0; r < std::max<int64_t>(q.m, 1); r += BM_ROW_TILE)
      rtile.push_back(BmTile{p, 0, r});
    E += q.nnz;
    R += q.m;
  }
  if (etile.size() >= (size_t(1) << 31) || rtile.size() >= (size_t(1) << 31))
    return bfail(SPGEMM_EOVERFLOW, "batch too large for one launch");

  // scratch of the analysis
  const int64_t ncnt = static_cast<int64_t>(count) * BM_NCLS;
  size_t off = 0;
  auto add = [&](size_t bytes) {
    const size_t o0 = off;
    off = round256(off + std::max<size_t>(bytes, 1));
    return o0;
  };
  const size_t o_prob = add(sizeof(BmProblem) * count);
  const size_t o_et = add(sizeof(BmTile) * etile.size());
  const size_t o_rt = add(sizeof(BmTile) * rtile.size());
  const size_t o_w = add(sizeof(int32_t) * E);
  const size_t o_P = add(sizeof(int64_t) * (E + 1));
  const size_t o_part = add(sizeof(int64_t) * scan_part_len(std::max<int64_t>(std::max(E, R), 1)));
  const size_t o_U = add(sizeof(int64_t) * R);
  const size_t o_CTO = add(sizeof(int64_t) * (R + 1));
  const size_t o_RN = add(sizeof(int64_t) * R);
  const size_t o_RO = add(sizeof(int64_t) * (R + 1));
  const size_t o_cnt = add(sizeof(unsigned long long) * (ncnt + count));  // counts, then sums of u
  const size_t o_cur = add(sizeof(unsigned long long) * ncnt);
  const size_t o_io = add(sizeof(int64_t) * ncnt);
  const size_t o_list = add(sizeof(int32_t) * R);
  const size_t o_g = add(sizeof(int64_t) * (count + 1));
  const size_t o_bp = add(sizeof(BatchProblem) * count);
  char *ws = static_cast<char *>(mem.get(off));
  if (!ws) return bfail(SPGEMM_ENOMEM, "batch scratch allocation failed");
  BmProblem *dprob = reinterpret_cast<BmProblem *>(ws + o_prob);
  BmTile *det = reinterpret_cast<BmTile *>(ws + o_et);
  BmTile *drt = reinterpret_cast<BmTile *>(ws + o_rt);
  int32_t *dw = reinterpret_cast<int32_t *>(ws + o_w);
  int64_t *dP = reinterpret_cast<int64_t *>(ws + o_P);
  int64_t *dpart = reinterpret_cast<int64_t *>(ws + o_part);
  int64_t *dU = reinterpret_cast<int64_t *>(ws + o_U);
  int64_t *dCTO = reinterpret_cast<int64_t *>(ws + o_CTO);
  int64_t *dRN = reinterpret_cast<int64_t *>(ws + o_RN);
  int64_t *dRO = reinterpret_cast<int64_t *>(ws + o_RO);
  unsigned long long *dcnt = reinterpret_cast<unsigned long long *>(ws + o_cnt);
  unsigned long long *dsumu = dcnt + ncnt;
  unsigned long long *dcur = reinterpret_cast<unsigned long long *>(ws + o_cur);
  int64_t *dio = reinterpret_cast<int64_t *>(ws + o_io);
  int32_t *dlist = reinterpret_cast<int32_t *>(ws + o_list);
  int64_t *dg = reinterpret_cast<int64_t *>(ws + o_g);
  BatchProblem *dbp = reinterpret_cast<BatchProblem *>(ws + o_bp);
  int64_t bytes_scratch = static_cast<int64_t>(off);

  auto h2d = [&](void *dst, const void *src, size_t bytes) {
    return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  if (!h2d(dprob, hp.data(), sizeof(BmProblem) * count) ||
      !h2d(det, etile.data(), sizeof(BmTile) * etile.size()) ||
      !h2d(drt, rtile.data(), sizeof(BmTile) * rtile.size()))
    return bfail(SPGEMM_EHIP, "batch table upload failed");
  launch_zero(dcnt, sizeof(unsigned long long) * (ncnt + count), s);

  // stage 1 over every problem: products per entry, their scan, u_i
  if (!etile.empty())
    hipLaunchKernelGGL(k_bm_entries, dim3(static_cast<unsigned int>(etile.size())), dim3(BM_NT),
                       0, s, det, dprob, dw);
  scan_i32(dw, E, dP, dpart, s);
  hipLaunchKernelGGL(k_bm_rows, dim3(static_cast<unsigned int>(rtile.size())), dim3(BM_NT), 0, s,
                     drt, dprob, dP, dU, dRN, dcnt, dsumu);
  std::vector<unsigned long long> hcnt(ncnt + count);
  if (hipMemcpyAsync(hcnt.data(), dcnt, sizeof(unsigned long long) * (ncnt + count),
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bfail(SPGEMM_EHIP, std::string("batch analysis failed: ") +
                                  hipGetErrorString(hipGetLastError()));

  // problems of the batched kernels (rows up to 1024 products, 32-bit keys);
  // C~ holds u_i entries for each of their rows (hybrid allocation)
  std::vector<int32_t> fallback;
  std::vector<int64_t> cbase(count, 0);
  int64_t ntilde = 0;  // entries of C~
  for (int32_t p = 0; p < count; ++p) {
    const bool keys32 = (static_cast<uint64_t>(B[p].cols) << 10) <= 0xffffffffull;
    hp[p].batched = keys32 && hcnt[static_cast<int64_t>(p) * BM_NCLS + kBatchNumClasses] == 0;
    st.flops += 2 * static_cast<int64_t>(hcnt[ncnt + p]);
    if (!hp[p].batched) {
      fallback.push_back(p);
      // no C~ entries and no row sizes for the rows of a fallback problem
      if (hp[p].m > 0) {
        launch_zero(dU + hp[p].ro, sizeof(int64_t) * hp[p].m, s);
        launch_zero(dRN + hp[p].ro, sizeof(int64_t) * hp[p].m, s);
      }
      continue;
    }
    cbase[p] = ntilde;
    ntilde += static_cast<int64_t>(hcnt[ncnt + p]);
  }
  // class lists grouped by class, then problem; items of at most 256 / G
  // rows, written on the device from each list's first item (-1: none)
  std::vector<unsigned long long> hcur(ncnt, 0);
  std::vector<int64_t> hio(ncnt, -1);
  int64_t cls_off[kBatchNumClasses + 1];
  int64_t nitems = 0;
  {
    int64_t pos = 0;
    for (int c = 0; c < kBatchNumClasses; ++c) {
      cls_off[c] = nitems;
      const int rpb = class_rpb(set, c);
      for (int32_t p = 0; p < count; ++p) {
        if (!hp[p].batched) continue;
        const int64_t k = static_cast<int64_t>(p) * BM_NCLS + c;
        const int64_t n = static_cast<int64_t>(hcnt[k]);
        hcur[k] = static_cast<unsigned long long>(pos);
        if (n > 0) hio[k] = nitems;
        nitems += (n + rpb - 1) / rpb;
        pos += n;
      }
    }
    cls_off[kBatchNumClasses] = nitems;
  }
  for (int c = 0; c < kBatchNumClasses; ++c)
    if (cls_off[c + 1] - cls_off[c] >= (int64_t(1) << 31))
      return bfail(SPGEMM_EOVERFLOW, "batch too large for one launch");

  // C~ (columns; values in 8-byte slots whatever the problem's type, so
  // that binary32 and binary64 problems share one offset space) and items
  char *tcol = static_cast<char *>(mem.get(std::max<int64_t>(ntilde, 1) * 4));
  char *tval = static_cast<char *>(mem.get(std::max<int64_t>(ntilde, 1) * 8));
  BatchItem *ditems =
      static_cast<BatchItem *>(mem.get(sizeof(BatchItem) * std::max<int64_t>(nitems, 1)));
  if (!tcol || !tval || !ditems) return bfail(SPGEMM_ENOMEM, "C~ allocation failed");
  bytes_scratch += static_cast<int64_t>(round256(std::max<int64_t>(ntilde, 1) * 4) +
                                        round256(std::max<int64_t>(ntilde, 1) * 8) +
                                        round256(sizeof(BatchItem) * std::max<int64_t>(nitems, 1)));
  std::vector<BatchProblem> hbp(count);
  for (int32_t p = 0; p < count; ++p) {
    // a binary32 problem's values at slot offset cbase + k sit at byte
    // 8 * cbase + 4 * k: inside its own slots
    const size_t vs = A[p].dtype == SPGEMM_F64 ? 8 : 4;
    hp[p].tval = tval + (8 - vs) * static_cast<size_t>(cbase[p]);
    BatchProblem &q = hbp[p];
    q.arp = A[p].row_ptr;
    q.acol = A[p].col_idx;
    q.aval = A[p].val;
    q.brp = B[p].row_ptr;
    q.bcol = B[p].col_idx;
    q.bval = B[p].val;
    q.P = dP + hp[p].eo;
    q.u = dU + hp[p].ro;
    q.rowoff = dCTO + hp[p].ro;
    q.ccol = reinterpret_cast<int32_t *>(tcol);
    q.cval = const_cast<void *>(hp[p].tval);
    q.rownnz = dRN + hp[p].ro;
    q.binlist = dlist;
    q.dtype = A[p].dtype;
    q.pad = 0;
  }
  if (!h2d(dprob, hp.data(), sizeof(BmProblem) * count) ||
      !h2d(dbp, hbp.data(), sizeof(BatchProblem) * count) ||
      !h2d(dcur, hcur.data(), sizeof(unsigned long long) * ncnt) ||
      !h2d(dio, hio.data(), sizeof(int64_t) * ncnt))
    return bfail(SPGEMM_EHIP, "batch table upload failed");
  hipLaunchKernelGGL(k_bm_items, dim3(static_cast<unsigned int>(ncnt)), dim3(BM_NT), 0, s, dcnt,
                     dcur, dio, set, ditems);

  // C~ offsets, class lists, the ESC per class, row sizes of C
  scan_i64(dU, R, dCTO, dpart, s);
  hipLaunchKernelGGL(k_bm_scatter, dim3(static_cast<unsigned int>(rtile.size())), dim3(BM_NT), 0,
                     s, drt, dprob, dU, dcur, dlist);
  launch_classes(s, ditems, dbp, cls_off, set);
  scan_i64(dRN, R, dRO, dpart, s);
  hipLaunchKernelGGL(k_bm_gather, dim3(static_cast<unsigned int>((count + 256) / 256)), dim3(256),
                     0, s, dprob, count, dRO, R, dg);
  std::vector<int64_t> hg(count + 1);
  if (hipMemcpyAsync(hg.data(), dg, sizeof(int64_t) * (count + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bfail(SPGEMM_EHIP, std::string("batch numeric stage failed: ") +
                                  hipGetErrorString(hipGetLastError()));

  // fallback problems through the plain path (their outputs are moved into
  // the output block below)
  std::vector<spgemm_csr_out> fb(count);
  struct FbGuard {
    std::vector<spgemm_csr_out> &v;
    BmMem &mem;
    ~FbGuard() {
      for (auto &c : v) {
        mem.put(c.row_ptr);
        mem.put(c.col_idx);
        mem.put(c.val);
      }
    }
  } fb_guard{fb, mem};
  std::vector<int64_t> nnz(count, 0);
  int64_t fb_scratch = 0;  // the largest plain-path peak, on top of what is held here
  for (int32_t p : fallback) {
    spgemm_info I;
    if ((rc = spgemm_multiply(&A[p], &B[p], &o, alloc_fn, free_fn, ctx, stream, &fb[p], &I)) !=
        SPGEMM_OK)
      return rc;
    nnz[p] = fb[p].nnz;
    fb_scratch = std::max(fb_scratch, I.bytes_scratch);
  }
  bytes_scratch += fb_scratch;
  for (int32_t p = 0; p < count; ++p) {
    if (!hp[p].batched) continue;
    nnz[p] = hg[p + 1] - hg[p];
    if (nnz[p] >= (int64_t(1) << 31))
      return bfail(SPGEMM_EOVERFLOW, "nnz(C) exceeds the int32 index range");
  }

  // one block for every output: row pointers, columns, values of each C_p
  size_t obytes = 0;
  std::vector<size_t> orp(count), ocol(count), oval(count);
  for (int32_t p = 0; p < count; ++p) {
    const size_t vs = A[p].dtype == SPGEMM_F64 ? 8 : 4;
    orp[p] = obytes;
    obytes += round256(sizeof(int32_t) * (hp[p].m + 1));
    ocol[p] = obytes;
    obytes += round256(sizeof(int32_t) * std::max<int64_t>(nnz[p], 1));
    oval[p] = obytes;
    obytes += round256(vs * std::max<int64_t>(nnz[p], 1));
  }
  char *ob = static_cast<char *>(mem.get(obytes));
  if (!ob) return bfail(SPGEMM_ENOMEM, "output allocation failed");
  for (int32_t p = 0; p < count; ++p) {
    const size_t vs = A[p].dtype == SPGEMM_F64 ? 8 : 4;
    C[p].rows = A[p].rows;
    C[p].cols = B[p].cols;
    C[p].nnz = nnz[p];
    C[p].row_ptr = reinterpret_cast<int32_t *>(ob + orp[p]);
    C[p].col_idx = reinterpret_cast<int32_t *>(ob + ocol[p]);
    C[p].val = ob + oval[p];
    C[p].dtype = A[p].dtype;
    hp[p].crp = C[p].row_ptr;
    hp[p].ccol = C[p].col_idx;
    hp[p].cval = C[p].val;
    if (!hp[p].batched) {
      bool ok = hipMemcpyAsync(C[p].row_ptr, fb[p].row_ptr, sizeof(int32_t) * (hp[p].m + 1),
                               hipMemcpyDeviceToDevice, s) == hipSuccess;
      if (ok && nnz[p] > 0)
        ok = hipMemcpyAsync(C[p].col_idx, fb[p].col_idx, sizeof(int32_t) * nnz[p],
                            hipMemcpyDeviceToDevice, s) == hipSuccess &&
             hipMemcpyAsync(C[p].val, fb[p].val, vs * nnz[p], hipMemcpyDeviceToDevice, s) ==
                 hipSuccess;
      if (!ok) return bfail(SPGEMM_EHIP, "output copy failed");
    }
  }
  if (!h2d(dprob, hp.data(), sizeof(BmProblem) * count))
    return bfail(SPGEMM_EHIP, "batch table upload failed");
  hipLaunchKernelGGL(k_bm_compact, dim3(static_cast<unsigned int>(rtile.size())), dim3(CP_NT), 0,
                     s, drt, dprob, reinterpret_cast<const int32_t *>(tcol), dCTO, dRO, dRN);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfail(SPGEMM_EHIP, std::string("batch multiply: ") + hipGetErrorString(e));
  mem.keep(ob);
  *out_mem = ob;

  st.fallback = static_cast<int32_t>(fallback.size());
  st.items = nitems;
  for (int c = 0; c < kBatchNumClasses; ++c) st.grid += cls_off[c + 1] > cls_off[c];
  for (int32_t p = 0; p < count; ++p) st.nnz_c += nnz[p];
  st.bytes_scratch = bytes_scratch;
  if (stats) *stats = st;
  return SPGEMM_OK;
}

}  // extern "C"
