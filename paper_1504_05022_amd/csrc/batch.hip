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
  // one launch per class, the largest rows first (their work-groups run
  // longest), one work-group per item
  auto enqueue = [&](hipStream_t st, const int64_t (&off)[kBatchNumClasses + 1], int set) {
    for (int c = kBatchNumClasses - 1; c >= 0; --c) {
      const int64_t n = off[c + 1] - off[c];
      if (n > 0)
        hipLaunchKernelGGL(batch_kernel(set, c), dim3(static_cast<unsigned int>(n)), dim3(ESC_NT),
                           0, st, ditems + off[c], static_cast<const BatchProblem *>(dprob));
    }
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
