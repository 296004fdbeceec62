// Host orchestration and C ABI of libspgemm (declared in include/spgemm.h).
//
// analyze: stage 1 (Algorithm 2, u_i through a scan of the B row lengths)
//          and stage 2 (Algorithm 3, bins; hybrid C~ sizes) on the device,
//          one read-back of a small summary.
// compute: stage 3 per bin group (wavefront ESC for rows up to the last
//          group-4 edge, the merge method for long rows), stage 4 (scan of
//          the row sizes, allocation of C, copy).  One read-back of nnz(C),
//          plus one per long-row pool exhaustion (pool grows 2x, failed
//          long rows resume from their checkpoints).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace spg;

// Fixed device scratch of spgemm_backward_static (one copy per GPU).  Host
// code never uses the symbol itself as an address: the device address is
// looked up once per device (static_scratch_ptr) and passed to the kernels.
static __device__ __align__(256) unsigned char scratch[SPGEMM_STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return SPGEMM_EHIP;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(_e, #expr);   \
  } while (0)

// Bytes requested from the allocator for a buffer of `bytes` (multiples of
// 256, at least 256).
inline size_t alloc_size(size_t bytes) {
  bytes = (bytes + 255) & ~static_cast<size_t>(255);
  return bytes == 0 ? 256 : bytes;
}

struct Allocator {
  spgemm_alloc_fn af = nullptr;
  spgemm_free_fn ff = nullptr;
  void *ctx = nullptr;
  void *get(size_t bytes, hipStream_t s) const {
    bytes = alloc_size(bytes);
    if (af) return af(bytes, ctx, reinterpret_cast<void *>(s));
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void put(void *p, hipStream_t s) const {
    if (!p) return;
    if (ff)
      ff(p, ctx, reinterpret_cast<void *>(s));
    else
      (void)hipFreeAsync(p, s);
  }
};

// Lays out several arrays inside one allocation (256-byte aligned pieces).
struct Layout {
  size_t off = 0;
  template <typename X> size_t add(int64_t n) {
    off = (off + 255) & ~static_cast<size_t>(255);
    const size_t o = off;
    off += static_cast<size_t>(n > 0 ? n : 1) * sizeof(X);
    return o;
  }
  size_t bytes() const { return (off + 255) & ~static_cast<size_t>(255); }
};

template <typename X> X *at(void *base, size_t off) {
  return reinterpret_cast<X *>(static_cast<char *>(base) + off);
}

int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

int dtype_bytes(int dt) { return dt == SPGEMM_F64 ? 8 : 4; }

// A pool chunk holds `entries` columns (int32) then `entries` values.
size_t pool_chunk_bytes(int64_t entries, size_t vbytes) {
  return ((static_cast<size_t>(entries) * 4 + 255) & ~static_cast<size_t>(255)) +
         static_cast<size_t>(entries) * vbytes;
}
Pool pool_view(void *chunk, int64_t entries) {
  Pool hp{};
  hp.col = static_cast<int32_t *>(chunk);
  hp.val = static_cast<char *>(chunk) +
           ((static_cast<size_t>(entries) * 4 + 255) & ~static_cast<size_t>(255));
  hp.cap = static_cast<unsigned long long>(entries);
  hp.top = 0;
  hp.fail_count = 0;
  hp.used = 0;
  return hp;
}

int check_csr(const spgemm_csr *M, const char *name) {
  if (!M) return fail(SPGEMM_EINVAL, std::string(name) + " is NULL");
  if (M->rows < 0 || M->cols < 0 || M->nnz < 0)
    return fail(SPGEMM_EINVAL, std::string(name) + ": negative size");
  if (M->rows >= (int64_t(1) << 31) - 1 || M->cols >= (int64_t(1) << 31) - 1 ||
      M->nnz >= (int64_t(1) << 31))
    return fail(SPGEMM_EOVERFLOW, std::string(name) + ": size exceeds the int32 index range");
  if (M->dtype != SPGEMM_F32 && M->dtype != SPGEMM_F64)
    return fail(SPGEMM_EINVAL, std::string(name) + ": unknown dtype");
  if (!M->row_ptr) return fail(SPGEMM_EINVAL, std::string(name) + ": row_ptr is NULL");
  if (M->nnz > 0 && (!M->col_idx || !M->val))
    return fail(SPGEMM_EINVAL, std::string(name) + ": col_idx/val is NULL");
  return SPGEMM_OK;
}

// Pinned staging for the small device<->host records, one per thread,
// allocated once (hipHostMalloc is far too slow to call per plan).
void *pinned_staging() {
  thread_local void *buf = nullptr;
  if (!buf) {
    if (hipHostMalloc(&buf, 4096, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      buf = nullptr;
    }
  }
  return buf;
}

// Device -> host copy of a small record through the pinned staging area;
// synchronizes the stream.
hipError_t read_small(void *dst, const void *src, size_t bytes, hipStream_t s) {
  void *stage = pinned_staging();
  if (!stage || bytes > 4096) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
  }
  hipError_t e = hipMemcpyAsync(stage, src, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) std::memcpy(dst, stage, bytes);
  return e;
}

}  // namespace

struct spgemm_plan_s {
  // identity of the analyzed inputs
  int64_t m = 0, k = 0, n = 0, nnzA = 0, nnzB = 0;
  const void *arp = nullptr, *acol = nullptr, *brp = nullptr, *bcol = nullptr;
  int dtype = 0;
  spgemm_options opt{};
  BinEdges be{};
  Allocator al;
  hipStream_t stream = nullptr;

  // analyze scratch (one allocation)
  void *ws = nullptr;
  size_t ws_bytes = 0;
  int64_t *P = nullptr, *u = nullptr, *h = nullptr, *cto = nullptr, *rownnz = nullptr,
          *rowoff = nullptr, *hist_scan = nullptr, *part = nullptr;
  int32_t *hist = nullptr, *binlist = nullptr;
  int64_t *bpart = nullptr;
  int64_t nblocks = 0;
  LongParams lp{};
  int l1cap = 0;
  Summary *dsum = nullptr;
  ComputeStatus *dstat = nullptr;
  Pool *dpool = nullptr;
  int64_t nwaves = 0;

  // host mirrors
  Summary *hsum = nullptr;
  ComputeStatus *hstat = nullptr;
  Pool *hpool = nullptr;
  Summary hsum_store{};
  ComputeStatus hstat_store{};
  Pool hpool_store{};

  // compute scratch
  void *cws = nullptr;
  size_t cws_bytes = 0;
  std::vector<void *> pool_chunks;
  size_t pool_bytes = 0;  // allocated for pool_chunks

  // backward scratch: A's transposed pattern, built on first use
  void *bws = nullptr;
  size_t bws_bytes = 0;
  int32_t *tcnt = nullptr, *trow = nullptr, *tpos = nullptr;
  int64_t *tptr = nullptr, *tpart = nullptr;

  // second stream for the short-row kernels (from a per-device pool) and
  // the events that fork it from and join it to the caller's stream
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;

  spgemm_info info{};
  hipEvent_t ev[2 * SPGEMM_NSTAGES] = {};
  bool events = false;
  int dev = 0;              // device the events belong to
  uint32_t tmask = 0;       // stages to time
  uint32_t stage_mask = 0;  // stages recorded since the last read-back
};

extern "C" {

void spgemm_default_options(spgemm_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->bin_edges[0] = 32;
  o->bin_edges[1] = 64;
  o->bin_edges[2] = 128;
  o->bin_edges[3] = 256;
  o->bin_edges[4] = 512;
  o->long_slot = 256;
  o->l1_cap = 0;
  o->seg = 0;
  o->pool_entries = 0;
  o->validate = 0;
  o->timing = 0;
}

const char *spgemm_strerror(int code) {
  switch (code) {
    case SPGEMM_OK: return "success";
    case SPGEMM_EINVAL: return "invalid argument";
    case SPGEMM_ENOMEM: return "device allocation failed";
    case SPGEMM_EOVERFLOW: return "size exceeds the index type";
    case SPGEMM_EHIP: return "HIP runtime error";
    case SPGEMM_ESTATE: return "plan used with other matrices";
    default: return "unknown status";
  }
}

const char *spgemm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

// Timing events outlive plans: created once per device and reused, since
// creating and destroying two dozen events per plan costs more host time
// than the kernels of a small product take.
std::mutex g_ev_mu;
std::vector<std::pair<int, hipEvent_t>> g_ev_free;

hipError_t take_event(int dev, hipEvent_t *e) {
  {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    for (size_t i = g_ev_free.size(); i-- > 0;) {
      if (g_ev_free[i].first == dev) {
        *e = g_ev_free[i].second;
        g_ev_free.erase(g_ev_free.begin() + static_cast<std::ptrdiff_t>(i));
        return hipSuccess;
      }
    }
  }
  return hipEventCreate(e);
}

void give_event(int dev, hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_ev_mu);
  g_ev_free.emplace_back(dev, e);
}

// Auxiliary streams outlive plans too (one is taken per plan that computes
// and returned when the plan is destroyed); default priority, not
// synchronized with the null stream.
std::vector<std::pair<int, hipStream_t>> g_aux_free;

hipError_t take_aux(int dev, hipStream_t *st) {
  {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    for (size_t i = g_aux_free.size(); i-- > 0;) {
      if (g_aux_free[i].first == dev) {
        *st = g_aux_free[i].second;
        g_aux_free.erase(g_aux_free.begin() + static_cast<std::ptrdiff_t>(i));
        return hipSuccess;
      }
    }
  }
  return hipStreamCreateWithFlags(st, hipStreamNonBlocking);
}

void give_aux(int dev, hipStream_t st) {
  if (!st) return;
  std::lock_guard<std::mutex> lk(g_ev_mu);
  g_aux_free.emplace_back(dev, st);
}

// Forks the plan's auxiliary stream from `s` (its work then follows
// everything enqueued on `s` so far).  False when no stream or event could
// be had: the caller then stays on `s`.
bool fork_aux(spgemm_plan p, hipStream_t s) {
  if (!p->aux) {
    hipStream_t st = nullptr;
    if (take_aux(p->dev, &st) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    p->aux = st;
  }
  if (!p->fork_ev && take_event(p->dev, &p->fork_ev) != hipSuccess) p->fork_ev = nullptr;
  if (!p->join_ev && take_event(p->dev, &p->join_ev) != hipSuccess) p->join_ev = nullptr;
  if (!p->fork_ev || !p->join_ev) {
    (void)hipGetLastError();
    return false;
  }
  return hipEventRecord(p->fork_ev, s) == hipSuccess &&
         hipStreamWaitEvent(p->aux, p->fork_ev, 0) == hipSuccess;
}

// Makes `s` wait for everything enqueued on the auxiliary stream.
void join_aux(spgemm_plan p, hipStream_t s) {
  if (!p->aux || !p->join_ev) return;
  (void)hipEventRecord(p->join_ev, p->aux);
  (void)hipStreamWaitEvent(s, p->join_ev, 0);
}

void release_compute(spgemm_plan p, hipStream_t s) {
  p->al.put(p->cws, s);
  p->cws = nullptr;
  p->cws_bytes = 0;
  for (void *c : p->pool_chunks) p->al.put(c, s);
  p->pool_chunks.clear();
  p->pool_bytes = 0;
}

// Device memory the plan holds now, as requested from the allocator
// (analysis, C~ and long-row tables, pool chunks, A's transposed pattern).
// At the end of compute (C~ still held, released on return) this is the
// call's peak apart from C itself.
int64_t held_bytes(spgemm_plan p) {
  size_t b = p->pool_bytes;
  if (p->ws) b += alloc_size(p->ws_bytes);
  if (p->cws) b += alloc_size(p->cws_bytes);
  if (p->bws) b += alloc_size(p->bws_bytes);
  return static_cast<int64_t>(b);
}

void destroy_plan(spgemm_plan p) {
  if (!p) return;
  release_compute(p, p->stream);
  p->al.put(p->ws, p->stream);
  p->al.put(p->bws, p->stream);
  if (p->events)
    for (auto &e : p->ev) give_event(p->dev, e);
  give_event(p->dev, p->fork_ev);
  give_event(p->dev, p->join_ev);
  give_aux(p->dev, p->aux);
  delete p;
}

int check_options(const spgemm_options &o) {
  const int32_t *e = o.bin_edges;
  if (e[0] < 1 || e[0] > 32) return fail(SPGEMM_EINVAL, "bin_edges[0] must be in [1, 32]");
  for (int i = 1; i < 5; ++i)
    if (e[i] <= e[i - 1]) return fail(SPGEMM_EINVAL, "bin_edges must increase");
  if (e[4] > 1024) return fail(SPGEMM_EINVAL, "bin_edges[4] must be <= 1024");
  if (o.long_slot < 1 || o.long_slot > (1 << 20))
    return fail(SPGEMM_EINVAL, "long_slot must be in [1, 2^20]");
  if (o.l1_cap != 0 && o.l1_cap != 2048 && o.l1_cap != 3072 && o.l1_cap != 5120 &&
      o.l1_cap != 7168)
    return fail(SPGEMM_EINVAL, "l1_cap must be 0, 2048, 3072, 5120 or 7168");
  if (o.pool_entries < 0) return fail(SPGEMM_EINVAL, "pool_entries must be >= 0");
  if (o.long_path < 0 || o.long_path > 2) return fail(SPGEMM_EINVAL, "long_path must be 0, 1 or 2");
  if (o.long_direct < 0 || o.long_direct > 1) return fail(SPGEMM_EINVAL, "long_direct must be 0 or 1");
  if (o.batch_shapes < 0 || o.batch_shapes > 3)
    return fail(SPGEMM_EINVAL, "batch_shapes must be 0 (autotune) or 1..3");
  if (o.timing_mask < 0 || o.timing_mask >= (1 << SPGEMM_NSTAGES))
    return fail(SPGEMM_EINVAL, "timing_mask has bits beyond the stage count");
  return SPGEMM_OK;
}

bool timed(spgemm_plan p, int st) { return p->events && (p->tmask & (1u << st)); }
void stage_begin(spgemm_plan p, int st, hipStream_t s) {
  if (!timed(p, st)) return;
  (void)hipEventRecord(p->ev[2 * st], s);
  p->stage_mask |= 1u << st;
}
void stage_end(spgemm_plan p, int st, hipStream_t s) {
  if (timed(p, st)) (void)hipEventRecord(p->ev[2 * st + 1], s);
}

}  // namespace

extern "C" int spgemm_analyze(const spgemm_csr *A, const spgemm_csr *B,
                              const spgemm_options *opt, spgemm_alloc_fn alloc_fn,
                              spgemm_free_fn free_fn, void *ctx, void *stream,
                              spgemm_plan *plan, spgemm_info *info) {
  if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
  *plan = nullptr;
  int rc;
  if ((rc = check_csr(A, "A")) != SPGEMM_OK) return rc;
  if ((rc = check_csr(B, "B")) != SPGEMM_OK) return rc;
  if (A->cols != B->rows)
    return fail(SPGEMM_EINVAL, "inner dimensions differ (A.cols != B.rows)");
  if (A->dtype != B->dtype) return fail(SPGEMM_EINVAL, "A and B have different dtypes");
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(SPGEMM_EINVAL, "alloc_fn and free_fn must both be set or both be NULL");
  spgemm_options o;
  spgemm_default_options(&o);
  if (opt) o = *opt;
  if ((rc = check_options(o)) != SPGEMM_OK) return rc;

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  spgemm_plan p = new (std::nothrow) spgemm_plan_s();
  if (!p) return fail(SPGEMM_ENOMEM, "host allocation failed");
  p->m = A->rows;
  p->k = A->cols;
  p->n = B->cols;
  p->nnzA = A->nnz;
  p->nnzB = B->nnz;
  p->arp = A->row_ptr;
  p->acol = A->col_idx;
  p->brp = B->row_ptr;
  p->bcol = B->col_idx;
  p->dtype = A->dtype;
  p->opt = o;
  for (int i = 0; i < 5; ++i) p->be.e[i] = o.bin_edges[i];
  p->al.af = alloc_fn;
  p->al.ff = free_fn;
  p->al.ctx = ctx;
  p->stream = s;

  const int64_t m = p->m;
  p->nwaves = (m + 63) / 64;  // one histogram column per 64-row wavefront
  p->nblocks = (m + 255) / 256;
  p->l1cap = o.l1_cap ? o.l1_cap : long_l1cap_default(dtype_bytes(p->dtype));
  // defaults: a row of up to kWaveTile products is one item; longer rows are
  // cut into segments of kWaveTile / 2 (one wavefront each, at twice the
  // occupancy of a full tile), and combine ranges aim at kWaveTile / 4
  p->lp.segp = o.seg < 0 ? -1 : (o.seg > 0 ? o.seg : kWaveTile / 2);
  p->lp.single = o.seg != 0 ? 0 : kWaveTile;
  p->lp.maxs = combine_maxs();
  p->lp.cb = kWaveTile / 4;
  p->lp.minw_shift = 4;
  p->lp.maxw_shift = 30;
  const int64_t nh = static_cast<int64_t>(NBINS) * p->nwaves;
  int64_t partn = scan_part_len(std::max<int64_t>({p->nnzA, m, nh, 1}));
  Layout L;
  const size_t oP = L.add<int64_t>(p->nnzA + 1);
  const size_t ou = L.add<int64_t>(m);
  const size_t oh = L.add<int64_t>(m);
  const size_t octo = L.add<int64_t>(m + 1);
  const size_t onnz = L.add<int64_t>(m);
  const size_t ooff = L.add<int64_t>(m + 1);
  const size_t ohs = L.add<int64_t>(nh + 1);
  const size_t opart = L.add<int64_t>(partn);
  const size_t ohist = L.add<int32_t>(nh);
  const size_t obl = L.add<int32_t>(m);
  const size_t obp = L.add<int64_t>(p->nblocks * kBlockStats);
  const size_t osum = L.add<Summary>(1);
  const size_t ostat = L.add<ComputeStatus>(1);
  const size_t opool = L.add<Pool>(1);
  p->ws_bytes = L.bytes();
  p->ws = p->al.get(p->ws_bytes, s);
  if (!p->ws) {
    destroy_plan(p);
    return fail(SPGEMM_ENOMEM, "analyze scratch allocation failed");
  }
  p->P = at<int64_t>(p->ws, oP);
  p->u = at<int64_t>(p->ws, ou);
  p->h = at<int64_t>(p->ws, oh);
  p->cto = at<int64_t>(p->ws, octo);
  p->rownnz = at<int64_t>(p->ws, onnz);
  p->rowoff = at<int64_t>(p->ws, ooff);
  p->hist_scan = at<int64_t>(p->ws, ohs);
  p->part = at<int64_t>(p->ws, opart);
  p->hist = at<int32_t>(p->ws, ohist);
  p->binlist = at<int32_t>(p->ws, obl);
  p->bpart = at<int64_t>(p->ws, obp);
  p->dsum = at<Summary>(p->ws, osum);
  p->dstat = at<ComputeStatus>(p->ws, ostat);
  p->dpool = at<Pool>(p->ws, opool);

  // host mirrors of the small records (read-backs go through pinned staging)
  p->hsum = &p->hsum_store;
  p->hstat = &p->hstat_store;
  p->hpool = &p->hpool_store;
  (void)hipGetDevice(&p->dev);
  if (o.timing) {
    p->tmask = o.timing_mask ? static_cast<uint32_t>(o.timing_mask)
                             : (1u << SPGEMM_NSTAGES) - 1u;
    for (auto &e : p->ev) {
      if (take_event(p->dev, &e) != hipSuccess) {
        destroy_plan(p);
        return fail(SPGEMM_EHIP, "hipEventCreate failed");
      }
    }
    p->events = true;
  }

  launch_zero(p->dsum, sizeof(Summary), s);
  if (o.validate) {
    // checked before any kernel indexes with the inputs
    launch_validate(A->row_ptr, A->col_idx, A->rows, A->cols, A->nnz, p->dsum, s);
    launch_validate(B->row_ptr, B->col_idx, B->rows, B->cols, B->nnz, p->dsum, s);
    hipError_t ve = read_small(p->hsum, p->dsum, sizeof(Summary), s);
    if (ve != hipSuccess) {
      destroy_plan(p);
      return hip_fail(ve, "validate");
    }
    if (p->hsum->err) {
      destroy_plan(p);
      return fail(SPGEMM_EINVAL, "input CSR failed validation (row_ptr or column order/range)");
    }
  }
  stage_begin(p, SPGEMM_T_UPPER, s);
  // stage 1 (Algorithm 2): P = exclusive scan of nnz(b_j*) over A's entries,
  // so u_i = P[arp[i+1]] - P[arp[i]].
  scan_row_lengths(A->col_idx, B->row_ptr, p->nnzA, p->P, p->part, s);
  {
    RowStatsArgs ra;
    ra.arp = A->row_ptr;
    ra.P = p->P;
    ra.m = m;
    ra.ncols = p->n;
    ra.be = p->be;
    ra.long_slot = o.long_slot;
    ra.l1cap = p->l1cap;
    ra.vbytes = dtype_bytes(p->dtype);
    ra.lp = p->lp;
    ra.u = p->u;
    ra.h = p->h;
    ra.hist = p->hist;
    ra.nwaves = p->nwaves;
    ra.rownnz = p->rownnz;
    ra.bpart = p->bpart;
    launch_row_stats(ra, s);
  }
  stage_end(p, SPGEMM_T_UPPER, s);
  // stage 2 (Algorithm 3): C~ offsets and the stable bin lists
  stage_begin(p, SPGEMM_T_BIN, s);
  scan_i64(p->h, m, p->cto, p->part, s);
  scan_i32(p->hist, nh, p->hist_scan, p->part, s);
  launch_bin_scatter(p->u, m, p->be, p->hist_scan, p->nwaves, p->binlist, s);
  launch_summary(p->P, p->nnzA, p->cto, m, p->hist_scan, p->nwaves, p->bpart, p->nblocks,
                 p->dsum, s);
  stage_end(p, SPGEMM_T_BIN, s);
  hipError_t e = read_small(p->hsum, p->dsum, sizeof(Summary), s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    destroy_plan(p);
    return hip_fail(e, "analyze");
  }
  const Summary &S = *p->hsum;
  if (S.err) {
    destroy_plan(p);
    return fail(SPGEMM_EINVAL, "input CSR failed validation (row_ptr or column order/range)");
  }
  if (S.max_u >= (1ull << 31)) {
    destroy_plan(p);
    return fail(SPGEMM_EOVERFLOW, "a row of C has 2^31 or more products");
  }
  spgemm_info &I = p->info;
  std::memset(&I, 0, sizeof(I));
  I.m = p->m;
  I.k = p->k;
  I.n = p->n;
  I.nnz_hat = S.sum_u;
  I.flops = 2 * S.sum_u;
  I.nnz_tilde = S.sum_h;
  I.nnz_c = -1;
  I.max_u = static_cast<int64_t>(S.max_u);
  for (int b = 0; b < NBINS; ++b) I.bin_count[b] = S.bin_off[b + 1] - S.bin_off[b];
  I.long_items = S.n_items;
  I.bytes_scratch = held_bytes(p);
  for (int st : {SPGEMM_T_UPPER, SPGEMM_T_BIN})
    if (timed(p, st)) (void)hipEventElapsedTime(&I.stage_ms[st], p->ev[2 * st], p->ev[2 * st + 1]);
  if (info) *info = I;
  *plan = p;
  return SPGEMM_OK;
}

namespace {

template <typename T>
int compute_t(spgemm_plan p, const spgemm_csr *A, const spgemm_csr *B, spgemm_csr_out *C,
              hipStream_t s) {
  const Summary &S = *p->hsum;
  spgemm_info &I = p->info;
  const int64_t m = p->m;
  const int64_t nlong = I.bin_count[LONG_BIN];
  release_compute(p, s);

  // long rows: column windows (by default when every long row is a direct
  // dense row, i.e. B has at most kDenseCols columns), else product
  // segments and column ranges with the merge method
  const int64_t kDenseCols = int64_t(1) << win_dense_log(static_cast<int>(sizeof(T)));
  const bool want_win = p->opt.long_path == 2 || (p->opt.long_path == 0 && p->n <= kDenseCols);
  const bool use_win = nlong > 0 && p->opt.seg == 0 && want_win && S.w_none == 0;
  const bool legacy = nlong > 0 && !use_win;
  // merge method with direct output: a counting pass sizes the pieces of
  // split rows after phase 1, and phase 2 writes them straight into C
  const bool direct =
      legacy && p->opt.long_direct && S.n_split > 0 && long_direct_ok(p->lp, p->n);
  // C~ (hybrid sizes) plus the long-row tables in one allocation
  const int64_t nitems = legacy ? S.n_items : 0;
  const int64_t npieces = legacy ? S.n_pieces : 0;
  const int64_t w_items = use_win ? S.w_items : 0;
  const int64_t w_segs = use_win ? S.w_segs : 0;
  const int64_t w_slots = use_win ? S.w_dslots : 0;
  const int64_t w_nwords = (p->n + 31) / 32;
  Layout L;
  const size_t octc = L.add<int32_t>(S.sum_h);
  const size_t octv = L.add<T>(S.sum_h);
  const size_t olr = L.add<LongRow>(nlong);
  const size_t oit = L.add<LongItem>(nitems);
  const size_t ost = L.add<LongState>(nitems);
  const size_t opa = L.add<Seq>(nitems);
  const size_t ofa = L.add<unsigned int>(nitems);
  const size_t ofb = L.add<unsigned int>(nitems);
  const size_t ocs = L.add<LongState>(npieces);
  const size_t of2a = L.add<unsigned int>(npieces);
  const size_t of2b = L.add<unsigned int>(npieces);
  const size_t opc = L.add<Piece>(npieces);
  const size_t opl = L.add<int32_t>(npieces);
  const size_t ops = L.add<int64_t>(npieces + 1);
  const size_t opp = L.add<int64_t>(scan_part_len(std::max<int64_t>(npieces, 1)));
  const size_t osp = L.add<int32_t>(legacy ? S.n_split : 0);
  const size_t opbc = L.add<int32_t>(legacy ? S.sum_u_multi : 0);
  const size_t opbv = L.add<T>(legacy ? S.sum_u_multi : 0);
  const size_t oobc = L.add<int32_t>(legacy && !direct ? S.sum_u_multi : 0);
  const size_t oobv = L.add<T>(legacy && !direct ? S.sum_u_multi : 0);
  const size_t otmp = L.add<int64_t>(legacy ? long_table_tmp_len(nlong) : 0);
  // window method
  const size_t owr = L.add<WinRow>(use_win ? nlong : 0);
  const size_t owi = L.add<WinWork>(w_items);
  const size_t ows = L.add<WinWork>(w_segs);
  const size_t owsl = L.add<int32_t>(w_slots);
  const size_t owb = L.add<int64_t>(use_win ? 5 * ((nlong + 255) / 256) : 0);
  const size_t owt = L.add<uint16_t>(use_win ? S.w_table : 0);
  const size_t owpk = L.add<uint32_t>(use_win ? S.w_partial : 0);
  const size_t owpv = L.add<T>(use_win ? S.w_partial : 0);
  const size_t owdb = L.add<uint32_t>(w_slots * w_nwords);
  const size_t owda = L.add<T>(w_slots * p->n);
  const size_t owc = L.add<int64_t>(w_items);
  const size_t owis = L.add<int64_t>(use_win ? w_items + 1 : 0);
  const size_t owpp = L.add<int64_t>(use_win ? scan_part_len(std::max<int64_t>(w_items, 1)) : 0);
  const size_t owl = L.add<uint32_t>(use_win ? w_items + 1 : 0);
  const size_t ocnt = L.add<LongCounters>(1);
  const size_t ogl = L.add<unsigned int>(nitems);
  const size_t ogl2 = L.add<unsigned int>(npieces);
  const size_t ol1 = L.add<unsigned int>(nitems);
  const size_t olw = L.add<unsigned int>(nitems);
  const size_t ol2 = L.add<unsigned int>(npieces);
  const size_t ol3 = L.add<unsigned int>(npieces);
  p->cws_bytes = L.bytes();
  p->cws = p->al.get(p->cws_bytes, s);
  if (!p->cws) return fail(SPGEMM_ENOMEM, "C~ allocation failed");
  int32_t *ct_col = at<int32_t>(p->cws, octc);
  T *ct_val = at<T>(p->cws, octv);
  LongRow *lrows = at<LongRow>(p->cws, olr);
  LongItem *items = at<LongItem>(p->cws, oit);
  LongState *states = at<LongState>(p->cws, ost);
  Seq *partials = at<Seq>(p->cws, opa);
  unsigned int *fail_a = at<unsigned int>(p->cws, ofa);
  unsigned int *fail_b = at<unsigned int>(p->cws, ofb);
  LongState *cstates = at<LongState>(p->cws, ocs);
  unsigned int *fail2_a = at<unsigned int>(p->cws, of2a);
  unsigned int *fail2_b = at<unsigned int>(p->cws, of2b);
  Piece *pieces = at<Piece>(p->cws, opc);
  int32_t *piece_lrow = at<int32_t>(p->cws, opl);
  int64_t *pscan = at<int64_t>(p->cws, ops);
  int64_t *ppart = at<int64_t>(p->cws, opp);
  int32_t *split = at<int32_t>(p->cws, osp);
  int32_t *pcol = at<int32_t>(p->cws, opbc);
  T *pval = at<T>(p->cws, opbv);
  int32_t *ocol = at<int32_t>(p->cws, oobc);
  T *oval = at<T>(p->cws, oobv);
  int64_t *lt_tmp = at<int64_t>(p->cws, otmp);
  LongCounters *lcnt = at<LongCounters>(p->cws, ocnt);
  unsigned int *glist = at<unsigned int>(p->cws, ogl);
  unsigned int *glist2 = at<unsigned int>(p->cws, ogl2);
  unsigned int *list1 = at<unsigned int>(p->cws, ol1);
  unsigned int *listw = at<unsigned int>(p->cws, olw);
  unsigned int *list2 = at<unsigned int>(p->cws, ol2);
  unsigned int *list3 = at<unsigned int>(p->cws, ol3);
  WinRow *wrows = at<WinRow>(p->cws, owr);
  WinWork *witems = at<WinWork>(p->cws, owi);
  WinWork *wsegs = at<WinWork>(p->cws, ows);
  int32_t *wslot = at<int32_t>(p->cws, owsl);
  int64_t *wbsum = at<int64_t>(p->cws, owb);
  uint16_t *wtable = at<uint16_t>(p->cws, owt);
  uint32_t *wpkey = at<uint32_t>(p->cws, owpk);
  T *wpval = at<T>(p->cws, owpv);
  uint32_t *wdbits = at<uint32_t>(p->cws, owdb);
  T *wdacc = at<T>(p->cws, owda);
  int64_t *wcnt = at<int64_t>(p->cws, owc);
  int64_t *wiscan = at<int64_t>(p->cws, owis);
  int64_t *wpart = at<int64_t>(p->cws, owpp);
  uint32_t *wlist = at<uint32_t>(p->cws, owl);  // [0]: count, then item ids

  EscArgs<T> ea;
  ea.arp = A->row_ptr;
  ea.acol = A->col_idx;
  ea.aval = static_cast<const T *>(A->val);
  ea.brp = B->row_ptr;
  ea.bcol = B->col_idx;
  ea.bval = static_cast<const T *>(B->val);
  ea.P = p->P;
  ea.u = p->u;
  ea.cto = p->cto;
  ea.ct_col = ct_col;
  ea.ct_val = ct_val;
  ea.rownnz = p->rownnz;

  // the short-row kernels run on a second stream, beside the long-row work
  // on the caller's stream: forked here, once C~ exists (the second stream
  // waits for what the caller's stream holds now, not for the long-row
  // kernels queued next), queued after the first long-row kernels so that
  // the host gets those going first, joined before the row sizes are scanned
  const hipStream_t es = fork_aux(p, s) ? p->aux : s;
  bool short_done = false;
  auto launch_short_rows = [&]() -> int {
    if (short_done) return SPGEMM_OK;
    short_done = true;
    // ---- bin group 4: the four range bins, the largest first: its kernel
    // runs long enough for the host to queue the short ones behind it
    stage_begin(p, SPGEMM_T_MEDIUM, es);
    for (int b = 36; b >= 33; --b) {
      const int cap = static_cast<int>(next_pow2(p->be.e[b - 32]));
      const int64_t r0 = S.bin_off[b], r1 = S.bin_off[b + 1];
      if (launch_esc<T>(ea, p->binlist + r0, r1 - r0, cap, p->n, es))
        return fail(SPGEMM_EINVAL, "no ESC kernel for this capacity");
    }
    stage_end(p, SPGEMM_T_MEDIUM, es);
    // ---- stage 3, bin groups 2-3: one launch per power-of-two capacity
    stage_begin(p, SPGEMM_T_TINY, es);
    if (p->opt.tiny_heap) {
      // bin 1 through the wavefront kernel, bins 2..edge[0] one kernel each
      if (launch_esc<T>(ea, p->binlist + S.bin_off[1], S.bin_off[2] - S.bin_off[1], 1, p->n, es))
        return fail(SPGEMM_EINVAL, "no ESC kernel for this capacity");
      for (int b = 2; b <= p->be.e[0]; ++b)
        if (launch_heap<T>(ea, p->binlist + S.bin_off[b], S.bin_off[b + 1] - S.bin_off[b], b, es))
          return fail(SPGEMM_EINVAL, "no heap kernel for this size");
    } else {
      int b = 1;
      while (b <= p->be.e[0]) {
        const int cap = static_cast<int>(next_pow2(b));
        const int hi = std::min<int>(cap, p->be.e[0]);
        const int64_t r0 = S.bin_off[b], r1 = S.bin_off[hi + 1];
        if (launch_esc<T>(ea, p->binlist + r0, r1 - r0, cap, p->n, es))
          return fail(SPGEMM_EINVAL, "no ESC kernel for this capacity");
        b = hi + 1;
      }
    }
    stage_end(p, SPGEMM_T_TINY, es);
    return SPGEMM_OK;
  };

  // ---- bin group 5: long rows (merge method, split over work-groups)
  int64_t pool_entries = 0;
  I.realloc_rounds = 0;
  I.long_launches = 0;
  I.long_kernel_ms = 0.f;
  LongArgs<T> la;
  la.e = ea;
  la.lrows = lrows;
  la.items = items;
  la.work = nullptr;
  la.state = states;
  la.pool = p->dpool;
  la.fail_list = fail_a;
  la.long_slot = p->opt.long_slot;
  la.partials = partials;
  la.pcol = pcol;
  la.pval = pval;
  la.ocol = ocol;
  la.oval = oval;
  la.split = split;
  la.pieces = pieces;
  la.piece_lrow = piece_lrow;
  la.cstate = cstates;
  la.fail_list2 = fail2_a;
  la.cnt = lcnt;
  la.glist = glist;
  la.glist2 = glist2;
  la.list1 = list1;
  la.listw = listw;
  la.list2 = list2;
  la.list3 = list3;
  la.ncols = p->n;
  la.direct = direct ? 1 : 0;
  la.c_col = nullptr;
  la.c_val = nullptr;
  la.rowoff = p->rowoff;
  la.pscan = pscan;
  const bool spill_expected = S.spill_bound > 0 || p->opt.pool_entries > 0;
  auto new_pool = [&](int64_t entries, unsigned long long used) -> int {
    void *chunk = p->al.get(pool_chunk_bytes(entries, sizeof(T)), s);
    if (!chunk) return fail(SPGEMM_ENOMEM, "long-row pool allocation failed");
    p->pool_chunks.push_back(chunk);
    p->pool_bytes += alloc_size(pool_chunk_bytes(entries, sizeof(T)));
    *p->hpool = pool_view(chunk, entries);
    p->hpool->used = used;
    launch_set_pool(p->dpool, *p->hpool, s);
    return SPGEMM_OK;
  };
  auto read_status = [&]() -> int {
    launch_status(p->rowoff, m, p->dpool, p->dstat, s);
    HIP_TRY(read_small(p->hstat, p->dstat, sizeof(ComputeStatus), s));
    HIP_TRY(hipGetLastError());
    return SPGEMM_OK;
  };
  auto finish_long = [&]() {
    // long-row sizes from their pieces
    scan_piece_counts(pieces, npieces, pscan, ppart, s);
    launch_long_rownnz(lrows, nlong, pscan, p->rownnz, s);
  };
  int rc;
  if (use_win) {
    // window method: plan, partition, symbolic pass, long-row sizes
    stage_begin(p, SPGEMM_T_LONG, s);
    win_plan_launch(p->binlist + S.bin_off[LONG_BIN], nlong, p->u, p->n, static_cast<int>(sizeof(T)),
                    wbsum, wrows, witems, w_items, wsegs, w_segs, wslot, w_slots, A->row_ptr, p->P,
                    s);
    if ((rc = launch_short_rows()) != SPGEMM_OK) return rc;
    stage_begin(p, SPGEMM_T_LONG_WAVE, s);
    win_partition<T>(ea, wrows, wsegs, w_segs, wtable, wpkey, wpval, s);
    stage_end(p, SPGEMM_T_LONG_WAVE, s);
    stage_begin(p, SPGEMM_T_LONG_SYM, s);
    win_symbolic<T>(ea, p->n, wrows, witems, w_items, wtable, wpkey, wslot, w_slots, wlist + 1,
                    wlist, wdbits, wcnt, s);
    stage_end(p, SPGEMM_T_LONG_SYM, s);
    scan_i64(wcnt, w_items, wiscan, wpart, s);
    win_rownnz(wrows, nlong, wiscan, p->rownnz, s);
    stage_end(p, SPGEMM_T_LONG, s);
  } else if (nlong > 0) {
    pool_entries = p->opt.pool_entries
                       ? p->opt.pool_entries
                       : S.pool_single + 3 * S.spill_bound + 65536;
    if ((rc = new_pool(pool_entries, 0)) != SPGEMM_OK) return rc;
    launch_long_table(p->binlist, S.bin_off[LONG_BIN], nlong, p->u, p->n, p->lp, lrows, nitems,
                      items, states, partials, npieces, piece_lrow, A->row_ptr, p->P, lt_tmp, s);
    launch_cstate_init(cstates, npieces, lcnt, s);
    // phase 1: every segment; one wavefront, else one work-group tile, else
    // the level-1 merge method
    stage_begin(p, SPGEMM_T_LONG, s);
    stage_begin(p, SPGEMM_T_LONG_WAVE, s);
    launch_long_wave<T>(la, nitems, s);
    stage_end(p, SPGEMM_T_LONG_WAVE, s);
    if ((rc = launch_short_rows()) != SPGEMM_OK) return rc;
    launch_long_wave_large<T>(la, nitems, s);
    launch_long_oneshot<T>(la, nitems, s);
    if (launch_long<T>(la, nitems, p->l1cap, s))
      return fail(SPGEMM_EINVAL, "no long-row kernel for this l1_cap");
    I.long_launches++;
    stage_end(p, SPGEMM_T_LONG, s);
    // pool exhaustion in phase 1 only when L1 can spill: relaunch from checkpoints
    if (spill_expected) {
      unsigned int *fl = fail_a, *fl_other = fail_b;
      for (;;) {
        if ((rc = read_status()) != SPGEMM_OK) return rc;
        const unsigned int nfail = p->hstat->fail_count;
        if (nfail == 0) break;
        if (++I.realloc_rounds > 64) return fail(SPGEMM_ENOMEM, "long-row pool keeps overflowing");
        pool_entries *= 2;
        if ((rc = new_pool(pool_entries, p->hstat->pool_used)) != SPGEMM_OK) return rc;
        la.work = reinterpret_cast<const int32_t *>(fl);
        la.fail_list = fl_other;
        if (launch_long<T>(la, nfail, p->l1cap, s))
          return fail(SPGEMM_EINVAL, "no long-row kernel for this l1_cap");
        I.long_launches++;
        std::swap(fl, fl_other);
      }
      la.work = nullptr;
      la.fail_list = fail_a;
    }
    // phase 2: every output piece of the multi-segment rows (with direct
    // output: only their sizes now, the pieces after C is allocated)
    if (direct) {
      stage_begin(p, SPGEMM_T_LONG_SYM, s);
      launch_piece_count<T>(la, npieces, s);
      stage_end(p, SPGEMM_T_LONG_SYM, s);
    } else if (S.n_split > 0) {  // some row was split
      stage_begin(p, SPGEMM_T_COMBINE, s);
      stage_begin(p, SPGEMM_T_COMBINE_WAVE, s);
      launch_combine_wave<T>(la, npieces, s);
      stage_end(p, SPGEMM_T_COMBINE_WAVE, s);
      launch_combine_wave_large<T>(la, npieces, s);
      launch_combine_oneshot<T>(la, npieces, s);
      launch_combine<T>(la, npieces, s);
      stage_end(p, SPGEMM_T_COMBINE, s);
    }
    finish_long();
  }

  // ---- stage 4a: row pointers of C (exclusive scan of the row sizes)
  if ((rc = launch_short_rows()) != SPGEMM_OK) return rc;  // no long rows
  if (es != s) join_aux(p, s);
  stage_begin(p, SPGEMM_T_SCAN, s);
  scan_i64(p->rownnz, m, p->rowoff, p->part, s);
  stage_end(p, SPGEMM_T_SCAN, s);
  // C's row pointers have a known size: allocated while the GPU is busy,
  // released again if anything below fails
  struct OwnedBuf {
    const Allocator &al;
    hipStream_t s;
    void *p;
    ~OwnedBuf() { al.put(p, s); }
  } crp_guard{p->al, s, p->al.get(static_cast<size_t>(m + 1) * 4, s)};
  if (!crp_guard.p) return fail(SPGEMM_ENOMEM, "allocation of C failed");
  {
    unsigned int *f2 = fail2_a, *f2_other = fail2_b;
    unsigned int *fl = fail_a, *fl_other = fail_b;
    for (;;) {
      if ((rc = read_status()) != SPGEMM_OK) return rc;
      const unsigned int nf1 = legacy ? p->hstat->fail_count : 0u;
      const unsigned int nf2 = legacy ? p->hstat->fail2 : 0u;
      if (nf1 == 0 && nf2 == 0) break;
      if (++I.realloc_rounds > 64) return fail(SPGEMM_ENOMEM, "long-row pool keeps overflowing");
      pool_entries *= 2;
      if ((rc = new_pool(pool_entries, p->hstat->pool_used)) != SPGEMM_OK) return rc;
      if (nf1 > 0) {
        // phase-1 items resume from their checkpoints; phase 2 then reruns
        la.work = reinterpret_cast<const int32_t *>(fl);
        la.fail_list = fl_other;
        launch_long<T>(la, nf1, p->l1cap, s);
        I.long_launches++;
        std::swap(fl, fl_other);
        la.work = nullptr;
        la.fail_list = fl;
        launch_cstate_init(cstates, npieces, lcnt, s);
        la.fail_list2 = f2;
        if (direct) {
          launch_piece_count<T>(la, npieces, s);
        } else if (S.n_split > 0) {  // some row was split
          launch_combine_wave<T>(la, npieces, s);
          launch_combine_wave_large<T>(la, npieces, s);
          launch_combine_oneshot<T>(la, npieces, s);
          launch_combine<T>(la, npieces, s);
        }
      } else {
        la.work = reinterpret_cast<const int32_t *>(f2);
        la.fail_list2 = f2_other;
        launch_combine<T>(la, nf2, s);
        std::swap(f2, f2_other);
        la.work = nullptr;
      }
      finish_long();
      scan_i64(p->rownnz, m, p->rowoff, p->part, s);
    }
  }
  const int64_t nnz = p->hstat->nnz_c;
  if (nnz >= (int64_t(1) << 31)) return fail(SPGEMM_EOVERFLOW, "nnz(C) exceeds 2^31 - 1");
  I.pool_used = legacy ? static_cast<int64_t>(p->hstat->pool_used) : 0;
  I.long_items = use_win ? S.w_items : (nlong > 0 ? S.n_items : 0);
  I.pool_entries = pool_entries;
  I.bytes_scratch = held_bytes(p);

  // ---- stage 4b: allocate C and copy C~ into it
  void *crp = crp_guard.p;
  void *ccol = p->al.get(static_cast<size_t>(nnz) * 4, s);
  void *cval = ccol ? p->al.get(static_cast<size_t>(nnz) * sizeof(T), s) : nullptr;
  if (!cval) {
    p->al.put(ccol, s);
    return fail(SPGEMM_ENOMEM, "allocation of C failed");
  }
  if (direct) {
    // phase 2 straight into C (pieces whose level-1 sequence spilled stay in
    // the pool and are copied below); pool exhaustion relaunches the failed
    // pieces until none is left
    la.c_col = static_cast<int32_t *>(ccol);
    la.c_val = static_cast<T *>(cval);
    stage_begin(p, SPGEMM_T_COMBINE, s);
    stage_begin(p, SPGEMM_T_COMBINE_WAVE, s);
    launch_combine_wave<T>(la, npieces, s);
    stage_end(p, SPGEMM_T_COMBINE_WAVE, s);
    launch_combine_wave_large<T>(la, npieces, s);
    launch_combine_oneshot<T>(la, npieces, s);
    launch_combine<T>(la, npieces, s);
    stage_end(p, SPGEMM_T_COMBINE, s);
    if (spill_expected) {
      unsigned int *f2 = fail2_a, *f2_other = fail2_b;
      for (;;) {
        if ((rc = read_status()) != SPGEMM_OK) {
          p->al.put(ccol, s);
          p->al.put(cval, s);
          return rc;
        }
        const unsigned int nf2 = p->hstat->fail2;
        if (nf2 == 0) break;
        if (++I.realloc_rounds > 64) {
          p->al.put(ccol, s);
          p->al.put(cval, s);
          return fail(SPGEMM_ENOMEM, "long-row pool keeps overflowing");
        }
        pool_entries *= 2;
        if ((rc = new_pool(pool_entries, p->hstat->pool_used)) != SPGEMM_OK) {
          p->al.put(ccol, s);
          p->al.put(cval, s);
          return rc;
        }
        la.work = reinterpret_cast<const int32_t *>(f2);
        la.fail_list2 = f2_other;
        launch_combine<T>(la, nf2, s);
        std::swap(f2, f2_other);
        la.work = nullptr;
      }
      I.pool_entries = pool_entries;
      I.pool_used = static_cast<int64_t>(p->hstat->pool_used);
      I.bytes_scratch = held_bytes(p);
    }
  }
  if (use_win) {
    // numeric pass of the long rows, straight into C
    stage_begin(p, SPGEMM_T_COMBINE, s);
    stage_begin(p, SPGEMM_T_COMBINE_WAVE, s);
    win_numeric<T>(ea, p->n, wrows, witems, w_items, wtable, wpkey, wpval, wslot, w_slots,
                   wlist + 1, wlist, wdbits, wdacc, wiscan, p->rowoff,
                   static_cast<int32_t *>(ccol), static_cast<T *>(cval), s);
    stage_end(p, SPGEMM_T_COMBINE_WAVE, s);
    stage_end(p, SPGEMM_T_COMBINE, s);
  }
  stage_begin(p, SPGEMM_T_COPY, s);
  CompactArgs<T> ca;
  ca.u = p->u;
  ca.cto = p->cto;
  ca.ct_col = ct_col;
  ca.ct_val = ct_val;
  ca.rowoff = p->rowoff;
  ca.long_min = p->be.e[4];
  ca.lrows = lrows;
  ca.pieces = pieces;
  ca.pscan = pscan;
  ca.c_rp = static_cast<int32_t *>(crp);
  ca.c_col = static_cast<int32_t *>(ccol);
  ca.c_val = static_cast<T *>(cval);
  if (m > 0)
    launch_compact<T>(ca, m, npieces, s);
  else
    launch_zero(crp, 4, s);
  stage_end(p, SPGEMM_T_COPY, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    p->al.put(ccol, s);
    p->al.put(cval, s);
    return hip_fail(e, "compute");
  }
  crp_guard.p = nullptr;  // C's arrays belong to the caller from here on
  C->rows = m;
  C->cols = p->n;
  C->nnz = nnz;
  C->row_ptr = static_cast<int32_t *>(crp);
  C->col_idx = static_cast<int32_t *>(ccol);
  C->val = cval;
  C->dtype = p->dtype;
  I.nnz_c = nnz;
  release_compute(p, s);
  return SPGEMM_OK;
}

}  // namespace

extern "C" int spgemm_compute(spgemm_plan plan, const spgemm_csr *A, const spgemm_csr *B,
                              spgemm_csr_out *C, void *stream, spgemm_info *info) {
  if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
  if (!C) return fail(SPGEMM_EINVAL, "C is NULL");
  int rc;
  if ((rc = check_csr(A, "A")) != SPGEMM_OK) return rc;
  if ((rc = check_csr(B, "B")) != SPGEMM_OK) return rc;
  spgemm_plan p = plan;
  if (A->rows != p->m || A->cols != p->k || B->cols != p->n || A->nnz != p->nnzA ||
      B->nnz != p->nnzB || A->row_ptr != p->arp || A->col_idx != p->acol ||
      B->row_ptr != p->brp || B->col_idx != p->bcol || A->dtype != p->dtype ||
      B->dtype != p->dtype)
    return fail(SPGEMM_ESTATE, "A/B differ from the analyzed matrices");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  p->stream = s;
  rc = p->dtype == SPGEMM_F64 ? compute_t<double>(p, A, B, C, s) : compute_t<float>(p, A, B, C, s);
  if (rc != SPGEMM_OK) {
    join_aux(p, s);  // nothing on the second stream may outlive the scratch
    release_compute(p, s);
    return rc;
  }
  if (p->events) {
    // waits only for the timed stages (the copy into C may still run)
    static const int kComputeStages[] = {SPGEMM_T_TINY,   SPGEMM_T_MEDIUM,    SPGEMM_T_LONG,
                                         SPGEMM_T_SCAN,   SPGEMM_T_COPY,      SPGEMM_T_LONG_WAVE,
                                         SPGEMM_T_COMBINE, SPGEMM_T_COMBINE_WAVE,
                                         SPGEMM_T_LONG_SYM};
    for (int st : kComputeStages) {
      p->info.stage_ms[st] = 0.f;
      if (p->stage_mask & (1u << st)) {
        HIP_TRY(hipEventSynchronize(p->ev[2 * st + 1]));
        (void)hipEventElapsedTime(&p->info.stage_ms[st], p->ev[2 * st], p->ev[2 * st + 1]);
      }
    }
    p->stage_mask = 0;
    p->info.long_kernel_ms = p->info.stage_ms[SPGEMM_T_LONG];
  }
  if (info) *info = p->info;
  return SPGEMM_OK;
}

extern "C" int spgemm_plan_info(spgemm_plan plan, spgemm_info *info) {
  if (!plan || !info) return fail(SPGEMM_EINVAL, "NULL argument");
  *info = plan->info;
  return SPGEMM_OK;
}

extern "C" int spgemm_plan_destroy(spgemm_plan plan) {
  destroy_plan(plan);
  return SPGEMM_OK;
}

extern "C" int spgemm_multiply(const spgemm_csr *A, const spgemm_csr *B,
                               const spgemm_options *opt, spgemm_alloc_fn alloc_fn,
                               spgemm_free_fn free_fn, void *ctx, void *stream, spgemm_csr_out *C,
                               spgemm_info *info) {
  if (!C) return fail(SPGEMM_EINVAL, "C is NULL");
  spgemm_plan plan = nullptr;
  int rc = spgemm_analyze(A, B, opt, alloc_fn, free_fn, ctx, stream, &plan, nullptr);
  if (rc != SPGEMM_OK) return rc;
  rc = spgemm_compute(plan, A, B, C, stream, info);
  spgemm_plan_destroy(plan);
  return rc;
}

namespace {

// A's transposed pattern (rows of every column, ascending), built once per plan.
int ensure_transpose(spgemm_plan p, const spgemm_csr *A, hipStream_t s) {
  if (p->bws) return SPGEMM_OK;
  Layout L;
  const size_t oc = L.add<int32_t>(p->k);
  const size_t ot = L.add<int64_t>(p->k + 1);
  const size_t orr = L.add<int32_t>(p->nnzA);
  const size_t op = L.add<int32_t>(p->nnzA);
  const size_t opa = L.add<int64_t>(scan_part_len(std::max<int64_t>(p->k, 1)));
  p->bws = p->al.get(L.bytes(), s);
  if (!p->bws) return fail(SPGEMM_ENOMEM, "backward scratch allocation failed");
  p->bws_bytes = L.bytes();
  p->tcnt = at<int32_t>(p->bws, oc);
  p->tptr = at<int64_t>(p->bws, ot);
  p->trow = at<int32_t>(p->bws, orr);
  p->tpos = at<int32_t>(p->bws, op);
  p->tpart = at<int64_t>(p->bws, opa);
  p->info.bytes_scratch = held_bytes(p);
  launch_transpose_pattern(A->row_ptr, A->col_idx, p->m, p->k, p->nnzA, p->tcnt, p->tptr,
                           p->trow, p->tpos, p->tpart, s);
  return SPGEMM_OK;
}

// Products of the dB sums are staged when they fit this budget (bytes);
// beyond it dB is gathered with binary searches instead.
constexpr int64_t kMaxStagedProducts = int64_t(1) << 36;

template <typename T>
int backward_t(spgemm_plan p, const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *C,
               void *dA_val, void *dB_val, hipStream_t s) {
  const bool want_a = dA_val && p->nnzA > 0;
  const bool want_b = dB_val && p->nnzB > 0;
  if (!want_a && !want_b) return SPGEMM_OK;
  const T *aval = static_cast<const T *>(A->val);
  const T *bval = static_cast<const T *>(B->val);
  const T *dc = static_cast<const T *>(C->val);
  T *dA = want_a ? static_cast<T *>(dA_val) : nullptr;
  T *dB = want_b ? static_cast<T *>(dB_val) : nullptr;
  int rc;
  if (want_b && (rc = ensure_transpose(p, A, s)) != SPGEMM_OK) return rc;
  const int64_t nprod = p->info.nnz_hat;
  T *W = nullptr;
  if (want_b && nprod > 0 && nprod * static_cast<int64_t>(sizeof(T)) <= kMaxStagedProducts)
    W = static_cast<T *>(p->al.get(static_cast<size_t>(nprod) * sizeof(T), s));
  // the call's peak: what the plan holds plus the staged products
  p->info.bytes_scratch =
      held_bytes(p) + (W ? static_cast<int64_t>(alloc_size(static_cast<size_t>(nprod) * sizeof(T))) : 0);
  if (want_a || W)
    launch_grad_entries<T>(A->row_ptr, A->col_idx, aval, p->m, p->nnzA, p->P, B->row_ptr,
                           B->col_idx, bval, p->n, C->row_ptr, C->col_idx, dc, dA, W, s);
  if (want_b) {
    if (W) {
      launch_grad_b_sum<T>(p->tptr, p->tpos, p->P, B->row_ptr, p->k, W, dB, s);
      p->al.put(W, s);
    } else {
      launch_grad_b<T>(p->tptr, p->trow, p->tpos, aval, B->row_ptr, B->col_idx, p->k,
                       C->row_ptr, C->col_idx, dc, dB, s);
    }
  }
  return SPGEMM_OK;
}

}  // namespace

extern "C" int spgemm_backward(spgemm_plan plan, const spgemm_csr *A, const spgemm_csr *B,
                               const spgemm_csr *C, void *dA_val, void *dB_val, void *stream) {
  if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
  int rc;
  if ((rc = check_csr(A, "A")) != SPGEMM_OK) return rc;
  if ((rc = check_csr(B, "B")) != SPGEMM_OK) return rc;
  if ((rc = check_csr(C, "C")) != SPGEMM_OK) return rc;
  spgemm_plan p = plan;
  if (A->rows != p->m || A->cols != p->k || B->cols != p->n || A->nnz != p->nnzA ||
      B->nnz != p->nnzB || A->row_ptr != p->arp || A->col_idx != p->acol ||
      B->row_ptr != p->brp || B->col_idx != p->bcol || A->dtype != p->dtype ||
      B->dtype != p->dtype)
    return fail(SPGEMM_ESTATE, "A/B differ from the analyzed matrices");
  if (C->rows != p->m || C->cols != p->n || C->dtype != p->dtype)
    return fail(SPGEMM_EINVAL, "C must be the m x n result of this plan, with A's dtype");
  if (p->info.nnz_c >= 0 && C->nnz != p->info.nnz_c)
    return fail(SPGEMM_EINVAL, "C has a different nnz than the computed product");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  p->stream = s;
  stage_begin(p, SPGEMM_T_BACKWARD, s);
  rc = p->dtype == SPGEMM_F64 ? backward_t<double>(p, A, B, C, dA_val, dB_val, s)
                              : backward_t<float>(p, A, B, C, dA_val, dB_val, s);
  if (rc != SPGEMM_OK) return rc;
  stage_end(p, SPGEMM_T_BACKWARD, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "backward");
  return SPGEMM_OK;
}

namespace {

// Device address of `scratch` on the current device, looked up on the first
// call per device (with that device current) and kept.
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;

int static_scratch_ptr(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (static_cast<int>(g_scratch_ptr.size()) <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SPGEMM_OK;
}

template <typename T>
int backward_static_t(spgemm_plan p, const spgemm_csr *A, const spgemm_csr *B,
                      const spgemm_csr *C, void *dA_val, void *dB_val, void *base,
                      hipStream_t s) {
  const bool want_a = dA_val && p->nnzA > 0;
  const bool want_b = dB_val && p->nnzB > 0;
  if (!want_a && !want_b) return SPGEMM_OK;
  const T *aval = static_cast<const T *>(A->val);
  const T *bval = static_cast<const T *>(B->val);
  const T *dc = static_cast<const T *>(C->val);
  T *dA = want_a ? static_cast<T *>(dA_val) : nullptr;
  T *dB = want_b ? static_cast<T *>(dB_val) : nullptr;
  if (!want_b) {
    launch_grad_entries<T>(A->row_ptr, A->col_idx, aval, p->m, p->nnzA, p->P, B->row_ptr,
                           B->col_idx, bval, p->n, C->row_ptr, C->col_idx, dc, dA, nullptr, s);
    return SPGEMM_OK;
  }
  // A's transposed pattern, then the staged dB products if they fit too
  Layout L;
  const size_t oc = L.add<int32_t>(p->k);
  const size_t ot = L.add<int64_t>(p->k + 1);
  const size_t orr = L.add<int32_t>(p->nnzA);
  const size_t op = L.add<int32_t>(p->nnzA);
  const size_t opa = L.add<int64_t>(scan_part_len(std::max<int64_t>(p->k, 1)));
  if (L.bytes() > SPGEMM_STATIC_SCRATCH_BYTES)
    return fail(SPGEMM_EINVAL, "A's transposed pattern needs " + std::to_string(L.bytes()) +
                                   " bytes, more than the static scratch (" +
                                   std::to_string(SPGEMM_STATIC_SCRATCH_BYTES) + " bytes)");
  const int64_t nprod = p->info.nnz_hat;
  const size_t ow = L.add<T>(nprod > 0 ? nprod : 0);
  T *W = (nprod > 0 && L.bytes() <= SPGEMM_STATIC_SCRATCH_BYTES) ? at<T>(base, ow) : nullptr;
  int32_t *cnt = at<int32_t>(base, oc);
  int64_t *tptr = at<int64_t>(base, ot);
  int32_t *trow = at<int32_t>(base, orr);
  int32_t *tpos = at<int32_t>(base, op);
  int64_t *tpart = at<int64_t>(base, opa);
  // rebuilt on every call: another call may have used the area since
  launch_transpose_pattern(A->row_ptr, A->col_idx, p->m, p->k, p->nnzA, cnt, tptr, trow, tpos,
                           tpart, s);
  if (want_a || W)
    launch_grad_entries<T>(A->row_ptr, A->col_idx, aval, p->m, p->nnzA, p->P, B->row_ptr,
                           B->col_idx, bval, p->n, C->row_ptr, C->col_idx, dc, dA, W, s);
  if (W)
    launch_grad_b_sum<T>(tptr, tpos, p->P, B->row_ptr, p->k, W, dB, s);
  else
    launch_grad_b<T>(tptr, trow, tpos, aval, B->row_ptr, B->col_idx, p->k, C->row_ptr,
                     C->col_idx, dc, dB, s);
  return SPGEMM_OK;
}

}  // namespace

extern "C" int spgemm_backward_static(spgemm_plan plan, const spgemm_csr *A,
                                      const spgemm_csr *B, const spgemm_csr *C, void *dA_val,
                                      void *dB_val, void *stream) {
  if (!plan) return fail(SPGEMM_EINVAL, "plan is NULL");
  int rc;
  if ((rc = check_csr(A, "A")) != SPGEMM_OK) return rc;
  if ((rc = check_csr(B, "B")) != SPGEMM_OK) return rc;
  if ((rc = check_csr(C, "C")) != SPGEMM_OK) return rc;
  spgemm_plan p = plan;
  if (A->rows != p->m || A->cols != p->k || B->cols != p->n || A->nnz != p->nnzA ||
      B->nnz != p->nnzB || A->row_ptr != p->arp || A->col_idx != p->acol ||
      B->row_ptr != p->brp || B->col_idx != p->bcol || A->dtype != p->dtype ||
      B->dtype != p->dtype)
    return fail(SPGEMM_ESTATE, "A/B differ from the analyzed matrices");
  if (C->rows != p->m || C->cols != p->n || C->dtype != p->dtype)
    return fail(SPGEMM_EINVAL, "C must be the m x n result of this plan, with A's dtype");
  if (p->info.nnz_c >= 0 && C->nnz != p->info.nnz_c)
    return fail(SPGEMM_EINVAL, "C has a different nnz than the computed product");
  void *base = nullptr;
  if ((rc = static_scratch_ptr(&base)) != SPGEMM_OK) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  p->stream = s;
  stage_begin(p, SPGEMM_T_BACKWARD, s);
  rc = p->dtype == SPGEMM_F64
           ? backward_static_t<double>(p, A, B, C, dA_val, dB_val, base, s)
           : backward_static_t<float>(p, A, B, C, dA_val, dB_val, base, s);
  if (rc != SPGEMM_OK) return rc;
  stage_end(p, SPGEMM_T_BACKWARD, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "backward_static");
  return SPGEMM_OK;
}

namespace spg {
const int64_t *plan_rowoff(spgemm_plan p) { return p->rowoff; }
const int64_t *plan_scan(spgemm_plan p) { return p->P; }
const int64_t *plan_upper(spgemm_plan p) { return p->u; }
int64_t *plan_rownnz(spgemm_plan p) { return p->rownnz; }
const int32_t *plan_binlist(spgemm_plan p) { return p->binlist; }
void set_last_error(const std::string &msg) { g_last_error = msg; }
// the input checks of spgemm_analyze, for the batched forms
int check_problem(const spgemm_csr *A, const spgemm_csr *B) {
  int rc;
  if ((rc = check_csr(A, "A")) != SPGEMM_OK) return rc;
  if ((rc = check_csr(B, "B")) != SPGEMM_OK) return rc;
  if (A->cols != B->rows)
    return fail(SPGEMM_EINVAL, "inner dimensions differ (A.cols != B.rows)");
  if (A->dtype != B->dtype) return fail(SPGEMM_EINVAL, "A and B have different dtypes");
  return SPGEMM_OK;
}
int check_opts(const spgemm_options &o) { return check_options(o); }
}  // namespace spg
