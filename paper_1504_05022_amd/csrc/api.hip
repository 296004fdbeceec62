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
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace spg;

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

struct Allocator {
  spgemm_alloc_fn af = nullptr;
  spgemm_free_fn ff = nullptr;
  void *ctx = nullptr;
  void *get(size_t bytes, hipStream_t s) const {
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
  Summary *dsum = nullptr;
  ComputeStatus *dstat = nullptr;
  Pool *dpool = nullptr;
  int64_t nwaves = 0;

  // pinned host mirrors
  Summary *hsum = nullptr;
  ComputeStatus *hstat = nullptr;
  Pool *hpool = nullptr;

  // compute scratch
  void *cws = nullptr;
  size_t cws_bytes = 0;
  std::vector<void *> pool_chunks;

  // backward scratch: A's transposed pattern, built on first use
  void *bws = nullptr;
  int32_t *tcnt = nullptr, *trow = nullptr, *tpos = nullptr;
  int64_t *tptr = nullptr, *tpart = nullptr;

  spgemm_info info{};
  hipEvent_t ev[2 * SPGEMM_NSTAGES] = {};
  bool events = false;
  std::vector<hipEvent_t> long_ev;
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
  o->seg = -1;
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

void release_compute(spgemm_plan p, hipStream_t s) {
  p->al.put(p->cws, s);
  p->cws = nullptr;
  p->cws_bytes = 0;
  for (void *c : p->pool_chunks) p->al.put(c, s);
  p->pool_chunks.clear();
}

void destroy_plan(spgemm_plan p) {
  if (!p) return;
  release_compute(p, p->stream);
  p->al.put(p->ws, p->stream);
  p->al.put(p->bws, p->stream);
  if (p->hsum) (void)hipHostFree(p->hsum);
  if (p->events)
    for (auto &e : p->ev) (void)hipEventDestroy(e);
  for (auto &e : p->long_ev) (void)hipEventDestroy(e);
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
  return SPGEMM_OK;
}

void stage_begin(spgemm_plan p, int st, hipStream_t s) {
  if (p->events) (void)hipEventRecord(p->ev[2 * st], s);
}
void stage_end(spgemm_plan p, int st, hipStream_t s) {
  if (p->events) (void)hipEventRecord(p->ev[2 * st + 1], s);
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
  p->dsum = at<Summary>(p->ws, osum);
  p->dstat = at<ComputeStatus>(p->ws, ostat);
  p->dpool = at<Pool>(p->ws, opool);

  // pinned host mirrors of the small records
  {
    void *hp = nullptr;
    hipError_t e = hipHostMalloc(&hp, sizeof(Summary) + sizeof(ComputeStatus) + sizeof(Pool) + 64,
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
      destroy_plan(p);
      return hip_fail(e, "hipHostMalloc");
    }
    p->hsum = static_cast<Summary *>(hp);
    p->hstat = reinterpret_cast<ComputeStatus *>(static_cast<char *>(hp) + sizeof(Summary));
    p->hpool = reinterpret_cast<Pool *>(static_cast<char *>(hp) + sizeof(Summary) +
                                        sizeof(ComputeStatus));
  }
  if (o.timing) {
    for (auto &e : p->ev) {
      if (hipEventCreate(&e) != hipSuccess) {
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
    hipError_t ve = hipMemcpyAsync(p->hsum, p->dsum, sizeof(Summary), hipMemcpyDeviceToHost, s);
    if (ve == hipSuccess) ve = hipStreamSynchronize(s);
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
  launch_row_stats(A->row_ptr, p->P, m, p->n, p->be, o.long_slot, p->u, p->h, p->hist, p->nwaves,
                   p->rownnz, p->dsum, s);
  stage_end(p, SPGEMM_T_UPPER, s);
  // stage 2 (Algorithm 3): C~ offsets and the stable bin lists
  stage_begin(p, SPGEMM_T_BIN, s);
  scan_i64(p->h, m, p->cto, p->part, s);
  scan_i32(p->hist, nh, p->hist_scan, p->part, s);
  launch_bin_scatter(p->u, m, p->be, p->hist_scan, p->nwaves, p->binlist, s);
  launch_summary(p->P, p->nnzA, p->cto, m, p->hist_scan, p->nwaves, p->dsum, s);
  stage_end(p, SPGEMM_T_BIN, s);
  hipError_t e = hipMemcpyAsync(p->hsum, p->dsum, sizeof(Summary), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
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
  I.long_items = I.bin_count[LONG_BIN];
  I.bytes_scratch = static_cast<int64_t>(p->ws_bytes);
  if (p->events) {
    (void)hipEventElapsedTime(&I.stage_ms[SPGEMM_T_UPPER], p->ev[0], p->ev[1]);
    (void)hipEventElapsedTime(&I.stage_ms[SPGEMM_T_BIN], p->ev[2], p->ev[3]);
  }
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

  // C~ (hybrid sizes) plus the long-row records in one allocation
  Layout L;
  const size_t octc = L.add<int32_t>(S.sum_h);
  const size_t octv = L.add<T>(S.sum_h);
  const size_t oit = L.add<LongItem>(nlong);
  const size_t ost = L.add<LongState>(nlong);
  const size_t ofa = L.add<unsigned int>(nlong);
  const size_t ofb = L.add<unsigned int>(nlong);
  const size_t orc = L.add<int32_t *>(nlong > 0 ? m : 0);
  const size_t orv = L.add<T *>(nlong > 0 ? m : 0);
  p->cws_bytes = L.bytes();
  p->cws = p->al.get(p->cws_bytes, s);
  if (!p->cws) return fail(SPGEMM_ENOMEM, "C~ allocation failed");
  int32_t *ct_col = at<int32_t>(p->cws, octc);
  T *ct_val = at<T>(p->cws, octv);
  LongItem *items = at<LongItem>(p->cws, oit);
  LongState *states = at<LongState>(p->cws, ost);
  unsigned int *fail_a = at<unsigned int>(p->cws, ofa);
  unsigned int *fail_b = at<unsigned int>(p->cws, ofb);
  int32_t **rsrc_col = at<int32_t *>(p->cws, orc);
  T **rsrc_val = at<T *>(p->cws, orv);

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

  // ---- stage 3, bin groups 2-3: one launch per power-of-two capacity
  stage_begin(p, SPGEMM_T_TINY, s);
  {
    int b = 1;
    while (b <= p->be.e[0]) {
      const int cap = static_cast<int>(next_pow2(b));
      const int hi = std::min<int>(cap, p->be.e[0]);
      const int64_t r0 = S.bin_off[b], r1 = S.bin_off[hi + 1];
      if (launch_esc<T>(ea, p->binlist + r0, r1 - r0, cap, p->n, s))
        return fail(SPGEMM_EINVAL, "no ESC kernel for this capacity");
      b = hi + 1;
    }
  }
  stage_end(p, SPGEMM_T_TINY, s);
  // ---- bin group 4: the four range bins
  stage_begin(p, SPGEMM_T_MEDIUM, s);
  for (int b = 33; b <= 36; ++b) {
    const int cap = static_cast<int>(next_pow2(p->be.e[b - 32]));
    const int64_t r0 = S.bin_off[b], r1 = S.bin_off[b + 1];
    if (launch_esc<T>(ea, p->binlist + r0, r1 - r0, cap, p->n, s))
      return fail(SPGEMM_EINVAL, "no ESC kernel for this capacity");
  }
  stage_end(p, SPGEMM_T_MEDIUM, s);

  // ---- bin group 5: long rows with the merge method and a growing pool
  int64_t pool_entries = 0;
  I.realloc_rounds = 0;
  I.long_launches = 0;
  I.long_kernel_ms = 0.f;
  const int l1cap = p->opt.l1_cap ? p->opt.l1_cap : long_l1cap_default(sizeof(T));
  LongArgs<T> la;
  la.e = ea;
  la.items = items;
  la.state = states;
  la.pool = p->dpool;
  la.long_slot = p->opt.long_slot;
  la.rsrc_col = rsrc_col;
  la.rsrc_val = rsrc_val;
  if (nlong > 0) {
    pool_entries = p->opt.pool_entries
                       ? p->opt.pool_entries
                       : std::max<int64_t>(3 * S.sum_r_long + nlong * p->opt.long_slot, 1 << 16);
    void *chunk = p->al.get(pool_chunk_bytes(pool_entries, sizeof(T)), s);
    if (!chunk) return fail(SPGEMM_ENOMEM, "long-row pool allocation failed");
    p->pool_chunks.push_back(chunk);
    *p->hpool = pool_view(chunk, pool_entries);
    HIP_TRY(hipMemcpyAsync(p->dpool, p->hpool, sizeof(Pool), hipMemcpyHostToDevice, s));
    launch_long_items(p->binlist, S.bin_off[LONG_BIN], nlong, p->u, items, s);
    launch_long_init(items, states, nlong, s);
  }
  int64_t nwork = nlong;
  const unsigned int *work = nullptr;
  unsigned int *fl = fail_a, *fl_other = fail_b;
  for (int round = 0;; ++round) {
    if (round == 0) stage_begin(p, SPGEMM_T_LONG, s);
    if (nwork > 0) {
      la.work = reinterpret_cast<const int32_t *>(work);
      la.fail_list = fl;
      if (launch_long<T>(la, nwork, p->n, l1cap, s))
        return fail(SPGEMM_EINVAL, "no long-row kernel for this l1_cap");
      I.long_launches++;
    }
    if (round == 0) {
      stage_end(p, SPGEMM_T_LONG, s);
      stage_begin(p, SPGEMM_T_SCAN, s);
    }
    // ---- stage 4a: row pointers of C (exclusive scan of the row sizes)
    scan_i64(p->rownnz, m, p->rowoff, p->part, s);
    launch_status(p->rowoff, m, p->dpool, p->dstat, s);
    if (round == 0) stage_end(p, SPGEMM_T_SCAN, s);
    HIP_TRY(hipMemcpyAsync(p->hstat, p->dstat, sizeof(ComputeStatus), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    const unsigned int nfail = nlong > 0 ? p->hstat->fail_count : 0u;
    if (nfail == 0) break;
    // pool exhausted: grow 2x, relaunch the failed items from their checkpoints
    I.realloc_rounds++;
    if (I.realloc_rounds > 64) return fail(SPGEMM_ENOMEM, "long-row pool keeps overflowing");
    const unsigned long long used = p->hstat->pool_used;
    pool_entries *= 2;
    void *chunk = p->al.get(pool_chunk_bytes(pool_entries, sizeof(T)), s);
    if (!chunk) return fail(SPGEMM_ENOMEM, "long-row pool growth failed");
    p->pool_chunks.push_back(chunk);
    *p->hpool = pool_view(chunk, pool_entries);
    p->hpool->used = used;
    HIP_TRY(hipMemcpyAsync(p->dpool, p->hpool, sizeof(Pool), hipMemcpyHostToDevice, s));
    work = fl;
    nwork = nfail;
    std::swap(fl, fl_other);
  }
  const int64_t nnz = p->hstat->nnz_c;
  if (nnz >= (int64_t(1) << 31)) return fail(SPGEMM_EOVERFLOW, "nnz(C) exceeds 2^31 - 1");
  I.pool_used = nlong > 0 ? static_cast<int64_t>(p->hstat->pool_used) : 0;
  I.pool_entries = pool_entries;

  // ---- stage 4b: allocate C and copy C~ into it
  void *crp = p->al.get(static_cast<size_t>(m + 1) * 4, s);
  void *ccol = crp ? p->al.get(static_cast<size_t>(nnz) * 4, s) : nullptr;
  void *cval = ccol ? p->al.get(static_cast<size_t>(nnz) * sizeof(T), s) : nullptr;
  if (!cval) {
    p->al.put(crp, s);
    p->al.put(ccol, s);
    return fail(SPGEMM_ENOMEM, "allocation of C failed");
  }
  stage_begin(p, SPGEMM_T_COPY, s);
  CompactArgs<T> ca;
  ca.u = p->u;
  ca.cto = p->cto;
  ca.ct_col = ct_col;
  ca.ct_val = ct_val;
  ca.rsrc_col = rsrc_col;
  ca.rsrc_val = rsrc_val;
  ca.rowoff = p->rowoff;
  ca.long_min = p->be.e[4];
  ca.c_rp = static_cast<int32_t *>(crp);
  ca.c_col = static_cast<int32_t *>(ccol);
  ca.c_val = static_cast<T *>(cval);
  if (m > 0)
    launch_compact<T>(ca, m, s);
  else
    launch_zero(crp, 4, s);
  stage_end(p, SPGEMM_T_COPY, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    p->al.put(crp, s);
    p->al.put(ccol, s);
    p->al.put(cval, s);
    return hip_fail(e, "compute");
  }
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
    release_compute(p, s);
    return rc;
  }
  if (p->events) {
    HIP_TRY(hipEventSynchronize(p->ev[2 * SPGEMM_T_COPY + 1]));
    for (int st = SPGEMM_T_TINY; st <= SPGEMM_T_COPY; ++st)
      (void)hipEventElapsedTime(&p->info.stage_ms[st], p->ev[2 * st], p->ev[2 * st + 1]);
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
  if (dA_val && p->nnzA > 0) {
    if (p->dtype == SPGEMM_F64)
      launch_grad_a<double>(A->row_ptr, A->col_idx, p->m, B->row_ptr, B->col_idx,
                            static_cast<const double *>(B->val), C->row_ptr, C->col_idx,
                            static_cast<const double *>(C->val), static_cast<double *>(dA_val), s);
    else
      launch_grad_a<float>(A->row_ptr, A->col_idx, p->m, B->row_ptr, B->col_idx,
                           static_cast<const float *>(B->val), C->row_ptr, C->col_idx,
                           static_cast<const float *>(C->val), static_cast<float *>(dA_val), s);
  }
  if (dB_val && p->nnzB > 0) {
    if (!p->bws) {
      Layout L;
      const size_t oc = L.add<int32_t>(p->k);
      const size_t ot = L.add<int64_t>(p->k + 1);
      const size_t orr = L.add<int32_t>(p->nnzA);
      const size_t op = L.add<int32_t>(p->nnzA);
      const size_t opa = L.add<int64_t>(scan_part_len(std::max<int64_t>(p->k, 1)));
      p->bws = p->al.get(L.bytes(), s);
      if (!p->bws) return fail(SPGEMM_ENOMEM, "backward scratch allocation failed");
      p->tcnt = at<int32_t>(p->bws, oc);
      p->tptr = at<int64_t>(p->bws, ot);
      p->trow = at<int32_t>(p->bws, orr);
      p->tpos = at<int32_t>(p->bws, op);
      p->tpart = at<int64_t>(p->bws, opa);
      p->info.bytes_scratch += static_cast<int64_t>(L.bytes());
      launch_transpose_pattern(A->row_ptr, A->col_idx, p->m, p->k, p->nnzA, p->tcnt, p->tptr,
                               p->trow, p->tpos, p->tpart, s);
    }
    if (p->dtype == SPGEMM_F64)
      launch_grad_b<double>(p->tptr, p->trow, p->tpos, static_cast<const double *>(A->val),
                            B->row_ptr, B->col_idx, p->k, C->row_ptr, C->col_idx,
                            static_cast<const double *>(C->val), static_cast<double *>(dB_val), s);
    else
      launch_grad_b<float>(p->tptr, p->trow, p->tpos, static_cast<const float *>(A->val),
                           B->row_ptr, B->col_idx, p->k, C->row_ptr, C->col_idx,
                           static_cast<const float *>(C->val), static_cast<float *>(dB_val), s);
  }
  stage_end(p, SPGEMM_T_BACKWARD, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "backward");
  return SPGEMM_OK;
}
