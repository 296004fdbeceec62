// Coalesced copy of many short CSR rows as one stream per wavefront: the
// copy step of stage 4 (Section 3.1), shared by the plain path's compaction
// and the batched form's.
#pragma once

#include "common.hpp"

namespace spg {

constexpr int CP_NT = 256;
constexpr int CP_ROWS = 32;    // short rows per wavefront
constexpr int CP_BATCH = 4;    // passes whose loads are issued before their stores

// LDS table of the sources of one wavefront.
template <int R> struct CopyTable {
  int64_t pre[R];   // first stream index of every source
  int64_t dst[R];   // destination index of its first entry
  int64_t col[R];   // source column / value pointers
  int64_t val[R];
};

// Copy up to R sources held one per lane (n entries from scol/sval to dst)
// as one stream: every pass moves 64 consecutive entries of their
// concatenation, one per lane, so loads and stores are coalesced along every
// source.  The source of an entry is found by a binary search in the
// wavefront's table, so passes are independent: the loads of the next
// CP_BATCH passes are issued before the stores of the current ones (the
// memory counter that a load waits on also counts earlier stores).
template <typename T, int R> struct StreamBatch {
  int32_t c[CP_BATCH];
  T v[CP_BATCH];
  int64_t d[CP_BATCH];
};

// Loads of one batch, without branches (a pass beyond the stream rereads its
// last entry and is not stored), so that the compiler can keep them in
// flight across the stores of the previous batch.
template <typename T, int R>
DEVI void stream_load(const CopyTable<R> &tb, int64_t x0, int64_t tot, StreamBatch<T, R> &sb) {
#pragma unroll
  for (int b = 0; b < CP_BATCH; ++b) {
    const int64_t xr = x0 + b * WAVE + lane();
    const int64_t x = xr < tot ? xr : tot - 1;
    int lo = 0;  // last source starting at or before x (it is not empty)
#pragma unroll
    for (int step = R / 2; step >= 1; step >>= 1)
      lo = tb.pre[lo + step] <= x ? lo + step : lo;
    const int64_t off = x - tb.pre[lo];
    sb.c[b] = as_global(reinterpret_cast<const int32_t *>(tb.col[lo]))[off];
    sb.v[b] = as_global(reinterpret_cast<const T *>(tb.val[lo]))[off];
    sb.d[b] = xr < tot ? tb.dst[lo] + off : -1;
  }
}

template <typename T, int R>
DEVI void stream_store(const StreamBatch<T, R> &sb, int32_t *dcol, T *dval) {
#pragma unroll
  for (int b = 0; b < CP_BATCH; ++b) {
    if (sb.d[b] >= 0) {
      dcol[sb.d[b]] = sb.c[b];
      dval[sb.d[b]] = sb.v[b];
    }
  }
}

template <typename T, int R>
DEVI void wave_stream_copy(int64_t n, const int32_t *scol, const T *sval, int64_t dst,
                           int32_t *dcol, T *dval, CopyTable<R> &tb) {
  static_assert((R & (R - 1)) == 0 && R <= WAVE, "R must be a power of two up to 64");
  const int ln = lane();
  const int64_t incl = group_incl_sum<WAVE>(n);
  const int64_t tot = __shfl(static_cast<long long>(incl), WAVE - 1, WAVE);
  if (ln < R) {
    tb.pre[ln] = incl - n;
    tb.dst[ln] = dst;
    tb.col[ln] = reinterpret_cast<int64_t>(scol);
    tb.val[ln] = reinterpret_cast<int64_t>(sval);
  }
  wave_sync();
  if (tot <= 0) return;
  constexpr int64_t STEP = static_cast<int64_t>(CP_BATCH) * WAVE;
  // two register batches in turn: the loads of one are in flight while the
  // other is stored
  StreamBatch<T, R> ba, bb;
  stream_load<T, R>(tb, 0, tot, ba);
  for (int64_t x0 = 0; x0 < tot; x0 += 2 * STEP) {
    if (x0 + STEP < tot) stream_load<T, R>(tb, x0 + STEP, tot, bb);
    stream_store<T, R>(ba, dcol, dval);
    if (x0 + STEP >= tot) break;
    if (x0 + 2 * STEP < tot) stream_load<T, R>(tb, x0 + 2 * STEP, tot, ba);
    stream_store<T, R>(bb, dcol, dval);
  }
}

}  // namespace spg
