// Stage 4 of the framework ("arranging data", Section 3.1): after the row
// sizes of C have been scanned into C's row pointers, copy every row from
// the temporary matrix C~ into C.  A wavefront takes 32 consecutive short
// rows and streams all their entries at once, so the copy is coalesced and
// no wavefront waits on one row's metadata; long rows are copied piece by
// piece, one wavefront each.
#include "common.hpp"
#include "internal.hpp"

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

// Row pointers of C, and the short rows (u <= long_min) copied from C~:
// CP_ROWS consecutive rows per wavefront.
template <typename T>
__global__ __launch_bounds__(CP_NT) void k_compact_rows(CompactArgs<T> a, int64_t m) {
  __shared__ CopyTable<CP_ROWS> tabs[CP_NT / WAVE];
  const int64_t w = (static_cast<int64_t>(blockIdx.x) * CP_NT + threadIdx.x) / WAVE;
  const int64_t r0 = w * CP_ROWS;
  if (r0 >= m) return;  // uniform across the wavefront
  const int64_t r = r0 + lane();
  int64_t n = 0, src = 0, o = 0;
  if (lane() < CP_ROWS && r < m) {
    o = a.rowoff[r];
    const int64_t o1 = a.rowoff[r + 1];
    a.c_rp[r] = static_cast<int32_t>(o);
    if (r == m - 1) a.c_rp[m] = static_cast<int32_t>(o1);
    if (a.u[r] <= a.long_min) {
      n = o1 - o;
      src = a.cto[r];
    }
  }
  wave_stream_copy<T, CP_ROWS>(n, a.ct_col + src, a.ct_val + src, o, a.c_col, a.c_val,
                               tabs[threadIdx.x / WAVE]);
}

// Long rows, piece by piece: one wavefront per piece (pieces hold a few
// hundred entries), loads of up to CP_PIECE_BATCH passes issued before
// their stores.
constexpr int CP_PIECE_BATCH = 8;

template <typename T>
__global__ __launch_bounds__(CP_NT) void k_compact_pieces(CompactArgs<T> a, int64_t npieces) {
  const int64_t pid = (static_cast<int64_t>(blockIdx.x) * CP_NT + threadIdx.x) / WAVE;
  if (pid >= npieces) return;  // uniform across the wavefront
  const Piece pc = a.pieces[pid];
  if (pc.cnt <= 0) return;
  const LongRow lr = a.lrows[pc.lrow];
  const int64_t dst = a.rowoff[lr.row] + a.pscan[pid] - a.pscan[lr.piece0];
  if (pc.col == a.c_col + dst) return;  // written in place (direct output)
  const GLOBAL_AS int32_t *sc = as_global(pc.col);
  const GLOBAL_AS T *sv = as_global(reinterpret_cast<const T *>(pc.val));
  GLOBAL_AS int32_t *dc = as_global_mut(a.c_col + dst);
  GLOBAL_AS T *dv = as_global_mut(a.c_val + dst);
  const int64_t n = pc.cnt;
  for (int64_t x0 = 0; x0 < n; x0 += CP_PIECE_BATCH * WAVE) {
    int32_t c[CP_PIECE_BATCH];
    T v[CP_PIECE_BATCH];
#pragma unroll
    for (int b = 0; b < CP_PIECE_BATCH; ++b) {
      const int64_t x = x0 + b * WAVE + lane();
      const int64_t xc = x < n ? x : n - 1;
      c[b] = sc[xc];
      v[b] = sv[xc];
    }
#pragma unroll
    for (int b = 0; b < CP_PIECE_BATCH; ++b) {
      const int64_t x = x0 + b * WAVE + lane();
      if (x < n) {
        dc[x] = c[b];
        dv[x] = v[b];
      }
    }
  }
}

template <typename T>
void launch_compact(const CompactArgs<T> &a, int64_t m, int64_t npieces, hipStream_t s) {
  if (m <= 0) return;
  const int64_t rwaves = (m + CP_ROWS - 1) / CP_ROWS;
  hipLaunchKernelGGL((k_compact_rows<T>), dim3((rwaves * WAVE + CP_NT - 1) / CP_NT), dim3(CP_NT),
                     0, s, a, m);
  if (npieces > 0)
    hipLaunchKernelGGL((k_compact_pieces<T>), dim3((npieces * WAVE + CP_NT - 1) / CP_NT),
                       dim3(CP_NT), 0, s, a, npieces);
}

template void launch_compact<float>(const CompactArgs<float> &, int64_t, int64_t, hipStream_t);
template void launch_compact<double>(const CompactArgs<double> &, int64_t, int64_t, hipStream_t);

}  // namespace spg
