// Stage 4 of the framework ("arranging data", Section 3.1): after the row
// sizes of C have been scanned into C's row pointers, copy every row from
// the temporary matrix C~ into C.  A wavefront takes 32 consecutive short
// rows and streams all their entries at once, so the copy is coalesced and
// no wavefront waits on one row's metadata; long rows are copied piece by
// piece, one wavefront each.
#include "common.hpp"
#include "internal.hpp"
#include "stream_copy.hpp"

namespace spg {

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
