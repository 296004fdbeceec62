// Stage 4 of the framework ("arranging data", Section 3.1): after the row
// sizes of C have been scanned into C's row pointers, copy every row from
// the temporary matrix C~ into C.  Short rows are copied by one wavefront
// each (in row order, so consecutive waves write consecutive parts of C);
// long rows are copied piece by piece by whole work-groups, so that the
// longest rows do not serialise on one wavefront.
#include "common.hpp"
#include "internal.hpp"

namespace spg {

template <typename T>
__global__ __launch_bounds__(256) void k_compact_rows(CompactArgs<T> a, int64_t m) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
  if (i >= m) return;
  const int64_t o = a.rowoff[i];
  if (lane() == 0) {
    a.c_rp[i] = static_cast<int32_t>(o);
    if (i == m - 1) a.c_rp[m] = static_cast<int32_t>(a.rowoff[m]);
  }
  if (a.u[i] > a.long_min) return;  // copied by k_compact_pieces
  const int64_t n = a.rowoff[i + 1] - o;
  const int64_t src = a.cto[i];
  for (int64_t x = lane(); x < n; x += WAVE) {
    a.c_col[o + x] = a.ct_col[src + x];
    a.c_val[o + x] = a.ct_val[src + x];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_compact_pieces(CompactArgs<T> a) {
  const Piece pc = a.pieces[blockIdx.x];
  if (pc.cnt <= 0) return;
  const LongRow lr = a.lrows[pc.lrow];
  const int64_t dst = a.rowoff[lr.row] + a.pscan[blockIdx.x] - a.pscan[lr.piece0];
  const T *sv = reinterpret_cast<const T *>(pc.val);
  for (int64_t x = threadIdx.x; x < pc.cnt; x += blockDim.x) {
    a.c_col[dst + x] = pc.col[x];
    a.c_val[dst + x] = sv[x];
  }
}

template <typename T>
void launch_compact(const CompactArgs<T> &a, int64_t m, int64_t npieces, hipStream_t s) {
  if (m <= 0) return;
  const int64_t nb = (m * WAVE + 255) / 256;
  hipLaunchKernelGGL((k_compact_rows<T>), dim3(nb), dim3(256), 0, s, a, m);
  if (npieces > 0)
    hipLaunchKernelGGL((k_compact_pieces<T>), dim3(npieces), dim3(256), 0, s, a);
}

template void launch_compact<float>(const CompactArgs<float> &, int64_t, int64_t, hipStream_t);
template void launch_compact<double>(const CompactArgs<double> &, int64_t, int64_t, hipStream_t);

}  // namespace spg
