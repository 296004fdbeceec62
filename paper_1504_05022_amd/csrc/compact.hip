// Stage 4 of the framework ("arranging data", Section 3.1): after the row
// sizes of C have been scanned into C's row pointers, copy every row from
// the temporary matrix C~ (or, for long rows, from wherever the long-row
// kernel left it) into C.  One wavefront per row.
#include "common.hpp"
#include "internal.hpp"

namespace spg {

template <typename T>
__global__ __launch_bounds__(256) void k_compact(CompactArgs<T> a, int64_t m) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
  if (i >= m) return;
  const int64_t o = a.rowoff[i];
  const int64_t n = a.rowoff[i + 1] - o;
  if (lane() == 0) {
    a.c_rp[i] = static_cast<int32_t>(o);
    if (i == m - 1) a.c_rp[m] = static_cast<int32_t>(a.rowoff[m]);
  }
  if (n == 0) return;
  const int32_t *sc;
  const T *sv;
  if (a.u[i] > a.long_min) {
    sc = a.rsrc_col[i];
    sv = a.rsrc_val[i];
  } else {
    sc = a.ct_col + a.cto[i];
    sv = a.ct_val + a.cto[i];
  }
  for (int64_t x = lane(); x < n; x += WAVE) {
    a.c_col[o + x] = sc[x];
    a.c_val[o + x] = sv[x];
  }
}

template <typename T> void launch_compact(const CompactArgs<T> &a, int64_t m, hipStream_t s) {
  if (m <= 0) return;
  const int64_t nb = (m * WAVE + 255) / 256;
  hipLaunchKernelGGL((k_compact<T>), dim3(nb), dim3(256), 0, s, a, m);
}

template void launch_compact<float>(const CompactArgs<float> &, int64_t, hipStream_t);
template void launch_compact<double>(const CompactArgs<double> &, int64_t, hipStream_t);

}  // namespace spg
