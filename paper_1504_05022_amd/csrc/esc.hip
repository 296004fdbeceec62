// Stage 3 for short rows (bin groups 2-4, Section 3.1): expand-sort-compress
// of each row of C inside an aligned group of G lanes of a wavefront.
//
// The paper gives one thread per row with a heap for sizes 2..32 and one
// thread group per row with a bitonic ESC in scratchpad memory for 33..512.
// Here one kernel template covers both: a row with u <= G*K products is
// handled by G lanes holding K products each.  Products are expanded into
// LDS (run starts of every b_j* row, then a segmented max-scan gives each
// product its a_ij), sorted with a bitonic network on the key
// (column, position in the expansion order) entirely in registers and
// cross-lane shuffles, and compressed: each column's products are folded in
// expansion order starting from +0.0 (so the values equal Gustavson's
// sequential sums exactly), and the unique columns are written to C~.
#include "esc_body.hpp"

namespace spg {

// Wavefronts per SIMD kept resident: the kernel waits on memory, so the
// register budget of the 8-products-per-lane tiles is held to 5 (LDS allows
// 6 for FP64); not for whole-wavefront rows, which would spill at 5.
template <int G, int K> constexpr int esc_occupancy() { return K >= 8 && G < 64 ? 5 : 1; }

template <typename T, int G, int K, typename Key>
__global__ __launch_bounds__(ESC_NT) __attribute__((amdgpu_waves_per_eu(esc_occupancy<G, K>())))
void k_esc(EscArgs<T> a, const int32_t *rows, int64_t nrows) {
  using Sh = EscShape<T, G, K, Key>;
  __shared__ __align__(16) unsigned char lds[Sh::lds_bytes];
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * Sh::RPB; base < nrows;
       base += static_cast<int64_t>(gridDim.x) * Sh::RPB)
    esc_rows<T, G, K, Key>(a, rows, base, nrows, lds);
}

template <typename T, int G, int K>
static void launch_gk(const EscArgs<T> &a, const int32_t *rows, int64_t nrows, int64_t ncols,
                      hipStream_t s) {
  constexpr int RPB = ESC_NT / G;
  constexpr int LOGU = Log2<G * K>::v;
  int64_t nb = (nrows + RPB - 1) / RPB;
  if (nb > 65536) nb = 65536;
  if ((static_cast<uint64_t>(ncols) << LOGU) <= 0xffffffffull)
    hipLaunchKernelGGL((k_esc<T, G, K, uint32_t>), dim3(nb), dim3(ESC_NT), 0, s, a, rows, nrows);
  else
    hipLaunchKernelGGL((k_esc<T, G, K, uint64_t>), dim3(nb), dim3(ESC_NT), 0, s, a, rows, nrows);
}

template <typename T>
int launch_esc(const EscArgs<T> &a, const int32_t *rows, int64_t nrows, int cap, int64_t ncols,
               hipStream_t s) {
  if (nrows <= 0) return 0;
  // lanes per row G and products per lane K for each capacity: several
  // rows per wavefront so that their memory latencies overlap
  switch (cap) {
    case 1: launch_gk<T, 1, 1>(a, rows, nrows, ncols, s); break;
    case 2: launch_gk<T, 2, 1>(a, rows, nrows, ncols, s); break;
    case 4: launch_gk<T, 4, 1>(a, rows, nrows, ncols, s); break;
    case 8: launch_gk<T, 4, 2>(a, rows, nrows, ncols, s); break;
    case 16: launch_gk<T, 4, 4>(a, rows, nrows, ncols, s); break;
    case 32: launch_gk<T, 8, 4>(a, rows, nrows, ncols, s); break;
    case 64: launch_gk<T, 16, 4>(a, rows, nrows, ncols, s); break;
    case 128: launch_gk<T, 16, 8>(a, rows, nrows, ncols, s); break;
    case 256: launch_gk<T, 32, 8>(a, rows, nrows, ncols, s); break;
    case 512: launch_gk<T, 64, 8>(a, rows, nrows, ncols, s); break;
    case 1024: launch_gk<T, 64, 16>(a, rows, nrows, ncols, s); break;
    default: return -1;
  }
  return 0;
}

template int launch_esc<float>(const EscArgs<float> &, const int32_t *, int64_t, int, int64_t,
                               hipStream_t);
template int launch_esc<double>(const EscArgs<double> &, const int32_t *, int64_t, int, int64_t,
                                hipStream_t);

}  // namespace spg
