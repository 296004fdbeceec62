// Stage 3 for bin group 3 as the paper gives it (Section 3.1, heap method,
// Fig. 2), kept beside the wavefront ESC as an ablation: one thread per row,
// one kernel per exact row size 2..32 (the 31 size-specialised programs).
//
// Every thread owns an implicit max-heap of (column, value) pairs in LDS,
// sized for its bin.  All products of the row are inserted (sift-up on the
// column).  A heapsort variant then builds the result in the tail of the
// same array: every delete-max either fuses the root into the first entry of
// the result, when both have the same column, or becomes the new first
// entry; the element that was last in the heap is sifted down from the
// root.  The tail ends up in ascending column order without duplicates and
// is copied to C~.
//
// Duplicates are added in heap-deletion order (starting from +0.0), not in
// Gustavson's order, so values can differ from sequential sums by rounding.
//
// LDS layout: entry e of thread t at e * HEAP_NT + t, so the lanes of a
// wavefront always touch distinct banks whatever their heap paths.
#include <utility>

#include "common.hpp"
#include "internal.hpp"

namespace spg {

constexpr int HEAP_NT = 64;

template <typename T, int USZ>
__global__ __launch_bounds__(HEAP_NT) void k_heap(EscArgs<T> a, const int32_t *rows,
                                                  int64_t nrows) {
  __shared__ int32_t hc[USZ * HEAP_NT];
  __shared__ T hv[USZ * HEAP_NT];
  const int t = threadIdx.x;
  auto at = [t](int e) { return e * HEAP_NT + t; };
  const GLOBAL_AS int32_t *garp = as_global(a.arp);
  const GLOBAL_AS int32_t *gacol = as_global(a.acol);
  const GLOBAL_AS T *gaval = as_global(a.aval);
  const GLOBAL_AS int32_t *gbrp = as_global(a.brp);
  const GLOBAL_AS int32_t *gbcol = as_global(a.bcol);
  const GLOBAL_AS T *gbval = as_global(a.bval);
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * HEAP_NT + t; r < nrows;
       r += static_cast<int64_t>(gridDim.x) * HEAP_NT) {
    const int32_t i = as_global(rows)[r];
    // rows of this bin have u == USZ; the check keeps LDS indexes in range
    if (as_global(a.u)[i] > USZ) continue;
    // insert every product (sift-up on the column: parents >= children)
    int h = 0;
    const int32_t e1 = garp[i + 1];
    for (int32_t e = garp[i]; e < e1; ++e) {
      const int32_t j = gacol[e];
      const T av = gaval[e];
      const int32_t q1 = gbrp[j + 1];
      for (int32_t q = gbrp[j]; q < q1; ++q) {
        const int32_t c = gbcol[q];
        const T v = av * gbval[q];
        int x = h++;
        while (x > 0) {
          const int par = (x - 1) >> 1;
          if (hc[at(par)] >= c) break;
          hc[at(x)] = hc[at(par)];
          hv[at(x)] = hv[at(par)];
          x = par;
        }
        hc[at(x)] = c;
        hv[at(x)] = v;
      }
    }
    // heapsort variant: the result grows downwards from the end of the array
    const int n0 = h;
    int rr = n0;
    while (h > 0) {
      const int32_t rc = hc[at(0)];
      const T rv = hv[at(0)];
      const int32_t lc = hc[at(h - 1)];
      const T lv = hv[at(h - 1)];
      --h;
      if (rr < n0 && hc[at(rr)] == rc) {
        hv[at(rr)] = hv[at(rr)] + rv;  // fuse into the first result entry
      } else {
        --rr;  // rr >= h: the slot is outside the heap
        hc[at(rr)] = rc;
        hv[at(rr)] = T(0) + rv;
      }
      if (h > 0) {
        int x = 0;
        for (;;) {
          int ch = 2 * x + 1;
          if (ch >= h) break;
          if (ch + 1 < h && hc[at(ch + 1)] > hc[at(ch)]) ++ch;
          if (hc[at(ch)] <= lc) break;
          hc[at(x)] = hc[at(ch)];
          hv[at(x)] = hv[at(ch)];
          x = ch;
        }
        hc[at(x)] = lc;
        hv[at(x)] = lv;
      }
    }
    const int64_t o = as_global(a.cto)[i];
    for (int k = rr; k < n0; ++k) {
      as_global_mut(a.ct_col)[o + k - rr] = hc[at(k)];
      as_global_mut(a.ct_val)[o + k - rr] = hv[at(k)];
    }
    as_global_mut(a.rownnz)[i] = n0 - rr;
  }
}

namespace {

template <typename T, int USZ>
void launch_one(const EscArgs<T> &a, const int32_t *rows, int64_t nrows, hipStream_t s) {
  int64_t nb = (nrows + HEAP_NT - 1) / HEAP_NT;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((k_heap<T, USZ>), dim3(nb), dim3(HEAP_NT), 0, s, a, rows, nrows);
}

template <typename T, int... S>
bool launch_size(int usz, const EscArgs<T> &a, const int32_t *rows, int64_t nrows, hipStream_t s,
                 std::integer_sequence<int, S...>) {
  bool done = false;
  ((usz == S + 2 ? (launch_one<T, S + 2>(a, rows, nrows, s), done = true) : false), ...);
  return done;
}

}  // namespace

template <typename T>
int launch_heap(const EscArgs<T> &a, const int32_t *rows, int64_t nrows, int usz, hipStream_t s) {
  if (nrows <= 0) return 0;
  return launch_size<T>(usz, a, rows, nrows, s, std::make_integer_sequence<int, 31>()) ? 0 : -1;
}

template int launch_heap<float>(const EscArgs<float> &, const int32_t *, int64_t, int,
                                hipStream_t);
template int launch_heap<double>(const EscArgs<double> &, const int32_t *, int64_t, int,
                                 hipStream_t);

}  // namespace spg
