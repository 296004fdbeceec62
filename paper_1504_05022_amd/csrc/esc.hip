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
#include "common.hpp"
#include "internal.hpp"

namespace spg {

constexpr int ESC_NT = 256;

template <typename T, int G, int K, typename Key>
__global__ __launch_bounds__(ESC_NT) void k_esc(EscArgs<T> a, const int32_t *rows,
                                                int64_t nrows) {
  constexpr int U = G * K;         // products per row capacity
  constexpr int LOGU = Log2<U>::v;
  constexpr int RPB = ESC_NT / G;  // rows per work-group
  constexpr Key KMAX = KeyMax<Key>::v;
  // Per row: region A holds the run starts (int32 index into B's arrays, -1
  // = none) and later the sorted keys; region B holds a_ij of each run and
  // later the product values.  A group's lanes share one wavefront, so all
  // reads of the first use precede the writes of the second in program
  // order.
  constexpr int KB = sizeof(Key) > 4 ? static_cast<int>(sizeof(Key)) : 4;
  __shared__ __align__(16) unsigned char s_a[RPB * U * KB];
  __shared__ __align__(16) T s_b[RPB * U];

  const int grp = threadIdx.x / G;
  const int pos = threadIdx.x & (G - 1);
  int32_t *rs = reinterpret_cast<int32_t *>(s_a + grp * U * KB);
  Key *sk = reinterpret_cast<Key *>(s_a + grp * U * KB);
  T *ra = s_b + grp * U;
  T *pv = s_b + grp * U;

  for (int64_t base = static_cast<int64_t>(blockIdx.x) * RPB; base < nrows;
       base += static_cast<int64_t>(gridDim.x) * RPB) {
    const int64_t r = base + grp;
    const int32_t i = r < nrows ? rows[r] : 0;
    // rows of this launch have u <= U by binning; the check keeps every LDS
    // and global index in range even if that were violated
    const bool act = r < nrows && a.u[i] <= U;
    const int u = act ? static_cast<int>(a.u[i]) : 0;
    const int32_t e0 = act ? a.arp[i] : 0;
    const int32_t e1 = act ? a.arp[i + 1] : 0;
    const int64_t pbase = act ? a.P[e0] : 0;

#pragma unroll
    for (int kk = 0; kk < K; ++kk) rs[pos * K + kk] = -1;
    __syncthreads();
    // run starts: entry e of row i contributes products [P[e]-P[e0], P[e+1]-P[e0])
    for (int32_t e = e0 + pos; e < e1; e += G) {
      const int64_t s0 = a.P[e] - pbase;
      const int64_t w = a.P[e + 1] - a.P[e];
      if (w > 0) {
        const int32_t j = a.acol[e];
        rs[s0] = a.brp[j];
        ra[s0] = a.aval[e];
      }
    }
    __syncthreads();

    // segmented max-scan: the run containing product l starts at s(l)
    int st[K];
    int run = -1;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int l = pos * K + kk;
      const int f = (l < u && rs[l] >= 0) ? l : -1;
      run = max(run, f);
      st[kk] = run;
    }
    const int incl = group_incl_max<G>(run);
    int prev = __shfl_up(incl, 1, WAVE);
    if (pos == 0) prev = -1;

    Key key[K];
    T prod[K];
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int l = pos * K + kk;
      key[kk] = KMAX;
      prod[kk] = T(0);
      const int s0 = max(prev, st[kk]);
      if (l < u && s0 >= 0) {
        const int32_t bidx = rs[s0] + (l - s0);
        const T av = ra[s0];
        const int32_t c = a.bcol[bidx];
        const T bv = a.bval[bidx];
        prod[kk] = av * bv;
        key[kk] = (static_cast<Key>(c) << LOGU) | static_cast<Key>(l);
      }
    }
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int l = pos * K + kk;
      if (l < u) pv[l] = prod[kk];
    }

    group_bitonic_sort<G, K, Key>(key);

#pragma unroll
    for (int kk = 0; kk < K; ++kk) sk[pos * K + kk] = key[kk];
    const Key pk = shfl_up_key<Key>(key[K - 1], 1);
    __syncthreads();

    // compress: count the distinct columns, place them with a group scan,
    // then fold every column's products in expansion order
    uint32_t hmask = 0;
    int nh = 0;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int l = pos * K + kk;
      const Key before = kk > 0 ? key[kk - 1] : pk;
      const bool head = l < u && (l == 0 || (before >> LOGU) != (key[kk] >> LOGU));
      hmask |= head ? (1u << kk) : 0u;
      nh += head ? 1 : 0;
    }
    const int incl_h = group_incl_sum<G>(nh);
    const int total = group_last<G>(incl_h);
    if (act) {
      int64_t o = a.cto[i] + (incl_h - nh);
#pragma unroll
      for (int kk = 0; kk < K; ++kk) {
        if (hmask & (1u << kk)) {
          const int l = pos * K + kk;
          const Key c = key[kk] >> LOGU;
          T v = T(0);
          v = v + pv[static_cast<int>(key[kk] & (U - 1))];
          for (int l2 = l + 1; l2 < u; ++l2) {
            const Key k2 = sk[l2];
            if ((k2 >> LOGU) != c) break;
            v = v + pv[static_cast<int>(k2 & (U - 1))];
          }
          a.ct_col[o] = static_cast<int32_t>(c);
          a.ct_val[o] = v;
          ++o;
        }
      }
      if (pos == 0) a.rownnz[i] = total;
    }
    __syncthreads();
  }
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
