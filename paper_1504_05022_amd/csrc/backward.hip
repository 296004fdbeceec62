// Backward of C = A*B for L = <dC, C> on the fixed patterns of A and B:
//   dA_ij = sum over stored b_jk of dC_ik * b_jk       ((dC B^T) on S(A))
//   dB_jk = sum over stored a_ij of a_ij * dC_ik       ((A^T dC) on S(B))
// Every (i, k) reached lies in S(C) because S(C) is the structural product.
// Both are gathers (no floating-point atomics).  dA, and the products
// a_ij dC_ik of dB, come from an entry-parallel pass over A; dB then adds
// those products per b_jk over A's transposed pattern (rows of each column in
// ascending order).  Without room for the products, dB is gathered per row
// of B with binary searches in C.  Each sum runs in the order of the
// definition (ascending k, ascending i), from +0.0.
#include "common.hpp"
#include "internal.hpp"

namespace spg {

DEVI int32_t find_col(const int32_t *col, int32_t lo, int32_t hi, int32_t c) {
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (col[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <typename T>
__global__ __launch_bounds__(256) void k_grad_b(const int64_t *tptr, const int32_t *trow,
                                                const int32_t *tpos, const T *aval,
                                                const int32_t *brp, const int32_t *bcol,
                                                int64_t kb, const int32_t *crp,
                                                const int32_t *ccol, const T *dc, T *dB) {
  const int64_t j = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
  if (j >= kb) return;
  const int64_t t0 = tptr[j], t1 = tptr[j + 1];
  for (int32_t q = brp[j] + lane(); q < brp[j + 1]; q += WAVE) {
    const int32_t c = bcol[q];
    T s = T(0);
    for (int64_t d = t0; d < t1; ++d) {
      const int32_t i = trow[d];
      const int32_t pc = find_col(ccol, crp[i], crp[i + 1], c);
      s = s + aval[tpos[d]] * dc[pc];
    }
    dB[q] = s;
  }
}

// ---------------------------------------------------------------------------
// Entry-parallel form.  One wavefront per chunk of BW_CH consecutive entries
// of A (rows found by a binary search on A's row pointers, so rows of any
// length are spread evenly).  For every entry e = (i, j) and every stored
// b_jk, y = dC_ik is looked up -- in a dense LDS copy of the row's dC when C
// has few columns, else by a binary search in c_i* -- and
//   dA_e += y * b_jk                  (ascending k, as in the definition)
//   W[P_e + q] = a_ij * y             (q = position of b_jk in b_j*)
// where P_e is the product offset of entry e from stage 1.  W holds every
// product a_ij dC_ik of the dB sums; k_grad_b_sum adds them per b_jk over
// A's transposed pattern (ascending i).  Sums, products and their order are
// those of the definition (and of k_grad_b).
constexpr int BW_CH = 512;
constexpr int BW_NT = 128;  // two wavefronts: 32 KB of dense rows per work-group
constexpr int BW_U = 8;  // entries of b_j* whose loads are in flight together
// with the dense dC row (16 KB of LDS per wavefront, so LDS, not registers,
// caps the kernel at two wavefronts per SIMD) a whole block of 32 entries
// of b_j* is loaded at once: fewer dependent round trips per entry
constexpr int BW_UD = 32;
constexpr int BW_SC = 8;  // passes of a dC row's scatter whose loads are in flight together
constexpr int BW_MAP_BYTES = 16384;  // dense dC row per wavefront

template <typename T> constexpr int bw_map_cols() { return BW_MAP_BYTES / static_cast<int>(sizeof(T)); }

template <typename T, bool DENSE>
__global__ __launch_bounds__(BW_NT) void k_grad_entries(
    const int32_t *arp, const int32_t *acol, const T *aval, int64_t m, int64_t nnz,
    const int64_t *P, const int32_t *brp, const int32_t *bcol, const T *bval, const int32_t *crp,
    const int32_t *ccol, const T *dc, T *dA, T *W) {
  constexpr int NWV = BW_NT / WAVE;
  constexpr int MAPC = DENSE ? bw_map_cols<T>() : 1;
  __shared__ T map[NWV * MAPC];
  const int w = threadIdx.x / WAVE;
  const int ln = lane();
  const int64_t e0 = (static_cast<int64_t>(blockIdx.x) * NWV + w) * BW_CH;
  if (e0 >= nnz) return;  // uniform across the wavefront; no work-group barriers here
  const int64_t e1 = e0 + BW_CH < nnz ? e0 + BW_CH : nnz;
  // dense dC row: every column a row looks up is one of its own C columns
  // (C holds every structural product), written by that row's scatter, so
  // the map is never cleared
  T *mp = map + w * MAPC;
  int64_t lo = 0, hi = m;  // the row holding e0: last i with arp[i] <= e0
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (arp[mid] <= e0)
      lo = mid;
    else
      hi = mid;
  }
  int64_t i = lo;
  int64_t e = e0;
  while (e < e1) {
    while (arp[i + 1] <= e) ++i;  // skip empty rows
    const int64_t re = arp[i + 1] < e1 ? static_cast<int64_t>(arp[i + 1]) : e1;
    const int32_t c0 = crp[i], c1 = crp[i + 1];
    if (DENSE) {
      // the row's dC entries, BW_SC passes of the wavefront loaded together
      // (clamped to the row) before they are written to the map
      for (int32_t xb = c0; xb < c1; xb += BW_SC * WAVE) {
        int32_t cc[BW_SC];
        T vv[BW_SC];
#pragma unroll
        for (int u = 0; u < BW_SC; ++u) {
          const int32_t x = xb + u * WAVE + ln;
          const int32_t xc = x < c1 ? x : c1 - 1;
          cc[u] = ccol[xc];
          vv[u] = dc[xc];
        }
#pragma unroll
        for (int u = 0; u < BW_SC; ++u)
          if (xb + u * WAVE + ln < c1) mp[cc[u]] = vv[u];
      }
      wave_sync();
    }
    for (int64_t ee = e + ln; ee < re; ee += WAVE) {
      const int32_t j = acol[ee];
      const T av = aval[ee];
      const int32_t q0 = brp[j], q1 = brp[j + 1];
      T *wp = W ? W + (P[ee] - q0) : nullptr;
      T s = T(0);
      int32_t from = c0;
      // blocks of UB entries of b_j*: their loads are issued together
      // (clamped to the row), then the block is added in order
      constexpr int UB = DENSE ? BW_UD : BW_U;
      for (int32_t qb = q0; qb < q1; qb += UB) {
        int32_t kk[UB];
        T bv[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int32_t q = qb + u < q1 ? qb + u : q1 - 1;
          kk[u] = bcol[q];
          bv[u] = bval[q];
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          if (qb + u < q1) {
            T y;
            if (DENSE) {
              y = mp[kk[u]];
            } else {
              const int32_t pc = find_col(ccol, from, c1, kk[u]);
              y = dc[pc];
              from = pc + 1;  // columns of b_j* ascend
            }
            s = s + y * bv[u];
            if (wp) wp[qb + u] = av * y;
          }
        }
      }
      if (dA) dA[ee] = s;
    }
    if (DENSE) wave_sync();  // this row's lookups precede the next row's scatter
    e = re;
  }
}

// dB_jk = sum over A's column j (ascending i) of the products a_ij dC_ik in W.
// BW_SUB lanes per row of B (each lane sums its own entries, so rows share
// a wavefront without any ordering between them).
constexpr int BW_SUB = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_grad_b_sum(const int64_t *tptr, const int32_t *tpos,
                                                    const int64_t *P, const int32_t *brp,
                                                    int64_t kb, const T *W, T *dB) {
  const int64_t j = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / BW_SUB;
  if (j >= kb) return;
  const int64_t t0 = tptr[j], t1 = tptr[j + 1];
  const int32_t q0 = brp[j], q1 = brp[j + 1];
  for (int32_t q = q0 + (lane() & (BW_SUB - 1)); q < q1; q += BW_SUB) {
    T s = T(0);
    // blocks of BW_U entries of A's column j: offsets, then products, each
    // loaded together (clamped to the column), then added in order
    for (int64_t db = t0; db < t1; db += BW_U) {
      int64_t off[BW_U];
#pragma unroll
      for (int u = 0; u < BW_U; ++u) off[u] = P[tpos[db + u < t1 ? db + u : t1 - 1]];
      T v[BW_U];
#pragma unroll
      for (int u = 0; u < BW_U; ++u) v[u] = W[off[u] + (q - q0)];
#pragma unroll
      for (int u = 0; u < BW_U; ++u)
        if (db + u < t1) s = s + v[u];
    }
    dB[q] = s;
  }
}

template <typename T>
void launch_grad_entries(const int32_t *arp, const int32_t *acol, const T *aval, int64_t m,
                         int64_t nnz, const int64_t *P, const int32_t *brp, const int32_t *bcol,
                         const T *bval, int64_t n, const int32_t *crp, const int32_t *ccol,
                         const T *dc, T *dA, T *W, hipStream_t s) {
  if (nnz <= 0) return;
  const int64_t waves = (nnz + BW_CH - 1) / BW_CH;
  const int64_t grid = (waves + BW_NT / WAVE - 1) / (BW_NT / WAVE);
  if (n <= bw_map_cols<T>())
    hipLaunchKernelGGL((k_grad_entries<T, true>), dim3(grid), dim3(BW_NT), 0, s, arp, acol, aval,
                       m, nnz, P, brp, bcol, bval, crp, ccol, dc, dA, W);
  else
    hipLaunchKernelGGL((k_grad_entries<T, false>), dim3(grid), dim3(BW_NT), 0, s, arp, acol,
                       aval, m, nnz, P, brp, bcol, bval, crp, ccol, dc, dA, W);
}

template <typename T>
void launch_grad_b_sum(const int64_t *tptr, const int32_t *tpos, const int64_t *P,
                       const int32_t *brp, int64_t kb, const T *W, T *dB, hipStream_t s) {
  if (kb <= 0) return;
  hipLaunchKernelGGL((k_grad_b_sum<T>), dim3((kb * BW_SUB + 255) / 256), dim3(256), 0, s, tptr,
                     tpos, P, brp, kb, W, dB);
}

template void launch_grad_entries<float>(const int32_t *, const int32_t *, const float *, int64_t,
                                         int64_t, const int64_t *, const int32_t *,
                                         const int32_t *, const float *, int64_t,
                                         const int32_t *, const int32_t *, const float *, float *,
                                         float *, hipStream_t);
template void launch_grad_entries<double>(const int32_t *, const int32_t *, const double *,
                                          int64_t, int64_t, const int64_t *, const int32_t *,
                                          const int32_t *, const double *, int64_t,
                                          const int32_t *, const int32_t *, const double *,
                                          double *, double *, hipStream_t);
template void launch_grad_b_sum<float>(const int64_t *, const int32_t *, const int64_t *,
                                       const int32_t *, int64_t, const float *, float *,
                                       hipStream_t);
template void launch_grad_b_sum<double>(const int64_t *, const int32_t *, const int64_t *,
                                        const int32_t *, int64_t, const double *, double *,
                                        hipStream_t);

// Column counts of A.
__global__ void k_col_count(const int32_t *acol, int64_t nnz, int32_t *cnt) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[acol[e]], 1);
}

// Scatter (row, position) of every entry into its column's segment, in any
// order; k_col_sort restores ascending rows.  One wavefront per chunk of
// TS_CH consecutive entries (rows found by one binary search per wavefront,
// then walked per lane), TS_U entries per lane whose column loads and slot
// atomics are in flight together.
constexpr int TS_U = 4;
constexpr int TS_CH = WAVE * TS_U;

__global__ __launch_bounds__(256) void k_col_scatter(const int32_t *arp, const int32_t *acol,
                                                     int64_t m, int64_t nnz, const int64_t *tptr,
                                                     int32_t *fill, int32_t *trow,
                                                     int32_t *tpos) {
  const int64_t e0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE * TS_CH;
  if (e0 >= nnz) return;  // uniform across the wavefront
  int64_t lo = 0, hi = m;  // the row holding e0: last i with arp[i] <= e0
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (arp[mid] <= e0)
      lo = mid;
    else
      hi = mid;
  }
  int64_t e[TS_U], row[TS_U];
  int32_t col[TS_U], slot[TS_U];
  int64_t i = lo;
#pragma unroll
  for (int u = 0; u < TS_U; ++u) {
    e[u] = e0 + u * WAVE + lane();
    if (e[u] < nnz)
      while (arp[i + 1] <= e[u]) ++i;  // entries ascend with u, so rows do too
    row[u] = i;
  }
#pragma unroll
  for (int u = 0; u < TS_U; ++u) col[u] = e[u] < nnz ? acol[e[u]] : 0;
#pragma unroll
  for (int u = 0; u < TS_U; ++u) slot[u] = e[u] < nnz ? atomicAdd(&fill[col[u]], 1) : 0;
#pragma unroll
  for (int u = 0; u < TS_U; ++u) {
    if (e[u] < nnz) {
      const int64_t d = tptr[col[u]] + slot[u];
      trow[d] = static_cast<int32_t>(row[u]);
      tpos[d] = static_cast<int32_t>(e[u]);
    }
  }
}

// Insertion sort of every column segment by row (rows are distinct).
__global__ void k_col_sort(const int64_t *tptr, int64_t k, int32_t *trow, int32_t *tpos) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const int64_t a = tptr[j], b = tptr[j + 1];
  for (int64_t x = a + 1; x < b; ++x) {
    const int32_t r = trow[x], p = tpos[x];
    int64_t y = x - 1;
    while (y >= a && trow[y] > r) {
      trow[y + 1] = trow[y];
      tpos[y + 1] = tpos[y];
      --y;
    }
    trow[y + 1] = r;
    tpos[y + 1] = p;
  }
}

void launch_transpose_pattern(const int32_t *arp, const int32_t *acol, int64_t m, int64_t k,
                              int64_t nnz, int32_t *cnt, int64_t *tptr, int32_t *trow,
                              int32_t *tpos, int64_t *part, hipStream_t s) {
  launch_zero(cnt, static_cast<size_t>(k) * 4, s);
  if (nnz > 0)
    hipLaunchKernelGGL(k_col_count, dim3((nnz + 255) / 256), dim3(256), 0, s, acol, nnz, cnt);
  scan_i32(cnt, k, tptr, part, s);
  launch_zero(cnt, static_cast<size_t>(k) * 4, s);
  if (nnz > 0) {
    const int64_t waves = (nnz + TS_CH - 1) / TS_CH;
    hipLaunchKernelGGL(k_col_scatter, dim3((waves * WAVE + 255) / 256), dim3(256), 0, s, arp,
                       acol, m, nnz, tptr, cnt, trow, tpos);
  }
  if (k > 0)
    hipLaunchKernelGGL(k_col_sort, dim3((k + 255) / 256), dim3(256), 0, s, tptr, k, trow, tpos);
}

template <typename T>
void launch_grad_b(const int64_t *tptr, const int32_t *trow, const int32_t *tpos, const T *aval,
                   const int32_t *brp, const int32_t *bcol, int64_t kb, const int32_t *crp,
                   const int32_t *ccol, const T *dc, T *dB, hipStream_t s) {
  if (kb <= 0) return;
  hipLaunchKernelGGL((k_grad_b<T>), dim3((kb * WAVE + 255) / 256), dim3(256), 0, s, tptr, trow,
                     tpos, aval, brp, bcol, kb, crp, ccol, dc, dB);
}

template void launch_grad_b<float>(const int64_t *, const int32_t *, const int32_t *,
                                   const float *, const int32_t *, const int32_t *, int64_t,
                                   const int32_t *, const int32_t *, const float *, float *,
                                   hipStream_t);
template void launch_grad_b<double>(const int64_t *, const int32_t *, const int32_t *,
                                    const double *, const int32_t *, const int32_t *, int64_t,
                                    const int32_t *, const int32_t *, const double *, double *,
                                    hipStream_t);

}  // namespace spg
