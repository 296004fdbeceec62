// Backward of C = A*B for L = <dC, C> on the fixed patterns of A and B:
//   dA_ij = sum over stored b_jk of dC_ik * b_jk       ((dC B^T) on S(A))
//   dB_jk = sum over stored a_ij of a_ij * dC_ik       ((A^T dC) on S(B))
// Every (i, k) reached lies in S(C) because S(C) is the structural product.
// Both are gathers (no floating-point atomics): one wavefront per row of A
// for dA, one per row of B for dB, the latter through A's transposed
// pattern (rows of each column in ascending order).  Each sum runs in the
// same order as the definition (ascending k, ascending i), from +0.0.
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
__global__ __launch_bounds__(256) void k_grad_a(const int32_t *arp, const int32_t *acol,
                                                int64_t m, const int32_t *brp,
                                                const int32_t *bcol, const T *bval,
                                                const int32_t *crp, const int32_t *ccol,
                                                const T *dc, T *dA) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
  if (i >= m) return;
  const int32_t c0 = crp[i], c1 = crp[i + 1];
  for (int32_t e = arp[i] + lane(); e < arp[i + 1]; e += WAVE) {
    const int32_t j = acol[e];
    T s = T(0);
    int32_t lo = c0;
    for (int32_t q = brp[j]; q < brp[j + 1]; ++q) {
      const int32_t pc = find_col(ccol, lo, c1, bcol[q]);
      s = s + dc[pc] * bval[q];
      lo = pc + 1;  // columns of b_j* ascend
    }
    dA[e] = s;
  }
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

// Column counts of A.
__global__ void k_col_count(const int32_t *acol, int64_t nnz, int32_t *cnt) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[acol[e]], 1);
}

// Scatter (row, position) of every entry into its column's segment, in any
// order; k_col_sort restores ascending rows.
__global__ __launch_bounds__(256) void k_col_scatter(const int32_t *arp, const int32_t *acol,
                                                     int64_t m, const int64_t *tptr,
                                                     int32_t *fill, int32_t *trow,
                                                     int32_t *tpos) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
  if (i >= m) return;
  for (int32_t e = arp[i] + lane(); e < arp[i + 1]; e += WAVE) {
    const int32_t j = acol[e];
    const int32_t slot = atomicAdd(&fill[j], 1);
    trow[tptr[j] + slot] = static_cast<int32_t>(i);
    tpos[tptr[j] + slot] = e;
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
  if (m > 0)
    hipLaunchKernelGGL(k_col_scatter, dim3((m * WAVE + 255) / 256), dim3(256), 0, s, arp, acol,
                       m, tptr, cnt, trow, tpos);
  if (k > 0)
    hipLaunchKernelGGL(k_col_sort, dim3((k + 255) / 256), dim3(256), 0, s, tptr, k, trow, tpos);
}

template <typename T>
void launch_grad_a(const int32_t *arp, const int32_t *acol, int64_t m, const int32_t *brp,
                   const int32_t *bcol, const T *bval, const int32_t *crp, const int32_t *ccol,
                   const T *dc, T *dA, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL((k_grad_a<T>), dim3((m * WAVE + 255) / 256), dim3(256), 0, s, arp, acol, m,
                     brp, bcol, bval, crp, ccol, dc, dA);
}

template <typename T>
void launch_grad_b(const int64_t *tptr, const int32_t *trow, const int32_t *tpos, const T *aval,
                   const int32_t *brp, const int32_t *bcol, int64_t kb, const int32_t *crp,
                   const int32_t *ccol, const T *dc, T *dB, hipStream_t s) {
  if (kb <= 0) return;
  hipLaunchKernelGGL((k_grad_b<T>), dim3((kb * WAVE + 255) / 256), dim3(256), 0, s, tptr, trow,
                     tpos, aval, brp, bcol, kb, crp, ccol, dc, dB);
}

template void launch_grad_a<float>(const int32_t *, const int32_t *, int64_t, const int32_t *,
                                   const int32_t *, const float *, const int32_t *,
                                   const int32_t *, const float *, float *, hipStream_t);
template void launch_grad_a<double>(const int32_t *, const int32_t *, int64_t, const int32_t *,
                                    const int32_t *, const double *, const int32_t *,
                                    const int32_t *, const double *, double *, hipStream_t);
template void launch_grad_b<float>(const int64_t *, const int32_t *, const int32_t *,
                                   const float *, const int32_t *, const int32_t *, int64_t,
                                   const int32_t *, const int32_t *, const float *, float *,
                                   hipStream_t);
template void launch_grad_b<double>(const int64_t *, const int32_t *, const int32_t *,
                                    const double *, const int32_t *, const int32_t *, int64_t,
                                    const int32_t *, const int32_t *, const double *, double *,
                                    hipStream_t);

}  // namespace spg
