// Stages 1-2 of the SpGEMM framework (Section 3.1): per-row upper bounds
// (Algorithm 2) through a device prefix scan, binning (Algorithm 3) as a
// per-wavefront histogram, a scan and a stable scatter, and the hybrid sizes
// of the temporary matrix C~.  Also the reduce-then-scan primitive used by
// every stage.
#include "common.hpp"
#include "internal.hpp"

namespace spg {

constexpr int SCAN_NT = 256;
constexpr int SCAN_IPT = 16;
constexpr int SCAN_TILE = SCAN_NT * SCAN_IPT;

int64_t scan_part_len(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

struct RowLenFn {
  const int32_t *acol;
  const int32_t *brp;
  DEVI int64_t operator()(int64_t e) const {
    const int32_t j = acol[e];
    return static_cast<int64_t>(brp[j + 1]) - brp[j];
  }
};
struct I64Fn {
  const int64_t *v;
  DEVI int64_t operator()(int64_t e) const { return v[e]; }
};
struct I32Fn {
  const int32_t *v;
  DEVI int64_t operator()(int64_t e) const { return v[e]; }
};

// Phase 1: sum of every tile.
template <typename F>
__global__ __launch_bounds__(SCAN_NT) void k_scan_reduce(F f, int64_t n, int64_t *part) {
  __shared__ int64_t sm[SCAN_NT / WAVE + 1];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE;
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_IPT; ++j) {
    const int64_t e = base + j * SCAN_NT + threadIdx.x;
    if (e < n) s += f(e);
  }
  int64_t tot;
  block_excl_sum<SCAN_NT>(s, sm, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Phase 2: exclusive scan of the tile sums by one work-group; part[nb] gets
// the grand total.
__global__ __launch_bounds__(SCAN_NT) void k_scan_part(int64_t *part, int64_t nb) {
  __shared__ int64_t sm[SCAN_NT / WAVE + 1];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += SCAN_NT) {
    const int64_t b = b0 + threadIdx.x;
    int64_t v = b < nb ? part[b] : 0;
    int64_t tot;
    int64_t ex = block_excl_sum<SCAN_NT>(v, sm, tot);
    if (b < nb) part[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[nb] = carry;
}

// Phase 3: rescan every tile from its offset.  Thread t owns the IPT
// consecutive elements t*IPT .. t*IPT+IPT-1 of the tile.
template <typename F>
__global__ __launch_bounds__(SCAN_NT) void k_scan_down(F f, int64_t n, const int64_t *part,
                                                       int64_t nb, int64_t *out) {
  __shared__ int64_t sm[SCAN_NT / WAVE + 1];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_IPT;
  int64_t v[SCAN_IPT];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_IPT; ++j) {
    const int64_t e = base + j;
    v[j] = e < n ? f(e) : 0;
    s += v[j];
  }
  int64_t tot;
  int64_t ex = block_excl_sum<SCAN_NT>(s, sm, tot) + part[blockIdx.x];
#pragma unroll
  for (int j = 0; j < SCAN_IPT; ++j) {
    const int64_t e = base + j;
    if (e < n) out[e] = ex;
    ex += v[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = part[nb];
}

template <typename F>
static void scan_with(F f, int64_t n, int64_t *out, int64_t *part, hipStream_t s) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 0) {
    // out[0] = 0
    hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(SCAN_NT), 0, s, part, int64_t(0));
    hipLaunchKernelGGL((k_scan_down<F>), dim3(1), dim3(SCAN_NT), 0, s, f, n, part,
                       int64_t(0), out);
    return;
  }
  hipLaunchKernelGGL((k_scan_reduce<F>), dim3(nb), dim3(SCAN_NT), 0, s, f, n, part);
  hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(SCAN_NT), 0, s, part, nb);
  hipLaunchKernelGGL((k_scan_down<F>), dim3(nb), dim3(SCAN_NT), 0, s, f, n, part, nb, out);
}

void scan_row_lengths(const int32_t *acol, const int32_t *brp, int64_t n, int64_t *out,
                      int64_t *part, hipStream_t s) {
  scan_with(RowLenFn{acol, brp}, n, out, part, s);
}
void scan_i64(const int64_t *v, int64_t n, int64_t *out, int64_t *part, hipStream_t s) {
  scan_with(I64Fn{v}, n, out, part, s);
}
void scan_i32(const int32_t *v, int64_t n, int64_t *out, int64_t *part, hipStream_t s) {
  scan_with(I32Fn{v}, n, out, part, s);
}

// ------------------------------------------------------------ validation

// One thread per row: row_ptr monotone and bounded, columns in range and
// strictly increasing.  Any violation sets sum->err.
__global__ void k_validate(const int32_t *rp, const int32_t *ci, int64_t rows, int64_t cols,
                           int64_t nnz, Summary *sum) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > rows) return;
  bool bad = false;
  if (i == 0 && rp[0] != 0) bad = true;
  if (i == rows && rp[rows] != nnz) bad = true;
  if (i < rows) {
    const int32_t a = rp[i], b = rp[i + 1];
    if (b < a || a < 0 || b > nnz) {
      bad = true;
    } else {
      int64_t prev = -1;
      for (int32_t p = a; p < b; ++p) {
        const int32_t c = ci[p];
        if (c < 0 || c >= cols || c <= prev) {
          bad = true;
          break;
        }
        prev = c;
      }
    }
  }
  if (bad) atomicOr(&sum->err, 1);
}

void launch_validate(const int32_t *rp, const int32_t *ci, int64_t rows, int64_t cols,
                     int64_t nnz, Summary *sum, hipStream_t s) {
  const int64_t nb = (rows + 1 + 255) / 256;
  hipLaunchKernelGGL(k_validate, dim3(nb), dim3(256), 0, s, rp, ci, rows, cols, nnz, sum);
}

// --------------------------------------------------------------- binning

// For each distinct bin present in the wavefront: its lane mask.  Calls
// `fn(bin, mask)` once per distinct bin (wave-uniform loop).
template <typename Fn> DEVI void for_each_bin_in_wave(bool valid, int bin, Fn fn) {
  uint64_t todo = __ballot(valid);
  while (todo) {
    const int leader = __ffsll(static_cast<long long>(todo)) - 1;
    const int b = __shfl(bin, leader, WAVE);
    const uint64_t mask = __ballot(valid && bin == b);
    fn(b, mask);
    todo &= ~mask;
  }
}

// Stage 1 result per row and the bin histogram of every wavefront.
// hist layout: hist[bin * nwaves + wave] so that one exclusive scan yields,
// for every (bin, wave), the start of that wave's rows in the bin list.
__global__ __launch_bounds__(256) void k_row_stats(const int32_t *arp, const int64_t *P,
                                                   int64_t m, int64_t ncols, BinEdges be,
                                                   int32_t long_slot, int64_t *u, int64_t *h,
                                                   int32_t *hist, int64_t nwaves,
                                                   int64_t *rownnz, Summary *sum) {
  __shared__ int32_t cnt[256 / WAVE][NBINS];
  const int w = threadIdx.x / WAVE;
  for (int b = lane(); b < NBINS; b += WAVE) cnt[w][b] = 0;
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool valid = i < m;
  int64_t ui = 0;
  int bin = 0;
  if (valid) {
    ui = P[arp[i + 1]] - P[arp[i]];
    bin = bin_of(ui, be);
    u[i] = ui;
    h[i] = bin == LONG_BIN ? static_cast<int64_t>(long_slot) : ui;
    if (ui == 0) rownnz[i] = 0;
  }
  for_each_bin_in_wave(valid, bin, [&](int b, uint64_t mask) {
    if (lane() == 0) cnt[w][b] = __popcll(mask);
  });
  __syncthreads();
  const int64_t gw = static_cast<int64_t>(blockIdx.x) * (256 / WAVE) + w;
  if (gw < nwaves) {
    for (int b = lane(); b < NBINS; b += WAVE) hist[b * nwaves + gw] = cnt[w][b];
  }
  // largest u: wave max then one atomic per wave
  unsigned long long mx = static_cast<unsigned long long>(ui);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long y = static_cast<unsigned long long>(
        __shfl_xor(static_cast<long long>(mx), o, WAVE));
    mx = mx > y ? mx : y;
  }
  if (lane() == 0 && mx > 0) atomicMax(&sum->max_u, mx);
  // products and result bound of the long rows (sizes the long-row pool)
  long long lu = bin == LONG_BIN ? static_cast<long long>(ui) : 0;
  long long lr = bin == LONG_BIN ? static_cast<long long>(ui < ncols ? ui : ncols) : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lu += __shfl_xor(lu, o, WAVE);
    lr += __shfl_xor(lr, o, WAVE);
  }
  if (lane() == 0 && lu > 0) {
    atomicAdd(reinterpret_cast<unsigned long long *>(&sum->sum_u_long),
              static_cast<unsigned long long>(lu));
    atomicAdd(reinterpret_cast<unsigned long long *>(&sum->sum_r_long),
              static_cast<unsigned long long>(lr));
  }
}

void launch_row_stats(const int32_t *arp, const int64_t *P, int64_t m, int64_t ncols,
                      BinEdges be, int32_t long_slot, int64_t *u, int64_t *h, int32_t *hist,
                      int64_t nwaves, int64_t *rownnz, Summary *sum, hipStream_t s) {
  const int64_t nb = (m + 255) / 256;
  if (nb == 0) return;
  hipLaunchKernelGGL(k_row_stats, dim3(nb), dim3(256), 0, s, arp, P, m, ncols, be, long_slot, u,
                     h, hist, nwaves, rownnz, sum);
}

// Stable scatter: rows keep ascending order inside each bin.
__global__ __launch_bounds__(256) void k_bin_scatter(const int64_t *u, int64_t m, BinEdges be,
                                                     const int64_t *hist_scan, int64_t nwaves,
                                                     int32_t *binlist) {
  const int w = threadIdx.x / WAVE;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool valid = i < m;
  const int bin = valid ? bin_of(u[i], be) : 0;
  const int64_t gw = static_cast<int64_t>(blockIdx.x) * (256 / WAVE) + w;
  const uint64_t lt = (lane() == 0) ? 0ull : (~0ull >> (WAVE - lane()));
  for_each_bin_in_wave(valid, bin, [&](int b, uint64_t mask) {
    if (valid && bin == b) {
      const int64_t pos = hist_scan[b * nwaves + gw] + __popcll(mask & lt);
      binlist[pos] = static_cast<int32_t>(i);
    }
  });
}

void launch_bin_scatter(const int64_t *u, int64_t m, BinEdges be, const int64_t *hist_scan,
                        int64_t nwaves, int32_t *binlist, hipStream_t s) {
  const int64_t nb = (m + 255) / 256;
  if (nb == 0) return;
  hipLaunchKernelGGL(k_bin_scatter, dim3(nb), dim3(256), 0, s, u, m, be, hist_scan, nwaves,
                     binlist);
}

__global__ void k_summary(const int64_t *P, int64_t nnzA, const int64_t *cto, int64_t m,
                          const int64_t *hist_scan, int64_t nwaves, Summary *sum) {
  const int t = threadIdx.x;
  if (t == 0) {
    sum->sum_u = P[nnzA];
    sum->sum_h = cto[m];
  }
  if (t <= NBINS) sum->bin_off[t] = (t < NBINS) ? hist_scan[t * nwaves] : hist_scan[NBINS * nwaves];
}

void launch_summary(const int64_t *P, int64_t nnzA, const int64_t *cto, int64_t m,
                    const int64_t *hist_scan, int64_t nwaves, Summary *sum, hipStream_t s) {
  hipLaunchKernelGGL(k_summary, dim3(1), dim3(64), 0, s, P, nnzA, cto, m, hist_scan, nwaves, sum);
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

void launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill_i64, dim3(nb), dim3(256), 0, s, p, n, v);
}

__global__ void k_zero(uint32_t *p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

void launch_zero(void *p, size_t bytes, hipStream_t s) {
  const int64_t n = static_cast<int64_t>((bytes + 3) / 4);
  if (n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, s, static_cast<uint32_t *>(p), n);
}

__global__ void k_status(const int64_t *rowoff, int64_t m, const Pool *pool, ComputeStatus *st) {
  st->nnz_c = rowoff[m];
  st->fail_count = pool->fail_count;
  st->pool_used = pool->used;
}

void launch_status(const int64_t *rowoff, int64_t m, const Pool *pool, ComputeStatus *st,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_status, dim3(1), dim3(1), 0, s, rowoff, m, pool, st);
}

}  // namespace spg
