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
struct PieceFn {
  const Piece *p;
  DEVI int64_t operator()(int64_t e) const { return p[e].cnt; }
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

// Phase 3: rescan every tile from its offset.  Loads and stores are
// coalesced (consecutive threads, consecutive elements); the tile goes
// through LDS so that thread t can scan its IPT consecutive elements
// t*IPT .. t*IPT+IPT-1 (one pad word per IPT elements keeps that access
// spread over the banks).
DEVI int scan_lds_ix(int i) { return i + i / SCAN_IPT; }

// SELF: `part` holds the raw tile sums and every work-group adds up those
// of the tiles before it (fine for a few thousand tiles; saves the launch of
// phase 2); otherwise `part` is phase 2's exclusive scan.
template <typename F, bool SELF>
__global__ __launch_bounds__(SCAN_NT) void k_scan_down(F f, int64_t n, const int64_t *part,
                                                       int64_t nb, int64_t *out) {
  __shared__ int64_t sm[SCAN_NT / WAVE + 1];
  __shared__ int64_t tile[SCAN_TILE + SCAN_TILE / SCAN_IPT];
  const int t = threadIdx.x;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE;
  int64_t offset = 0;
  if constexpr (SELF) {
    int64_t ps = 0;
    for (int64_t b = t; b < static_cast<int64_t>(blockIdx.x); b += SCAN_NT) ps += part[b];
    block_excl_sum<SCAN_NT>(ps, sm, offset);
  } else {
    offset = part[blockIdx.x];
  }
#pragma unroll
  for (int j = 0; j < SCAN_IPT; ++j) {
    const int i = j * SCAN_NT + t;
    const int64_t e = base + i;
    tile[scan_lds_ix(i)] = e < n ? f(e) : 0;
  }
  __syncthreads();
  int64_t v[SCAN_IPT];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_IPT; ++j) {
    v[j] = tile[scan_lds_ix(t * SCAN_IPT + j)];
    s += v[j];
  }
  int64_t tot;
  int64_t ex = block_excl_sum<SCAN_NT>(s, sm, tot) + offset;
#pragma unroll
  for (int j = 0; j < SCAN_IPT; ++j) {
    tile[scan_lds_ix(t * SCAN_IPT + j)] = ex;  // the slots this thread read
    ex += v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < SCAN_IPT; ++j) {
    const int i = j * SCAN_NT + t;
    const int64_t e = base + i;
    if (e < n) out[e] = tile[scan_lds_ix(i)];
  }
  if constexpr (SELF) {
    if (blockIdx.x == nb - 1 && t == 0) out[n] = offset + tot;
  } else {
    if (blockIdx.x == 0 && t == 0) out[n] = part[nb];
  }
}

// tiles up to which a work-group of phase 3 sums the earlier tile sums itself
constexpr int64_t SCAN_SELF_MAX_TILES = 4096;

template <typename F>
static void scan_with(F f, int64_t n, int64_t *out, int64_t *part, hipStream_t s) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 0) {
    // out[0] = 0
    hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(SCAN_NT), 0, s, part, int64_t(0));
    hipLaunchKernelGGL((k_scan_down<F, false>), dim3(1), dim3(SCAN_NT), 0, s, f, n, part,
                       int64_t(0), out);
    return;
  }
  hipLaunchKernelGGL((k_scan_reduce<F>), dim3(nb), dim3(SCAN_NT), 0, s, f, n, part);
  if (nb <= SCAN_SELF_MAX_TILES) {
    hipLaunchKernelGGL((k_scan_down<F, true>), dim3(nb), dim3(SCAN_NT), 0, s, f, n, part, nb,
                       out);
    return;
  }
  hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(SCAN_NT), 0, s, part, nb);
  hipLaunchKernelGGL((k_scan_down<F, false>), dim3(nb), dim3(SCAN_NT), 0, s, f, n, part, nb,
                     out);
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
void scan_piece_counts(const Piece *pieces, int64_t n, int64_t *out, int64_t *part,
                       hipStream_t s) {
  scan_with(PieceFn{pieces}, n, out, part, s);
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
// Also per-block sums that size the long-row work (reduced by k_summary).
__global__ __launch_bounds__(256) void k_row_stats(RowStatsArgs a) {
  __shared__ int32_t cnt[256 / WAVE][NBINS];
  __shared__ int64_t red[256 / WAVE][kBlockStats];
  const int w = threadIdx.x / WAVE;
  for (int b = lane(); b < NBINS; b += WAVE) cnt[w][b] = 0;
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool valid = i < a.m;
  int64_t ui = 0;
  int bin = 0;
  if (valid) {
    ui = a.P[a.arp[i + 1]] - a.P[a.arp[i]];
    bin = bin_of(ui, a.be);
    a.u[i] = ui;
    a.h[i] = bin == LONG_BIN ? static_cast<int64_t>(a.long_slot) : ui;
    if (ui == 0) a.rownnz[i] = 0;
  }
  for_each_bin_in_wave(valid, bin, [&](int b, uint64_t mask) {
    if (lane() == 0) cnt[w][b] = __popcll(mask);
  });
  __syncthreads();
  const int64_t gw = static_cast<int64_t>(blockIdx.x) * (256 / WAVE) + w;
  if (gw < a.nwaves) {
    for (int b = lane(); b < NBINS; b += WAVE) a.hist[b * a.nwaves + gw] = cnt[w][b];
  }
  // long-row planning sums
  int64_t v[kBlockStats];
#pragma unroll
  for (int k = 0; k < kBlockStats; ++k) v[k] = 0;
  v[0] = ui;
  if (bin == LONG_BIN) {
    const int64_t rmax = ui < a.ncols ? ui : a.ncols;
    int64_t segp;
    int32_t nseg, shift, npiece;
    long_row_plan(ui, a.ncols, a.lp, segp, nseg, shift, npiece);
    v[1] = ui;
    v[2] = rmax;
    v[3] = nseg;
    v[4] = npiece;
    if (nseg > 1) {
      v[5] = ui;
      v[6] = static_cast<int64_t>(nseg) * (npiece + 1);
      v[8] = rmax;
    } else if (ui <= kOneShot) {
      v[5] = rmax;  // one-tile row: its result has a place of its own
    } else if (rmax > a.long_slot) {
      int64_t cap = a.long_slot;
      while (cap < rmax) cap *= 2;
      v[7] = cap;
    }
    const int64_t segr = segp < a.ncols ? segp : a.ncols;
    if (segr > a.l1cap - kLongTile) v[9] = segr * nseg;
    const WinPlan wp = win_plan(ui, a.ncols, a.vbytes);
    v[10] = wp.nitem;
    v[11] = wp.nseg;
    v[12] = wp.table;
    v[13] = wp.partial;
    v[14] = wp.dslots;
    v[15] = wp.mode == WIN_NONE ? 1 : 0;
  }
#pragma unroll
  for (int k = 0; k < kBlockStats; ++k) {
    int64_t x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int64_t y = __shfl_xor(x, o, WAVE);
      x = k == 0 ? (x > y ? x : y) : x + y;
    }
    if (lane() == 0) red[w][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < kBlockStats) {
    const int k = threadIdx.x;
    int64_t x = red[0][k];
    for (int q = 1; q < 256 / WAVE; ++q) x = k == 0 ? (x > red[q][k] ? x : red[q][k]) : x + red[q][k];
    a.bpart[static_cast<int64_t>(blockIdx.x) * kBlockStats + k] = x;
  }
}

void launch_row_stats(const RowStatsArgs &a, hipStream_t s) {
  const int64_t nb = (a.m + 255) / 256;
  if (nb == 0) return;
  hipLaunchKernelGGL(k_row_stats, dim3(nb), dim3(256), 0, s, a);
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

__global__ __launch_bounds__(256) void k_summary(const int64_t *P, int64_t nnzA,
                                                 const int64_t *cto, int64_t m,
                                                 const int64_t *hist_scan, int64_t nwaves,
                                                 const int64_t *bpart, int64_t nblocks,
                                                 Summary *sum) {
  __shared__ int64_t red[256 / WAVE][kBlockStats];
  const int t = threadIdx.x;
  if (t == 0) {
    sum->sum_u = P[nnzA];
    sum->sum_h = cto[m];
  }
  if (t <= NBINS) sum->bin_off[t] = (t < NBINS) ? hist_scan[t * nwaves] : hist_scan[NBINS * nwaves];
  int64_t v[kBlockStats];
#pragma unroll
  for (int k = 0; k < kBlockStats; ++k) v[k] = 0;
  for (int64_t b = t; b < nblocks; b += 256) {
#pragma unroll
    for (int k = 0; k < kBlockStats; ++k) {
      const int64_t x = bpart[b * kBlockStats + k];
      v[k] = k == 0 ? (v[k] > x ? v[k] : x) : v[k] + x;
    }
  }
#pragma unroll
  for (int k = 0; k < kBlockStats; ++k) {
    int64_t x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int64_t y = __shfl_xor(x, o, WAVE);
      x = k == 0 ? (x > y ? x : y) : x + y;
    }
    if (lane() == 0) red[t / WAVE][k] = x;
  }
  __syncthreads();
  if (t < kBlockStats) {
    int64_t x = red[0][t];
    for (int q = 1; q < 256 / WAVE; ++q) x = t == 0 ? (x > red[q][t] ? x : red[q][t]) : x + red[q][t];
    switch (t) {
      case 0: sum->max_u = static_cast<unsigned long long>(x); break;
      case 1: sum->sum_u_long = x; break;
      case 2: sum->sum_r_long = x; break;
      case 3: sum->n_items = x; break;
      case 4: sum->n_pieces = x; break;
      case 5: sum->sum_u_multi = x; break;
      case 6: sum->n_split = x; break;
      case 7: sum->pool_single = x; break;
      case 8: sum->sum_r_multi = x; break;
      case 9: sum->spill_bound = x; break;
      case 10: sum->w_items = x; break;
      case 11: sum->w_segs = x; break;
      case 12: sum->w_table = x; break;
      case 13: sum->w_partial = x; break;
      case 14: sum->w_dslots = x; break;
      case 15: sum->w_none = x; break;
    }
  }
}

void launch_summary(const int64_t *P, int64_t nnzA, const int64_t *cto, int64_t m,
                    const int64_t *hist_scan, int64_t nwaves, const int64_t *bpart,
                    int64_t nblocks, Summary *sum, hipStream_t s) {
  hipLaunchKernelGGL(k_summary, dim3(1), dim3(256), 0, s, P, nnzA, cto, m, hist_scan, nwaves,
                     bpart, nblocks, sum);
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

__global__ void k_set_pool(Pool *dst, Pool value) { *dst = value; }

void launch_set_pool(Pool *dst, Pool value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_pool, dim3(1), dim3(1), 0, s, dst, value);
}

__global__ void k_status(const int64_t *rowoff, int64_t m, const Pool *pool, ComputeStatus *st) {
  st->nnz_c = rowoff[m];
  st->fail_count = pool->fail_count;
  st->fail2 = pool->fail2;
  st->pool_used = pool->used;
}

void launch_status(const int64_t *rowoff, int64_t m, const Pool *pool, ComputeStatus *st,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_status, dim3(1), dim3(1), 0, s, rowoff, m, pool, st);
}

}  // namespace spg
