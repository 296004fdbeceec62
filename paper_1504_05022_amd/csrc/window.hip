// Long rows (bin group 5) by windows of columns: the default method for rows
// above the last group-4 edge.
//
// The paper gives a long row one thread group and merges its products into
// a sequence that spills to global memory (Section 3.1, merge method).  On
// gfx950 a few rows hold most of the products of irregular inputs, and a
// work-group that walks one row through many dependent memory and LDS steps
// leaves the CU waiting, so a row is cut into items, each a window of
// columns that ONE WAVEFRONT finishes (many independent wavefronts per CU,
// wavefront-local LDS ordering only):
//
//  * direct sparse rows (u <= kWinDirect): one item; the products are
//    gathered from the B rows into LDS in expansion order, ordered by a
//    counting sort on the high column bits (kWinBuckets buckets) and a rank
//    among the few entries of each bucket, then every column is folded in
//    expansion order;
//  * partitioned rows: segments of kWinSeg consecutive products are
//    scattered stably (expansion order kept inside every bucket, ranks from
//    wavefront ballots) by column piece (2^shift columns) into a partial
//    array, with a piece-start table; a piece then gathers its share of every
//    segment in segment order -- again expansion order -- and is finished
//    like a direct sparse row;
//  * direct dense rows (n <= the dense window) and pieces with more products
//    than a wavefront stages are listed and finished by work-groups with a
//    dense accumulator that persists across chunks of products; dense rows
//    above kWinSplit products are cut into product ranges whose dense
//    partial rows are added in range order by a reduction.
//
// Within a column the products are always added in expansion order
// (ascending j, then the position inside b_j*), from +0.0, without fused
// multiply-add: every value equals Gustavson's sequential sum, except for
// direct dense rows cut into product ranges.
//
// A symbolic pass (the same ordering, counting distinct columns; a bitmap
// in the work-group kernel) sizes every item first, so that C can be
// allocated before the numeric pass, which writes every item straight to
// its place in C.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace spg {

namespace {

constexpr int WNT = 256;            // threads of the work-group kernels
constexpr int WG_STAGE = 2048;      // products staged per chunk (work-group kernels)
constexpr int WKP = WG_STAGE / WNT; // products per thread and round (work-group kernels)
constexpr int WVK = kWinStage / WAVE; // products per lane (wavefront kernels)

template <typename T> struct ValTraits;
template <> struct ValTraits<float> { static constexpr int dl = 12; };
template <> struct ValTraits<double> { static constexpr int dl = 11; };

DEVI uint64_t lanes_below() { return lane() == 0 ? 0ull : (~0ull >> (WAVE - lane())); }

// Largest k in [0, n) with pre[k] <= x.
DEVI int batch_find(const int32_t *pre, int n, int32_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- planning

__host__ __device__ inline void plan_values(const WinPlan &p, int64_t (&v)[5]) {
  v[0] = p.nitem;
  v[1] = p.nseg;
  v[2] = p.table;
  v[3] = p.partial;
  v[4] = p.dslots;
}

// Per block of 256 long rows: the five plan sums.
__global__ __launch_bounds__(256) void k_wplan_count(const int32_t *lrows, int64_t nlong,
                                                     const int64_t *u, int64_t n, int vbytes,
                                                     int64_t *bsum) {
  __shared__ int64_t red[256 / WAVE][5];
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  int64_t v[5] = {0, 0, 0, 0, 0};
  if (k < nlong) plan_values(win_plan(u[lrows[k]], n, vbytes), v);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const int64_t x = group_incl_sum<WAVE>(v[q]);
    if (lane() == WAVE - 1) red[threadIdx.x / WAVE][q] = x;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    int64_t x = 0;
    for (int w = 0; w < 256 / WAVE; ++w) x += red[w][threadIdx.x];
    bsum[static_cast<int64_t>(blockIdx.x) * 5 + threadIdx.x] = x;
  }
}

// Exclusive scan of the block sums (one work-group, in rounds of 256).
__global__ __launch_bounds__(256) void k_wplan_scan(int64_t *bsum, int64_t nblk) {
  __shared__ int64_t sm[256 / WAVE + 1];
  for (int q = 0; q < 5; ++q) {
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nblk; b0 += 256) {
      const int64_t b = b0 + threadIdx.x;
      const int64_t x = b < nblk ? bsum[b * 5 + q] : 0;
      int64_t tot;
      const int64_t ex = block_excl_sum<256, int64_t>(x, sm, tot);
      if (b < nblk) bsum[b * 5 + q] = carry + ex;
      carry += tot;
    }
  }
}

// Row records (one thread per long row).
__global__ __launch_bounds__(256) void k_wplan_write(const int32_t *lrows, int64_t nlong,
                                                     const int64_t *u, int64_t n, int vbytes,
                                                     const int64_t *bsum, WinRow *rows) {
  __shared__ int64_t sm[256 / WAVE + 1];
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  WinPlan p{};
  p.mode = WIN_NONE;
  int64_t ui = 0;
  int32_t row = 0;
  if (k < nlong) {
    row = lrows[k];
    ui = u[row];
    p = win_plan(ui, n, vbytes);
  }
  int64_t v[5];
  plan_values(p, v);
  int64_t off[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    int64_t tot;
    off[q] = block_excl_sum<256, int64_t>(v[q], sm, tot) + bsum[static_cast<int64_t>(blockIdx.x) * 5 + q];
  }
  if (k >= nlong) return;
  WinRow r;
  r.row = row;
  r.mode = p.mode;
  r.nitem = p.nitem;
  r.shift = p.shift;
  r.nseg = p.nseg;
  r.pad = 0;
  r.u = ui;
  r.item0 = off[0];
  r.seg0 = off[1];
  r.tbase = off[2];
  r.pbase = off[3];
  r.dslot0 = off[4];
  rows[k] = r;
}

// First entry of A whose products reach product q0 of its row: the entry e
// of row i with P[e] - P[rp(i)] <= q0 < P[e+1] - P[rp(i)] (binary search).
DEVI int32_t entry_of(const int32_t *arp, const int64_t *P, int32_t row, int64_t q0) {
  int64_t lo = arp[row], hi = static_cast<int64_t>(arp[row + 1]) - 1;
  const int64_t target = P[lo] + q0;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (P[mid + 1] > target)
      hi = mid;
    else
      lo = mid + 1;
  }
  return static_cast<int32_t>(lo);
}

// The long row that owns work unit t of a list whose per-row starts are
// first(k) (non-decreasing): the last k with first(k) <= t, which is the row
// holding t because every later row starts beyond t.
template <typename First> DEVI int64_t owner_row(int64_t nlong, int64_t t, First first) {
  int64_t lo = 0, hi = nlong - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (first(mid) <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// One thread per work unit: items (WHAT 0; e0 set for the product ranges
// of direct dense rows), segments (WHAT 1; e0 always) or dense partial rows
// (WHAT 2; the owning long row in slot_row).
template <int WHAT>
__global__ __launch_bounds__(256) void k_wplan_units(const WinRow *rows, int64_t nlong,
                                                     int64_t nunits, const int32_t *arp,
                                                     const int64_t *P, WinWork *work,
                                                     int32_t *slot_row) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t >= nunits) return;
  const int64_t k = owner_row(nlong, t, [&](int64_t x) {
    return WHAT == 0 ? rows[x].item0 : WHAT == 1 ? rows[x].seg0 : rows[x].dslot0;
  });
  const WinRow r = rows[k];
  if (WHAT == 2) {
    slot_row[t] = static_cast<int32_t>(k);
    return;
  }
  const int32_t q = static_cast<int32_t>(t - (WHAT == 0 ? r.item0 : r.seg0));
  int32_t e0 = -1;
  if (WHAT == 1)
    e0 = entry_of(arp, P, r.row, static_cast<int64_t>(q) * kWinSeg);
  else if (r.mode == WIN_DD)
    e0 = entry_of(arp, P, r.row, static_cast<int64_t>(q) * kWinSplit);
  work[t] = WinWork{static_cast<int32_t>(k), q, e0, 0};
}

// ---------------------------------------------- wavefront product sources

// Batch of entries (direct) or segment buckets (partitioned) in LDS.
template <typename T> struct WaveBatch {
  int32_t pre[WAVE];  // exclusive prefix of the products of the batch
  int64_t src[WAVE];  // position of the first product in B or in the partials
  T av[WAVE];         // a_ij (direct)
};

// Products [q0, q1) of row `row` (positions in the row's expansion order;
// q1 - q0 <= kWinStage), from entry e_start on.  fn(x, col, val) gets the
// position relative to q0.  Lanes take consecutive products (coalesced
// loads along every b_j*), each lane's loads are issued together.
template <typename T, bool WANT_VAL, typename Fn>
DEVI void wave_direct(const EscArgs<T> &e, int32_t row, int64_t q0, int64_t q1,
                      int32_t e_start, WaveBatch<T> &wb, Fn fn) {
  const int ln = lane();
  const int32_t e_end = e.arp[row + 1];
  const int64_t P0 = e.P[e.arp[row]];
  for (int32_t eb = e_start; eb < e_end; eb += WAVE) {
    const int32_t ee = eb + ln;
    int32_t len = 0;
    int64_t src = 0, pstart = 0;
    T av = T(0);
    if (ee < e_end) {
      const int64_t ps = e.P[ee] - P0, pe = e.P[ee + 1] - P0;
      const int64_t lo = ps > q0 ? ps : q0, hi = pe < q1 ? pe : q1;
      if (hi > lo) {
        const int32_t j = e.acol[ee];
        len = static_cast<int32_t>(hi - lo);
        src = static_cast<int64_t>(e.brp[j]) + (lo - ps);
        if (WANT_VAL) av = e.aval[ee];
      }
      pstart = lo - q0;
    }
    const int32_t incl = group_incl_sum<WAVE>(len);
    wb.pre[ln] = incl - len;
    wb.src[ln] = src;
    if (WANT_VAL) wb.av[ln] = av;
    const int32_t btot = __shfl(incl, WAVE - 1, WAVE);
    const int64_t base = __shfl(static_cast<long long>(pstart), 0, WAVE);
    const int nb = (e_end - eb) < WAVE ? (e_end - eb) : WAVE;
    wave_sync();
    for (int32_t r0 = 0; r0 < btot; r0 += WVK * WAVE) {
      int64_t pos[WVK];
      T a[WVK];
#pragma unroll
      for (int q = 0; q < WVK; ++q) {
        const int32_t bx = r0 + q * WAVE + ln;
        const int32_t bxc = bx < btot ? bx : btot - 1;
        const int k = batch_find(wb.pre, nb, bxc);
        pos[q] = wb.src[k] + (bxc - wb.pre[k]);
        a[q] = WANT_VAL ? wb.av[k] : T(0);
      }
      int32_t col[WVK];
      T bv[WVK];
#pragma unroll
      for (int q = 0; q < WVK; ++q) {
        col[q] = as_global(e.bcol)[pos[q]];
        bv[q] = WANT_VAL ? as_global(e.bval)[pos[q]] : T(0);
      }
#pragma unroll
      for (int q = 0; q < WVK; ++q) {
        const int32_t bx = r0 + q * WAVE + ln;
        if (bx < btot) fn(static_cast<int32_t>(base + bx), col[q], a[q] * bv[q]);
      }
    }
    wave_sync();
    if (e.P[eb + nb] - P0 >= q1) break;
  }
}

// Products of piece r of a partitioned row (at most kWinStage): bucket r
// of every segment, in segment order, which is expansion order because the
// partition is stable.  fn(x, key, val) gets the position in the piece.
template <typename T, bool WANT_VAL, typename Fn>
DEVI void wave_partial(const WinRow &wr, int32_t r, const uint16_t *table, const uint32_t *pkey,
                       const T *pval, WaveBatch<T> &wb, Fn fn) {
  const int ln = lane();
  const uint16_t *t0 = table + wr.tbase + static_cast<int64_t>(r) * wr.nseg;
  const uint16_t *t1 = t0 + wr.nseg;
  int32_t base = 0;
  for (int32_t sb = 0; sb < wr.nseg; sb += WAVE) {
    const int32_t s = sb + ln;
    int32_t len = 0;
    int64_t src = 0;
    if (s < wr.nseg) {
      const int32_t a = t0[s];
      len = static_cast<int32_t>(t1[s]) - a;
      src = wr.pbase + static_cast<int64_t>(s) * kWinSeg + a;
    }
    const int32_t incl = group_incl_sum<WAVE>(len);
    wb.pre[ln] = incl - len;
    wb.src[ln] = src;
    const int32_t btot = __shfl(incl, WAVE - 1, WAVE);
    const int nb = (wr.nseg - sb) < WAVE ? (wr.nseg - sb) : WAVE;
    wave_sync();
    for (int32_t r0 = 0; r0 < btot; r0 += WVK * WAVE) {
      int64_t pos[WVK];
#pragma unroll
      for (int q = 0; q < WVK; ++q) {
        const int32_t bx = r0 + q * WAVE + ln;
        const int32_t bxc = bx < btot ? bx : btot - 1;
        const int k = batch_find(wb.pre, nb, bxc);
        pos[q] = wb.src[k] + (bxc - wb.pre[k]);
      }
      uint32_t key[WVK];
      T v[WVK];
#pragma unroll
      for (int q = 0; q < WVK; ++q) {
        key[q] = as_global(pkey)[pos[q]];
        v[q] = WANT_VAL ? as_global(pval)[pos[q]] : T(0);
      }
#pragma unroll
      for (int q = 0; q < WVK; ++q) {
        const int32_t bx = r0 + q * WAVE + ln;
        if (bx < btot) fn(base + bx, key[q], v[q]);
      }
    }
    base += btot;
    wave_sync();
  }
}

// Products of piece r of a partitioned row: the sum of its buckets.
DEVI int64_t piece_total(const WinRow &wr, int32_t r, const uint16_t *table) {
  const uint16_t *t0 = table + wr.tbase + static_cast<int64_t>(r) * wr.nseg;
  const uint16_t *t1 = t0 + wr.nseg;
  int64_t c = 0;
  for (int32_t s = lane(); s < wr.nseg; s += WAVE) c += static_cast<int64_t>(t1[s]) - t0[s];
  return __shfl(static_cast<long long>(group_incl_sum<WAVE>(c)), WAVE - 1, WAVE);
}

// ------------------------------------------- wavefront sort and fold

template <typename T, bool NUM> struct WaveLds {
  uint32_t coff[kWinStage];   // column offset in the window (sorted in place)
  T val[NUM ? kWinStage : 1];
  uint16_t idx[kWinStage];    // staging positions in counting-sort order
  uint32_t cnt[kWinBuckets];  // histogram, then bucket ends
  WaveBatch<T> wb;
};

// Order the staged products [0, ns) on (column offset, staging position):
// a counting sort on coff >> sh, then every product counts the entries of
// its (small) bucket that precede it and moves there.
template <typename T, bool NUM> DEVI void wave_sort(WaveLds<T, NUM> &L, int ns, int sh) {
  const int ln = lane();
  for (int b = ln; b < kWinBuckets; b += WAVE) L.cnt[b] = 0u;
  wave_sync();
#pragma unroll
  for (int q = 0; q < WVK; ++q) {
    const int x = q * WAVE + ln;
    if (x < ns) atomicAdd(&L.cnt[L.coff[x] >> sh], 1u);
  }
  wave_sync();
  uint32_t run = 0;
#pragma unroll
  for (int c0 = 0; c0 < kWinBuckets; c0 += WAVE) {
    const uint32_t v = L.cnt[c0 + ln];
    const uint32_t inc = group_incl_sum<WAVE>(v);
    L.cnt[c0 + ln] = run + inc - v;
    run += __shfl(inc, WAVE - 1, WAVE);
  }
  wave_sync();
#pragma unroll
  for (int q = 0; q < WVK; ++q) {
    const int x = q * WAVE + ln;
    if (x < ns) {
      const uint32_t slot = atomicAdd(&L.cnt[L.coff[x] >> sh], 1u);
      L.idx[slot] = static_cast<uint16_t>(x);
    }
  }
  wave_sync();
  uint32_t c[WVK];
  T v[WVK];
  int dst[WVK];
#pragma unroll
  for (int q = 0; q < WVK; ++q) {
    const int x = q * WAVE + ln;
    dst[q] = -1;
    c[q] = 0u;
    v[q] = T(0);
    if (x < ns) {
      c[q] = L.coff[x];
      if (NUM) v[q] = L.val[x];
      const uint32_t bk = c[q] >> sh;
      const int bs = bk == 0 ? 0 : static_cast<int>(L.cnt[bk - 1]);
      const int be = static_cast<int>(L.cnt[bk]);
      int r = 0;
      for (int y = bs; y < be; ++y) {
        const int z = L.idx[y];
        const uint32_t cz = L.coff[z];
        r += (cz < c[q]) || (cz == c[q] && z < x);
      }
      dst[q] = bs + r;
    }
  }
  wave_sync();
#pragma unroll
  for (int q = 0; q < WVK; ++q) {
    if (dst[q] >= 0) {
      L.coff[dst[q]] = c[q];
      if (NUM) L.val[dst[q]] = v[q];
    }
  }
  wave_sync();
}

// Distinct columns of the sorted products [0, ns), or (NUM) every column
// folded in order and written to dst in column order (lanes take
// consecutive run heads, so the stores are coalesced).  Returns the count.
template <typename T, bool NUM>
DEVI int64_t wave_fold(WaveLds<T, NUM> &L, int ns, int64_t lo, int32_t *dcol, T *dval) {
  const int ln = lane();
  int64_t run = 0;
#pragma unroll
  for (int q = 0; q < WVK; ++q) {
    const int x = q * WAVE + ln;
    const bool head = x < ns && (x == 0 || L.coff[x] != L.coff[x - 1]);
    const uint64_t m = __ballot(head);
    if (NUM && head) {
      const uint32_t c = L.coff[x];
      T v = T(0);
      int y = x;
      do {
        v = v + L.val[y];
        ++y;
      } while (y < ns && L.coff[y] == c);
      const int64_t o = run + __popcll(m & lanes_below());
      as_global_mut(dcol)[o] = static_cast<int32_t>(lo + c);
      as_global_mut(dval)[o] = v;
    }
    run += __popcll(m);
  }
  return run;
}

// ------------------------------------------------------ wavefront kernels

// Work the wavefront kernels hand to the work-group kernels (direct dense
// rows, pieces too large for one wavefront's staging), listed by the
// symbolic pass.
struct WinList {
  uint32_t *ids;
  uint32_t *count;
};

template <typename T> struct WinArgsW {
  EscArgs<T> e;
  int64_t n;
  const WinRow *rows;
  const WinWork *items;
  int64_t nitems;
  const uint16_t *table;
  const uint32_t *pkey;
  const T *pval;
  WinList list;
  int64_t *cnt;           // symbolic: output count per item
  const int64_t *iscan;   // numeric: exclusive scan of the counts
  const int64_t *rowoff;  // numeric: row offsets of C
  int32_t *c_col;
  T *c_val;
};

// One wavefront per item of a direct sparse row or a piece of a partitioned
// row.  Symbolic (NUM false): its distinct columns; numeric: its entries of
// C.  Items for the work-group kernels are listed (symbolic) or skipped.
template <typename T, bool NUM>
__global__ __launch_bounds__(WAVE) void k_witem(WinArgsW<T> a) {
  __shared__ WaveLds<T, NUM> L;
  const int64_t it = xcd_block_id<16>();
  if (it >= a.nitems) return;
  const WinWork w = a.items[it];
  const WinRow wr = a.rows[w.wrow];
  const int ln = lane();
  int ns, sh;
  int64_t lo = 0;
  if (wr.mode == WIN_DS) {
    ns = static_cast<int>(wr.u);
    sh = ceil_log2_i64(a.n) - kWinBucketLog;
    wave_direct<T, NUM>(a.e, wr.row, 0, wr.u, a.e.arp[wr.row], L.wb,
                        [&](int32_t x, int32_t col, T val) {
                          L.coff[x] = static_cast<uint32_t>(col);
                          if (NUM) L.val[x] = val;
                        });
  } else {
    const int64_t total = wr.mode == WIN_PT ? piece_total(wr, w.k, a.table) : 0;
    if (wr.mode != WIN_PT || total > kWinStage) {
      if (!NUM && ln == 0) a.list.ids[atomicAdd(a.list.count, 1u)] = static_cast<uint32_t>(it);
      return;
    }
    ns = static_cast<int>(total);
    lo = static_cast<int64_t>(w.k) << wr.shift;
    sh = wr.shift - kWinBucketLog;
    wave_partial<T, NUM>(wr, w.k, a.table, a.pkey, a.pval, L.wb,
                         [&](int32_t x, uint32_t key, T val) {
                           L.coff[x] = key;
                           if (NUM) L.val[x] = val;
                         });
  }
  if (sh < 0) sh = 0;
  wave_sync();
  wave_sort(L, ns, sh);
  if (NUM) {
    const int64_t out = a.rowoff[wr.row] + a.iscan[it] - a.iscan[wr.item0];
    wave_fold(L, ns, lo, a.c_col + out, a.c_val + out);
  } else {
    const int64_t c = wave_fold(L, ns, lo, static_cast<int32_t *>(nullptr), static_cast<T *>(nullptr));
    if (ln == 0) a.cnt[it] = c;
  }
}

// One wavefront per segment of a partitioned row: its products are staged,
// counted per piece (the piece starts go to the table, one column of it per
// segment), then scattered stably in rounds of 64 in expansion order (the
// rank among the lanes of a round with the same piece comes from ballots)
// and copied to the segment's partial region as (column offset in the
// piece, value).
template <typename T> struct PartLds {
  uint32_t col[kWinSeg];
  T val[kWinSeg];
  uint32_t okey[kWinSeg];
  T oval[kWinSeg];
  uint32_t hist[kWinMaxPieces + 1];
  WaveBatch<T> wb;
};

template <typename T>
__global__ __launch_bounds__(WAVE) void k_wpart(EscArgs<T> e, const WinRow *rows,
                                                const WinWork *segs, int64_t nsegs,
                                                uint16_t *table, uint32_t *pkey, T *pval) {
  __shared__ PartLds<T> L;
  const int64_t sid = xcd_block_id<16>();
  if (sid >= nsegs) return;
  const WinWork w = segs[sid];
  const WinRow wr = rows[w.wrow];
  const int ln = lane();
  const int R = wr.nitem;
  const int sh = wr.shift;
  for (int q = ln; q <= R; q += WAVE) L.hist[q] = 0u;
  const int64_t q0 = static_cast<int64_t>(w.k) * kWinSeg;
  const int64_t q1 = (q0 + kWinSeg) < wr.u ? (q0 + kWinSeg) : wr.u;
  const int ns = static_cast<int>(q1 - q0);
  wave_sync();
  wave_direct<T, true>(e, wr.row, q0, q1, w.e0, L.wb, [&](int32_t x, int32_t col, T val) {
    L.col[x] = static_cast<uint32_t>(col);
    L.val[x] = val;
    atomicAdd(&L.hist[static_cast<uint32_t>(col) >> sh], 1u);
  });
  wave_sync();
  // piece starts: exclusive scan of hist[0, R] (hist[R] is 0), one table
  // column per segment
  {
    uint32_t run = 0;
    uint16_t *tcol = table + wr.tbase + w.k;
    for (int c0 = 0; c0 <= R; c0 += WAVE) {
      const int c = c0 + ln;
      const uint32_t v = c <= R ? L.hist[c] : 0u;
      const uint32_t inc = group_incl_sum<WAVE>(v);
      if (c <= R) {
        L.hist[c] = run + inc - v;
        tcol[static_cast<int64_t>(c) * wr.nseg] = static_cast<uint16_t>(run + inc - v);
      }
      run += __shfl(inc, WAVE - 1, WAVE);
    }
  }
  wave_sync();
  // stable scatter: rounds of 64 consecutive products
  const int nbits = ceil_log2_i64(R);
  const uint32_t mask = (1u << sh) - 1u;
  for (int x0 = 0; x0 < ns; x0 += WAVE) {
    const int x = x0 + ln;
    const bool ok = x < ns;
    const uint32_t c = ok ? L.col[x] : 0u;
    const uint32_t p = c >> sh;
    uint64_t m = __ballot(ok);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (p >> b) & 1u;
      const uint64_t bb = __ballot(ok && bit);
      m &= bit ? bb : ~bb;
    }
    if (ok) {
      const uint32_t slot = L.hist[p] + static_cast<uint32_t>(__popcll(m & lanes_below()));
      L.okey[slot] = c & mask;
      L.oval[slot] = L.val[x];
    }
    wave_sync();
    // the highest lane of every group advances its piece's cursor
    if (ok && (m >> ln) == 1ull) L.hist[p] += static_cast<uint32_t>(__popcll(m));
    wave_sync();
  }
  const int64_t base = wr.pbase + q0;
  for (int x = ln; x < ns; x += WAVE) {
    as_global_mut(pkey)[base + x] = L.okey[x];
    as_global_mut(pval)[base + x] = L.oval[x];
  }
}

// ------------------------------------------- direct dense rows (n <= DW)
//
// One wavefront per item (a direct dense row, or one product range of one):
// a dense accumulator of all n columns in LDS, updated A entry by A entry
// in expansion order with the lanes on consecutive products of one b_j*
// row.  Those columns are distinct, so one round of plain LDS
// read-add-write updates never has two lanes on one column, and the LDS
// unit executes one wavefront's accesses in issue order: every column is
// summed in expansion order.  No LDS atomics (they run at about one lane
// per clock): the symbolic pass stores a byte of 1 per column hit; the
// numeric pass starts every column at a signalling-NaN pattern that no
// arithmetic result has (results are quiet NaNs), replaced by +0.0 + p at
// the column's first product, so the columns hit are those that lost it.
// The loads of GE entries are issued together, one group ahead.

constexpr int GE = 16;

DEVI float readlane_val(float v, int t) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t));
}
DEVI double readlane_val(double v, int t) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffll), t);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), t);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<uint32_t>(lo));
}

// Keeps the compiler from moving LDS accesses across it (no wait).
DEVI void order_lds() { asm volatile("" ::: "memory"); }

template <typename T> struct Untouched;
template <> struct Untouched<float> {
  using U = uint32_t;
  static constexpr U bits = 0x7fa5a5a5u;
};
template <> struct Untouched<double> {
  using U = uint64_t;
  static constexpr U bits = 0x7ff4a5a5a5a5a5a5ull;
};

template <typename T> DEVI bool untouched(T v) {
  typename Untouched<T>::U b;
  __builtin_memcpy(&b, &v, sizeof(T));
  return b == Untouched<T>::bits;
}
template <typename T> DEVI T untouched_value() {
  const typename Untouched<T>::U b = Untouched<T>::bits;
  T v;
  __builtin_memcpy(&v, &b, sizeof(T));
  return v;
}

template <typename T, bool NUM> struct DenseLds {
  static constexpr int DW = 1 << ValTraits<T>::dl;
  alignas(16) T acc[NUM ? DW : 1];             // numeric: the sums (untouched until hit)
  alignas(16) uint32_t hit[NUM ? 4 : DW / 4];  // symbolic: one byte per column
};

// Wavefronts per work-group of the dense kernels (numeric ones may share
// one accumulator between NWV wavefronts, each owning every NWV-th block of
// 32 columns: measured slower at 2 than at 1, as every wavefront gathers
// every product), and wavefronts per SIMD their registers are held to (the
// LDS allows about 2.5 numeric ones, 16 KB accumulator, and 9 symbolic).
template <bool NUM> constexpr int dense_nwv() { return 1; }
template <bool NUM> constexpr int dense_waves_per_simd() { return NUM ? 2 : 5; }

// One work-group per item (the hardware deals new work-groups to CUs as
// others finish, which balances items of very different sizes; a shared
// item counter would serialize them on one address).
// Symbolic (NUM false): the item's columns counted (one-range items) or
// kept as a bitmap for the reduction (product ranges).  Numeric: the row
// written to C in column order (one-range items) or the dense partial row
// of the range.
template <typename T, bool NUM>
__global__ __launch_bounds__(WAVE * dense_nwv<NUM>())
__attribute__((amdgpu_waves_per_eu(dense_waves_per_simd<NUM>())))
void k_wdense(WinArgsW<T> a, uint32_t *dbits, T *dacc) {
  constexpr int G = GE;  // entries per load group
  constexpr int NWV = dense_nwv<NUM>();
  __shared__ DenseLds<T, NUM> L;
  const int ln = lane();
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / WAVE));
  const int n = static_cast<int>(a.n);
  if (a.n > DenseLds<T, NUM>::DW) return;  // launched only for n <= DW
  const int64_t it = xcd_block_id<16>();
  if (it >= a.nitems) return;
  auto group_sync = [&]() {
    if (NWV > 1)
      __syncthreads();
    else
      wave_sync();
  };
  const int nwords = (n + 31) >> 5;
  const int nhit = (n + 3) >> 2;
  uint8_t *hit = reinterpret_cast<uint8_t *>(L.hit);
  // clear with 16-byte stores (n rounded up to 16 bytes stays inside the
  // arrays, whose sizes are multiples of 16 bytes)
  if (NUM) {
    constexpr int PER = 16 / static_cast<int>(sizeof(T));
    const typename Untouched<T>::U pat = Untouched<T>::bits;
    uint4 v;
    __builtin_memcpy(&v, &pat, sizeof(pat));
    if (sizeof(T) == 4) v.y = v.z = v.w = v.x;
    else { v.z = v.x; v.w = v.y; }
    uint4 *dst = reinterpret_cast<uint4 *>(L.acc);
    for (int q = threadIdx.x; q < (n + PER - 1) / PER; q += WAVE * NWV) dst[q] = v;
  } else {
    uint4 *dst = reinterpret_cast<uint4 *>(L.hit);
    for (int q = ln; q < (n + 15) / 16; q += WAVE) dst[q] = make_uint4(0u, 0u, 0u, 0u);
  }
  group_sync();
  const GLOBAL_AS int32_t *bcol = as_global(a.e.bcol);
  const GLOBAL_AS T *bval = as_global(a.e.bval);
  // numeric: wavefront wv owns the columns with (c / 32) % NWV == wv, so
  // the wavefronts of a work-group never touch one column
  auto update = [&](int32_t c, T p) {
    if (NUM) {
      if (((c >> 5) & (NWV - 1)) == wv) {
        const T o = L.acc[c];
        L.acc[c] = (untouched(o) ? T(0) : o) + p;
      }
    } else {
      hit[c] = 1;
    }
  };
  {
    const WinWork w = a.items[it];
    const WinRow wr = a.rows[w.wrow];
    const int64_t q0 = static_cast<int64_t>(w.k) * kWinSplit;
    const int64_t q1 = (q0 + kWinSplit) < wr.u ? (q0 + kWinSplit) : wr.u;
    const int32_t e_end = a.e.arp[wr.row + 1];
    const int64_t P0 = a.e.P[a.e.arp[wr.row]];
    for (int32_t eb = w.e0; eb < e_end; eb += WAVE) {
      // lane t: entry eb + t, its products inside [q0, q1) and where they
      // start in B
      const int32_t ee = eb + ln;
      int32_t start = 0, len = 0;
      T av = T(0);
      if (ee < e_end) {
        const int64_t ps = a.e.P[ee] - P0, pe = a.e.P[ee + 1] - P0;
        const int64_t lo = ps > q0 ? ps : q0, hi = pe < q1 ? pe : q1;
        if (hi > lo) {
          const int32_t j = a.e.acol[ee];
          start = a.e.brp[j] + static_cast<int32_t>(lo - ps);
          len = static_cast<int32_t>(hi - lo);
          if (NUM) av = a.e.aval[ee];
        }
      }
      const int nb = (e_end - eb) < WAVE ? (e_end - eb) : WAVE;
      // groups of G entries, double-buffered: the loads of the next group
      // are in flight while the current one is added
      struct Group {
        int32_t st[G], ls[G], bc[G];
        T as[G], bv[G];
      };
      auto load_group = [&](int t0, Group &g_) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int t = t0 + g < nb ? t0 + g : nb - 1;
          g_.st[g] = __builtin_amdgcn_readlane(start, t);
          g_.ls[g] = t0 + g < nb ? __builtin_amdgcn_readlane(len, t) : 0;
          g_.as[g] = NUM ? readlane_val(av, t) : T(0);
          // clamped, not branched around: the loads of a group stay in
          // flight together (B has entries whenever the item has products)
          const int32_t idx = ln < g_.ls[g] ? g_.st[g] + ln : 0;
          g_.bc[g] = bcol[idx];
          g_.bv[g] = NUM ? bval[idx] : T(0);
        }
      };
      Group cur, nxt;
      load_group(0, cur);
      for (int t0 = 0; t0 < nb; t0 += G) {
        if (t0 + G < nb) load_group(t0 + G, nxt);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (ln < cur.ls[g]) update(cur.bc[g], cur.as[g] * cur.bv[g]);
          order_lds();
          // b_j* rows longer than a wavefront: the rest of the row, in order
          for (int x0 = WAVE; x0 < cur.ls[g]; x0 += WAVE) {
            const int x = x0 + ln;
            if (x < cur.ls[g]) {
              const int32_t c = bcol[cur.st[g] + x];
              const T v = NUM ? bval[cur.st[g] + x] : T(0);
              update(c, cur.as[g] * v);
            }
            order_lds();
          }
        }
        cur = nxt;
      }
      if (a.e.P[eb + nb] - P0 >= q1) break;
    }
    group_sync();
    if (wr.nitem > 1) {
      // one range of a row cut into product ranges
      if (NUM) {
        T *dst = dacc + (wr.dslot0 + w.k) * static_cast<int64_t>(n);
        for (int c = threadIdx.x; c < n; c += WAVE * NWV) {
          const T v = L.acc[c];
          dst[c] = untouched(v) ? T(0) : v;
        }
      } else {
        // the range's columns as a bitmap, for the reduction
        uint32_t *dst = dbits + (wr.dslot0 + w.k) * static_cast<int64_t>(nwords);
        for (int q = ln; q < nwords; q += WAVE) {
          uint32_t b = 0;
          for (int x = 0; x < 32; ++x)
            if (q * 32 + x < n && hit[q * 32 + x]) b |= 1u << x;
          dst[q] = b;
        }
      }
    } else if (!NUM) {
      int64_t c = 0;
      for (int q = ln; q < nhit; q += WAVE) c += __popc(L.hit[q] & 0x01010101u);
      c = __shfl(static_cast<long long>(group_incl_sum<WAVE>(c)), WAVE - 1, WAVE);
      if (ln == 0) a.cnt[it] = c;
    } else if (wv == 0) {
      // the row in column order (lanes on consecutive columns, coalesced
      // stores); eight columns per lane read ahead
      int32_t *dcol = a.c_col + a.rowoff[wr.row];
      T *dval = a.c_val + a.rowoff[wr.row];
      int64_t base = 0;
      for (int c0 = 0; c0 < n; c0 += 8 * WAVE) {
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = c0 + k * WAVE + ln;
          v[k] = c < n ? L.acc[c] : untouched_value<T>();
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int c = c0 + k * WAVE + ln;
          const bool on = !untouched(v[k]);
          const uint64_t m = __ballot(on);
          if (on) {
            const int64_t o = base + __popcll(m & lanes_below());
            dcol[o] = c;
            dval[o] = v[k];
          }
          base += __popcll(m);
        }
      }
    }
    wave_sync();
  }
}

// ----------------------------------------- work-group kernels (listed items)
//
// Direct dense rows and pieces too large for one wavefront: a work-group
// streams the products in chunks of WG_STAGE into a dense accumulator of
// 2048 (binary64) / 4096 (binary32) columns.

// Batch of entries (direct) or buckets (partitioned) in LDS.
template <typename T> struct BatchLds {
  int32_t pre[WNT + 1];  // exclusive prefix of the products of the batch
  int64_t src[WNT];      // position of the first product in B (direct) or the partials
  T av[WNT];             // a_ij (direct)
  int32_t seg[WNT];      // segment index (partitioned)
  int64_t red[WNT / WAVE + 1];
};

// Products of piece r of a partitioned row (any number), bucket r of every
// segment in segment order, in rounds of at most WG_STAGE; `fits(first,
// len)` is called (by every thread) before each round.  fn(x, key, val)
// gets the position in the piece.
template <typename T, bool WANT_VAL, typename Fits, typename Fn>
DEVI void partial_products_g(const WinRow &wr, int32_t r, const uint16_t *table,
                             const uint32_t *pkey, const T *pval, BatchLds<T> &bl, Fits fits,
                             Fn fn) {
  const int t = threadIdx.x;
  const uint16_t *t0 = table + wr.tbase + static_cast<int64_t>(r) * wr.nseg;
  const uint16_t *t1 = t0 + wr.nseg;
  int64_t base = 0;
  for (int32_t sb = 0; sb < wr.nseg; sb += WNT) {
    const int32_t s = sb + t;
    int32_t len = 0;
    int64_t src = 0;
    if (s < wr.nseg) {
      const int32_t a = t0[s];
      len = static_cast<int32_t>(t1[s]) - a;
      src = wr.pbase + static_cast<int64_t>(s) * kWinSeg + a;
    }
    int64_t tot;
    const int64_t ex = block_excl_sum<WNT, int64_t>(static_cast<int64_t>(len), bl.red, tot);
    bl.pre[t] = static_cast<int32_t>(ex);
    bl.src[t] = src;
    __syncthreads();
    const int nb = (wr.nseg - sb) < WNT ? (wr.nseg - sb) : WNT;
    const int32_t btot = static_cast<int32_t>(tot);
    for (int32_t r0 = 0; r0 < btot; r0 += WG_STAGE) {
      const int32_t rl = (btot - r0) < WG_STAGE ? (btot - r0) : WG_STAGE;
      fits(base + r0, rl);
      const int32_t kp = (rl + WNT - 1) / WNT;
      const int32_t x0 = r0 + t * kp, x1 = (x0 + kp) < (r0 + rl) ? (x0 + kp) : (r0 + rl);
      if (x0 < x1) {
        int k = batch_find(bl.pre, nb, x0);
        int32_t kend = (k + 1 < nb) ? bl.pre[k + 1] : btot;
        int64_t pos[WKP];
#pragma unroll
        for (int q = 0; q < WKP; ++q) {
          const int32_t x = (x0 + q) < x1 ? (x0 + q) : (x1 - 1);
          while (x >= kend) {
            ++k;
            kend = (k + 1 < nb) ? bl.pre[k + 1] : btot;
          }
          pos[q] = bl.src[k] + (x - bl.pre[k]);
        }
        uint32_t key[WKP];
        T val[WKP];
#pragma unroll
        for (int q = 0; q < WKP; ++q) {
          key[q] = as_global(pkey)[pos[q]];
          val[q] = WANT_VAL ? as_global(pval)[pos[q]] : T(0);
        }
#pragma unroll
        for (int q = 0; q < WKP; ++q)
          if (x0 + q < x1) fn(base + x0 + q, key[q], val[q]);
      }
    }
    base += btot;
    __syncthreads();
  }
}

struct SymLds {
  uint32_t bits[(1 << kWinBitmapLog) / 32];
};

// Symbolic pass of the listed pieces (too many products for one
// wavefront): one bit per column of the piece (up to 2^kWinBitmapLog),
// counted.
template <typename T>
__global__ __launch_bounds__(WNT) void k_wsym_g(EscArgs<T> e, int64_t n, const WinRow *rows,
                                                const WinWork *items, const uint16_t *table,
                                                const uint32_t *pkey, WinList list,
                                                int64_t *cnt) {
  __shared__ SymLds sl;
  __shared__ BatchLds<T> bl;
  const uint32_t count = *list.count;
  const int t = threadIdx.x;
  for (uint32_t li = blockIdx.x; li < count; li += gridDim.x) {
    const int64_t it = list.ids[li];
    const WinWork w = items[it];
    const WinRow wr = rows[w.wrow];
    const int64_t lo = static_cast<int64_t>(w.k) << wr.shift;
    const int64_t width = (n - lo) < (int64_t(1) << wr.shift) ? (n - lo) : (int64_t(1) << wr.shift);
    const int nwords = static_cast<int>((width + 31) >> 5);
    for (int q = t; q < nwords; q += WNT) sl.bits[q] = 0u;
    __syncthreads();
    partial_products_g<T, false>(wr, w.k, table, pkey, static_cast<const T *>(nullptr), bl,
                                 [](int64_t, int32_t) {}, [&](int64_t, uint32_t c, T) {
                                   atomicOr(&sl.bits[c >> 5], 1u << (c & 31));
                                 });
    __syncthreads();
    int64_t c = 0;
    for (int q = t; q < nwords; q += WNT) c += __popc(sl.bits[q]);
    int64_t tot;
    (void)block_excl_sum<WNT, int64_t>(c, bl.red, tot);
    if (t == 0) cnt[it] = tot;
    __syncthreads();
  }
}

// Dense partial rows of a direct dense row: OR of their bitmaps (kept in
// the first one) and the row's count (on its first item; the others 0).
__global__ __launch_bounds__(WNT) void k_wsym_reduce(const WinRow *rows, const int32_t *slot_row,
                                                     int64_t nslots, int64_t n, uint32_t *dbits,
                                                     int64_t *cnt) {
  __shared__ int64_t red[WNT / WAVE + 1];
  const int64_t sl = blockIdx.x;
  if (sl >= nslots) return;
  const WinRow wr = rows[slot_row[sl]];
  if (sl != wr.dslot0) return;  // one work-group per row
  const int nwords = static_cast<int>((n + 31) >> 5);
  int64_t c = 0;
  for (int q = threadIdx.x; q < nwords; q += WNT) {
    uint32_t x = 0;
    for (int32_t k = 0; k < wr.nitem; ++k) x |= dbits[(wr.dslot0 + k) * static_cast<int64_t>(nwords) + q];
    dbits[wr.dslot0 * static_cast<int64_t>(nwords) + q] = x;
    c += __popc(x);
  }
  int64_t tot;
  (void)block_excl_sum<WNT, int64_t>(c, red, tot);
  if (threadIdx.x == 0) {
    cnt[wr.item0] = tot;
    for (int32_t k = 1; k < wr.nitem; ++k) cnt[wr.item0 + k] = 0;
  }
}

// Long-row sizes from their items' counts (iscan: exclusive scan of cnt).
__global__ __launch_bounds__(256) void k_wrownnz(const WinRow *rows, int64_t nlong,
                                                 const int64_t *iscan, int64_t *rownnz) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (k >= nlong) return;
  const WinRow wr = rows[k];
  rownnz[wr.row] = iscan[wr.item0 + wr.nitem] - iscan[wr.item0];
}

template <typename T> struct NumLds {
  static constexpr int DW = 1 << ValTraits<T>::dl;
  uint32_t coff[WG_STAGE];  // column offset in the window
  T val[WG_STAGE];
  uint16_t idx[WG_STAGE];   // staging positions in counting-sort order
  uint32_t cnt[DW];          // histogram, then bucket ends
  T acc[DW];                 // dense accumulator
  uint32_t touched[DW / 32];
  int64_t wsum[WNT / WAVE + 1];
};

// Exclusive scan of cnt[0, nbk) in place, conflict-free: each wavefront
// scans a contiguous quarter 64 consecutive counters at a time (DPP), then
// the quarters are offset by the totals before them.  Contains barriers.
template <typename T> DEVI void scan_counters(NumLds<T> &L, int nbk) {
  constexpr int NW = WNT / WAVE;
  const int w = threadIdx.x / WAVE, ln = lane();
  const int per = (nbk + NW - 1) / NW;
  const int c0 = w * per, c1 = (c0 + per) < nbk ? (c0 + per) : nbk;
  uint32_t run = 0;
  for (int cb = c0; cb < c1; cb += WAVE) {
    const int c = cb + ln;
    const uint32_t x = c < c1 ? L.cnt[c] : 0u;
    const uint32_t inc = group_incl_sum<WAVE>(x);
    if (c < c1) L.cnt[c] = run + inc - x;
    run += __shfl(inc, WAVE - 1, WAVE);
  }
  if (ln == 0) L.wsum[w] = run;
  __syncthreads();
  uint32_t before = 0;
  for (int q = 0; q < w; ++q) before += static_cast<uint32_t>(L.wsum[q]);
  if (before)
    for (int c = c0 + ln; c < c1; c += WAVE) L.cnt[c] += before;
  __syncthreads();
}

// Counting sort of the staged products [0, ns) on coff >> sh into nbk
// buckets (products whose bucket is nbk or more are left out): afterwards
// idx holds staging positions bucket by bucket and cnt[b] the end of
// bucket b.  Contains barriers.
template <typename T> DEVI void count_sort(NumLds<T> &L, int ns, int sh, int nbk) {
  const int t = threadIdx.x;
  for (int q = t; q < nbk; q += WNT) L.cnt[q] = 0u;
  __syncthreads();
  for (int p = t; p < ns; p += WNT) {
    const uint32_t bk = L.coff[p] >> sh;
    if (bk < static_cast<uint32_t>(nbk)) atomicAdd(&L.cnt[bk], 1u);
  }
  __syncthreads();
  scan_counters(L, nbk);
  for (int p = t; p < ns; p += WNT) {
    const uint32_t bk = L.coff[p] >> sh;
    if (bk < static_cast<uint32_t>(nbk)) {
      const uint32_t slot = atomicAdd(&L.cnt[bk], 1u);
      L.idx[slot] = static_cast<uint16_t>(p);
    }
  }
  __syncthreads();
}

// Sort of the staged products on (column offset, staging position): a
// counting sort on coff >> sh, then every product counts the entries of its
// (small) bucket that precede it and moves there.  Afterwards positions [0, nk)
// hold the kept products in order.  Returns nk.  Contains barriers.
template <typename T> DEVI int rank_sort(NumLds<T> &L, int ns, int sh, int nbk) {
  count_sort(L, ns, sh, nbk);
  constexpr int PP = WG_STAGE / WNT;
  const int t = threadIdx.x;
  uint32_t c[PP];
  T v[PP];
  int dst[PP];
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = t + q * WNT;
    dst[q] = -1;
    c[q] = 0u;
    v[q] = T(0);
    if (p < ns) {
      c[q] = L.coff[p];
      v[q] = L.val[p];
      const uint32_t bk = c[q] >> sh;
      if (bk < static_cast<uint32_t>(nbk)) {
        const int bs = bk == 0 ? 0 : static_cast<int>(L.cnt[bk - 1]);
        const int be = static_cast<int>(L.cnt[bk]);
        int r = 0;
        for (int x = bs; x < be; ++x) {
          const int y = L.idx[x];
          const uint32_t cy = L.coff[y];
          r += (cy < c[q]) || (cy == c[q] && y < p);
        }
        dst[q] = bs + r;
      }
    }
  }
  const int nk = static_cast<int>(L.cnt[nbk - 1]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    if (dst[q] >= 0) {
      L.coff[dst[q]] = c[q];
      L.val[dst[q]] = v[q];
    }
  }
  __syncthreads();
  return nk;
}

// Dense window: fold the staged chunk into the accumulator, every column's
// products in staging order (thread t folds the columns whose first
// sorted entry lies in its block of WG_STAGE / WNT positions).  Contains
// barriers.
template <typename T> DEVI void dense_fold(NumLds<T> &L, int ns, int width) {
  const int nk = rank_sort(L, ns, 0, width);
  constexpr int PP = WG_STAGE / WNT;
  const int x0 = threadIdx.x * PP;
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int x = x0 + q;
    if (x < nk && (x == 0 || L.coff[x] != L.coff[x - 1])) {
      const uint32_t c = L.coff[x];
      T v = L.acc[c];
      int y = x;
      do {
        v = v + L.val[y];
        ++y;
      } while (y < nk && L.coff[y] == c);
      L.acc[c] = v;
      atomicOr(&L.touched[c >> 5], 1u << (c & 31));
    }
  }
  __syncthreads();
}

// Columns of a dense window that were touched go to dst (column lo + c),
// in column order; the accumulator is cleared.  Each wavefront takes a
// contiguous block of columns.  Returns the number written.  Contains
// barriers.
template <typename T>
DEVI int64_t dense_extract(NumLds<T> &L, int width, int64_t lo, int32_t *dcol, T *dval) {
  constexpr int NW = WNT / WAVE;
  const int w = threadIdx.x / WAVE, ln = lane();
  const int per = ((width + NW - 1) / NW + 63) & ~63;  // columns per wavefront
  const int c0 = w * per, c1 = (c0 + per) < width ? (c0 + per) : width;
  int64_t cw = 0;
  for (int c = c0 + ln; c < c1; c += WAVE) cw += (L.touched[c >> 5] >> (c & 31)) & 1u;
  int64_t tot;
  int64_t base = block_excl_sum<WNT, int64_t>(cw, L.wsum, tot);
  // every lane holds the exclusive prefix of its own count; the wavefront's
  // start is that of its first lane
  base = __shfl(static_cast<long long>(base), 0, WAVE);
  for (int cb = c0; cb < c1; cb += WAVE) {
    const int c = cb + ln;
    const bool on = c < c1 && ((L.touched[c >> 5] >> (c & 31)) & 1u);
    const uint64_t m = __ballot(on);
    if (on) {
      const int64_t o = base + __popcll(m & ((1ull << ln) - 1ull));
      dcol[o] = static_cast<int32_t>(lo + c);
      dval[o] = L.acc[c];
    }
    base += __popcll(m);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < width; c += WNT) L.acc[c] = T(0);
  for (int q = threadIdx.x; q < (width + 31) / 32; q += WNT) L.touched[q] = 0u;
  __syncthreads();
  return tot;
}

template <typename T> struct WinNumArgs {
  EscArgs<T> e;
  int64_t n;
  const WinRow *rows;
  const WinWork *items;
  const uint16_t *table;
  const uint32_t *pkey;
  const T *pval;
  WinList list;
  const int64_t *iscan;   // exclusive scan of the item counts
  const int64_t *rowoff;  // row offsets of C
  int32_t *c_col;
  T *c_val;
};

// Numeric pass of the listed items (work-group per item).
template <typename T>
__global__ __launch_bounds__(WNT) void k_wnum_g(WinNumArgs<T> a) {
  __shared__ NumLds<T> L;
  __shared__ BatchLds<T> bl;
  constexpr int DW = NumLds<T>::DW;
  const uint32_t count = *a.list.count;
  const int t = threadIdx.x;
  for (uint32_t li = blockIdx.x; li < count; li += gridDim.x) {
    const int64_t it = a.list.ids[li];
    const WinWork w = a.items[it];
    const WinRow wr = a.rows[w.wrow];
    const int64_t out = a.rowoff[wr.row] + a.iscan[it] - a.iscan[wr.item0];
    int32_t *dcol = a.c_col + out;
    T *dval = a.c_val + out;
    for (int c = t; c < DW; c += WNT) L.acc[c] = T(0);
    for (int q = t; q < DW / 32; q += WNT) L.touched[q] = 0u;
    __syncthreads();
    // a piece too large for one wavefront: dense sub-windows of DW columns
    // over the columns its products span, each streaming the piece's
    // products and keeping those that fall into it
    const int64_t lo = static_cast<int64_t>(w.k) << wr.shift;
    __shared__ uint32_t span[2];
    if (t == 0) {
      span[0] = 0xffffffffu;
      span[1] = 0u;
    }
    __syncthreads();
    partial_products_g<T, false>(wr, w.k, a.table, a.pkey, static_cast<const T *>(nullptr), bl,
                                 [](int64_t, int32_t) {}, [&](int64_t, uint32_t c, T) {
                                   atomicMin(&span[0], c);
                                   atomicMax(&span[1], c);
                                 });
    __syncthreads();
    const int64_t sw0 = (span[0] / DW) * static_cast<int64_t>(DW);
    const int64_t sw1 = static_cast<int64_t>(span[1]) + 1;
    __syncthreads();
    int64_t written = 0;
    for (int64_t sw = sw0; sw < sw1; sw += DW) {
      const int ww = static_cast<int>((sw1 - sw) < DW ? (sw1 - sw) : DW);
      int64_t cbase = 0;
      int64_t total = 0;
      partial_products_g<T, true>(
          wr, w.k, a.table, a.pkey, a.pval, bl,
          [&](int64_t first, int32_t len) {
            if (first + len - cbase > WG_STAGE) {
              __syncthreads();
              dense_fold(L, static_cast<int>(first - cbase), ww);
              cbase = first;
            }
            total = first + len;
          },
          [&](int64_t x, uint32_t c, T val) {
            const int p = static_cast<int>(x - cbase);
            const bool in = c >= static_cast<uint32_t>(sw) && c < static_cast<uint32_t>(sw + ww);
            // products of other sub-windows are parked and left out of the fold
            L.coff[p] = in ? c - static_cast<uint32_t>(sw) : 0xffffffffu;
            L.val[p] = val;
          });
      __syncthreads();
      dense_fold(L, static_cast<int>(total - cbase), ww);
      written += dense_extract(L, ww, lo + sw, dcol + written, dval + written);
    }
  }
}

// Dense partial rows of a direct dense row added in range order, written
// to C in column order: one work-group per block of WNT columns of a row
// (launched for every slot; only the row's first slot's blocks work).
template <typename T>
__global__ __launch_bounds__(WNT) void k_wnum_reduce(const WinRow *rows, const int32_t *slot_row,
                                                     int64_t nslots, int64_t n,
                                                     const uint32_t *dbits, const T *dacc,
                                                     const int64_t *rowoff, int32_t *c_col,
                                                     T *c_val) {
  __shared__ int64_t red[WNT / WAVE + 1];
  const int64_t nblk = (n + WNT - 1) / WNT;
  const int64_t sl = blockIdx.x / nblk;
  const int64_t cb = blockIdx.x % nblk;
  if (sl >= nslots) return;
  const WinRow wr = rows[slot_row[sl]];
  if (sl != wr.dslot0) return;  // uniform across the work-group
  const int64_t nwords = (n + 31) >> 5;
  const uint32_t *bits = dbits + wr.dslot0 * nwords;
  const int t = threadIdx.x;
  // entries of the row in the blocks before this one
  int64_t x = 0;
  for (int64_t q = t; q < cb * (WNT / 32); q += WNT) x += __popc(bits[q]);
  int64_t before;
  (void)block_excl_sum<WNT, int64_t>(x, red, before);
  const int64_t c = cb * WNT + t;
  const bool on = c < n && ((bits[c >> 5] >> (c & 31)) & 1u);
  int64_t tot;
  const int64_t o = block_excl_sum<WNT, int64_t>(on ? 1 : 0, red, tot);
  if (!on) return;
  const T *src = dacc + wr.dslot0 * n + c;
  T v = src[0];
#pragma unroll 8
  for (int32_t k = 1; k < wr.nitem; ++k) v = v + src[static_cast<int64_t>(k) * n];
  const int64_t dst = rowoff[wr.row] + before + o;
  c_col[dst] = static_cast<int32_t>(c);
  c_val[dst] = v;
}

}  // namespace

// ---------------------------------------------------------------- launchers

void win_plan_launch(const int32_t *lrows, int64_t nlong, const int64_t *u, int64_t n,
                     int vbytes, int64_t *bsum, WinRow *rows, WinWork *items, int64_t nitems,
                     WinWork *segs, int64_t nsegs, int32_t *slot_row, int64_t nslots,
                     const int32_t *arp, const int64_t *P, hipStream_t s) {
  if (nlong <= 0) return;
  const int64_t nb = (nlong + 255) / 256;
  hipLaunchKernelGGL(k_wplan_count, dim3(nb), dim3(256), 0, s, lrows, nlong, u, n, vbytes, bsum);
  hipLaunchKernelGGL(k_wplan_scan, dim3(1), dim3(256), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_wplan_write, dim3(nb), dim3(256), 0, s, lrows, nlong, u, n, vbytes, bsum,
                     rows);
  if (nitems > 0)
    hipLaunchKernelGGL(k_wplan_units<0>, dim3((nitems + 255) / 256), dim3(256), 0, s, rows, nlong,
                       nitems, arp, P, items, static_cast<int32_t *>(nullptr));
  if (nsegs > 0)
    hipLaunchKernelGGL(k_wplan_units<1>, dim3((nsegs + 255) / 256), dim3(256), 0, s, rows, nlong,
                       nsegs, arp, P, segs, static_cast<int32_t *>(nullptr));
  if (nslots > 0)
    hipLaunchKernelGGL(k_wplan_units<2>, dim3((nslots + 255) / 256), dim3(256), 0, s, rows, nlong,
                       nslots, arp, P, static_cast<WinWork *>(nullptr), slot_row);
}

template <typename T>
void win_partition(const EscArgs<T> &e, const WinRow *rows, const WinWork *segs, int64_t nsegs,
                   uint16_t *table, uint32_t *pkey, T *pval, hipStream_t s) {
  if (nsegs <= 0) return;
  hipLaunchKernelGGL((k_wpart<T>), dim3(nsegs), dim3(WAVE), 0, s, e, rows, segs, nsegs, table,
                     pkey, pval);
}

// work-groups of the kernels for listed items (they read the list length
// on the device and loop over it)
constexpr int kListGrid = 512;

template <typename T>
void win_symbolic(const EscArgs<T> &e, int64_t n, const WinRow *rows, const WinWork *items,
                  int64_t nitems, const uint16_t *table, const uint32_t *pkey,
                  const int32_t *slot_row, int64_t nslots, uint32_t *list_ids,
                  uint32_t *list_count, uint32_t *dbits, int64_t *cnt, hipStream_t s) {
  if (nitems <= 0) return;
  launch_zero(list_count, sizeof(uint32_t), s);
  WinArgsW<T> a{};
  a.e = e;
  a.n = n;
  a.rows = rows;
  a.items = items;
  a.nitems = nitems;
  a.table = table;
  a.pkey = pkey;
  a.list = WinList{list_ids, list_count};
  a.cnt = cnt;
  if (n <= (int64_t(1) << ValTraits<T>::dl)) {
    // every long row is a direct dense row
    hipLaunchKernelGGL((k_wdense<T, false>), dim3(nitems), dim3(WAVE), 0, s, a, dbits,
                       static_cast<T *>(nullptr));
    if (nslots > 0)
      hipLaunchKernelGGL(k_wsym_reduce, dim3(nslots), dim3(WNT), 0, s, rows, slot_row, nslots, n,
                         dbits, cnt);
    return;
  }
  hipLaunchKernelGGL((k_witem<T, false>), dim3(nitems), dim3(WAVE), 0, s, a);
  hipLaunchKernelGGL((k_wsym_g<T>), dim3(kListGrid), dim3(WNT), 0, s, e, n, rows, items, table,
                     pkey, WinList{list_ids, list_count}, cnt);
}

void win_rownnz(const WinRow *rows, int64_t nlong, const int64_t *iscan, int64_t *rownnz,
                hipStream_t s) {
  if (nlong <= 0) return;
  hipLaunchKernelGGL(k_wrownnz, dim3((nlong + 255) / 256), dim3(256), 0, s, rows, nlong, iscan,
                     rownnz);
}

template <typename T>
void win_numeric(const EscArgs<T> &e, int64_t n, const WinRow *rows, const WinWork *items,
                 int64_t nitems, const uint16_t *table, const uint32_t *pkey, const T *pval,
                 const int32_t *slot_row, int64_t nslots, uint32_t *list_ids,
                 uint32_t *list_count, const uint32_t *dbits, T *dacc, const int64_t *iscan,
                 const int64_t *rowoff, int32_t *c_col, T *c_val, hipStream_t s) {
  if (nitems <= 0) return;
  WinArgsW<T> a{};
  a.e = e;
  a.n = n;
  a.rows = rows;
  a.items = items;
  a.nitems = nitems;
  a.table = table;
  a.pkey = pkey;
  a.pval = pval;
  a.list = WinList{list_ids, list_count};
  a.iscan = iscan;
  a.rowoff = rowoff;
  a.c_col = c_col;
  a.c_val = c_val;
  if (n <= (int64_t(1) << ValTraits<T>::dl)) {
    hipLaunchKernelGGL((k_wdense<T, true>), dim3(nitems), dim3(WAVE * dense_nwv<true>()), 0, s,
                       a, static_cast<uint32_t *>(nullptr), dacc);
    if (nslots > 0)
      hipLaunchKernelGGL((k_wnum_reduce<T>), dim3(nslots * ((n + WNT - 1) / WNT)), dim3(WNT), 0, s,
                         rows, slot_row, nslots, n, dbits, dacc, rowoff, c_col, c_val);
    return;
  }
  hipLaunchKernelGGL((k_witem<T, true>), dim3(nitems), dim3(WAVE), 0, s, a);
  WinNumArgs<T> g;
  g.e = e;
  g.n = n;
  g.rows = rows;
  g.items = items;
  g.table = table;
  g.pkey = pkey;
  g.pval = pval;
  g.list = WinList{list_ids, list_count};
  g.iscan = iscan;
  g.rowoff = rowoff;
  g.c_col = c_col;
  g.c_val = c_val;
  hipLaunchKernelGGL((k_wnum_g<T>), dim3(kListGrid), dim3(WNT), 0, s, g);
}

#define WIN_INST(T)                                                                             \
  template void win_partition<T>(const EscArgs<T> &, const WinRow *, const WinWork *, int64_t,  \
                                 uint16_t *, uint32_t *, T *, hipStream_t);                     \
  template void win_symbolic<T>(const EscArgs<T> &, int64_t, const WinRow *, const WinWork *,   \
                                int64_t, const uint16_t *, const uint32_t *, const int32_t *,   \
                                int64_t, uint32_t *, uint32_t *, uint32_t *, int64_t *,         \
                                hipStream_t);                                                   \
  template void win_numeric<T>(const EscArgs<T> &, int64_t, const WinRow *, const WinWork *,    \
                               int64_t, const uint16_t *, const uint32_t *, const T *,          \
                               const int32_t *, int64_t, uint32_t *, uint32_t *,                \
                               const uint32_t *, T *, const int64_t *, const int64_t *,         \
                               int32_t *, T *, hipStream_t);
WIN_INST(float)
WIN_INST(double)

}  // namespace spg
