// Long rows (bin group 5) by windows of columns: the default method for rows
// above the last group-4 edge.
//
// The paper gives a long row one thread group and merges its products into
// a sequence that spills to global memory (Section 3.1, merge method).  On
// gfx950 a few rows hold most of the products of irregular inputs, so a row
// is cut into items, each a window of columns that one work-group finishes:
//
//  * direct sparse rows (u <= kWinDirect): one item; the products are
//    gathered from the B rows into LDS, put in order by a counting sort on
//    the high column bits (kWinBuckets buckets), every bucket is ordered on
//    (column, position) and each column is folded in position order;
//  * direct dense rows (n <= the dense window): one window holds all
//    columns; products are staged in chunks, each chunk is counting-sorted
//    by column, and every column adds its products in position order to a
//    dense accumulator that persists across chunks.  Rows above kWinSplit
//    products are cut into product ranges whose dense partial rows are added
//    in range order by a reduction;
//  * partitioned rows: segments of kWinSeg consecutive products scatter
//    their products by column piece (2^shift columns) into a partial array
//    and record where every piece starts (a piece-start table); a piece then
//    gathers its share of every segment, in segment order, and is finished
//    like a window above (dense when 2^shift is the dense window width,
//    sparse otherwise).
//
// Within a column the products are always added in expansion order
// (ascending j, then the position inside b_j*), from +0.0, without fused
// multiply-add: every value equals Gustavson's sequential sum, except for
// direct dense rows cut into product ranges.
//
// A symbolic pass sets one bit per output column of every item (an LDS
// bitmap) and counts them, so that C can be allocated before the numeric
// pass, which writes every item straight to its place in C.
#include "common.hpp"
#include "internal.hpp"

namespace spg {

namespace {

constexpr int WNT = 256;             // threads of the window kernels
constexpr int WKP = kWinStage / WNT; // products per thread and round

template <typename T> struct ValTraits;
template <> struct ValTraits<float> { static constexpr int dl = 12; };
template <> struct ValTraits<double> { static constexpr int dl = 11; };

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

// Row records, the item list and the segment list.
__global__ __launch_bounds__(256) void k_wplan_write(const int32_t *lrows, int64_t nlong,
                                                     const int64_t *u, int64_t n, int vbytes,
                                                     const int64_t *bsum, WinRow *rows,
                                                     WinWork *items, WinWork *segs,
                                                     int32_t *slot_row) {
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
  for (int32_t q = 0; q < p.nitem; ++q) items[off[0] + q] = WinWork{static_cast<int32_t>(k), q, -1, 0};
  for (int32_t q = 0; q < p.nseg; ++q) segs[off[1] + q] = WinWork{static_cast<int32_t>(k), q, -1, 0};
  for (int64_t q = 0; q < p.dslots; ++q) slot_row[off[4] + q] = static_cast<int32_t>(k);
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

// e0 of every segment (stride kWinSeg) or direct dense item (stride kWinSplit).
__global__ __launch_bounds__(256) void k_wplan_entry(WinWork *work, int64_t nwork,
                                                     const WinRow *rows, const int32_t *arp,
                                                     const int64_t *P, int only_dd) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t >= nwork) return;
  WinWork w = work[t];
  const WinRow r = rows[w.wrow];
  if (only_dd && r.mode != WIN_DD) return;
  const int64_t q0 = static_cast<int64_t>(w.k) * (only_dd ? kWinSplit : kWinSeg);
  work[t].e0 = entry_of(arp, P, r.row, q0);
}

// ------------------------------------------------------ product sources
//
// A source streams the products of an item in expansion order, in rounds:
// each round hands every thread up to WKP consecutive products (lane
// blocked), together with the round's first position.  `fits(len)` is asked
// before every round with the round's product count, and the consumer may
// flush its staging (a block-wide operation) before saying yes.

// Batch of entries (direct) or buckets (partitioned) in LDS.
template <typename T> struct BatchLds {
  int32_t pre[WNT + 1];  // exclusive prefix of the products of the batch
  int64_t src[WNT];      // position of the first product in B (direct) or the partials
  T av[WNT];             // a_ij (direct)
  int32_t seg[WNT];      // segment index (partitioned)
  int64_t red[WNT / WAVE + 1];
};

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

// Products [q0, q1) of row `row` (positions in the row's expansion), entries
// from e_start on.  fn(x, col, val) gets the position relative to q0.
template <typename T, bool WANT_VAL, typename Fits, typename Fn>
DEVI void direct_products(const EscArgs<T> &e, int32_t row, int64_t q0, int64_t q1,
                          int32_t e_start, BatchLds<T> &bl, Fits fits, Fn fn) {
  const int32_t e_end = e.arp[row + 1];
  const int64_t P0 = e.P[e.arp[row]];
  const int t = threadIdx.x;
  for (int32_t eb = e_start; eb < e_end; eb += WNT) {
    const int32_t ee = eb + t;
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
    int64_t tot;
    const int64_t ex = block_excl_sum<WNT, int64_t>(static_cast<int64_t>(len), bl.red, tot);
    bl.pre[t] = static_cast<int32_t>(ex);
    bl.src[t] = src;
    if (WANT_VAL) bl.av[t] = av;
    // position (relative to q0) of the batch's first product
    int64_t base = 0;
    if (t == 0) bl.red[0] = pstart;
    __syncthreads();
    base = bl.red[0];
    const int nb = (e_end - eb) < WNT ? (e_end - eb) : WNT;
    const int32_t btot = static_cast<int32_t>(tot);
    for (int32_t r0 = 0; r0 < btot; r0 += kWinStage) {
      const int32_t rl = (btot - r0) < kWinStage ? (btot - r0) : kWinStage;
      fits(base + r0, rl);
      const int32_t x0 = r0 + t * WKP;
      if (x0 < r0 + rl) {
        int k = batch_find(bl.pre, nb, x0);
        int32_t kend = bl.pre[k] + ((k + 1 < nb) ? (bl.pre[k + 1] - bl.pre[k]) : (btot - bl.pre[k]));
#pragma unroll
        for (int q = 0; q < WKP; ++q) {
          const int32_t x = x0 + q;
          if (x < r0 + rl) {
            while (x >= kend) {
              ++k;
              kend = (k + 1 < nb) ? bl.pre[k + 1] : btot;
            }
            const int64_t pos = bl.src[k] + (x - bl.pre[k]);
            const int32_t col = as_global(e.bcol)[pos];
            T val = T(0);
            if (WANT_VAL) val = bl.av[k] * as_global(e.bval)[pos];
            fn(static_cast<int32_t>(base + x), col, val);
          }
        }
      }
    }
    __syncthreads();
    if (e.P[eb + nb] - P0 >= q1) break;
  }
}

// Products of piece r of a partitioned row, segment by segment: bucket r of
// every segment.  Chunks may only end at bucket boundaries (a bucket is not
// ordered inside), so each round takes the whole buckets that `room`
// allows; fn(x, key, val) gets the round-relative position, the partial key
// (column offset << kWinSegLog | position in the segment) and the
// segment index.
template <typename T, bool WANT_VAL, typename Room, typename Fn>
DEVI void partial_products(const WinRow &wr, int32_t r, const uint16_t *table,
                           const uint32_t *pkey, const T *pval, BatchLds<T> &bl, Room room,
                           Fn fn) {
  const int t = threadIdx.x;
  const int64_t stride = wr.nitem + 1;
  for (int32_t sb = 0; sb < wr.nseg; sb += WNT) {
    const int32_t s = sb + t;
    int32_t len = 0;
    int64_t src = 0;
    if (s < wr.nseg) {
      const uint16_t *row = table + wr.tbase + static_cast<int64_t>(s) * stride;
      const int32_t a = row[r], b = row[r + 1];
      len = b - a;
      src = wr.pbase + static_cast<int64_t>(s) * kWinSeg + a;
    }
    int64_t tot;
    const int64_t ex = block_excl_sum<WNT, int64_t>(static_cast<int64_t>(len), bl.red, tot);
    bl.pre[t] = static_cast<int32_t>(ex);
    bl.src[t] = src;
    bl.seg[t] = s;
    if (t == 0) bl.pre[WNT] = static_cast<int32_t>(tot);
    __syncthreads();
    const int nb = (wr.nseg - sb) < WNT ? (wr.nseg - sb) : WNT;
    const int32_t btot = static_cast<int32_t>(tot);
    int k0 = 0;  // first bucket of the round
    while (k0 < nb) {
      // whole buckets that fit the room the consumer offers
      const int32_t cap = room();
      // last bucket k1 (exclusive) with pre[k1] - pre[k0] <= cap
      int lo = k0, hi = nb;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int32_t end = mid < nb ? bl.pre[mid] : btot;
        if (end - bl.pre[k0] <= cap)
          lo = mid;
        else
          hi = mid - 1;
      }
      int k1 = lo;
      if (k1 == k0) {
        // the next bucket does not fit: the consumer must flush first
        room.flush();
        continue;
      }
      const int32_t r0 = bl.pre[k0];
      const int32_t r1 = k1 < nb ? bl.pre[k1] : btot;
      const int32_t rl = r1 - r0;
      // lane-blocked positions, at most kWinStage per round
      const int32_t kp = (rl + WNT - 1) / WNT;
      const int32_t x0 = r0 + t * kp;
      if (x0 < r1) {
        int k = batch_find(bl.pre, nb, x0);
        int32_t kend = (k + 1 < nb) ? bl.pre[k + 1] : btot;
        for (int q = 0; q < kp; ++q) {
          const int32_t x = x0 + q;
          if (x >= r1) break;
          while (x >= kend) {
            ++k;
            kend = (k + 1 < nb) ? bl.pre[k + 1] : btot;
          }
          const int64_t pos = bl.src[k] + (x - bl.pre[k]);
          const uint32_t key = as_global(pkey)[pos];
          T val = T(0);
          if (WANT_VAL) val = as_global(pval)[pos];
          fn(x - r0, key, bl.seg[k], val);
        }
      }
      room.advance(rl);
      k0 = k1;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------ symbolic kernel

struct SymLds {
  uint32_t bits[(1 << kWinBitmapLog) / 32];
};

template <typename T>
__global__ __launch_bounds__(WNT) void k_wsym(EscArgs<T> e, int64_t n, const WinRow *rows,
                                              const WinWork *items, int64_t nitems,
                                              const uint16_t *table, const uint32_t *pkey,
                                              uint32_t *dbits, int64_t *cnt) {
  __shared__ SymLds sl;
  __shared__ BatchLds<T> bl;
  const int64_t it = xcd_block_id<4>();
  if (it >= nitems) return;
  const WinWork w = items[it];
  const WinRow wr = rows[w.wrow];
  const int t = threadIdx.x;
  int64_t lo = 0, width = n;
  if (wr.mode == WIN_PT) {
    lo = static_cast<int64_t>(w.k) << wr.shift;
    width = (n - lo) < (int64_t(1) << wr.shift) ? (n - lo) : (int64_t(1) << wr.shift);
  }
  const int nwords = static_cast<int>((width + 31) >> 5);
  for (int q = t; q < nwords; q += WNT) sl.bits[q] = 0u;
  __syncthreads();
  if (wr.mode == WIN_PT) {
    struct Room {
      __device__ int32_t operator()() const { return kWinStage; }
      __device__ void flush() const {}
      __device__ void advance(int32_t) const {}
    } room;
    partial_products<T, false>(wr, w.k, table, pkey, static_cast<const T *>(nullptr), bl, room,
                               [&](int32_t, uint32_t key, int32_t, T) {
                                 const uint32_t c = key >> kWinSegLog;
                                 atomicOr(&sl.bits[c >> 5], 1u << (c & 31));
                               });
  } else {
    int64_t q0 = 0, q1 = wr.u;
    int32_t e0 = e.arp[wr.row];
    if (wr.mode == WIN_DD) {
      q0 = static_cast<int64_t>(w.k) * kWinSplit;
      q1 = (q0 + kWinSplit) < wr.u ? (q0 + kWinSplit) : wr.u;
      e0 = w.e0;
    }
    direct_products<T, false>(e, wr.row, q0, q1, e0, bl, [](int64_t, int32_t) {},
                              [&](int32_t, int32_t col, T) {
                                const uint32_t c = static_cast<uint32_t>(col);
                                atomicOr(&sl.bits[c >> 5], 1u << (c & 31));
                              });
  }
  __syncthreads();
  if (wr.mode == WIN_DD && wr.nitem > 1) {
    // dense partial row: its bitmap, ORed with the others by the reduction
    uint32_t *dst = dbits + (wr.dslot0 + w.k) * static_cast<int64_t>(nwords);
    for (int q = t; q < nwords; q += WNT) dst[q] = sl.bits[q];
    return;
  }
  int64_t c = 0;
  for (int q = t; q < nwords; q += WNT) c += __popc(sl.bits[q]);
  int64_t tot;
  (void)block_excl_sum<WNT, int64_t>(c, bl.red, tot);
  if (t == 0) cnt[it] = tot;
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

// ------------------------------------------------------ partition kernel

// One work-group per segment of a partitioned row: its products are
// staged in LDS, counted per piece, the piece starts are written to the
// table and every product goes to its piece's bucket in the segment's
// partial region as (column offset in the piece << kWinSegLog | position in
// the segment, value).
template <typename T> struct PartLds {
  uint32_t col[kWinSeg];
  T val[kWinSeg];
  uint32_t hist[kWinMaxPieces + 1];
};

template <typename T>
__global__ __launch_bounds__(WNT) void k_wpart(EscArgs<T> e, const WinRow *rows,
                                               const WinWork *segs, int64_t nsegs,
                                               uint16_t *table, uint32_t *pkey, T *pval) {
  __shared__ PartLds<T> L;
  __shared__ BatchLds<T> bl;
  const int64_t sid = xcd_block_id<8>();
  if (sid >= nsegs) return;
  const WinWork w = segs[sid];
  const WinRow wr = rows[w.wrow];
  const int t = threadIdx.x;
  const int R = wr.nitem;
  const int sh = wr.shift;
  for (int q = t; q <= R; q += WNT) L.hist[q] = 0u;
  const int64_t q0 = static_cast<int64_t>(w.k) * kWinSeg;
  const int64_t q1 = (q0 + kWinSeg) < wr.u ? (q0 + kWinSeg) : wr.u;
  const int ns = static_cast<int>(q1 - q0);
  __syncthreads();
  direct_products<T, true>(e, wr.row, q0, q1, w.e0, bl, [](int64_t, int32_t) {},
                           [&](int32_t x, int32_t col, T val) {
                             L.col[x] = static_cast<uint32_t>(col);
                             L.val[x] = val;
                             atomicAdd(&L.hist[static_cast<uint32_t>(col) >> sh], 1u);
                           });
  __syncthreads();
  // piece starts: exclusive scan of the histogram (R + 1 entries, the last 0)
  {
    const int per = (R + 1 + WNT - 1) / WNT;
    const int b0 = t * per;
    uint32_t loc = 0;
    for (int q = 0; q < per; ++q)
      if (b0 + q <= R) loc += L.hist[b0 + q];
    int64_t tot;
    uint32_t run = static_cast<uint32_t>(block_excl_sum<WNT, int64_t>(loc, bl.red, tot));
    uint16_t *trow = table + wr.tbase + static_cast<int64_t>(w.k) * (R + 1);
    for (int q = 0; q < per; ++q) {
      const int b = b0 + q;
      if (b <= R) {
        const uint32_t h = L.hist[b];
        L.hist[b] = run;
        trow[b] = static_cast<uint16_t>(run);
        run += h;
      }
    }
  }
  __syncthreads();
  const int64_t base = wr.pbase + q0;
  const uint32_t mask = (1u << sh) - 1u;
  for (int x = t; x < ns; x += WNT) {
    const uint32_t c = L.col[x];
    const uint32_t slot = atomicAdd(&L.hist[c >> sh], 1u);
    pkey[base + slot] = ((c & mask) << kWinSegLog) | static_cast<uint32_t>(x);
    pval[base + slot] = L.val[x];
  }
}

// ------------------------------------------------------ numeric kernel

template <typename T> struct NumLds {
  static constexpr int DW = 1 << ValTraits<T>::dl;
  static constexpr int NC = DW > kWinBuckets ? DW : kWinBuckets;
  uint32_t coff[kWinStage];  // column offset in the window
  uint32_t skey[kWinStage];  // order key among equal columns
  T val[kWinStage];
  uint16_t idx[kWinStage];   // staging positions in counting-sort order
  uint32_t cnt[NC];          // histogram, then bucket ends
  T acc[DW];                 // dense accumulator
  uint32_t touched[DW / 32];
  int64_t wsum[WNT / WAVE + 1];
};

// Order of two staged products of one bucket: (column, order key).
template <typename T> DEVI bool stage_less(const NumLds<T> &L, uint32_t a, uint32_t b) {
  const uint32_t ca = L.coff[a], cb = L.coff[b];
  if (ca != cb) return ca < cb;
  return L.skey[a] < L.skey[b];
}

// Sort idx[b, e) by (column, order key): insertion sort for short ranges,
// heapsort beyond (one thread).
template <typename T> DEVI void sort_bucket(NumLds<T> &L, int b, int e) {
  const int k = e - b;
  if (k <= 1) return;
  if (k <= 32) {
    for (int x = b + 1; x < e; ++x) {
      const uint16_t v = L.idx[x];
      int y = x - 1;
      while (y >= b && stage_less(L, v, L.idx[y])) {
        L.idx[y + 1] = L.idx[y];
        --y;
      }
      L.idx[y + 1] = v;
    }
    return;
  }
  uint16_t *h = L.idx + b;
  auto sift = [&](int root, int end) {
    for (;;) {
      int child = 2 * root + 1;
      if (child >= end) break;
      if (child + 1 < end && stage_less(L, h[child], h[child + 1])) ++child;
      if (!stage_less(L, h[root], h[child])) break;
      const uint16_t tmp = h[root];
      h[root] = h[child];
      h[child] = tmp;
      root = child;
    }
  };
  for (int s = k / 2 - 1; s >= 0; --s) sift(s, k);
  for (int end = k - 1; end > 0; --end) {
    const uint16_t tmp = h[0];
    h[0] = h[end];
    h[end] = tmp;
    sift(0, end);
  }
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
  {
    const int per = (nbk + WNT - 1) / WNT;
    const int b0 = t * per;
    uint32_t loc = 0;
    for (int q = 0; q < per; ++q)
      if (b0 + q < nbk) loc += L.cnt[b0 + q];
    int64_t tot;
    uint32_t run = static_cast<uint32_t>(block_excl_sum<WNT, int64_t>(loc, L.wsum, tot));
    for (int q = 0; q < per; ++q) {
      if (b0 + q < nbk) {
        const uint32_t h = L.cnt[b0 + q];
        L.cnt[b0 + q] = run;
        run += h;
      }
    }
  }
  __syncthreads();
  for (int p = t; p < ns; p += WNT) {
    const uint32_t bk = L.coff[p] >> sh;
    if (bk < static_cast<uint32_t>(nbk)) {
      const uint32_t slot = atomicAdd(&L.cnt[bk], 1u);
      L.idx[slot] = static_cast<uint16_t>(p);
    }
  }
  __syncthreads();
}

// Dense window: fold the staged chunk into the accumulator, column by
// column in order-key order.  Contains barriers.
template <typename T> DEVI void dense_fold(NumLds<T> &L, int ns, int width) {
  count_sort(L, ns, 0, width);
  for (int c = threadIdx.x; c < width; c += WNT) {
    const int b = c == 0 ? 0 : static_cast<int>(L.cnt[c - 1]);
    const int e = static_cast<int>(L.cnt[c]);
    if (e > b) {
      sort_bucket(L, b, e);
      T v = L.acc[c];
      for (int x = b; x < e; ++x) v = v + L.val[L.idx[x]];
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

// Sparse window: the staged products [0, ns) (all of the item) sorted by
// buckets of 2^sh columns, folded, written to dst in column order.
// Contains barriers.
template <typename T>
DEVI void sparse_finish(NumLds<T> &L, int ns, int sh, int64_t lo, int32_t *dcol, T *dval) {
  constexpr int NW = WNT / WAVE;
  count_sort(L, ns, sh, kWinBuckets);
  const int w = threadIdx.x / WAVE, ln = lane();
  constexpr int per = kWinBuckets / NW;
  const int b0 = w * per;
  // pass 1: order every bucket, count its distinct columns
  int64_t cw = 0;
  for (int b = b0 + ln; b < b0 + per; b += WAVE) {
    const int s = b == 0 ? 0 : static_cast<int>(L.cnt[b - 1]);
    const int e = static_cast<int>(L.cnt[b]);
    if (e > s) {
      sort_bucket(L, s, e);
      int d = 1;
      for (int x = s + 1; x < e; ++x) d += L.coff[L.idx[x]] != L.coff[L.idx[x - 1]];
      cw += d;
    }
  }
  int64_t tot;
  int64_t base = block_excl_sum<WNT, int64_t>(cw, L.wsum, tot);
  base = __shfl(static_cast<long long>(base), 0, WAVE);
  // pass 2: fold and write, 64 consecutive buckets per round
  for (int bb = b0; bb < b0 + per; bb += WAVE) {
    const int b = bb + ln;
    const int s = b == 0 ? 0 : static_cast<int>(L.cnt[b - 1]);
    const int e = static_cast<int>(L.cnt[b]);
    int d = 0;
    if (e > s) {
      d = 1;
      for (int x = s + 1; x < e; ++x) d += L.coff[L.idx[x]] != L.coff[L.idx[x - 1]];
    }
    const int64_t incl = group_incl_sum<WAVE>(static_cast<int64_t>(d));
    int64_t o = base + incl - d;
    if (e > s) {
      int x = s;
      while (x < e) {
        const uint32_t c = L.coff[L.idx[x]];
        T v = T(0);
        while (x < e && L.coff[L.idx[x]] == c) {
          v = v + L.val[L.idx[x]];
          ++x;
        }
        dcol[o] = static_cast<int32_t>(lo + c);
        dval[o] = v;
        ++o;
      }
    }
    base += __shfl(static_cast<long long>(incl), WAVE - 1, WAVE);
  }
  __syncthreads();
}

template <typename T> struct WinNumArgs {
  EscArgs<T> e;
  int64_t n;
  const WinRow *rows;
  const WinWork *items;
  int64_t nitems;
  const uint16_t *table;
  const uint32_t *pkey;
  const T *pval;
  T *dacc;                // dense partial rows (direct dense rows cut into ranges)
  const int64_t *iscan;   // exclusive scan of the item counts
  const int64_t *rowoff;  // row offsets of C
  int32_t *c_col;
  T *c_val;
};

template <typename T>
__global__ __launch_bounds__(WNT) void k_wnum(WinNumArgs<T> a) {
  __shared__ NumLds<T> L;
  __shared__ BatchLds<T> bl;
  constexpr int DW = NumLds<T>::DW;
  const int64_t it = xcd_block_id<4>();
  if (it >= a.nitems) return;
  const WinWork w = a.items[it];
  const WinRow wr = a.rows[w.wrow];
  const int t = threadIdx.x;
  const int64_t n = a.n;
  const int64_t out = a.rowoff[wr.row] + a.iscan[it] - a.iscan[wr.item0];
  int32_t *dcol = a.c_col + out;
  T *dval = a.c_val + out;
  int ns = 0;  // staged products (uniform)

  if (wr.mode == WIN_DS) {
    // one chunk holds the whole row (u <= kWinDirect)
    direct_products<T, true>(a.e, wr.row, 0, wr.u, a.e.arp[wr.row], bl, [](int64_t, int32_t) {},
                             [&](int32_t x, int32_t col, T val) {
                               L.coff[x] = static_cast<uint32_t>(col);
                               L.skey[x] = static_cast<uint32_t>(x);
                               L.val[x] = val;
                             });
    __syncthreads();
    int sh = ceil_log2_i64(n) - kWinBucketLog;
    if (sh < 0) sh = 0;
    sparse_finish(L, static_cast<int>(wr.u), sh, 0, dcol, dval);
    return;
  }

  if (wr.mode == WIN_DD) {
    const int width = static_cast<int>(n);
    for (int c = t; c < width; c += WNT) L.acc[c] = T(0);
    for (int q = t; q < (width + 31) / 32; q += WNT) L.touched[q] = 0u;
    __syncthreads();
    const int64_t q0 = static_cast<int64_t>(w.k) * kWinSplit;
    const int64_t q1 = (q0 + kWinSplit) < wr.u ? (q0 + kWinSplit) : wr.u;
    int64_t cbase = 0;  // position of the chunk's first product (relative to q0)
    direct_products<T, true>(
        a.e, wr.row, q0, q1, w.e0, bl,
        [&](int64_t first, int32_t len) {
          if (first + len - cbase > kWinStage) {
            __syncthreads();
            dense_fold(L, static_cast<int>(first - cbase), width);
            cbase = first;
          }
        },
        [&](int32_t x, int32_t col, T val) {
          const int p = static_cast<int>(x - cbase);
          L.coff[p] = static_cast<uint32_t>(col);
          L.skey[p] = static_cast<uint32_t>(p);
          L.val[p] = val;
        });
    __syncthreads();
    dense_fold(L, static_cast<int>((q1 - q0) - cbase), width);
    if (wr.nitem == 1) {
      dense_extract(L, width, 0, dcol, dval);
    } else {
      T *dst = a.dacc + (wr.dslot0 + w.k) * n;
      for (int c = t; c < width; c += WNT) dst[c] = L.acc[c];
    }
    return;
  }

  // partitioned row, piece w.k
  const int64_t lo = static_cast<int64_t>(w.k) << wr.shift;
  const int64_t pw = int64_t(1) << wr.shift;
  const int width = static_cast<int>((n - lo) < pw ? (n - lo) : pw);
  // products of the piece: sum of its buckets over the segments
  int64_t total = 0;
  {
    const int64_t stride = wr.nitem + 1;
    int64_t loc = 0;
    for (int32_t s = t; s < wr.nseg; s += WNT) {
      const uint16_t *row = a.table + wr.tbase + static_cast<int64_t>(s) * stride;
      loc += static_cast<int64_t>(row[w.k + 1]) - row[w.k];
    }
    (void)block_excl_sum<WNT, int64_t>(loc, bl.red, total);
  }
  const bool dense = width <= DW;
  if (!dense && total <= kWinStage) {
    // sparse piece: one chunk
    struct Room {
      int32_t *ns;
      __device__ int32_t operator()() const { return kWinStage - *ns; }
      __device__ void flush() const {}
      __device__ void advance(int32_t l) const { *ns += l; }
    } room{&ns};
    partial_products<T, true>(wr, w.k, a.table, a.pkey, a.pval, bl, room,
                              [&](int32_t x, uint32_t key, int32_t seg, T val) {
                                const int p = ns + x;
                                L.coff[p] = key >> kWinSegLog;
                                L.skey[p] = (static_cast<uint32_t>(seg) << kWinSegLog) |
                                            (key & ((1u << kWinSegLog) - 1u));
                                L.val[p] = val;
                              });
    __syncthreads();
    sparse_finish(L, ns, wr.shift - kWinBucketLog, lo, dcol, dval);
    return;
  }
  // dense piece (or a sparse piece too large for one chunk): dense windows
  // of DW columns, each gathering the piece's products that fall into it
  for (int c = t; c < DW; c += WNT) L.acc[c] = T(0);
  for (int q = t; q < DW / 32; q += WNT) L.touched[q] = 0u;
  __syncthreads();
  int64_t written = 0;
  for (int64_t sw = 0; sw < width; sw += DW) {
    const int ww = static_cast<int>((width - sw) < DW ? (width - sw) : DW);
    ns = 0;
    struct Room {
      int32_t *ns;
      NumLds<T> *L;
      int ww;
      __device__ int32_t operator()() const { return kWinStage - *ns; }
      __device__ void flush() const {
        __syncthreads();
        dense_fold(*L, *ns, ww);
        *ns = 0;
      }
      __device__ void advance(int32_t l) const { *ns += l; }
    } room{&ns, &L, ww};
    // every product of a round keeps its slot; those of other sub-windows
    // are parked (column offset 0xffffffff) and left out of the fold
    partial_products<T, true>(wr, w.k, a.table, a.pkey, a.pval, bl, room,
                              [&](int32_t x, uint32_t key, int32_t seg, T val) {
                                const uint32_t c = key >> kWinSegLog;
                                const int p = ns + x;
                                const bool in = c >= static_cast<uint32_t>(sw) &&
                                                c < static_cast<uint32_t>(sw + ww);
                                L.coff[p] = in ? c - static_cast<uint32_t>(sw) : 0xffffffffu;
                                L.skey[p] = (static_cast<uint32_t>(seg) << kWinSegLog) |
                                            (key & ((1u << kWinSegLog) - 1u));
                                L.val[p] = val;
                              });
    __syncthreads();
    dense_fold(L, ns, ww);
    written += dense_extract(L, ww, lo + sw, dcol + written, dval + written);
  }
}

// Dense partial rows of a direct dense row added in range order, written
// to C in column order.
template <typename T>
__global__ __launch_bounds__(WNT) void k_wnum_reduce(const WinRow *rows, const int32_t *slot_row,
                                                     int64_t nslots, int64_t n,
                                                     const uint32_t *dbits, const T *dacc,
                                                     const int64_t *rowoff, int32_t *c_col,
                                                     T *c_val) {
  __shared__ int64_t wsum[WNT / WAVE + 1];
  const int64_t sl = blockIdx.x;
  if (sl >= nslots) return;
  const WinRow wr = rows[slot_row[sl]];
  if (sl != wr.dslot0) return;
  const int nwords = static_cast<int>((n + 31) >> 5);
  const uint32_t *bits = dbits + wr.dslot0 * static_cast<int64_t>(nwords);
  constexpr int NW = WNT / WAVE;
  const int w = threadIdx.x / WAVE, ln = lane();
  const int width = static_cast<int>(n);
  const int per = ((width + NW - 1) / NW + 63) & ~63;
  const int c0 = w * per, c1 = (c0 + per) < width ? (c0 + per) : width;
  int64_t cw = 0;
  for (int c = c0 + ln; c < c1; c += WAVE) cw += (bits[c >> 5] >> (c & 31)) & 1u;
  int64_t tot;
  int64_t base = block_excl_sum<WNT, int64_t>(cw, wsum, tot);
  base = __shfl(static_cast<long long>(base), 0, WAVE) + rowoff[wr.row];
  for (int cb = c0; cb < c1; cb += WAVE) {
    const int c = cb + ln;
    const bool on = c < c1 && ((bits[c >> 5] >> (c & 31)) & 1u);
    const uint64_t m = __ballot(on);
    if (on) {
      T v = dacc[wr.dslot0 * n + c];
      for (int32_t k = 1; k < wr.nitem; ++k) v = v + dacc[(wr.dslot0 + k) * n + c];
      const int64_t o = base + __popcll(m & ((1ull << ln) - 1ull));
      c_col[o] = c;
      c_val[o] = v;
    }
    base += __popcll(m);
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

void win_plan_launch(const int32_t *lrows, int64_t nlong, const int64_t *u, int64_t n,
                     int vbytes, int64_t *bsum, WinRow *rows, WinWork *items, int64_t nitems,
                     WinWork *segs, int64_t nsegs, int32_t *slot_row, const int32_t *arp,
                     const int64_t *P, hipStream_t s) {
  if (nlong <= 0) return;
  const int64_t nb = (nlong + 255) / 256;
  hipLaunchKernelGGL(k_wplan_count, dim3(nb), dim3(256), 0, s, lrows, nlong, u, n, vbytes, bsum);
  hipLaunchKernelGGL(k_wplan_scan, dim3(1), dim3(256), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_wplan_write, dim3(nb), dim3(256), 0, s, lrows, nlong, u, n, vbytes, bsum,
                     rows, items, segs, slot_row);
  if (nsegs > 0)
    hipLaunchKernelGGL(k_wplan_entry, dim3((nsegs + 255) / 256), dim3(256), 0, s, segs, nsegs,
                       rows, arp, P, 0);
  if (nitems > 0)
    hipLaunchKernelGGL(k_wplan_entry, dim3((nitems + 255) / 256), dim3(256), 0, s, items, nitems,
                       rows, arp, P, 1);
}

template <typename T>
void win_partition(const EscArgs<T> &e, const WinRow *rows, const WinWork *segs, int64_t nsegs,
                   uint16_t *table, uint32_t *pkey, T *pval, hipStream_t s) {
  if (nsegs <= 0) return;
  hipLaunchKernelGGL((k_wpart<T>), dim3(nsegs), dim3(WNT), 0, s, e, rows, segs, nsegs, table,
                     pkey, pval);
}

template <typename T>
void win_symbolic(const EscArgs<T> &e, int64_t n, const WinRow *rows, const WinWork *items,
                  int64_t nitems, const uint16_t *table, const uint32_t *pkey,
                  const int32_t *slot_row, int64_t nslots, uint32_t *dbits, int64_t *cnt,
                  hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL((k_wsym<T>), dim3(nitems), dim3(WNT), 0, s, e, n, rows, items, nitems,
                     table, pkey, dbits, cnt);
  if (nslots > 0)
    hipLaunchKernelGGL(k_wsym_reduce, dim3(nslots), dim3(WNT), 0, s, rows, slot_row, nslots, n,
                       dbits, cnt);
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
                 const int32_t *slot_row, int64_t nslots, const uint32_t *dbits, T *dacc,
                 const int64_t *iscan, const int64_t *rowoff, int32_t *c_col, T *c_val,
                 hipStream_t s) {
  if (nitems <= 0) return;
  WinNumArgs<T> a;
  a.e = e;
  a.n = n;
  a.rows = rows;
  a.items = items;
  a.nitems = nitems;
  a.table = table;
  a.pkey = pkey;
  a.pval = pval;
  a.dacc = dacc;
  a.iscan = iscan;
  a.rowoff = rowoff;
  a.c_col = c_col;
  a.c_val = c_val;
  hipLaunchKernelGGL((k_wnum<T>), dim3(nitems), dim3(WNT), 0, s, a);
  if (nslots > 0)
    hipLaunchKernelGGL((k_wnum_reduce<T>), dim3(nslots), dim3(WNT), 0, s, rows, slot_row, nslots,
                       n, dbits, dacc, rowoff, c_col, c_val);
}

#define WIN_INST(T)                                                                            \
  template void win_partition<T>(const EscArgs<T> &, const WinRow *, const WinWork *, int64_t, \
                                 uint16_t *, uint32_t *, T *, hipStream_t);                    \
  template void win_symbolic<T>(const EscArgs<T> &, int64_t, const WinRow *, const WinWork *,  \
                                int64_t, const uint16_t *, const uint32_t *, const int32_t *,  \
                                int64_t, uint32_t *, int64_t *, hipStream_t);                  \
  template void win_numeric<T>(const EscArgs<T> &, int64_t, const WinRow *, const WinWork *,   \
                               int64_t, const uint16_t *, const uint32_t *, const T *,         \
                               const int32_t *, int64_t, const uint32_t *, T *,                \
                               const int64_t *, const int64_t *, int32_t *, T *, hipStream_t);
WIN_INST(float)
WIN_INST(double)

}  // namespace spg
