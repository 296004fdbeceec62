// Stage 3 for long rows (bin group 5, u > 512 by default): the merge method
// of Section 3.1, split over work-groups.
//
// Merge method (one work-group per work item):
//  * products are taken in expansion order in tiles of TILE; every tile is
//    sorted on (column, position) and its products are folded per column;
//  * every distinct column of the tile is binary-searched in the level-1
//    sequence L1 held in LDS: found columns are fused in place (the running
//    value continues with the tile's products in order), missing ones are
//    tagged, compacted with a prefix sum and merged into L1 with merge path;
//  * before a tile could overflow L1, L1 is merged into the item's global
//    sequence G (merge path again, fusing columns present in both), which
//    lives in blocks carved from a device pool and grows 2x at a time
//    (progressive allocation);
//  * when the pool is exhausted the item records a checkpoint (the position
//    right after its last successful spill, with L1 empty, and G) and quits;
//    the host grows the pool and relaunches the failed items, which resume
//    from their checkpoints;
//  * at the end L1 is merged into G once more, or, if G was never used,
//    written out directly.
//
// Splitting (so that rows far longer than the average are balanced): a row
// of up to 1024 products is one work item; a longer row is cut into product
// segments of 512 (more when it would need over 512 segments).
//  * phase 1: every item by one wavefront (k_long_w: a pass with 512-entry
//    tiles, then one with 1024-entry tiles over the items it listed), by a
//    work-group radix sort in LDS up to 4096 products (k_long1), else by the
//    merge method above (k_long).  An item of a split row writes its
//    products sorted on (column, position) but not folded, and where every
//    output column range starts in them; a one-item row is folded straight
//    into a place of its own.
//  * phase 2: for split rows, every column range of the row (about 256
//    entries) gathers its part of every segment in segment order, sorts it
//    on (column, stream index) and folds it, with the same cascade of
//    wavefront (k_combine_w), work-group (k_combine1) and merge-method
//    (k_combine) kernels.
//
// Products of one column are thus added in Gustavson's order (ascending j)
// from +0.0, exactly as a sequential sum, except where the merge method
// handles the work (items or ranges above 4096 entries, or splitting turned
// off): there partial sums are added in segment order, deterministically.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"
#include "radix.hpp"

namespace spg {

// Where piece pid of a split row writes its result: straight into C with
// direct output, else at its place in the range buffer.
template <typename T>
DEVI void piece_out(const LongArgs<T> &a, int64_t pid, const LongRow &lr, int64_t obase,
                    int32_t *&dcol, T *&dval) {
  if (a.direct) {
    const int64_t d = a.rowoff[lr.row] + a.pscan[pid] - a.pscan[lr.piece0];
    dcol = a.c_col + d;
    dval = a.c_val + d;
  } else {
    dcol = a.ocol + lr.pbase + obase;
    dval = a.oval + lr.pbase + obase;
  }
}


// Number of X elements among the first d outputs when merging sorted X and
// Y with no common keys.
DEVI int split_disjoint(const int32_t *xc, int nx, const int32_t *yc, int ny, int d) {
  int lo = d > ny ? d - ny : 0;
  int hi = d < nx ? d : nx;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (xc[mid] < yc[d - mid - 1])
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Split of diagonal d when merging sorted, duplicate-free X and Y that may
// share keys: X goes first on ties, and a tied pair is never separated (the
// Y element moves to the earlier side).  Returns xi, sets yi.
DEVI int64_t split_fuse(const int32_t *xc, int64_t nx, const int32_t *yc, int64_t ny, int64_t d,
                        int64_t &yi) {
  int64_t lo = d > ny ? d - ny : 0;
  int64_t hi = d < nx ? d : nx;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (xc[mid] <= yc[d - mid - 1])
      lo = mid + 1;
    else
      hi = mid;
  }
  yi = d - lo;
  if (lo > 0 && yi < ny && xc[lo - 1] == yc[yi]) yi += 1;
  return lo;
}

// Merge X and Y into Z fusing equal columns (value X + Y), by the whole
// work-group.  Rounds of NT*E input positions; every thread merges one
// diagonal range twice: once to count its outputs, once (after a block scan)
// to write them.  Returns the output size.  Contains barriers.
template <int NT, int E, typename T>
DEVI int64_t merge_fuse(const int32_t *xc, const T *xv, int64_t nx, const int32_t *yc,
                        const T *yv, int64_t ny, int32_t *zc, T *zv, int64_t *smem) {
  const int64_t total = nx + ny;
  int64_t zo = 0;
  for (int64_t d0 = 0; d0 < total; d0 += static_cast<int64_t>(NT) * E) {
    int64_t da = d0 + static_cast<int64_t>(threadIdx.x) * E;
    int64_t db = da + E;
    if (da > total) da = total;
    if (db > total) db = total;
    int64_t ya, yb;
    const int64_t xa = split_fuse(xc, nx, yc, ny, da, ya);
    const int64_t xb = split_fuse(xc, nx, yc, ny, db, yb);
    int64_t cnt = 0;
    {
      int64_t x = xa, y = ya;
      while (x < xb || y < yb) {
        if (y >= yb || (x < xb && xc[x] < yc[y])) {
          ++x;
        } else if (x >= xb || yc[y] < xc[x]) {
          ++y;
        } else {
          ++x;
          ++y;
        }
        ++cnt;
      }
    }
    int64_t tot;
    int64_t o = zo + block_excl_sum<NT>(cnt, smem, tot);
    {
      int64_t x = xa, y = ya;
      while (x < xb || y < yb) {
        if (y >= yb || (x < xb && xc[x] < yc[y])) {
          zc[o] = xc[x];
          zv[o] = xv[x];
          ++x;
        } else if (x >= xb || yc[y] < xc[x]) {
          zc[o] = yc[y];
          zv[o] = yv[y];
          ++y;
        } else {
          zc[o] = xc[x];
          zv[o] = xv[x] + yv[y];
          ++x;
          ++y;
        }
        ++o;
      }
    }
    zo += tot;
  }
  __syncthreads();
  return zo;
}

// Work-group state broadcast through LDS.
template <typename T> struct MergeShared {
  int64_t scan[16];
  int32_t imax[16];
  int32_t *zcol;
  T *zval;
  int64_t zcap;
  int32_t ok;
  int32_t next_first;
  int64_t total;
};

template <typename T>
DEVI bool pool_alloc(Pool *pool, uint64_t cap, int32_t *&col, T *&val) {
  const unsigned long long off = atomicAdd(&pool->top, static_cast<unsigned long long>(cap));
  if (off + cap > pool->cap) return false;
  atomicAdd(&pool->used, static_cast<unsigned long long>(cap));
  col = pool->col + off;
  val = reinterpret_cast<T *>(pool->val) + off;
  return true;
}

// Tile element l lives at (l mod KT) * NT + l / KT: the KT elements of a
// thread are NT apart, so the threads of a wavefront touch consecutive words
// (no LDS bank conflicts on the regular accesses).
template <int NT, int KT> DEVI int tix(int l) { return (l & (KT - 1)) * NT + (l >> Log2<KT>::v); }

// Sort a tile (keys col << LOGT | position, values pv[position] in LDS),
// fold every column into L1 (binary-search fuse; new columns are compacted
// with a prefix sum) and merge the new columns into L1 with merge path.
// `sk`/`ncol` share LDS region A, `pv`/`nval` region B.  All reads of the
// tile's staging data must be complete before the call.  Contains barriers.
template <typename T, int NT, int TILE, int L1CAP, typename Key>
DEVI void tile_insert(Key (&key)[TILE / NT], const int tn, Key *sk, T *pv, int32_t *ncol,
                      T *nval, int32_t *l1c, T *l1v, int &r, const int32_t col_base,
                      int64_t *scan_smem) {
  constexpr int KT = TILE / NT;
  constexpr int LOGT = Log2<TILE>::v;
  constexpr int EO = (L1CAP + NT - 1) / NT;
  const int t = threadIdx.x;
  block_bitonic_sort<NT, KT, Key>(key, sk);
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) sk[kk * NT + t] = key[kk];
  __syncthreads();

  bool isnew[KT];
  int32_t nc[KT];
  T nv[KT];
  int nn = 0;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    isnew[kk] = false;
    nc[kk] = 0;
    nv[kk] = T(0);
    if (l < tn) {
      const Key c = key[kk] >> LOGT;
      const bool head = (l == 0) || ((sk[tix<NT, KT>(l - 1)] >> LOGT) != c);
      if (head) {
        const int32_t col = col_base + static_cast<int32_t>(c);
        int lo = 0, hi = r;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (l1c[mid] < col)
            lo = mid + 1;
          else
            hi = mid;
        }
        const bool found = lo < r && l1c[lo] == col;
        T v = found ? l1v[lo] : T(0);
        v = v + pv[tix<NT, KT>(static_cast<int>(key[kk] & (TILE - 1)))];
        for (int l2 = l + 1; l2 < tn; ++l2) {
          const Key k2 = sk[tix<NT, KT>(l2)];
          if ((k2 >> LOGT) != c) break;
          v = v + pv[tix<NT, KT>(static_cast<int>(k2 & (TILE - 1)))];
        }
        if (found) {
          l1v[lo] = v;
        } else {
          isnew[kk] = true;
          nc[kk] = col;
          nv[kk] = v;
          ++nn;
        }
      }
    }
  }
  int64_t qtot;
  int o = static_cast<int>(block_excl_sum<NT>(static_cast<int64_t>(nn), scan_smem, qtot));
  const int q = static_cast<int>(qtot);
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    if (isnew[kk]) {
      ncol[o] = nc[kk];
      nval[o] = nv[kk];
      ++o;
    }
  }
  __syncthreads();
  if (q > 0) {
    const int tot = r + q;
    const int d = t * EO;
    int32_t oc[EO];
    T ov[EO];
    if (d < tot) {
      int x = split_disjoint(l1c, r, ncol, q, d);
      int y = d - x;
#pragma unroll
      for (int j = 0; j < EO; ++j) {
        if (d + j < tot) {
          if (y >= q || (x < r && l1c[x] < ncol[y])) {
            oc[j] = l1c[x];
            ov[j] = l1v[x];
            ++x;
          } else {
            oc[j] = ncol[y];
            ov[j] = nval[y];
            ++y;
          }
        }
      }
    }
    __syncthreads();
    if (d < tot) {
#pragma unroll
      for (int j = 0; j < EO; ++j) {
        if (d + j < tot) {
          l1c[d + j] = oc[j];
          l1v[d + j] = ov[j];
        }
      }
    }
    __syncthreads();
    r = tot;
  }
}

// Merge L1 into G (into the spare block if large enough, else a new block of
// twice G's capacity or more); false if the pool is exhausted (G unchanged).
template <typename T, int NT>
DEVI bool spill_l1(LongState &st, int r, const int32_t *l1c, const T *l1v, Pool *pool,
                   int32_t slot, MergeShared<T> &sh) {
  const int64_t need = st.gcnt + r;
  if (threadIdx.x == 0) {
    sh.ok = 1;
    if (st.scap >= need) {
      sh.zcol = st.scol;
      sh.zval = reinterpret_cast<T *>(st.sval);
      sh.zcap = st.scap;
    } else {
      int64_t cap = st.gcap * 2;
      if (cap < slot) cap = slot;
      while (cap < need) cap *= 2;
      int32_t *zc = nullptr;
      T *zv = nullptr;
      if (pool_alloc<T>(pool, static_cast<uint64_t>(cap), zc, zv)) {
        sh.zcol = zc;
        sh.zval = zv;
        sh.zcap = cap;
      } else {
        sh.ok = 0;
      }
    }
  }
  __syncthreads();
  const bool ok = sh.ok != 0;
  int32_t *zc = sh.zcol;
  T *zv = sh.zval;
  const int64_t zcap = sh.zcap;
  __syncthreads();
  if (!ok) return false;
  const int64_t z = merge_fuse<NT, 8, T>(st.gcol, reinterpret_cast<const T *>(st.gval), st.gcnt,
                                         l1c, l1v, r, zc, zv, sh.scan);
  if (st.gcap > 0) {
    st.scol = st.gcol;
    st.sval = st.gval;
    st.scap = st.gcap;
  } else {
    st.scol = nullptr;
    st.sval = nullptr;
    st.scap = 0;
  }
  st.gcol = zc;
  st.gval = zv;
  st.gcap = zcap;
  st.gcnt = z;
  return true;
}

// Copy L1 to a destination chosen by thread 0 (`dst` set in sh.zcol/zval).
template <typename T, int NT>
DEVI void copy_l1(const int32_t *l1c, const T *l1v, int r, int32_t *dc, T *dv) {
  for (int x = threadIdx.x; x < r; x += NT) {
    dc[x] = l1c[x];
    dv[x] = l1v[x];
  }
}

// Record where every combine range starts in a partial held in LDS:
// pos[b * nseg + s] = first position with column >= b << shift, b = 0..np.
template <int NT>
DEVI void split_points_lds(const int32_t *c, int r, int shift, int32_t np, int32_t *pos,
                           int32_t nseg, int32_t s) {
  const int t = threadIdx.x;
  if (t == 0) {
    pos[s] = 0;
    pos[static_cast<int64_t>(np) * nseg + s] = r;
  }
  for (int x = t; x < r; x += NT) {
    const int32_t b = c[x] >> shift;
    const int32_t bp = x > 0 ? (c[x - 1] >> shift) : 0;
    // ranges bp+1 .. b start at x (ranges before the first entry start at 0)
    for (int32_t q = (x > 0 ? bp + 1 : 1); q <= b && q < np; ++q)
      pos[static_cast<int64_t>(q) * nseg + s] = x;
  }
  // ranges after the last entry start at r
  if (t == 0) {
    const int32_t blast = r > 0 ? (c[r - 1] >> shift) : 0;
    for (int32_t q = (r > 0 ? blast + 1 : 1); q < np; ++q) pos[static_cast<int64_t>(q) * nseg + s] = r;
  }
}

// Same for a partial in device memory (after a spill): binary searches.
template <int NT>
DEVI void split_points_global(const int32_t *c, int64_t cnt, int shift, int32_t np, int32_t *pos,
                              int32_t nseg, int32_t s) {
  for (int32_t b = threadIdx.x; b <= np; b += NT) {
    int64_t lo = 0, hi = cnt;
    if (b == np) {
      lo = cnt;
    } else {
      const int32_t key = b << shift;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (c[mid] < key)
          lo = mid + 1;
        else
          hi = mid;
      }
    }
    pos[static_cast<int64_t>(b) * nseg + s] = static_cast<int32_t>(lo);
  }
}

// ------------------------------------------------------------ phase 1

template <typename T, int NT, int TILE, int L1CAP, typename Key>
DEVI void long_item(LongArgs<T> &a, const int32_t item_id) {
  constexpr int KT = TILE / NT;
  constexpr int LOGT = Log2<TILE>::v;
  constexpr Key KMAX = KeyMax<Key>::v;
  constexpr int KB = sizeof(Key) > 4 ? static_cast<int>(sizeof(Key)) : 4;

  __shared__ int32_t l1c[L1CAP];
  __shared__ T l1v[L1CAP];
  __shared__ __align__(16) unsigned char s_a[TILE * KB];  // run starts / keys / new columns
  __shared__ __align__(16) T s_b[TILE];                    // a_ij of runs / products / new values
  __shared__ MergeShared<T> sh;

  int32_t *rs = reinterpret_cast<int32_t *>(s_a);
  Key *sk = reinterpret_cast<Key *>(s_a);
  int32_t *ncol = reinterpret_cast<int32_t *>(s_a);
  T *ra = s_b;
  T *pv = s_b;
  T *nval = s_b;

  const int t = threadIdx.x;
  const LongItem item = a.items[item_id];
  const LongRow lr = a.lrows[item.lrow];
  LongState st = a.state[item_id];
  const int32_t i = item.row;
  const int32_t e0 = a.e.arp[i];
  const int32_t e1 = a.e.arp[i + 1];
  const int64_t pbase = a.e.P[e0];
  const int64_t p1 = item.p1;
  int64_t pos = st.pos;
  int64_t last_clean = pos;
  int r = 0;

  // entry containing product `pos`: the last e with P[e] <= pbase + pos
  if (t == 0) {
    int32_t lo = e0, hi = e1;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (a.e.P[mid] - pbase <= pos)
        lo = mid;
      else
        hi = mid;
    }
    sh.next_first = lo;
  }
  __syncthreads();
  int32_t e_first = sh.next_first;
  bool failed = false;

  while (pos < p1) {
    if (r + TILE > L1CAP) {
      if (!spill_l1<T, NT>(st, r, l1c, l1v, a.pool, a.long_slot, sh)) {
        failed = true;
        break;
      }
      r = 0;
      last_clean = pos;
    }
    const int tn = static_cast<int>(p1 - pos < TILE ? p1 - pos : TILE);

    // run starts of the entries overlapping [pos, pos+tn)
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) rs[kk * NT + t] = -1;
    if (t == 0) sh.next_first = e_first;
    __syncthreads();
    for (int32_t e = e_first + t; e < e1; e += NT) {
      const int64_t s0 = a.e.P[e] - pbase;
      if (s0 > pos + tn) break;
      const int64_t s1 = a.e.P[e + 1] - pbase;
      if (s0 <= pos + tn && pos + tn < s1) sh.next_first = e;
      if (s0 < pos + tn && s1 > pos && s1 > s0) {
        const int32_t j = a.e.acol[e];
        int64_t ls = s0 - pos;
        int32_t off = 0;
        if (ls < 0) {
          off = static_cast<int32_t>(-ls);
          ls = 0;
        }
        rs[tix<NT, KT>(static_cast<int>(ls))] = a.e.brp[j] + off;
        ra[tix<NT, KT>(static_cast<int>(ls))] = a.e.aval[e];
      }
    }
    __syncthreads();
    e_first = sh.next_first;

    int st_run[KT];
    int run = -1;
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = t * KT + kk;
      const int f = (l < tn && rs[tix<NT, KT>(l)] >= 0) ? l : -1;
      run = max(run, f);
      st_run[kk] = run;
    }
    const int before = block_excl_max<NT>(run, sh.imax);
    Key key[KT];
    T prod[KT];
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = t * KT + kk;
      key[kk] = KMAX;
      prod[kk] = T(0);
      const int s0 = max(before, st_run[kk]);
      if (l < tn && s0 >= 0) {
        const int32_t bidx = rs[tix<NT, KT>(s0)] + (l - s0);
        const T av = ra[tix<NT, KT>(s0)];
        const int32_t c = a.e.bcol[bidx];
        const T bv = a.e.bval[bidx];
        prod[kk] = av * bv;
        key[kk] = (static_cast<Key>(c) << LOGT) | static_cast<Key>(l);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = t * KT + kk;
      if (l < tn) pv[tix<NT, KT>(l)] = prod[kk];
    }
    tile_insert<T, NT, TILE, L1CAP, Key>(key, tn, sk, pv, ncol, nval, l1c, l1v, r, 0, sh.scan);
    pos += tn;
  }

  const bool single = lr.nseg <= 1;
  int32_t *dcol = nullptr;
  T *dval = nullptr;
  int64_t cnt = 0;
  bool in_lds = false;
  if (!failed) {
    if (st.gcnt == 0) {
      // the whole result is in L1
      if (t == 0) {
        sh.ok = 1;
        if (!single) {
          sh.zcol = a.pcol + lr.pbase + item.p0;
          sh.zval = a.pval + lr.pbase + item.p0;
        } else if (r <= a.long_slot) {
          sh.zcol = a.e.ct_col + a.e.cto[i];
          sh.zval = a.e.ct_val + a.e.cto[i];
        } else {
          int64_t cap = a.long_slot;
          while (cap < r) cap *= 2;
          int32_t *zc = nullptr;
          T *zv = nullptr;
          if (pool_alloc<T>(a.pool, static_cast<uint64_t>(cap), zc, zv)) {
            sh.zcol = zc;
            sh.zval = zv;
          } else {
            sh.ok = 0;
          }
        }
      }
      __syncthreads();
      if (sh.ok) {
        dcol = sh.zcol;
        dval = sh.zval;
        copy_l1<T, NT>(l1c, l1v, r, dcol, dval);
        cnt = r;
        in_lds = true;
      } else {
        failed = true;
      }
    } else {
      if (r > 0 && !spill_l1<T, NT>(st, r, l1c, l1v, a.pool, a.long_slot, sh)) {
        failed = true;
      } else {
        dcol = st.gcol;
        dval = reinterpret_cast<T *>(st.gval);
        cnt = st.gcnt;
        if (!single) {
          // a partial always sits at its products' place, where phase 2
          // finds it without a pointer (cnt <= the item's products)
          int32_t *pc = a.pcol + lr.pbase + item.p0;
          T *pv2 = a.pval + lr.pbase + item.p0;
          for (int64_t x = t; x < cnt; x += NT) {
            pc[x] = dcol[x];
            pv2[x] = dval[x];
          }
          dcol = pc;
          dval = pv2;
          __syncthreads();  // the range starts are read from the copy
        }
      }
    }
  }

  if (failed) {
    if (t == 0) {
      st.pos = last_clean;
      st.status = 1;
      a.state[item_id] = st;
      const unsigned int k = atomicAdd(&a.pool->fail_count, 1u);
      a.fail_list[k] = static_cast<unsigned int>(item_id);
    }
    return;
  }
  if (!single) {
    // where every combine range starts in this partial
    const int32_t s = static_cast<int32_t>(item_id - lr.item0);
    int32_t *pos_tab = a.split + lr.sbase;
    if (in_lds)
      split_points_lds<NT>(l1c, r, lr.shift, lr.npiece, pos_tab, lr.nseg, s);
    else
      split_points_global<NT>(dcol, cnt, lr.shift, lr.npiece, pos_tab, lr.nseg, s);
  }
  if (t == 0) {
    st.pos = p1;
    st.status = 0;
    a.state[item_id] = st;
    if (single) {
      Piece pc;
      pc.col = dcol;
      pc.val = dval;
      pc.cnt = cnt;
      pc.lrow = item.lrow;
      pc.pad = 0;
      a.pieces[lr.piece0] = pc;
    } else {
      Seq q;
      q.col = dcol;
      q.val = dval;
      q.cnt = cnt;
      a.partials[item_id] = q;
    }
  }
}

// ------------------------------------------------------------ phase 2

// One work-group per output piece of a multi-segment row: entries of the
// piece's column range from all partials, in segment order, through the
// merge method.  Pieces of one-segment rows are skipped (phase 1 wrote them).
template <typename T, int NT, int TILE, int L1CAP, typename Key, int MAXS>
DEVI void combine_piece(LongArgs<T> &a, const int32_t pid) {
  constexpr int KT = TILE / NT;
  constexpr int LOGT = Log2<TILE>::v;
  constexpr Key KMAX = KeyMax<Key>::v;
  constexpr int KB = sizeof(Key) > 4 ? static_cast<int>(sizeof(Key)) : 4;

  __shared__ int32_t l1c[L1CAP];
  __shared__ T l1v[L1CAP];
  __shared__ __align__(16) unsigned char s_a[TILE * KB];
  __shared__ __align__(16) T s_b[TILE];
  __shared__ int32_t sg_off[MAXS + 1];  // first entry of segment s in this piece's stream
  __shared__ int32_t sg_lo[MAXS];       // start of the range in partial s
  __shared__ const int32_t *sg_col[MAXS];
  __shared__ const T *sg_val[MAXS];
  __shared__ MergeShared<T> sh;

  Key *sk = reinterpret_cast<Key *>(s_a);
  int32_t *ncol = reinterpret_cast<int32_t *>(s_a);
  T *pv = s_b;
  T *nval = s_b;

  const int t = threadIdx.x;
  const int32_t lri = a.piece_lrow[pid];
  const LongRow lr = a.lrows[lri];
  if (lr.nseg <= 1) return;  // uniform across the block
  LongState st = a.cstate[pid];
  const int32_t b = static_cast<int32_t>(pid - lr.piece0);
  const int32_t c0 = b << lr.shift;
  const int32_t nseg = lr.nseg;
  const int32_t *pos_tab = a.split + lr.sbase;

  // segment table and the stream length
  int64_t carry = 0;
  int64_t obase = 0;  // sum of the range starts: where this piece's result goes
  for (int32_t s0 = 0; s0 < nseg; s0 += NT) {
    const int32_t s = s0 + t;
    int64_t len = 0, start = 0;
    if (s < nseg) {
      const Seq q = a.partials[lr.item0 + s];
      int64_t lo = 0, hi = 0;
      if (q.cnt > 0 && q.col != nullptr) {
        // range starts were recorded by the item that produced the partial;
        // clamped so that a partial that is not there reads nothing
        lo = pos_tab[static_cast<int64_t>(b) * nseg + s];
        hi = pos_tab[static_cast<int64_t>(b + 1) * nseg + s];
        lo = lo < 0 ? 0 : (lo > q.cnt ? q.cnt : lo);
        hi = hi < lo ? lo : (hi > q.cnt ? q.cnt : hi);
      }
      sg_lo[s] = static_cast<int32_t>(lo);
      sg_col[s] = q.col;
      sg_val[s] = reinterpret_cast<const T *>(q.val);
      len = hi - lo;
      start = lo;
    }
    int64_t tot;
    const int64_t ex = block_excl_sum<NT>(len, sh.scan, tot);
    if (s < nseg) sg_off[s] = static_cast<int32_t>(carry + ex);
    carry += tot;
    block_excl_sum<NT>(start, sh.scan, tot);
    obase += tot;
  }
  if (t == 0) sg_off[nseg] = static_cast<int32_t>(carry);
  __syncthreads();
  const int64_t E = carry;
  int64_t pos = st.pos;
  int64_t last_clean = pos;
  int r = 0;
  bool failed = false;

  while (pos < E) {
    if (r + TILE > L1CAP) {
      if (!spill_l1<T, NT>(st, r, l1c, l1v, a.pool, a.long_slot, sh)) {
        failed = true;
        break;
      }
      r = 0;
      last_clean = pos;
    }
    const int tn = static_cast<int>(E - pos < TILE ? E - pos : TILE);
    Key key[KT];
    T val[KT];
    {
      // segment of this thread's first entry, then walk forward
      const int64_t g0 = pos + t * KT;
      int lo = 0, hi = nseg;  // last s with sg_off[s] <= g0
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sg_off[mid] <= g0)
          lo = mid;
        else
          hi = mid;
      }
      int s = lo;
#pragma unroll
      for (int kk = 0; kk < KT; ++kk) {
        const int l = t * KT + kk;
        key[kk] = KMAX;
        val[kk] = T(0);
        if (l < tn) {
          const int64_t g = pos + l;
          while (s + 1 < nseg && sg_off[s + 1] <= g) ++s;
          const int64_t idx = sg_lo[s] + (g - sg_off[s]);
          const int32_t c = sg_col[s][idx];
          val[kk] = sg_val[s][idx];
          key[kk] = (static_cast<Key>(c - c0) << LOGT) | static_cast<Key>(l);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = t * KT + kk;
      if (l < tn) pv[tix<NT, KT>(l)] = val[kk];
    }
    tile_insert<T, NT, TILE, L1CAP, Key>(key, tn, sk, pv, ncol, nval, l1c, l1v, r, c0, sh.scan);
    pos += tn;
  }

  int32_t *dcol = nullptr;
  T *dval = nullptr;
  int64_t cnt = 0;
  if (!failed) {
    if (st.gcnt == 0) {
      // never spilled: L1 goes to the piece's own place (E entries)
      piece_out(a, pid, lr, obase, dcol, dval);
      if (r > 0) copy_l1<T, NT>(l1c, l1v, r, dcol, dval);
      cnt = r;
    } else {
      if (r > 0 && !spill_l1<T, NT>(st, r, l1c, l1v, a.pool, a.long_slot, sh)) {
        failed = true;
      } else {
        dcol = st.gcol;
        dval = reinterpret_cast<T *>(st.gval);
        cnt = st.gcnt;
      }
    }
  }
  if (failed) {
    if (t == 0) {
      st.pos = last_clean;
      st.status = 1;
      a.cstate[pid] = st;
      const unsigned int k = atomicAdd(&a.pool->fail2, 1u);
      a.fail_list2[k] = static_cast<unsigned int>(pid);
    }
    return;
  }
  if (t == 0) {
    st.pos = E;
    st.status = 0;
    a.cstate[pid] = st;
    Piece pc;
    pc.col = dcol;
    pc.val = dval;
    pc.cnt = cnt;
    pc.lrow = lri;
    pc.pad = 0;
    a.pieces[pid] = pc;
  }
}

// General kernels: an explicit work list (relaunch after pool exhaustion),
// or the work the one-tile kernels left behind, in a grid-stride loop.
template <typename T, int NT, int TILE, int L1CAP, typename Key>
__global__ __launch_bounds__(NT) void k_long(LongArgs<T> a) {
  if (a.work) {
    long_item<T, NT, TILE, L1CAP, Key>(a, a.work[blockIdx.x]);
    return;
  }
  const unsigned int n = a.cnt->glong;
  for (unsigned int w = blockIdx.x; w < n; w += gridDim.x) {
    __syncthreads();
    long_item<T, NT, TILE, L1CAP, Key>(a, static_cast<int32_t>(a.glist[w]));
  }
}

template <typename T, int NT, int TILE, int L1CAP, typename Key, int MAXS>
__global__ __launch_bounds__(NT) void k_combine(LongArgs<T> a) {
  if (a.work) {
    combine_piece<T, NT, TILE, L1CAP, Key, MAXS>(a, a.work[blockIdx.x]);
    return;
  }
  const unsigned int n = a.cnt->gcomb;
  for (unsigned int w = blockIdx.x; w < n; w += gridDim.x) {
    __syncthreads();
    combine_piece<T, NT, TILE, L1CAP, Key, MAXS>(a, static_cast<int32_t>(a.glist2[w]));
  }
}

// ------------------------------------------------------- one-tile paths
// An item (or a combine piece) with at most TILE entries needs no level-1
// sequence: all its products are sorted at once, folded, and written
// straight to their destination.  Anything larger, and any item whose
// destination block cannot be allocated, is left to the general kernel.

// Output of a one-tile pass: head flags and the running output index.
// Writes the range starts of a multi-segment row's partial from the heads.
template <typename Key, int NT, int KT, int LOGT>
DEVI void oneshot_split_points(const Key (&key)[KT], const bool (&hd)[KT], const int32_t (&ho)[KT],
                               const Key *sk, int tn, int r, int32_t col_base, int shift,
                               int32_t np, int32_t *pos, int32_t nseg, int32_t s) {
  const int t = threadIdx.x;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    if (l < tn && hd[kk]) {
      const int32_t c = col_base + static_cast<int32_t>(key[kk] >> LOGT);
      const int32_t b = c >> shift;
      const int32_t bp =
          l > 0 ? ((col_base + static_cast<int32_t>(sk[tix<NT, KT>(l - 1)] >> LOGT)) >> shift) : -1;
      for (int32_t q = bp + 1; q <= b && q < np; ++q)
        pos[static_cast<int64_t>(q) * nseg + s] = ho[kk];
    }
    if (l == tn - 1) {
      const int32_t c = col_base + static_cast<int32_t>(key[kk] >> LOGT);
      for (int32_t q = (c >> shift) + 1; q < np; ++q) pos[static_cast<int64_t>(q) * nseg + s] = r;
      pos[static_cast<int64_t>(np) * nseg + s] = r;
    }
  }
}

template <typename T, int NT, int KT, typename Key>
DEVI void long1_body(LongArgs<T> &a, const int32_t item_id, const LongItem &item,
                     unsigned char *s_a, T *s_b, MergeShared<T> &sh) {
  constexpr int TILE = NT * KT;
  constexpr int LOGT = Log2<TILE>::v;
  constexpr Key KMAX = KeyMax<Key>::v;
  int32_t *rs = reinterpret_cast<int32_t *>(s_a);
  Key *sk = reinterpret_cast<Key *>(s_a);
  T *ra = s_b;
  T *pv = s_b;
  const int t = threadIdx.x;
  const int64_t p0 = item.p0, p1 = item.p1;
  const LongRow lr = a.lrows[item.lrow];
  const int32_t i = item.row;
  const int32_t e1 = a.e.arp[i + 1];
  const int64_t pbase = a.e.P[a.e.arp[i]];
  const int tn = static_cast<int>(p1 - p0);

#pragma unroll
  for (int kk = 0; kk < KT; ++kk) rs[kk * NT + t] = -1;
  __syncthreads();
  for (int32_t e = item.e_first + t; e < e1; e += NT) {
    const int64_t s0 = a.e.P[e] - pbase;
    if (s0 >= p1) break;
    const int64_t s1 = a.e.P[e + 1] - pbase;
    if (s1 > p0 && s1 > s0) {
      int64_t ls = s0 - p0;
      int32_t off = 0;
      if (ls < 0) {
        off = static_cast<int32_t>(-ls);
        ls = 0;
      }
      rs[tix<NT, KT>(static_cast<int>(ls))] = a.e.brp[a.e.acol[e]] + off;
      ra[tix<NT, KT>(static_cast<int>(ls))] = a.e.aval[e];
    }
  }
  __syncthreads();
  int st_run[KT];
  int run = -1;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    const int f = (l < tn && rs[tix<NT, KT>(l)] >= 0) ? l : -1;
    run = max(run, f);
    st_run[kk] = run;
  }
  const int before = block_excl_max<NT>(run, sh.imax);
  Key key[KT];
  T prod[KT];
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    key[kk] = KMAX;
    prod[kk] = T(0);
    const int s0 = max(before, st_run[kk]);
    if (l < tn && s0 >= 0) {
      const int32_t bidx = rs[tix<NT, KT>(s0)] + (l - s0);
      const T av = ra[tix<NT, KT>(s0)];
      const int32_t c = a.e.bcol[bidx];
      prod[kk] = av * a.e.bval[bidx];
      key[kk] = (static_cast<Key>(c) << LOGT) | static_cast<Key>(l);
    }
  }
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    if (l < tn) pv[tix<NT, KT>(l)] = prod[kk];
  }
  block_bitonic_sort<NT, KT, Key>(key, sk);
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) sk[kk * NT + t] = key[kk];
  __syncthreads();

  bool hd[KT];
  int nh = 0;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    hd[kk] = l < tn && (l == 0 || (sk[tix<NT, KT>(l - 1)] >> LOGT) != (key[kk] >> LOGT));
    nh += hd[kk] ? 1 : 0;
  }
  int64_t rtot;
  int o = static_cast<int>(block_excl_sum<NT>(static_cast<int64_t>(nh), sh.scan, rtot));
  const int r = static_cast<int>(rtot);
  const bool single = lr.nseg <= 1;
  // partial of a split row at its products' place; a whole row at its own
  // place of min(u, n) entries
  int32_t *dcol = a.pcol + lr.pbase + (single ? 0 : p0);
  T *dval = a.pval + lr.pbase + (single ? 0 : p0);
  int32_t ho[KT];
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    ho[kk] = o;
    if (hd[kk]) {
      const Key c = key[kk] >> LOGT;
      T v = T(0);
      v = v + pv[tix<NT, KT>(static_cast<int>(key[kk] & (TILE - 1)))];
      for (int l2 = l + 1; l2 < tn; ++l2) {
        const Key k2 = sk[tix<NT, KT>(l2)];
        if ((k2 >> LOGT) != c) break;
        v = v + pv[tix<NT, KT>(static_cast<int>(k2 & (TILE - 1)))];
      }
      dcol[o] = static_cast<int32_t>(c);
      dval[o] = v;
      ++o;
    }
  }
  if (!single)
    oneshot_split_points<Key, NT, KT, LOGT>(key, hd, ho, sk, tn, r, 0, lr.shift, lr.npiece,
                                        a.split + lr.sbase, lr.nseg,
                                        static_cast<int32_t>(item_id - lr.item0));
  if (t == 0) {
    LongState st = a.state[item_id];
    st.pos = p1;
    st.status = 0;
    a.state[item_id] = st;
    if (single) {
      Piece pc;
      pc.col = dcol;
      pc.val = dval;
      pc.cnt = r;
      pc.lrow = item.lrow;
      pc.pad = 0;
      a.pieces[lr.piece0] = pc;
    } else {
      Seq q;
      q.col = dcol;
      q.val = dval;
      q.cnt = r;
      a.partials[item_id] = q;
    }
  }
}


// Radix variant of the one-tile pass (column offsets fit the packed 32-bit
// key).  A row with one segment is sorted on the column and folded in
// sequence order straight into its destination.  A segment of a split row
// is only partitioned by output range (stable, so every range keeps the
// sequence order of its products): phase 2 then sorts each range once and
// folds it in sequence order, which gives Gustavson's sums exactly.
constexpr int kRadixBits = 8;

template <typename T, int NT, int KT>
DEVI void long1_radix(LongArgs<T> &a, const int32_t item_id, const LongItem &item, uint32_t *ka,
                      uint32_t *kb, T *pv, uint32_t *cnt, MergeShared<T> &sh) {
  constexpr int TILE = NT * KT;
  constexpr int LOGT = Log2<TILE>::v;
  constexpr int NW = NT / WAVE;
  int32_t *rs = reinterpret_cast<int32_t *>(ka);
  T *ra = pv;
  const int t = threadIdx.x;
  const int w = t / WAVE;
  const int ln = lane();
  const int64_t p0 = item.p0, p1 = item.p1;
  const LongRow lr = a.lrows[item.lrow];
  const int32_t i = item.row;
  const int32_t e1 = a.e.arp[i + 1];
  const int64_t pbase = a.e.P[a.e.arp[i]];
  const int tn = static_cast<int>(p1 - p0);

  // expansion: run starts, then a max-scan gives every product its run
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) rs[kk * NT + t] = -1;
  __syncthreads();
  for (int32_t e = item.e_first + t; e < e1; e += NT) {
    const int64_t s0 = a.e.P[e] - pbase;
    if (s0 >= p1) break;
    const int64_t s1 = a.e.P[e + 1] - pbase;
    if (s1 > p0 && s1 > s0) {
      int64_t ls = s0 - p0;
      int32_t off = 0;
      if (ls < 0) {
        off = static_cast<int32_t>(-ls);
        ls = 0;
      }
      rs[tix<NT, KT>(static_cast<int>(ls))] = a.e.brp[a.e.acol[e]] + off;
      ra[tix<NT, KT>(static_cast<int>(ls))] = a.e.aval[e];
    }
  }
  __syncthreads();
  int st_run[KT];
  int run = -1;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    const int f = (l < tn && rs[tix<NT, KT>(l)] >= 0) ? l : -1;
    run = max(run, f);
    st_run[kk] = run;
  }
  const int before = block_excl_max<NT>(run, sh.imax);
  int32_t col[KT];
  T prod[KT];
  int cmin = 0x7fffffff, cmax = -1;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    col[kk] = 0;
    prod[kk] = T(0);
    const int s0 = max(before, st_run[kk]);
    if (l < tn && s0 >= 0) {
      const int32_t bidx = rs[tix<NT, KT>(s0)] + (l - s0);
      const T av = ra[tix<NT, KT>(s0)];
      col[kk] = a.e.bcol[bidx];
      prod[kk] = av * a.e.bval[bidx];
      cmin = min(cmin, col[kk]);
      cmax = max(cmax, col[kk]);
    }
  }
  block_minmax<NT>(cmin, cmax, sh.imax);  // also orders the staging reads before the writes
  if (tn <= 0) {
    cmin = 0;
    cmax = 0;
  }
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    if (l < tn) {
      ka[l] = (static_cast<uint32_t>(col[kk] - cmin) << LOGT) | static_cast<uint32_t>(l);
      pv[l] = prod[kk];
    }
  }
  __syncthreads();

  const bool single = lr.nseg <= 1;
  if (!single) {
    // partition by output range; the partial keeps every product
    const int shift = lr.shift;
    const int32_t qlo = cmin >> shift;
    const int bits = bit_width(static_cast<uint32_t>((cmax >> shift) - qlo));
    const uint32_t *R = radix_sort<NT, KT, kRadixBits>(
        ka, kb, tn, bits,
        [&](uint32_t k) {
          return static_cast<uint32_t>(((static_cast<int32_t>(k >> LOGT) + cmin) >> shift) - qlo);
        },
        cnt, sh.scan);
    int32_t *dcol = a.pcol + lr.pbase + p0;
    T *dval = a.pval + lr.pbase + p0;
    const int32_t np = lr.npiece;
    const int32_t nseg = lr.nseg;
    const int32_t s = static_cast<int32_t>(item_id - lr.item0);
    int32_t *pos = a.split + lr.sbase;
    for (int e = t; e < tn; e += NT) {
      const uint32_t k = R[e];
      const int32_t c = static_cast<int32_t>(k >> LOGT) + cmin;
      dcol[e] = c;
      dval[e] = pv[k & (TILE - 1)];
      const int32_t q = c >> shift;
      const int32_t qp = e > 0 ? ((static_cast<int32_t>(R[e - 1] >> LOGT) + cmin) >> shift) : -1;
      for (int32_t qq = qp + 1; qq <= q && qq < np; ++qq)
        pos[static_cast<int64_t>(qq) * nseg + s] = e;
      if (e == tn - 1)
        for (int32_t qq = q + 1; qq <= np; ++qq) pos[static_cast<int64_t>(qq) * nseg + s] = tn;
    }
    if (tn <= 0)
      for (int32_t qq = t; qq <= np; qq += NT) pos[static_cast<int64_t>(qq) * nseg + s] = 0;
    if (t == 0) {
      LongState st = a.state[item_id];
      st.pos = p1;
      st.status = 0;
      a.state[item_id] = st;
      Seq q;
      q.col = dcol;
      q.val = dval;
      q.cnt = tn;
      a.partials[item_id] = q;
    }
    return;
  }

  // whole row: sort on the column, fold every column in sequence order
  const uint32_t *R = radix_sort<NT, KT, kRadixBits>(
      ka, kb, tn, bit_width(static_cast<uint32_t>(cmax - cmin)),
      [](uint32_t k) { return k >> LOGT; }, cnt, sh.scan);
  const uint64_t below_mask = ln == 0 ? 0ull : (~0ull >> (WAVE - ln));
  bool hd[KT];
  int pre[KT];
  int wcount = 0;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int e = (w * KT + kk) * WAVE + ln;
    hd[kk] = e < tn && (e == 0 || (R[e - 1] >> LOGT) != (R[e] >> LOGT));
    const uint64_t m = __ballot(hd[kk]);
    pre[kk] = wcount + __popcll(m & below_mask);
    wcount += __popcll(m);
  }
  if (ln == 0) sh.imax[w] = wcount;
  __syncthreads();
  int woff = 0, r = 0;
#pragma unroll
  for (int x = 0; x < NW; ++x) {
    woff += x < w ? sh.imax[x] : 0;
    r += sh.imax[x];
  }
  // the row's own place (min(u, n) entries), so no allocation is needed
  int32_t *dcol = a.pcol + lr.pbase;
  T *dval = a.pval + lr.pbase;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    if (hd[kk]) {
      const int e = (w * KT + kk) * WAVE + ln;
      const uint32_t k = R[e];
      const uint32_t c = k >> LOGT;
      T v = T(0);
      v = v + pv[k & (TILE - 1)];
      for (int e2 = e + 1; e2 < tn; ++e2) {
        const uint32_t k2 = R[e2];
        if ((k2 >> LOGT) != c) break;
        v = v + pv[k2 & (TILE - 1)];
      }
      const int o = woff + pre[kk];
      dcol[o] = static_cast<int32_t>(c) + cmin;
      dval[o] = v;
    }
  }
  if (t == 0) {
    LongState st = a.state[item_id];
    st.pos = p1;
    st.status = 0;
    a.state[item_id] = st;
    Piece pc;
    pc.col = dcol;
    pc.val = dval;
    pc.cnt = r;
    pc.lrow = item.lrow;
    pc.pad = 0;
    a.pieces[lr.piece0] = pc;
  }
}

// radix: two key buffers and the digit counters; bitonic: one key buffer
template <int NT, int TILE, typename Key> struct Long1Lds {
  static constexpr size_t bytes_a =
      sizeof(Key) == 4 ? static_cast<size_t>(TILE) * 8 + RadixCounters<NT, kRadixBits>::count * 4
                       : static_cast<size_t>(TILE) * sizeof(Key);
};

template <typename T, int NT, int TILE, typename Key>
DEVI void long1_item(LongArgs<T> &a, const int32_t item_id, unsigned char *s_a, T *s_b,
                     MergeShared<T> &sh) {
  constexpr int KT = TILE / NT;
  constexpr bool kRadix = sizeof(Key) == 4;
  const LongItem item = a.items[item_id];
  const int64_t size = item.p1 - item.p0;
  if (size > TILE) {
    if (threadIdx.x == 0)
      a.glist[atomicAdd(&a.cnt->glong, 1u)] = static_cast<unsigned int>(item_id);
    return;
  }
  if constexpr (kRadix) {
    uint32_t *ka = reinterpret_cast<uint32_t *>(s_a);
    long1_radix<T, NT, KT>(a, item_id, item, ka, ka + TILE, s_b, ka + 2 * TILE, sh);
    return;
  }
  // the sorting network only as large as the item needs
  if (size <= TILE / 4)
    long1_body<T, NT, KT / 4, Key>(a, item_id, item, s_a, s_b, sh);
  else if (size <= TILE / 2)
    long1_body<T, NT, KT / 2, Key>(a, item_id, item, s_a, s_b, sh);
  else
    long1_body<T, NT, KT, Key>(a, item_id, item, s_a, s_b, sh);
}

// One item per work-group, or (list1 set) the items listed by the
// wavefront kernel, in a grid-stride loop.
template <typename T, int NT, int TILE, typename Key>
__global__ __launch_bounds__(NT) void k_long1(LongArgs<T> a) {
  __shared__ __align__(16) unsigned char s_a[Long1Lds<NT, TILE, Key>::bytes_a];  // run starts / keys
  __shared__ __align__(16) T s_b[TILE];  // a_ij of runs / products
  __shared__ MergeShared<T> sh;
  if (a.list1 == nullptr) {
    long1_item<T, NT, TILE, Key>(a, static_cast<int32_t>(blockIdx.x), s_a, s_b, sh);
    return;
  }
  const unsigned int n = a.cnt->l1;
  for (unsigned int w = blockIdx.x; w < n; w += gridDim.x) {
    __syncthreads();
    long1_item<T, NT, TILE, Key>(a, static_cast<int32_t>(a.list1[w]), s_a, s_b, sh);
  }
}

template <typename T, int NT, int KT, typename Key, int MAXS>
DEVI void combine1_body(LongArgs<T> &a, const int32_t pid, const int32_t lri, const int32_t c0,
                        const int32_t nseg, const int64_t E, const int64_t obase,
                        const int32_t *sg_off,
                        const int32_t *sg_lo, const int32_t *const *sg_col,
                        const T *const *sg_val, unsigned char *s_a, T *s_b,
                        MergeShared<T> &sh) {
  constexpr int TILE = NT * KT;
  constexpr int LOGT = Log2<TILE>::v;
  constexpr Key KMAX = KeyMax<Key>::v;
  Key *sk = reinterpret_cast<Key *>(s_a);
  T *pv = s_b;
  const int t = threadIdx.x;
  const int tn = static_cast<int>(E);
  Key key[KT];
  T val[KT];
  {
    const int g0 = t * KT;
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (sg_off[mid] <= g0)
        lo = mid;
      else
        hi = mid;
    }
    int s = lo;
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = t * KT + kk;
      key[kk] = KMAX;
      val[kk] = T(0);
      if (l < tn) {
        while (s + 1 < nseg && sg_off[s + 1] <= l) ++s;
        const int64_t idx = sg_lo[s] + (l - sg_off[s]);
        const int32_t c = sg_col[s][idx];
        val[kk] = sg_val[s][idx];
        key[kk] = (static_cast<Key>(c - c0) << LOGT) | static_cast<Key>(l);
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    if (l < tn) pv[tix<NT, KT>(l)] = val[kk];
  }
  block_bitonic_sort<NT, KT, Key>(key, sk);
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) sk[kk * NT + t] = key[kk];
  __syncthreads();
  bool hd[KT];
  int nh = 0;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    hd[kk] = l < tn && (l == 0 || (sk[tix<NT, KT>(l - 1)] >> LOGT) != (key[kk] >> LOGT));
    nh += hd[kk] ? 1 : 0;
  }
  int64_t rtot;
  int o = static_cast<int>(block_excl_sum<NT>(static_cast<int64_t>(nh), sh.scan, rtot));
  const int r = static_cast<int>(rtot);
  const LongRow lr = a.lrows[lri];
  int32_t *dcol;
  T *dval;
  piece_out(a, pid, lr, obase, dcol, dval);
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    if (hd[kk]) {
      const Key c = key[kk] >> LOGT;
      T v = T(0);
      v = v + pv[tix<NT, KT>(static_cast<int>(key[kk] & (TILE - 1)))];
      for (int l2 = l + 1; l2 < tn; ++l2) {
        const Key k2 = sk[tix<NT, KT>(l2)];
        if ((k2 >> LOGT) != c) break;
        v = v + pv[tix<NT, KT>(static_cast<int>(k2 & (TILE - 1)))];
      }
      dcol[o] = c0 + static_cast<int32_t>(c);
      dval[o] = v;
      ++o;
    }
  }
  if (t == 0) {
    LongState st = a.cstate[pid];
    st.pos = E;
    a.cstate[pid] = st;
    Piece pc;
    pc.col = dcol;
    pc.val = dval;
    pc.cnt = r;
    pc.lrow = lri;
    pc.pad = 0;
    a.pieces[pid] = pc;
  }
}


// Radix variant of the one-tile combine: the range's entries of all
// partials, concatenated in segment order, sorted on the column (stable)
// and folded in that order.
template <typename T, int NT, int KT, int MAXS>
DEVI void combine1_radix(LongArgs<T> &a, const int32_t pid, const int32_t lri, const int32_t c0,
                         const int32_t nseg, const int64_t E, const int64_t obase,
                         const int32_t *sg_off,
                         const int32_t *sg_lo, const int32_t *const *sg_col,
                         const T *const *sg_val, uint32_t *ka, uint32_t *kb, T *pv,
                         uint32_t *cnt, MergeShared<T> &sh) {
  constexpr int TILE = NT * KT;
  constexpr int LOGT = Log2<TILE>::v;
  constexpr int NW = NT / WAVE;
  const int t = threadIdx.x;
  const int w = t / WAVE;
  const int ln = lane();
  const int tn = static_cast<int>(E);
  int32_t col[KT];
  T val[KT];
  int cmin = 0x7fffffff, cmax = -1;
  {
    const int g0 = t * KT;
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (sg_off[mid] <= g0)
        lo = mid;
      else
        hi = mid;
    }
    int sgi = lo;
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = t * KT + kk;
      col[kk] = 0;
      val[kk] = T(0);
      if (l < tn) {
        while (sgi + 1 < nseg && sg_off[sgi + 1] <= l) ++sgi;
        const int64_t idx = sg_lo[sgi] + (l - sg_off[sgi]);
        col[kk] = sg_col[sgi][idx] - c0;
        val[kk] = sg_val[sgi][idx];
        cmin = min(cmin, col[kk]);
        cmax = max(cmax, col[kk]);
      }
    }
  }
  block_minmax<NT>(cmin, cmax, sh.imax);  // the segment tables are dead after this
  if (tn <= 0) {
    cmin = 0;
    cmax = 0;
  }
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int l = t * KT + kk;
    if (l < tn) {
      ka[l] = (static_cast<uint32_t>(col[kk] - cmin) << LOGT) | static_cast<uint32_t>(l);
      pv[l] = val[kk];
    }
  }
  __syncthreads();
  const uint32_t *R = radix_sort<NT, KT, kRadixBits>(
      ka, kb, tn, bit_width(static_cast<uint32_t>(cmax - cmin)),
      [](uint32_t k) { return k >> LOGT; }, cnt, sh.scan);
  const uint64_t below_mask = ln == 0 ? 0ull : (~0ull >> (WAVE - ln));
  bool hd[KT];
  int pre[KT];
  int wcount = 0;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int e = (w * KT + kk) * WAVE + ln;
    hd[kk] = e < tn && (e == 0 || (R[e - 1] >> LOGT) != (R[e] >> LOGT));
    const uint64_t m = __ballot(hd[kk]);
    pre[kk] = wcount + __popcll(m & below_mask);
    wcount += __popcll(m);
  }
  if (ln == 0) sh.imax[w] = wcount;
  __syncthreads();
  int woff = 0, r = 0;
#pragma unroll
  for (int x = 0; x < NW; ++x) {
    woff += x < w ? sh.imax[x] : 0;
    r += sh.imax[x];
  }
  const LongRow lr = a.lrows[lri];
  int32_t *dcol;
  T *dval;
  piece_out(a, pid, lr, obase, dcol, dval);
  const int32_t cb = c0 + cmin;
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    if (hd[kk]) {
      const int e = (w * KT + kk) * WAVE + ln;
      const uint32_t k = R[e];
      const uint32_t c = k >> LOGT;
      T v = T(0);
      v = v + pv[k & (TILE - 1)];
      for (int e2 = e + 1; e2 < tn; ++e2) {
        const uint32_t k2 = R[e2];
        if ((k2 >> LOGT) != c) break;
        v = v + pv[k2 & (TILE - 1)];
      }
      const int o = woff + pre[kk];
      dcol[o] = cb + static_cast<int32_t>(c);
      dval[o] = v;
    }
  }
  if (t == 0) {
    LongState st = a.cstate[pid];
    st.pos = E;
    a.cstate[pid] = st;
    Piece pc;
    pc.col = dcol;
    pc.val = dval;
    pc.cnt = r;
    pc.lrow = lri;
    pc.pad = 0;
    a.pieces[pid] = pc;
  }
}

// segment tables: (MAXS + 1) offsets, MAXS range starts, 2 MAXS pointers;
// with radix sorting they live in the second key buffer (dead by then)
template <int NT, int TILE, typename Key, int MAXS> struct Combine1Lds {
  static constexpr size_t tab = (MAXS + 1) * 4 + MAXS * 4 + 2 * MAXS * sizeof(void *);
  static constexpr size_t tab_al = (tab + 15) & ~static_cast<size_t>(15);
  static constexpr size_t bytes_a =
      sizeof(Key) == 4 ? static_cast<size_t>(TILE) * 8 + RadixCounters<NT, kRadixBits>::count * 4
                       : static_cast<size_t>(TILE) * sizeof(Key) + tab_al;
  static_assert(sizeof(Key) != 4 || tab <= static_cast<size_t>(TILE) * 4,
                "tables exceed key buffer");
};

template <typename T, int NT, int TILE, typename Key, int MAXS>
DEVI void combine1_piece(LongArgs<T> &a, const int32_t pid, unsigned char *s_a, T *s_b,
                         MergeShared<T> &sh) {
  constexpr int KT = TILE / NT;
  constexpr bool kRadix = sizeof(Key) == 4;
  unsigned char *tab = kRadix ? s_a + static_cast<size_t>(TILE) * 4
                              : s_a + static_cast<size_t>(TILE) * sizeof(Key);
  const T **sg_val = reinterpret_cast<const T **>(tab);
  const int32_t **sg_col = reinterpret_cast<const int32_t **>(tab + MAXS * sizeof(void *));
  int32_t *sg_off = reinterpret_cast<int32_t *>(tab + 2 * MAXS * sizeof(void *));
  int32_t *sg_lo = sg_off + (MAXS + 1);
  const int t = threadIdx.x;
  const int32_t lri = a.piece_lrow[pid];
  const LongRow lr = a.lrows[lri];
  if (lr.nseg <= 1) return;
  const int32_t b = static_cast<int32_t>(pid - lr.piece0);
  const int32_t c0 = b << lr.shift;
  const int32_t nseg = lr.nseg;
  const int32_t *pos_tab = a.split + lr.sbase;
  int64_t carry = 0;
  int64_t obase = 0;  // sum of the range starts: where this piece's result goes
  for (int32_t s0 = 0; s0 < nseg; s0 += NT) {
    const int32_t s = s0 + t;
    int64_t len = 0, start = 0;
    if (s < nseg) {
      const Seq q = a.partials[lr.item0 + s];
      int64_t lo = 0, hi = 0;
      if (q.cnt > 0 && q.col != nullptr) {
        lo = pos_tab[static_cast<int64_t>(b) * nseg + s];
        hi = pos_tab[static_cast<int64_t>(b + 1) * nseg + s];
        lo = lo < 0 ? 0 : (lo > q.cnt ? q.cnt : lo);
        hi = hi < lo ? lo : (hi > q.cnt ? q.cnt : hi);
      }
      sg_lo[s] = static_cast<int32_t>(lo);
      sg_col[s] = q.col;
      sg_val[s] = reinterpret_cast<const T *>(q.val);
      len = hi - lo;
      start = lo;
    }
    int64_t tot;
    const int64_t ex = block_excl_sum<NT>(len, sh.scan, tot);
    if (s < nseg) sg_off[s] = static_cast<int32_t>(carry + ex);
    carry += tot;
    block_excl_sum<NT>(start, sh.scan, tot);
    obase += tot;
  }
  if (t == 0) sg_off[nseg] = static_cast<int32_t>(carry);
  __syncthreads();
  const int64_t E = carry;
  if (E > TILE) {
    if (t == 0) a.glist2[atomicAdd(&a.cnt->gcomb, 1u)] = static_cast<unsigned int>(pid);
    return;
  }
  if constexpr (kRadix) {
    uint32_t *ka = reinterpret_cast<uint32_t *>(s_a);
    combine1_radix<T, NT, KT, MAXS>(a, pid, lri, c0, nseg, E, obase, sg_off, sg_lo, sg_col, sg_val, ka,
                                    ka + TILE, s_b, ka + 2 * TILE, sh);
    return;
  }
  if (E <= TILE / 4)
    combine1_body<T, NT, KT / 4, Key, MAXS>(a, pid, lri, c0, nseg, E, obase, sg_off, sg_lo, sg_col,
                                            sg_val, s_a, s_b, sh);
  else if (E <= TILE / 2)
    combine1_body<T, NT, KT / 2, Key, MAXS>(a, pid, lri, c0, nseg, E, obase, sg_off, sg_lo, sg_col,
                                            sg_val, s_a, s_b, sh);
  else
    combine1_body<T, NT, KT, Key, MAXS>(a, pid, lri, c0, nseg, E, obase, sg_off, sg_lo, sg_col,
                                        sg_val, s_a, s_b, sh);
}

// One piece per work-group, or (list3 set) the pieces listed by the
// wavefront kernels, in a grid-stride loop.
template <typename T, int NT, int TILE, typename Key, int MAXS>
__global__ __launch_bounds__(NT) void k_combine1(LongArgs<T> a) {
  __shared__ __align__(16) unsigned char s_a[Combine1Lds<NT, TILE, Key, MAXS>::bytes_a];
  __shared__ __align__(16) T s_b[TILE];
  __shared__ MergeShared<T> sh;
  if (a.list3 == nullptr) {
    combine1_piece<T, NT, TILE, Key, MAXS>(a, static_cast<int32_t>(blockIdx.x), s_a, s_b, sh);
    return;
  }
  const unsigned int n = a.cnt->l3;
  for (unsigned int w = blockIdx.x; w < n; w += gridDim.x) {
    __syncthreads();
    combine1_piece<T, NT, TILE, Key, MAXS>(a, static_cast<int32_t>(a.list3[w]), s_a, s_b, sh);
  }
}

// ------------------------------------------------------ wavefront items
//
// The common case of both phases fits one wavefront: an item or piece of at
// most kWaveTile entries is sorted by one wavefront on (column, position)
// with a register bitonic network (16 keys per lane) and never waits for
// the other wavefronts of its work-group.  A one-item row is folded into its
// result.  An item of a split row is only sorted: its partial keeps every
// product, in (column, position) order, so that phase 2 sees each column's
// products in sequence order and its sums are Gustavson's.

constexpr int WAVE_NT = 256;  // four independent wavefronts per work-group
constexpr int WAVE_K = kWaveTile / WAVE;

// Element l of a wavefront tile lives at (l mod K) * 64 + l / K (lanes touch
// consecutive words).
template <int K> DEVI int wix(int l) { return (l & (K - 1)) * WAVE + (l >> Log2<K>::v); }

// Rank r of a sorted wavefront tile lives at r + r / 64: lane-blocked writes
// (lane p, ranks p*K ..) and lane-striped reads (lane p, ranks k*64 + p)
// are both free of LDS bank conflicts.  A tile needs U + U / 64 slots.
DEVI int wpad(int r) { return r + (r >> 6); }

// Wavefronts per SIMD that the tile's LDS allows (FP64 values): the register
// budget of the wavefront kernels is held to it, since they wait on memory
// and need every resident wavefront they can get.
template <int K> constexpr int wave_occupancy() { return K <= 8 ? 6 : 3; }

template <typename T, int K, typename Key>
DEVI void wave_item(LongArgs<T> &a, const int32_t item_id, const LongItem &item,
                    unsigned char *lds_a, T *lds_b) {
  constexpr int U = WAVE * K;
  constexpr int LOGU = Log2<U>::v;
  constexpr Key KMAX = KeyMax<Key>::v;
  const int pos = lane();
  int32_t *rs = reinterpret_cast<int32_t *>(lds_a);
  Key *sk = reinterpret_cast<Key *>(lds_a);
  T *ra = lds_b;
  T *pv = lds_b;
  const int64_t p0 = item.p0, p1 = item.p1;
  const int tn = static_cast<int>(p1 - p0);
  const LongRow lr = a.lrows[item.lrow];
  const int32_t i = item.row;
  const int32_t e1 = a.e.arp[i + 1];
  const int64_t pbase = a.e.P[a.e.arp[i]];

#pragma unroll
  for (int kk = 0; kk < K; ++kk) rs[kk * WAVE + pos] = -1;
  wave_sync();
  // run starts of the b_j* rows that overlap [p0, p1); the loads of a
  // chunk of 64 entries are issued together (clamped, not branched on)
  const GLOBAL_AS int64_t *gP = as_global(a.e.P);
  for (int32_t e0 = item.e_first; e0 < e1; e0 += WAVE) {
    const int32_t e = e0 + pos;
    const bool in = e < e1;
    const int32_t ec = in ? e : e1 - 1;
    const int64_t s0 = gP[ec] - pbase;
    const int64_t s1 = gP[ec + 1] - pbase;
    const int32_t j = as_global(a.e.acol)[ec];
    const T av = as_global(a.e.aval)[ec];
    if (in && s0 < p1 && s1 > p0 && s1 > s0) {
      int64_t ls = s0 - p0;
      int32_t off = 0;
      if (ls < 0) {
        off = static_cast<int32_t>(-ls);
        ls = 0;
      }
      rs[wix<K>(static_cast<int>(ls))] = as_global(a.e.brp)[j] + off;
      ra[wix<K>(static_cast<int>(ls))] = av;
    }
    if (!__any(in && s1 < p1)) break;  // the next chunk starts at or after p1
  }
  wave_sync();
  int st[K];
  int run = -1;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = pos * K + kk;
    const int f = (l < tn && rs[wix<K>(l)] >= 0) ? l : -1;
    run = max(run, f);
    st[kk] = run;
  }
  const int incl = group_incl_max<WAVE>(run);
  int prev = wave_shr1(incl, -1);
  if (pos == 0) prev = -1;
  // B index and a_ij of every product, resolved in lane-blocked order and
  // handed over through LDS so that consecutive lanes gather consecutive
  // products (coalesced loads along each b_j* row)
  int32_t gbx[K];
  T gav[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = pos * K + kk;
    const int s0 = max(prev, st[kk]);
    const bool ok = l < tn && s0 >= 0;
    gbx[kk] = ok ? rs[wix<K>(s0)] + (l - s0) : 0;
    gav[kk] = ok ? ra[wix<K>(s0)] : T(0);
  }
  int32_t *gb = rs;  // product l at gb[l] / ga[l]
  T *ga = ra;
  wave_sync();
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = pos * K + kk;
    if (l < tn) {
      gb[l] = gbx[kk];
      ga[l] = gav[kk];
    }
  }
  wave_sync();
  // every load of the tile is issued before any is used: positions past
  // the end load B's entry 0 (there are products, so B has one) and are
  // then ignored
  int32_t bc[K];
  T bv[K], av[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = kk * WAVE + pos;
    const int32_t g = gb[l];
    const int32_t bidx = l < tn ? g : 0;
    av[kk] = ga[l];
    bc[kk] = as_global(a.e.bcol)[bidx];
    bv[kk] = as_global(a.e.bval)[bidx];
  }
  Key key[K];
  T prod[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = kk * WAVE + pos;
    const bool ok = l < tn;
    prod[kk] = ok ? av[kk] * bv[kk] : T(0);
    key[kk] = ok ? ((static_cast<Key>(bc[kk]) << LOGU) | static_cast<Key>(l)) : KMAX;
  }
  wave_sync();  // pv takes the place of ga
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = kk * WAVE + pos;
    if (l < tn) pv[l] = prod[kk];
  }
  // a tile inside one sorted run of B (about a fifth of the tiles of
  // power-law rows) is already in order: it only changes lanes
  bool ordered = true;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = kk * WAVE + pos;
    const Key right = shfl_key<Key>(key[kk], (pos + 1) & (WAVE - 1));
    const Key wrap = shfl_key<Key>(key[kk + 1 < K ? kk + 1 : kk], 0);
    const Key next = pos < WAVE - 1 ? right : wrap;
    if (l + 1 < tn && !(key[kk] < next)) ordered = false;
  }
  if (__all(ordered)) {
    wave_sync();  // gb is dead
#pragma unroll
    for (int kk = 0; kk < K; ++kk) sk[wpad(kk * WAVE + pos)] = key[kk];
    wave_sync();
#pragma unroll
    for (int kk = 0; kk < K; ++kk) key[kk] = sk[wpad(pos * K + kk)];
  } else {
    group_bitonic_sort<WAVE, K, Key>(key);
  }
  // sorted keys by rank (rank pos * K + kk is in key[kk])
  wave_sync();
#pragma unroll
  for (int kk = 0; kk < K; ++kk) sk[wpad(pos * K + kk)] = key[kk];
  wave_sync();

  if (lr.nseg > 1) {
    // item of a split row: every product, sorted, plus the range starts
    const int32_t s = static_cast<int32_t>(item_id - lr.item0);
    const int shift = lr.shift;
    const int32_t np = lr.npiece;
    const int32_t nseg = lr.nseg;
    int32_t *ptab = a.split + lr.sbase;
    int32_t *dcol = a.pcol + lr.pbase + p0;
    T *dval = a.pval + lr.pbase + p0;
    // rank r = kk * 64 + lane: consecutive lanes write consecutive entries;
    // every LDS read is issued before the stores
    Key krs[K];
    T vrs[K];
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int r = kk * WAVE + pos;
      const Key kv = sk[wpad(r)];
      krs[kk] = r < tn ? kv : KMAX;
    }
#pragma unroll
    for (int kk = 0; kk < K; ++kk) vrs[kk] = pv[static_cast<int>(krs[kk] & (U - 1))];
    Key carry = 0;  // key of the rank before this pass's first
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int r = kk * WAVE + pos;
      const Key kr = krs[kk];
      Key before = shfl_up_key<Key>(kr, 1);
      if (pos == 0) before = carry;
      carry = shfl_key<Key>(kr, WAVE - 1);
      if (r < tn) {
        const int32_t c = static_cast<int32_t>(kr >> LOGU);
        dcol[r] = c;
        dval[r] = vrs[kk];
        const int32_t q = c >> shift;
        const int32_t qp = r > 0 ? (static_cast<int32_t>(before >> LOGU) >> shift) : -1;
        for (int32_t qq = qp + 1; qq <= q && qq < np; ++qq)
          ptab[static_cast<int64_t>(qq) * nseg + s] = r;
        if (r == tn - 1)
          for (int32_t qq = q + 1; qq <= np; ++qq) ptab[static_cast<int64_t>(qq) * nseg + s] = tn;
      }
    }
    if (pos == 0) {
      LongState stt = a.state[item_id];
      stt.pos = p1;
      stt.status = 0;
      a.state[item_id] = stt;
      Seq q;
      q.col = dcol;
      q.val = dval;
      q.cnt = tn;
      a.partials[item_id] = q;
    }
    return;
  }

  // one-item row: fold every column in position order into the row's place
  int32_t *sc = reinterpret_cast<int32_t *>(lds_a);
  const int r = fold_runs<T, WAVE, K, Key>(key, tn, pv, sc, lds_b, 0);
  int32_t *dcol = a.pcol + lr.pbase;
  T *dval = a.pval + lr.pbase;
  for (int x = pos; x < r; x += WAVE) {
    dcol[x] = sc[x];
    dval[x] = lds_b[x];
  }
  if (pos == 0) {
    LongState stt = a.state[item_id];
    stt.pos = p1;
    stt.status = 0;
    a.state[item_id] = stt;
    Piece pc;
    pc.col = dcol;
    pc.val = dval;
    pc.cnt = r;
    pc.lrow = item.lrow;
    pc.pad = 0;
    a.pieces[lr.piece0] = pc;
  }
}

// Every item (in_list == nullptr), or the listed ones in a grid-stride
// loop; items above 64 K products go to out_list.
template <typename T, typename Key, int K>
__global__ __launch_bounds__(WAVE_NT) __attribute__((amdgpu_waves_per_eu(wave_occupancy<K>())))
void k_long_w(LongArgs<T> a, int64_t nitems,
                                                    const unsigned int *in_list,
                                                    const unsigned int *in_cnt,
                                                    unsigned int *out_list,
                                                    unsigned int *out_cnt) {
  constexpr int NWV = WAVE_NT / WAVE;
  constexpr int U = WAVE * K;
  constexpr int KB = sizeof(Key) > 4 ? static_cast<int>(sizeof(Key)) : 4;
  __shared__ __align__(16) unsigned char s_a[NWV][(U + U / WAVE) * KB];
  __shared__ __align__(16) T s_b[NWV][U];
  // wave-uniform (so item and row records are read through the scalar cache)
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / WAVE));
  const int64_t id0 = xcd_block_id<16>() * NWV + w;
  const int64_t n = in_list ? static_cast<int64_t>(*in_cnt) : nitems;
  const int64_t stride = in_list ? static_cast<int64_t>(gridDim.x) * NWV : n;
  // uniform across the wavefront; no work-group barriers here
  for (int64_t x = id0; x < n; x += stride) {
    const int32_t id = static_cast<int32_t>(in_list ? in_list[x] : x);
    const LongItem item = a.items[id];
    if (item.p1 - item.p0 > U) {
      if (lane() == 0) out_list[atomicAdd(out_cnt, 1u)] = static_cast<unsigned int>(id);
      continue;
    }
    wave_item<T, K, Key>(a, id, item, s_a[w], s_b[w]);
  }
}

// The gather, sort, fold and output of a piece whose stream (tn entries,
// at most WAVE * K) the segment table of wave_piece describes: seg_at in
// lds_a, tbase in lds_b.
template <typename T, int K, typename Key>
DEVI void piece_body(LongArgs<T> &a, const int32_t pid, const LongRow &lr, const int32_t lri,
                     const int32_t c0, const int tn, const int64_t E, const int64_t obase,
                     unsigned char *lds_a, T *lds_b) {
  constexpr int U = WAVE * K;
  constexpr int LOGU = Log2<U>::v;
  constexpr Key KMAX = KeyMax<Key>::v;
  const int pos = lane();
  const int32_t *seg_at = reinterpret_cast<const int32_t *>(lds_a);
  const int32_t *tbase = reinterpret_cast<const int32_t *>(lds_b);
  const int32_t *pcol = a.pcol + lr.pbase;
  const T *pval = a.pval + lr.pbase;
  // partial-buffer index of every stream entry: the segment is the last one
  // starting at or before it (a max-scan in lane-blocked order), handed over
  // through LDS so that the loads below read consecutive entries with
  // consecutive lanes
  int32_t gix[K];
  {
    int run = -1;
    int sgk[K];
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int l = pos * K + kk;
      const int v = seg_at[l];
      run = max(run, l < tn ? v : -1);
      sgk[kk] = run;
    }
    const int inc = group_incl_max<WAVE>(run);
    int prev = wave_shr1(inc, -1);
    if (pos == 0) prev = -1;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int l = pos * K + kk;
      const int sg = max(prev, sgk[kk]);
      const int32_t tb = tbase[sg > 0 ? sg : 0];
      gix[kk] = l < tn ? tb + l : 0;
    }
  }
  int32_t *gi = reinterpret_cast<int32_t *>(lds_a);
  wave_sync();  // the segment table is dead from here on
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = pos * K + kk;
    if (l < tn) gi[l] = gix[kk];
  }
  wave_sync();
  // every load is issued before any is used (entries past the end reload
  // entry 0 and are ignored)
  int32_t cv[K];
  T vv[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = kk * WAVE + pos;
    const int32_t g = gi[l];
    const int32_t idx = l < tn ? g : 0;
    cv[kk] = as_global(pcol)[idx];
    vv[kk] = as_global(pval)[idx];
  }
  Key key[K];
  T *pv = lds_b;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = kk * WAVE + pos;
    key[kk] = KMAX;
    if (l < tn) {
      pv[l] = vv[kk];
      key[kk] = (static_cast<Key>(cv[kk] - c0) << LOGU) | static_cast<Key>(l);
    }
  }
  group_bitonic_sort<WAVE, K, Key>(key);
  wave_sync();  // gi is dead from here on
  int32_t *sc = reinterpret_cast<int32_t *>(lds_a);
  T *sv = lds_b;
  const int r = fold_runs<T, WAVE, K, Key>(key, tn, pv, sc, sv, c0);
  int32_t *dcol;
  T *dval;
  piece_out(a, pid, lr, obase, dcol, dval);
  for (int x = pos; x < r; x += WAVE) {
    dcol[x] = sc[x];
    dval[x] = sv[x];
  }
  if (pos == 0) {
    LongState stt = a.cstate[pid];
    stt.pos = E;
    a.cstate[pid] = stt;
    Piece pc;
    pc.col = dcol;
    pc.val = dval;
    pc.cnt = r;
    pc.lrow = lri;
    pc.pad = 0;
    a.pieces[pid] = pc;
  }
}

// One piece of a split row by one wavefront: the piece's range of every
// partial, concatenated in segment order, sorted on (column, stream index),
// folded in that order.  Larger pieces are listed for the work-group kernel.
template <typename T, int K, typename Key, int MAXS>
DEVI void wave_piece(LongArgs<T> &a, const int32_t pid, unsigned char *lds_a, T *lds_b,
                     unsigned int *olist, unsigned int *ocnt) {
  constexpr int U = WAVE * K;
  constexpr int LOGU = Log2<U>::v;
  constexpr Key KMAX = KeyMax<Key>::v;
  static_assert(MAXS <= U, "segment table exceeds the tile buffers");
  const int pos = lane();
  const int32_t lri = a.piece_lrow[pid];
  const LongRow lr = a.lrows[lri];
  if (lr.nseg <= 1) return;
  const int32_t b = static_cast<int32_t>(pid - lr.piece0);
  const int32_t c0 = b << lr.shift;
  const int32_t nseg = lr.nseg;
  const int32_t *ptab = a.split + lr.sbase;
  // segment table: lane p holds segments p*KS .. p*KS+KS-1, whose range
  // bounds are loaded together (one memory round trip); the stream is the
  // concatenation of the segments' parts of the range, in segment order
  constexpr int KS = MAXS / WAVE;
  static_assert(MAXS % WAVE == 0, "segment table rows must fill lanes evenly");
  const GLOBAL_AS int32_t *lo_row = as_global(ptab + static_cast<int64_t>(b) * nseg);
  const GLOBAL_AS int32_t *hi_row = as_global(ptab + static_cast<int64_t>(b + 1) * nseg);
  int32_t slo[KS], slen[KS];
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    const int32_t sg = pos * KS + j;
    const int32_t sc = sg < nseg ? sg : nseg - 1;
    slo[j] = lo_row[sc];
    slen[j] = hi_row[sc];
  }
  int32_t tot_len = 0, tot_lo = 0;
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    const bool in = pos * KS + j < nseg;
    const int32_t lo = in ? max(slo[j], 0) : 0;
    slen[j] = in ? max(slen[j] - lo, 0) : 0;
    slo[j] = lo;
    tot_len += slen[j];
    tot_lo += lo;
  }
  // one scan for both sums (each below 2^31, so the halves never carry):
  // stream length and this lane's first stream index in the low half, the
  // sum of the range starts (where this range's output begins) in the high
  const int64_t packed = (static_cast<int64_t>(tot_lo) << 32) | static_cast<uint32_t>(tot_len);
  const int64_t incl = group_incl_sum<WAVE>(packed);
  const int64_t last = group_last<WAVE>(incl);
  const int64_t E = last & 0xffffffffll;
  const int64_t obase = last >> 32;
  if (E > U) {
    if (pos == 0) olist[atomicAdd(ocnt, 1u)] = static_cast<unsigned int>(pid);
    return;
  }
  const int tn = static_cast<int>(E);
  // seg_at[t] = segment whose part starts at stream index t (non-empty parts
  // start at distinct indices), tbase[s] = partial-buffer index of stream
  // index 0 for segment s; both in the tile buffers, dead before those are
  // used
  int32_t *seg_at = reinterpret_cast<int32_t *>(lds_a);
  int32_t *tbase = reinterpret_cast<int32_t *>(lds_b);
#pragma unroll
  for (int kk = 0; kk < K; ++kk) seg_at[pos * K + kk] = -1;
  wave_sync();
  {
    int32_t run = static_cast<int32_t>((incl - packed) & 0xffffffffll);
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      const int32_t sg = pos * KS + j;
      if (sg < nseg) {
        tbase[sg] = static_cast<int32_t>(static_cast<int64_t>(sg) * lr.segp + slo[j] - run);
        if (slen[j] > 0) seg_at[run] = sg;
      }
      run += slen[j];
    }
  }
  wave_sync();
  // in the 512-entry pass, a stream that fits half the tile takes the
  // half-size network (fewer keys per lane to gather, sort and fold); the
  // 1024-entry pass only receives streams above 512
  if constexpr (K == 8) {
    if (tn <= WAVE * (K / 2)) {
      piece_body<T, K / 2, Key>(a, pid, lr, lri, c0, tn, E, obase, lds_a, lds_b);
      return;
    }
  }
  piece_body<T, K, Key>(a, pid, lr, lri, c0, tn, E, obase, lds_a, lds_b);
}

// Every piece (in_list == nullptr), or the listed ones in a grid-stride
// loop; pieces above 64 K entries go to out_list.
template <typename T, typename Key, int MAXS, int K>
__global__ __launch_bounds__(WAVE_NT) __attribute__((amdgpu_waves_per_eu(wave_occupancy<K>())))
void k_combine_w(LongArgs<T> a, int64_t npieces,
                                                       const unsigned int *in_list,
                                                       const unsigned int *in_cnt,
                                                       unsigned int *out_list,
                                                       unsigned int *out_cnt) {
  constexpr int NWV = WAVE_NT / WAVE;
  constexpr int U = WAVE * K;
  constexpr int KB = sizeof(Key) > 4 ? static_cast<int>(sizeof(Key)) : 4;
  __shared__ __align__(16) unsigned char s_a[NWV][U * KB];
  __shared__ __align__(16) T s_b[NWV][U];
  // wave-uniform (so piece and row records are read through the scalar cache);
  // runs of 4 work-groups (16 neighbouring ranges, which read neighbouring
  // entries of every segment) share an XCD
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / WAVE));
  const int64_t id = xcd_block_id<4>() * NWV + w;
  if (in_list == nullptr) {
    if (id >= npieces) return;  // uniform across the wavefront; no work-group barriers here
    wave_piece<T, K, Key, MAXS>(a, static_cast<int32_t>(id), s_a[w], s_b[w], out_list, out_cnt);
    return;
  }
  const int64_t n = *in_cnt;
  for (int64_t x = id; x < n; x += static_cast<int64_t>(gridDim.x) * NWV)
    wave_piece<T, K, Key, MAXS>(a, static_cast<int32_t>(in_list[x]), s_a[w], s_b[w], out_list,
                                out_cnt);
}

// ------------------------------------------------------------ long table

int64_t long_table_tmp_len(int64_t nlong) { return 4 * ((nlong + 255) / 256 + 1); }

struct LtSums {
  int64_t items, pieces, umulti, split;
};

DEVI LtSums lt_plan(const int32_t *binlist, int64_t off, int64_t t, int64_t nlong,
                    const int64_t *u, int64_t ncols, const LongParams &lp, LongRow &lr) {
  LtSums z{0, 0, 0, 0};
  if (t >= nlong) return z;
  const int32_t row = binlist[off + t];
  const int64_t ui = u[row];
  int64_t segp;
  int32_t nseg, shift, npiece;
  long_row_plan(ui, ncols, lp, segp, nseg, shift, npiece);
  lr.row = row;
  lr.nseg = nseg;
  lr.npiece = npiece;
  lr.shift = shift;
  lr.u = ui;
  lr.segp = segp;
  z.items = nseg;
  z.pieces = npiece;
  // output space of the one-tile paths (same rule as the analysis summary)
  z.umulti = nseg > 1 ? ui : (ui <= kOneShot ? (ui < ncols ? ui : ncols) : 0);
  z.split = nseg > 1 ? static_cast<int64_t>(nseg) * (npiece + 1) : 0;
  return z;
}

__global__ __launch_bounds__(256) void k_lt_reduce(const int32_t *binlist, int64_t off,
                                                   int64_t nlong, const int64_t *u,
                                                   int64_t ncols, LongParams lp, int64_t *tmp) {
  __shared__ int64_t sm[256 / WAVE + 1];
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  LongRow lr;
  const LtSums z = lt_plan(binlist, off, t, nlong, u, ncols, lp, lr);
  int64_t tot;
  block_excl_sum<256>(z.items, sm, tot);
  if (threadIdx.x == 0) tmp[4 * blockIdx.x + 0] = tot;
  block_excl_sum<256>(z.pieces, sm, tot);
  if (threadIdx.x == 0) tmp[4 * blockIdx.x + 1] = tot;
  block_excl_sum<256>(z.umulti, sm, tot);
  if (threadIdx.x == 0) tmp[4 * blockIdx.x + 2] = tot;
  block_excl_sum<256>(z.split, sm, tot);
  if (threadIdx.x == 0) tmp[4 * blockIdx.x + 3] = tot;
}

__global__ void k_lt_scan(int64_t *tmp, int64_t nb) {
  const int c = threadIdx.x;
  if (c >= 4) return;
  int64_t run = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t v = tmp[4 * b + c];
    tmp[4 * b + c] = run;
    run += v;
  }
}

// SELF: tmp holds the raw block sums and every work-group adds up those of
// the blocks before it (few blocks; saves the launch of k_lt_scan).
template <bool SELF>
__global__ __launch_bounds__(256) void k_lt_write(const int32_t *binlist, int64_t off,
                                                  int64_t nlong, const int64_t *u, int64_t ncols,
                                                  LongParams lp, const int64_t *tmp,
                                                  LongRow *lrows) {
  __shared__ int64_t sm[256 / WAVE + 1];
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  int64_t base[4];
  if constexpr (SELF) {
    int64_t ps[4] = {0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < static_cast<int64_t>(blockIdx.x); b += 256)
#pragma unroll
      for (int c = 0; c < 4; ++c) ps[c] += tmp[4 * b + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) block_excl_sum<256>(ps[c], sm, base[c]);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) base[c] = tmp[4 * blockIdx.x + c];
  }
  LongRow lr;
  const LtSums z = lt_plan(binlist, off, t, nlong, u, ncols, lp, lr);
  int64_t tot;
  const int64_t i0 = block_excl_sum<256>(z.items, sm, tot) + base[0];
  const int64_t p0 = block_excl_sum<256>(z.pieces, sm, tot) + base[1];
  const int64_t u0 = block_excl_sum<256>(z.umulti, sm, tot) + base[2];
  const int64_t s0 = block_excl_sum<256>(z.split, sm, tot) + base[3];
  if (t >= nlong) return;
  lr.item0 = i0;
  lr.piece0 = p0;
  lr.pbase = u0;
  lr.sbase = s0;
  lrows[t] = lr;
}

// Work items (one thread each): product range, first entry of A's row that
// reaches it, an empty checkpoint and an empty partial.
__global__ __launch_bounds__(256) void k_lt_items(const LongRow *lrows, int64_t nlong,
                                                  int64_t nitems, const int32_t *arp,
                                                  const int64_t *P, LongItem *items,
                                                  LongState *state, Seq *partials) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (x >= nitems) return;
  int64_t lo = 0, hi = nlong;  // the row whose items include x
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (lrows[mid].item0 <= x)
      lo = mid;
    else
      hi = mid;
  }
  const LongRow lr = lrows[lo];
  LongItem it;
  it.row = lr.row;
  it.lrow = static_cast<int32_t>(lo);
  it.p0 = (x - lr.item0) * lr.segp;
  it.p1 = it.p0 + lr.segp < lr.u ? it.p0 + lr.segp : lr.u;
  {
    const int32_t e0 = arp[lr.row], e1 = arp[lr.row + 1];
    const int64_t pbase = P[e0];
    int32_t a = e0, b = e1;  // last entry whose products start at or before p0
    while (b - a > 1) {
      const int32_t mid = (a + b) >> 1;
      if (P[mid] - pbase <= it.p0)
        a = mid;
      else
        b = mid;
    }
    it.e_first = a;
  }
  it.pad = 0;
  items[x] = it;
  LongState st;
  st.pos = it.p0;
  st.gcnt = 0;
  st.gcap = 0;
  st.gcol = nullptr;
  st.gval = nullptr;
  st.scap = 0;
  st.scol = nullptr;
  st.sval = nullptr;
  st.status = 0;
  st.pad = 0;
  state[x] = st;
  Seq q;
  q.col = nullptr;
  q.val = nullptr;
  q.cnt = 0;
  partials[x] = q;
}

// Row of every output piece (one thread each).
__global__ __launch_bounds__(256) void k_lt_pieces(const LongRow *lrows, int64_t nlong,
                                                   int64_t npieces, int32_t *piece_lrow) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (x >= npieces) return;
  int64_t lo = 0, hi = nlong;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (lrows[mid].piece0 <= x)
      lo = mid;
    else
      hi = mid;
  }
  piece_lrow[x] = static_cast<int32_t>(lo);
}

void launch_long_table(const int32_t *binlist, int64_t off, int64_t nlong, const int64_t *u,
                       int64_t ncols, LongParams lp, LongRow *lrows, int64_t nitems,
                       LongItem *items, LongState *state, Seq *partials, int64_t npieces,
                       int32_t *piece_lrow, const int32_t *arp, const int64_t *P, int64_t *tmp,
                       hipStream_t s) {
  if (nlong <= 0) return;
  const int64_t nb = (nlong + 255) / 256;
  hipLaunchKernelGGL(k_lt_reduce, dim3(nb), dim3(256), 0, s, binlist, off, nlong, u, ncols, lp,
                     tmp);
  if (nb <= 1024) {
    hipLaunchKernelGGL(k_lt_write<true>, dim3(nb), dim3(256), 0, s, binlist, off, nlong, u,
                       ncols, lp, tmp, lrows);
  } else {
    hipLaunchKernelGGL(k_lt_scan, dim3(1), dim3(64), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_lt_write<false>, dim3(nb), dim3(256), 0, s, binlist, off, nlong, u,
                       ncols, lp, tmp, lrows);
  }
  if (nitems > 0)
    hipLaunchKernelGGL(k_lt_items, dim3((nitems + 255) / 256), dim3(256), 0, s, lrows, nlong,
                       nitems, arp, P, items, state, partials);
  if (npieces > 0)
    hipLaunchKernelGGL(k_lt_pieces, dim3((npieces + 255) / 256), dim3(256), 0, s, lrows, nlong,
                       npieces, piece_lrow);
}

// Checkpoints of the combine pieces: start of the stream, empty G; and the
// work-list counters cleared in the same launch.
__global__ void k_cstate_init(LongState *state, int64_t n, unsigned int *cnt, int ncnt) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x < ncnt) cnt[x] = 0u;
  if (x >= n) return;
  LongState s;
  s.pos = 0;
  s.gcnt = 0;
  s.gcap = 0;
  s.gcol = nullptr;
  s.gval = nullptr;
  s.scap = 0;
  s.scol = nullptr;
  s.sval = nullptr;
  s.status = 0;
  s.pad = 0;
  state[x] = s;
}

void launch_cstate_init(LongState *state, int64_t n, LongCounters *cnt, hipStream_t s) {
  constexpr int ncnt = static_cast<int>(sizeof(LongCounters) / sizeof(unsigned int));
  static_assert(ncnt <= 256, "counters are cleared by the first work-group");
  const int64_t nb = n > 0 ? (n + 255) / 256 : 1;
  hipLaunchKernelGGL(k_cstate_init, dim3(nb), dim3(256), 0, s, state, n,
                     reinterpret_cast<unsigned int *>(cnt), ncnt);
}

// rownnz of long rows = sum of their pieces (from the exclusive piece scan)
__global__ void k_long_rownnz(const LongRow *lrows, int64_t nlong, const int64_t *pscan,
                              int64_t *rownnz) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nlong) return;
  const LongRow lr = lrows[t];
  rownnz[lr.row] = pscan[lr.piece0 + lr.npiece] - pscan[lr.piece0];
}

void launch_long_rownnz(const LongRow *lrows, int64_t nlong, const int64_t *pscan,
                        int64_t *rownnz, hipStream_t s) {
  if (nlong <= 0) return;
  hipLaunchKernelGGL(k_long_rownnz, dim3((nlong + 255) / 256), dim3(256), 0, s, lrows, nlong,
                     pscan, rownnz);
}

// ------------------------------------------------------------ launchers

int long_l1cap_default(int dtype_bytes) { return dtype_bytes == 8 ? 5120 : 7168; }

constexpr int LONG_NT = 256;
constexpr int LONG_TILE = kLongTile;
constexpr int COMBINE_L1 = 3072;
constexpr int COMBINE_MAXS = 512;

constexpr int ONESHOT_NT = 512;
constexpr int GENERAL_GRID = 512;  // grid of the general kernels without a work list

template <typename T, int L1CAP>
static void launch_cfg(const LongArgs<T> &a, int64_t nwork, hipStream_t s) {
  const int64_t grid = a.work ? nwork : GENERAL_GRID;
  if ((static_cast<uint64_t>(a.ncols) << Log2<LONG_TILE>::v) <= 0xffffffffull)
    hipLaunchKernelGGL((k_long<T, LONG_NT, LONG_TILE, L1CAP, uint32_t>), dim3(grid),
                       dim3(LONG_NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_long<T, LONG_NT, LONG_TILE, L1CAP, uint64_t>), dim3(grid),
                       dim3(LONG_NT), 0, s, a);
}

constexpr int64_t LIST_GRID = 1024;  // grid of the one-tile kernels over a list

template <typename T> void launch_long_oneshot(const LongArgs<T> &a, int64_t nitems, hipStream_t s) {
  if (nitems <= 0) return;
  const int64_t grid = a.list1 ? std::min<int64_t>(nitems, LIST_GRID) : nitems;
  if ((static_cast<uint64_t>(a.ncols) << Log2<kOneShot>::v) <= 0xffffffffull)
    hipLaunchKernelGGL((k_long1<T, ONESHOT_NT, kOneShot, uint32_t>), dim3(grid),
                       dim3(ONESHOT_NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_long1<T, ONESHOT_NT, kOneShot, uint64_t>), dim3(grid),
                       dim3(ONESHOT_NT), 0, s, a);
}

template <typename T>
void launch_combine_oneshot(const LongArgs<T> &a, int64_t npieces, hipStream_t s) {
  if (npieces <= 0) return;
  const int64_t grid = a.list3 ? std::min<int64_t>(npieces, LIST_GRID) : npieces;
  if ((static_cast<uint64_t>(a.ncols) << Log2<kOneShot>::v) <= 0xffffffffull)
    hipLaunchKernelGGL((k_combine1<T, ONESHOT_NT, kOneShot, uint32_t, COMBINE_MAXS>),
                       dim3(grid), dim3(ONESHOT_NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_combine1<T, ONESHOT_NT, kOneShot, uint64_t, COMBINE_MAXS>),
                       dim3(grid), dim3(ONESHOT_NT), 0, s, a);
}

template <typename T, int K>
static void long_wave_k(const LongArgs<T> &a, int64_t nitems, int64_t grid,
                        const unsigned int *in_list, const unsigned int *in_cnt,
                        unsigned int *out_list, unsigned int *out_cnt, hipStream_t s) {
  if ((static_cast<uint64_t>(a.ncols) << Log2<WAVE * K>::v) <= 0xffffffffull)
    hipLaunchKernelGGL((k_long_w<T, uint32_t, K>), dim3(grid), dim3(WAVE_NT), 0, s, a, nitems,
                       in_list, in_cnt, out_list, out_cnt);
  else
    hipLaunchKernelGGL((k_long_w<T, uint64_t, K>), dim3(grid), dim3(WAVE_NT), 0, s, a, nitems,
                       in_list, in_cnt, out_list, out_cnt);
}

// Items of up to 512 products (every segment of a split row) in one pass,
// larger ones (one-item rows up to 1024) in a second, then the lists.
template <typename T> void launch_long_wave(const LongArgs<T> &a, int64_t nitems, hipStream_t s) {
  if (nitems <= 0) return;
  const int64_t grid = (nitems + WAVE_NT / WAVE - 1) / (WAVE_NT / WAVE);
  long_wave_k<T, WAVE_K / 2>(a, nitems, grid, nullptr, nullptr, a.listw, &a.cnt->lw, s);
}

template <typename T>
void launch_long_wave_large(const LongArgs<T> &a, int64_t nitems, hipStream_t s) {
  if (nitems <= 0) return;
  const int64_t grid =
      std::min<int64_t>((nitems + WAVE_NT / WAVE - 1) / (WAVE_NT / WAVE), LIST_GRID);
  long_wave_k<T, WAVE_K>(a, nitems, grid, a.listw, &a.cnt->lw, a.list1, &a.cnt->l1, s);
}

template <typename T, int K>
static void combine_wave_k(const LongArgs<T> &a, int64_t npieces, int64_t grid,
                           const unsigned int *in_list, const unsigned int *in_cnt,
                           unsigned int *out_list, unsigned int *out_cnt, hipStream_t s) {
  if ((static_cast<uint64_t>(a.ncols) << Log2<WAVE * K>::v) <= 0xffffffffull)
    hipLaunchKernelGGL((k_combine_w<T, uint32_t, COMBINE_MAXS, K>), dim3(grid), dim3(WAVE_NT), 0,
                       s, a, npieces, in_list, in_cnt, out_list, out_cnt);
  else
    hipLaunchKernelGGL((k_combine_w<T, uint64_t, COMBINE_MAXS, K>), dim3(grid), dim3(WAVE_NT), 0,
                       s, a, npieces, in_list, in_cnt, out_list, out_cnt);
}

template <typename T>
void launch_combine_wave(const LongArgs<T> &a, int64_t npieces, hipStream_t s) {
  if (npieces <= 0) return;
  const int64_t grid = (npieces + WAVE_NT / WAVE - 1) / (WAVE_NT / WAVE);
  combine_wave_k<T, WAVE_K / 2>(a, npieces, grid, nullptr, nullptr, a.list2, &a.cnt->l2, s);
}

template <typename T>
void launch_combine_wave_large(const LongArgs<T> &a, int64_t npieces, hipStream_t s) {
  if (npieces <= 0) return;
  const int64_t grid =
      std::min<int64_t>((npieces + WAVE_NT / WAVE - 1) / (WAVE_NT / WAVE), LIST_GRID);
  combine_wave_k<T, WAVE_K>(a, npieces, grid, a.list2, &a.cnt->l2, a.list3, &a.cnt->l3, s);
}

template <typename T>
int launch_long(const LongArgs<T> &a, int64_t nwork, int l1cap, hipStream_t s) {
  if (a.work && nwork <= 0) return 0;
  switch (l1cap) {
    case 2048: launch_cfg<T, 2048>(a, nwork, s); break;
    case 3072: launch_cfg<T, 3072>(a, nwork, s); break;
    case 5120: launch_cfg<T, 5120>(a, nwork, s); break;
    case 7168: launch_cfg<T, 7168>(a, nwork, s); break;
    default: return -1;
  }
  return 0;
}

template <typename T>
int launch_combine(const LongArgs<T> &a, int64_t npieces, hipStream_t s) {
  if (a.work && npieces <= 0) return 0;
  const int64_t grid = a.work ? npieces : GENERAL_GRID;
  if ((static_cast<uint64_t>(a.ncols) << Log2<LONG_TILE>::v) <= 0xffffffffull)
    hipLaunchKernelGGL(
        (k_combine<T, LONG_NT, LONG_TILE, COMBINE_L1, uint32_t, COMBINE_MAXS>),
        dim3(grid), dim3(LONG_NT), 0, s, a);
  else
    hipLaunchKernelGGL(
        (k_combine<T, LONG_NT, LONG_TILE, COMBINE_L1, uint64_t, COMBINE_MAXS>),
        dim3(grid), dim3(LONG_NT), 0, s, a);
  return 0;
}

int combine_maxs() { return COMBINE_MAXS; }
int combine_l1cap() { return COMBINE_L1; }

template int launch_long<float>(const LongArgs<float> &, int64_t, int, hipStream_t);
template int launch_long<double>(const LongArgs<double> &, int64_t, int, hipStream_t);
template int launch_combine<float>(const LongArgs<float> &, int64_t, hipStream_t);
template int launch_combine<double>(const LongArgs<double> &, int64_t, hipStream_t);
template void launch_long_oneshot<float>(const LongArgs<float> &, int64_t, hipStream_t);
template void launch_long_oneshot<double>(const LongArgs<double> &, int64_t, hipStream_t);
template void launch_combine_oneshot<float>(const LongArgs<float> &, int64_t, hipStream_t);
template void launch_combine_oneshot<double>(const LongArgs<double> &, int64_t, hipStream_t);
template void launch_long_wave<float>(const LongArgs<float> &, int64_t, hipStream_t);
template void launch_long_wave<double>(const LongArgs<double> &, int64_t, hipStream_t);
template void launch_long_wave_large<float>(const LongArgs<float> &, int64_t, hipStream_t);
template void launch_long_wave_large<double>(const LongArgs<double> &, int64_t, hipStream_t);
template void launch_combine_wave<float>(const LongArgs<float> &, int64_t, hipStream_t);
template void launch_combine_wave<double>(const LongArgs<double> &, int64_t, hipStream_t);
template void launch_combine_wave_large<float>(const LongArgs<float> &, int64_t, hipStream_t);
template void launch_combine_wave_large<double>(const LongArgs<double> &, int64_t, hipStream_t);


// ------------------------------------------------------- counting pass
//
// Distinct columns of each piece (column range) of a split row, from the
// sorted segments phase 1 wrote: every entry of the range in every segment
// sets its bit in a wavefront's LDS bitmap of the range's 2^shift columns
// (at most 2^kPieceCountLog, checked on the host), and the bits are
// counted.  A segment's part of the range is one run of its sorted
// partial.  Pieces of one-segment rows keep the count phase 1 wrote.
constexpr int PC_KS = 8;  // segments per lane (PC_KS * 64 >= the most segments of a row)

template <typename T>
__global__ __launch_bounds__(WAVE) void k_piece_count(LongArgs<T> a, int64_t npieces) {
  constexpr int NWORDS = (1 << kPieceCountLog) / 32;
  constexpr int MAXSEG = PC_KS * WAVE;
  __shared__ uint32_t bm[NWORDS];
  __shared__ int32_t pre[MAXSEG];  // start of each segment's part in the range's stream
  __shared__ int32_t src[MAXSEG];  // its first entry in the row's partials
  const int ln = lane();
  const int64_t pid = xcd_block_id<16>();
  if (pid >= npieces) return;
  const int32_t lri = a.piece_lrow[pid];
  const LongRow lr = a.lrows[lri];
  if (lr.nseg <= 1 || lr.shift > kPieceCountLog || lr.nseg > MAXSEG) return;  // (host rules out)
  const int32_t b = static_cast<int32_t>(pid - lr.piece0);
  const int64_t c0 = static_cast<int64_t>(b) << lr.shift;
  const int64_t width64 = (int64_t(1) << lr.shift) < (a.ncols - c0) ? (int64_t(1) << lr.shift)
                                                                   : (a.ncols - c0);
  const int nwords = static_cast<int>((width64 + 31) >> 5);
  for (int q = ln; q < nwords; q += WAVE) bm[q] = 0u;
  const int32_t nseg = lr.nseg;
  const GLOBAL_AS int32_t *lo_row = as_global(a.split + lr.sbase + static_cast<int64_t>(b) * nseg);
  const GLOBAL_AS int32_t *hi_row = as_global(a.split + lr.sbase + static_cast<int64_t>(b + 1) * nseg);
  const GLOBAL_AS int32_t *pcol = as_global(a.pcol + lr.pbase);
  // every segment's bounds in one round trip (lane p: segments p*KS ..),
  // then the parts laid end to end by one scan
  int32_t slo[PC_KS], slen[PC_KS];
#pragma unroll
  for (int j = 0; j < PC_KS; ++j) {
    const int32_t sg = ln * PC_KS + j;
    const int32_t sc = sg < nseg ? sg : nseg - 1;
    slo[j] = lo_row[sc];
    slen[j] = hi_row[sc];
  }
  int32_t tot_len = 0;
#pragma unroll
  for (int j = 0; j < PC_KS; ++j) {
    const bool in = ln * PC_KS + j < nseg;
    const int32_t lo = in ? max(slo[j], 0) : 0;
    slen[j] = in ? max(slen[j] - lo, 0) : 0;
    slo[j] = lo;
    tot_len += slen[j];
  }
  const int32_t incl = group_incl_sum<WAVE>(tot_len);
  const int32_t E = __shfl(incl, WAVE - 1, WAVE);
  {
    int32_t run = incl - tot_len;
#pragma unroll
    for (int j = 0; j < PC_KS; ++j) {
      const int32_t sg = ln * PC_KS + j;
      if (sg < nseg) {
        pre[sg] = run;
        src[sg] = static_cast<int32_t>(static_cast<int64_t>(sg) * lr.segp + slo[j]);
      }
      run += slen[j];
    }
  }
  wave_sync();
  // lanes on consecutive entries of the stream, four at a time; the entry's
  // part is the last one starting at or before it
  for (int32_t x0 = 0; x0 < E; x0 += 4 * WAVE) {
    int32_t c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t x = x0 + u * WAVE + ln;
      const int32_t xc = x < E ? x : E - 1;
      int lo = 0, hi = nseg - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= xc)
          lo = mid;
        else
          hi = mid - 1;
      }
      c[u] = pcol[src[lo] + (xc - pre[lo])];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (x0 + u * WAVE + ln < E) {
        const uint32_t x = static_cast<uint32_t>(c[u] - c0);
        atomicOr(&bm[x >> 5], 1u << (x & 31));
      }
    }
  }
  wave_sync();
  int64_t cnt = 0;
  for (int q = ln; q < nwords; q += WAVE) cnt += __popc(bm[q]);
  cnt = __shfl(static_cast<long long>(group_incl_sum<WAVE>(cnt)), WAVE - 1, WAVE);
  if (ln == 0) {
    Piece pc;
    pc.col = nullptr;
    pc.val = nullptr;
    pc.cnt = cnt;
    pc.lrow = lri;
    pc.pad = 0;
    a.pieces[pid] = pc;
  }
}

template <typename T>
void launch_piece_count(const LongArgs<T> &a, int64_t npieces, hipStream_t s) {
  if (npieces <= 0) return;
  hipLaunchKernelGGL((k_piece_count<T>), dim3(npieces), dim3(WAVE), 0, s, a, npieces);
}

bool long_direct_ok(const LongParams &lp, int64_t ncols) {
  if (lp.segp < 0) return false;
  // rows are split only above max(segp, single) products; the range width
  // shrinks as u grows
  const int64_t umin = std::max<int64_t>(lp.segp, lp.single) + 1;
  const int64_t w = (ncols * lp.cb + umin - 1) / umin;
  int32_t shift = ceil_log2_i64(w > 1 ? w : 1);
  if (shift < lp.minw_shift) shift = lp.minw_shift;
  if (shift > lp.maxw_shift) shift = lp.maxw_shift;
  return shift <= kPieceCountLog && lp.maxs <= PC_KS * WAVE;
}

template void launch_piece_count<float>(const LongArgs<float> &, int64_t, hipStream_t);
template void launch_piece_count<double>(const LongArgs<double> &, int64_t, hipStream_t);

}  // namespace spg
