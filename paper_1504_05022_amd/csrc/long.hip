// Stage 3 for long rows (bin group 5, u > 512 by default): the merge method
// of Section 3.1.  One work-group owns a work item (a long row, or a range
// of its products) and inserts its products into a sorted, duplicate-free
// result sequence:
//
//  * products are taken in expansion order in tiles of TILE; every tile is
//    sorted on (column, expansion position) and its products are folded per
//    column;
//  * every distinct column of the tile is binary-searched in the level-1
//    sequence L1 held in LDS: found columns are fused in place (the running
//    value continues with the tile's products in order), missing ones are
//    tagged, compacted with a prefix sum and merged into L1 with merge path;
//  * before a tile could overflow L1, L1 is merged into the item's global
//    sequence G (merge path again, fusing columns present in both), which
//    lives in blocks carved from a device pool and grows 2x at a time
//    (progressive allocation);
//  * when the pool is exhausted the item records a checkpoint (the product
//    position right after its last successful spill, with L1 empty, and G)
//    and quits; the host grows the pool and relaunches the failed items,
//    which resume from their checkpoints;
//  * at the end L1 is merged into G once more, or, if G was never used,
//    written to the row's 256-entry C~ slot or a pool block.
//
// Values of items that never spill are Gustavson's sequential sums exactly;
// spilled items add two partial sums per column (rounding may differ).
#include "common.hpp"
#include "internal.hpp"

namespace spg {

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

// Shared state of a work-group, broadcast through LDS.
template <typename T> struct LongShared {
  int64_t scan[16];
  int32_t imax[16];
  int32_t *zcol;
  T *zval;
  int64_t zcap;
  int32_t ok;
  int32_t next_first;
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

template <typename T, int NT, int TILE, int L1CAP, typename Key>
__global__ __launch_bounds__(NT) void k_long(LongArgs<T> a) {
  constexpr int KT = TILE / NT;        // products per thread per tile
  constexpr int LOGT = Log2<TILE>::v;
  constexpr int EO = (L1CAP + NT - 1) / NT;  // L1 entries per thread in the L1 merge
  constexpr Key KMAX = KeyMax<Key>::v;
  constexpr int KB = sizeof(Key) > 4 ? static_cast<int>(sizeof(Key)) : 4;

  __shared__ int32_t l1c[L1CAP];
  __shared__ T l1v[L1CAP];
  // region A: run starts (int32) / sort scratch and sorted keys / new columns
  __shared__ __align__(16) unsigned char s_a[TILE * KB];
  // region B: a_ij of each run / product values / new values
  __shared__ __align__(16) T s_b[TILE];
  __shared__ LongShared<T> sh;

  int32_t *rs = reinterpret_cast<int32_t *>(s_a);
  Key *sk = reinterpret_cast<Key *>(s_a);
  int32_t *ncol = reinterpret_cast<int32_t *>(s_a);
  T *ra = s_b;
  T *pv = s_b;
  T *nval = s_b;

  const int t = threadIdx.x;
  const int32_t item_id = a.work ? a.work[blockIdx.x] : static_cast<int32_t>(blockIdx.x);
  const LongItem item = a.items[item_id];
  LongState st = a.state[item_id];
  const int32_t i = item.row;
  const int32_t e0 = a.e.arp[i];
  const int32_t e1 = a.e.arp[i + 1];
  const int64_t pbase = a.e.P[e0];
  const int64_t p1 = item.p1;
  int64_t pos = st.pos;
  int64_t last_clean = pos;
  int r = 0;  // entries in L1

  // entry containing product `pos`: the last e with P[e] <= pbase + pos
  if (t == 0) {
    int32_t lo = e0, hi = e1;  // search in [e0, e1)
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

  // Merge L1 into G (into the spare block or a new 2x block); false if the
  // pool is exhausted (G unchanged).
  auto spill = [&]() -> bool {
    const int64_t need = st.gcnt + r;
    if (t == 0) {
      sh.ok = 1;
      if (st.scap >= need) {
        sh.zcol = st.scol;
        sh.zval = reinterpret_cast<T *>(st.sval);
        sh.zcap = st.scap;
      } else {
        int64_t cap = st.gcap * 2;
        if (cap < a.long_slot) cap = a.long_slot;
        while (cap < need) cap *= 2;
        int32_t *zc = nullptr;
        T *zv = nullptr;
        if (pool_alloc<T>(a.pool, static_cast<uint64_t>(cap), zc, zv)) {
          sh.zcol = zc;
          sh.zval = zv;
          sh.zcap = cap;
        } else {
          sh.ok = 0;
        }
      }
    }
    __syncthreads();
    if (!sh.ok) return false;
    int32_t *zc = sh.zcol;
    T *zv = sh.zval;
    const int64_t zcap = sh.zcap;
    const int64_t z = merge_fuse<NT, 8, T>(st.gcol, reinterpret_cast<const T *>(st.gval),
                                           st.gcnt, l1c, l1v, r, zc, zv, sh.scan);
    // the old G becomes the spare block
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
  };

  while (pos < p1) {
    if (r + TILE > L1CAP) {
      if (!spill()) {
        failed = true;
        break;
      }
      r = 0;
      last_clean = pos;
    }
    const int tn = static_cast<int>(p1 - pos < TILE ? p1 - pos : TILE);

    // ---- expansion: run starts of the entries overlapping [pos, pos+tn)
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) rs[t * KT + kk] = -1;
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
        rs[ls] = a.e.brp[j] + off;
        ra[ls] = a.e.aval[e];
      }
    }
    __syncthreads();
    e_first = sh.next_first;

    int st_run[KT];
    int run = -1;
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = t * KT + kk;
      const int f = (l < tn && rs[l] >= 0) ? l : -1;
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
        const int32_t bidx = rs[s0] + (l - s0);
        const T av = ra[s0];
        const int32_t c = a.e.bcol[bidx];
        const T bv = a.e.bval[bidx];
        prod[kk] = av * bv;
        key[kk] = (static_cast<Key>(c) << LOGT) | static_cast<Key>(l);
      }
    }
    __syncthreads();  // all reads of rs / ra done
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = t * KT + kk;
      if (l < tn) pv[l] = prod[kk];
    }
    block_bitonic_sort<NT, KT, Key>(key, sk);
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) sk[t * KT + kk] = key[kk];
    __syncthreads();

    // ---- fold every column of the tile, continuing L1's running value
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
        const bool head = (l == 0) || ((sk[l - 1] >> LOGT) != c);
        if (head) {
          const int32_t col = static_cast<int32_t>(c);
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
          v = v + pv[static_cast<int>(key[kk] & (TILE - 1))];
          for (int l2 = l + 1; l2 < tn; ++l2) {
            const Key k2 = sk[l2];
            if ((k2 >> LOGT) != c) break;
            v = v + pv[static_cast<int>(k2 & (TILE - 1))];
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
    int o = static_cast<int>(block_excl_sum<NT>(static_cast<int64_t>(nn), sh.scan, qtot));
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

    // ---- merge path of L1 (r) and the new columns (q) back into L1
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
    pos += tn;
  }

  // ---- final placement of the result
  int32_t *dcol = nullptr;
  T *dval = nullptr;
  int64_t cnt = 0;
  if (!failed) {
    if (st.gcnt == 0) {
      if (t == 0) {
        sh.ok = 1;
        if (r <= a.long_slot && item.part == 0 && item.p0 == 0 && item.p1 == a.e.u[i]) {
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
        for (int x = t; x < r; x += NT) {
          dcol[x] = l1c[x];
          dval[x] = l1v[x];
        }
        cnt = r;
      } else {
        failed = true;
      }
    } else {
      if (r > 0 && !spill()) {
        failed = true;
      } else {
        dcol = st.gcol;
        dval = reinterpret_cast<T *>(st.gval);
        cnt = st.gcnt;
      }
    }
  }

  if (failed) {
    // checkpoint: resume at the last position where L1 was empty, with G as
    // it was then (G only changes in a successful spill)
    if (t == 0) {
      st.pos = last_clean;
      st.status = 1;
      a.state[item_id] = st;
      const unsigned int k = atomicAdd(&a.pool->fail_count, 1u);
      a.fail_list[k] = static_cast<unsigned int>(item_id);
    }
    return;
  }
  if (t == 0) {
    st.pos = p1;
    st.status = 0;
    a.state[item_id] = st;
    a.e.rownnz[i] = cnt;
    a.rsrc_col[i] = dcol;
    a.rsrc_val[i] = dval;
  }
}

// Initial checkpoints: every item starts at its first product with empty G.
__global__ void k_long_init(const LongItem *items, LongState *state, int64_t n) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= n) return;
  LongState s;
  s.pos = items[x].p0;
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

int long_l1cap_default(int dtype_bytes) { return dtype_bytes == 8 ? 5120 : 7168; }

template <typename T, int L1CAP>
static void launch_cfg(const LongArgs<T> &a, int64_t nwork, int64_t ncols, hipStream_t s) {
  constexpr int NT = 256, TILE = 1024;
  if ((static_cast<uint64_t>(ncols) << Log2<TILE>::v) <= 0xffffffffull)
    hipLaunchKernelGGL((k_long<T, NT, TILE, L1CAP, uint32_t>), dim3(nwork), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_long<T, NT, TILE, L1CAP, uint64_t>), dim3(nwork), dim3(NT), 0, s, a);
}

template <typename T>
int launch_long(const LongArgs<T> &a, int64_t nwork, int64_t ncols, int l1cap, hipStream_t s) {
  if (nwork <= 0) return 0;
  switch (l1cap) {
    case 2048: launch_cfg<T, 2048>(a, nwork, ncols, s); break;
    case 3072: launch_cfg<T, 3072>(a, nwork, ncols, s); break;
    case 5120: launch_cfg<T, 5120>(a, nwork, ncols, s); break;
    case 7168: launch_cfg<T, 7168>(a, nwork, ncols, s); break;
    default: return -1;
  }
  return 0;
}

void launch_long_init(const LongItem *items, LongState *state, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_long_init, dim3((n + 255) / 256), dim3(256), 0, s, items, state, n);
}

// One work item per long row: the rows of bin 37 in the (stable) bin list.
__global__ void k_long_items(const int32_t *binlist, int64_t off, int64_t n, const int64_t *u,
                             LongItem *items) {
  const int64_t x = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const int32_t row = binlist[off + x];
  LongItem it;
  it.row = row;
  it.part = 0;
  it.p0 = 0;
  it.p1 = u[row];
  items[x] = it;
}

void launch_long_items(const int32_t *binlist, int64_t off, int64_t n, const int64_t *u,
                       LongItem *items, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_long_items, dim3((n + 255) / 256), dim3(256), 0, s, binlist, off, n, u,
                     items);
}

template int launch_long<float>(const LongArgs<float> &, int64_t, int64_t, int, hipStream_t);
template int launch_long<double>(const LongArgs<double> &, int64_t, int64_t, int, hipStream_t);

}  // namespace spg
