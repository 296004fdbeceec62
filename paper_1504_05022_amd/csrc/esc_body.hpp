// Expand-sort-compress of up to G*K products per row by an aligned group of
// G lanes of a wavefront (K products per lane), shared by the per-bin
// kernels and the batched per-class kernels.  See esc.hip.
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace spg {

constexpr int ESC_NT = 256;

template <typename T, int G, int K, typename Key> struct EscShape {
  static constexpr int U = G * K;
  static constexpr int RPB = ESC_NT / G;  // rows per work-group pass
  static constexpr int KB = sizeof(Key) > 4 ? static_cast<int>(sizeof(Key)) : 4;
  static constexpr size_t a_bytes = static_cast<size_t>(RPB) * U * KB;
  static constexpr size_t lds_bytes = a_bytes + static_cast<size_t>(RPB) * U * sizeof(T);
};

// One pass of a work-group over the rows rows[base .. base + RPB) (those
// below nrows).  A row's G lanes never leave their wavefront (G <= 64) and
// its LDS is its own, so only wavefront-level ordering is needed: the
// wavefronts of a work-group do not wait for each other.  LDS per row: region A holds the run starts (int32 index
// into B's arrays, -1 = none) and later the sorted keys; region B holds a_ij
// of each run and later the product values.  A group's lanes share one
// wavefront, so all reads of the first use precede the writes of the second
// in program order.
template <typename T, int G, int K, typename Key>
DEVI void esc_rows(const EscArgs<T> &a, const int32_t *rows, const int64_t base,
                   const int64_t nrows, unsigned char *lds) {
  using Sh = EscShape<T, G, K, Key>;
  constexpr int U = Sh::U;
  constexpr int LOGU = Log2<U>::v;
  constexpr int KB = Sh::KB;
  constexpr Key KMAX = KeyMax<Key>::v;
  const int grp = threadIdx.x / G;
  const int pos = threadIdx.x & (G - 1);
  int32_t *rs = reinterpret_cast<int32_t *>(lds + grp * U * KB);
  Key *sk = reinterpret_cast<Key *>(lds + grp * U * KB);
  T *ra = reinterpret_cast<T *>(lds + Sh::a_bytes) + grp * U;
  T *pv = ra;
  // element l of a row lives at (l mod K) * G + l / K: the K elements of a
  // lane are G apart, so lanes touch consecutive words (no bank conflicts)
  constexpr int LOGK = Log2<K>::v;
  auto ix = [](int l) { return (l & (K - 1)) * G + (l >> LOGK); };
  // every array is in global memory (the batched kernel reads these
  // pointers from memory, which would otherwise make them generic)
  const GLOBAL_AS int64_t *gu = as_global(a.u);
  const GLOBAL_AS int32_t *garp = as_global(a.arp);
  const GLOBAL_AS int64_t *gP = as_global(a.P);
  const GLOBAL_AS int32_t *gacol = as_global(a.acol);
  const GLOBAL_AS T *gaval = as_global(a.aval);
  const GLOBAL_AS int32_t *gbrp = as_global(a.brp);
  const GLOBAL_AS int32_t *gbcol = as_global(a.bcol);
  const GLOBAL_AS T *gbval = as_global(a.bval);
  const GLOBAL_AS int64_t *gcto = as_global(a.cto);
  GLOBAL_AS int32_t *gct_col = as_global_mut(a.ct_col);
  GLOBAL_AS T *gct_val = as_global_mut(a.ct_val);
  GLOBAL_AS int64_t *grownnz = as_global_mut(a.rownnz);
  const int64_t r = base + grp;
  const int32_t i = r < nrows ? as_global(rows)[r] : 0;
  // rows of this launch have u <= U by binning; the check keeps every LDS
  // and global index in range even if that were violated
  const bool act = r < nrows && gu[i] <= U;
  const int u = act ? static_cast<int>(gu[i]) : 0;
  const int32_t e0 = act ? garp[i] : 0;
  const int32_t e1 = act ? garp[i + 1] : 0;
  const int64_t pbase = act ? gP[e0] : 0;

#pragma unroll
  for (int kk = 0; kk < K; ++kk) rs[kk * G + pos] = -1;
  wave_sync();
  // run starts: entry e of row i contributes products [P[e]-P[e0], P[e+1]-P[e0]);
  // the loads of G entries are issued together (clamped, not branched on)
  for (int32_t eb = e0; eb < e1; eb += G) {
    const int32_t e = eb + pos;
    const bool in = e < e1;
    const int32_t ec = in ? e : e1 - 1;
    const int64_t q0 = gP[ec], q1 = gP[ec + 1];
    const int32_t j = gacol[ec];
    const T av = gaval[ec];
    if (in && q1 > q0) {
      rs[ix(static_cast<int>(q0 - pbase))] = gbrp[j];
      ra[ix(static_cast<int>(q0 - pbase))] = av;
    }
  }
  wave_sync();

  // segmented max-scan: the run containing product l starts at s(l)
  int st[K];
  int run = -1;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = pos * K + kk;
    const int f = (l < u && rs[ix(l)] >= 0) ? l : -1;
    run = max(run, f);
    st[kk] = run;
  }
  const int incl = group_incl_max<G>(run);
  int prev = wave_shr1(incl, -1);
  if (pos == 0) prev = -1;

  // B index and a_ij of every product, resolved in this lane-blocked order
  // and handed over through LDS, so that the gather below reads consecutive
  // products with consecutive lanes (coalesced loads along each b_j* row)
  int32_t gbx[K];
  T gav[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = pos * K + kk;
    const int s0 = max(prev, st[kk]);
    const bool ok = l < u && s0 >= 0;
    gbx[kk] = ok ? rs[ix(s0)] + (l - s0) : 0;
    gav[kk] = ok ? ra[ix(s0)] : T(0);
  }
  int32_t *gb = rs;  // product l at gb[l] / ga[l]
  T *ga = ra;
  wave_sync();
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = pos * K + kk;
    if (l < u) {
      gb[l] = gbx[kk];
      ga[l] = gav[kk];
    }
  }
  wave_sync();
  // every load of the row is issued before any is used: positions past the
  // end load B's entry 0 (a row with products implies that B has one) and
  // are then ignored
  int32_t bc[K];
  T bv[K], av[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    bc[kk] = 0;
    bv[kk] = T(0);
    av[kk] = T(0);
  }
  if (u > 0) {
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int l = kk * G + pos;
      const int32_t g = gb[l];
      const int32_t bidx = l < u ? g : 0;
      av[kk] = ga[l];
      bc[kk] = gbcol[bidx];
      bv[kk] = gbval[bidx];
    }
  }
  Key key[K];
  T prod[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = kk * G + pos;
    const bool ok = l < u;
    prod[kk] = ok ? av[kk] * bv[kk] : T(0);
    key[kk] = ok ? ((static_cast<Key>(bc[kk]) << LOGU) | static_cast<Key>(l)) : KMAX;
  }
  wave_sync();  // pv takes the place of ga
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = kk * G + pos;
    if (l < u) pv[l] = prod[kk];
  }

  group_bitonic_sort<G, K, Key>(key);
  wave_sync();  // every product is in pv

  // compress: fold every column's products in expansion order (registers),
  // stage the distinct columns in LDS, store them with consecutive lanes
  int32_t *sc = reinterpret_cast<int32_t *>(sk);
  const int total = fold_runs<T, G, K, Key>(key, act ? u : 0, pv, sc, pv, 0);
  if (act) {
    const int64_t o = gcto[i];
    for (int x = pos; x < total; x += G) {
      gct_col[o + x] = sc[x];
      gct_val[o + x] = pv[x];
    }
    if (pos == 0) grownnz[i] = total;
  }
  wave_sync();
}

}  // namespace spg
