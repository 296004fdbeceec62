// Work-group radix sorting of packed 32-bit keys in LDS, for the long-row
// kernels.  Keys are (column offset << LOGT) | position; sorting is stable
// on a bit field of the key, so equal fields keep position order, which is
// the expansion (sequence) order of the products.
//
// Ranking is done per wavefront with ballots: for every 64 consecutive
// elements, the lanes holding the same digit are found by intersecting one
// ballot per digit bit; the lowest such lane bumps the wavefront's counter
// of that digit by the group size, and every lane's rank is the counter
// value plus the number of equal-digit lanes below it.  Counters are kept
// per (digit, wavefront); an exclusive scan in digit-major order gives every
// (digit, wavefront) pair its output offset.  Element e of the sequence is
// handled by wavefront e / (64 KT), iteration (e / 64) mod KT, lane e mod 64,
// so the scan order equals the sequence order (the sort is stable).
#pragma once

#include "common.hpp"

namespace spg {

// Work-group minimum and maximum of one int per thread.  `smem` holds
// 2 * (NT / 64) ints.  Contains barriers: every thread must call it.
template <int NT> DEVI void block_minmax(int &mn, int &mx, int *smem) {
  constexpr int NW = NT / WAVE;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    mn = min(mn, __shfl_xor(mn, o, WAVE));
    mx = max(mx, __shfl_xor(mx, o, WAVE));
  }
  const int w = threadIdx.x / WAVE;
  if (lane() == 0) {
    smem[w] = mn;
    smem[NW + w] = mx;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    mn = min(mn, smem[i]);
    mx = max(mx, smem[NW + i]);
  }
  __syncthreads();
}

// Number of bits needed to hold values 0..x (0 for x <= 0).
DEVI int bit_width(uint32_t x) { return x == 0 ? 0 : 32 - __clz(static_cast<int>(x)); }

// Exclusive scan in place of c[0 .. len), len <= NT * CPT, by the work-group.
// Contains barriers.
template <int NT, int CPT> DEVI void block_scan_counts(uint32_t *c, int len, int64_t *smem) {
  const int b = threadIdx.x * CPT;
  uint32_t loc[CPT];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    loc[j] = b + j < len ? c[b + j] : 0u;
    s += loc[j];
  }
  int64_t tot;
  uint32_t run = static_cast<uint32_t>(block_excl_sum<NT>(static_cast<int64_t>(s), smem, tot));
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    if (b + j < len) c[b + j] = run;
    run += loc[j];
  }
}

// LDS counters of one pass: (1 << RB) digits per wavefront.
template <int NT, int RB> struct RadixCounters {
  static constexpr int count = (1 << RB) * (NT / WAVE);
};

// One stable counting pass: src[0 .. n) -> dst, ordered by digit(key) in
// [0, 1 << rb), rb <= RB.  `cnt` holds RadixCounters<NT, RB>::count words.
// Contains barriers.
template <int NT, int KT, int RB, typename DigitFn>
DEVI void radix_pass(const uint32_t *src, uint32_t *dst, const int n, const int rb,
                     DigitFn digit, uint32_t *cnt, int64_t *smem) {
  constexpr int NW = NT / WAVE;
  constexpr int CPT = (RadixCounters<NT, RB>::count + NT - 1) / NT;
  const int w = threadIdx.x / WAVE;
  const int ln = lane();
  const int nc = (1 << rb) * NW;
  for (int i = threadIdx.x; i < nc; i += NT) cnt[i] = 0u;
  __syncthreads();
  const uint64_t below_mask = ln == 0 ? 0ull : (~0ull >> (WAVE - ln));
  uint32_t key[KT];
  int dig[KT];
  int rk[KT];
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int e0 = (w * KT + kk) * WAVE;
    const int e = e0 + ln;
    const bool v = e < n;
    key[kk] = v ? src[e] : 0u;
    const int d = v ? digit(key[kk]) : 0;
    dig[kk] = d;
    rk[kk] = 0;
    if (e0 < n) {  // uniform across the wavefront
      uint64_t m = __ballot(v);
      for (int b = 0; b < rb; ++b) {
        const bool bit = (d >> b) & 1;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
      }
      const int leader = v ? static_cast<int>(__builtin_ctzll(m)) : ln;
      int base = 0;
      if (v && ln == leader) {
        base = static_cast<int>(cnt[d * NW + w]);
        cnt[d * NW + w] = static_cast<uint32_t>(base + __popcll(m));
      }
      base = __shfl(base, leader, WAVE);
      rk[kk] = base + __popcll(m & below_mask);
    }
  }
  __syncthreads();
  block_scan_counts<NT, CPT>(cnt, nc, smem);
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < KT; ++kk) {
    const int e = (w * KT + kk) * WAVE + ln;
    if (e < n) dst[cnt[dig[kk] * NW + w] + rk[kk]] = key[kk];
  }
  __syncthreads();
}

// Stable LSD sort of a[0 .. n) on field(key), a value of `bits` bits, in
// passes of at most RB bits; `b` is scratch of the same size.  Returns the
// buffer that holds the result.  `bits` must be uniform across the
// work-group.  Contains barriers.
template <int NT, int KT, int RB, typename FieldFn>
DEVI uint32_t *radix_sort(uint32_t *a, uint32_t *b, const int n, const int bits, FieldFn field,
                          uint32_t *cnt, int64_t *smem) {
  if (bits <= 0 || n <= 1) return a;
  const int passes = (bits + RB - 1) / RB;
  const int rb0 = (bits + passes - 1) / passes;
  int done = 0;
  for (int p = 0; p < passes; ++p) {
    const int rb = min(rb0, bits - done);
    const int sh = done;
    const uint32_t mask = (1u << rb) - 1u;
    radix_pass<NT, KT, RB>(
        a, b, n, rb, [&](uint32_t k) { return static_cast<int>((field(k) >> sh) & mask); }, cnt,
        smem);
    uint32_t *t = a;
    a = b;
    b = t;
    done += rb;
  }
  return a;
}

}  // namespace spg
