// Merge-algorithm microbenchmark (Section 3.2, Fig. 5): the five ways of
// merging two sorted sequences of length l in scratchpad memory that the
// paper compares before choosing merge path for its long-row kernels.
//
// A work-group takes a tile of consecutive pairs (tile = max(2l, 2 x its
// thread count) entries), loads it from HBM into LDS with coalesced loads,
// merges every pair in LDS with one algorithm, and stores the tile back.
// Keys are 32-bit unsigned; each key may carry a 32- or 64-bit value.
//
//  * ranking merge: every element finds its rank in the other sequence by
//    binary search (lower bound from the first sequence, upper bound from
//    the second, so ties keep the first sequence first) and is written to a
//    second LDS buffer (out of place);
//  * merge path: every thread owns a run of consecutive outputs, finds where
//    its run starts in both inputs by a binary search along the cross
//    diagonal of the merge grid, merges its run into registers and writes
//    it back in place after a barrier (stable);
//  * odd-even merge: the last merging network of Batcher's odd-even merge
//    sort (compare i with i + l, then for k = l/2 .. 1 the pairs
//    (j + i, j + i + k) with j = k, 3k, 5k, ..), one barrier per stage;
//  * bitonic merge: compare i with 2l - 1 - i (which turns two ascending
//    runs into a bitonic sequence), then half-cleaners i, i + k for
//    k = l/2 .. 1, one barrier per stage;
//  * advanced bitonic merge: the same network, but after the first stage
//    every thread loads 8 entries that three consecutive half-cleaner stages
//    combine only among themselves, runs those stages in registers and
//    writes back, so three stages cost one LDS round trip and one barrier.
//
// The networks are not stable: entries with equal keys may leave in either
// order.  l must be a power of two for every algorithm here.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace spg {

template <int VB> struct MergeVal {
  using type = typename std::conditional<VB == 8, uint64_t, uint32_t>::type;
};

constexpr int MERGE_PATH_EMAX = 32;  // outputs per thread held in registers

template <int VB> struct Tile {
  uint32_t *k;
  typename MergeVal<VB>::type *v;
  DEVI void swap_if(int64_t a, int64_t b) {
    const uint32_t ka = k[a], kb = k[b];
    if (kb < ka) {
      k[a] = kb;
      k[b] = ka;
      if constexpr (VB != 0) {
        const auto va = v[a];
        v[a] = v[b];
        v[b] = va;
      }
    }
  }
};

// lower bound (upper = false: first position with key >= x) or upper bound
// (upper = true: first position with key > x) in s[0 .. n)
DEVI int64_t bound(const uint32_t *s, int64_t n, uint32_t x, bool upper) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (s[mid] < x || (upper && s[mid] == x))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <int ALG, int VB>
__global__ __launch_bounds__(1024) void k_merge(const uint32_t *kin, const void *vin,
                                                uint32_t *kout, void *vout, int64_t l,
                                                int64_t total, int64_t tile) {
  using V = typename MergeVal<VB>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nt = blockDim.x, t = threadIdx.x;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * tile;
  const int64_t valid = total - base < tile ? total - base : tile;
  const int64_t two_l = 2 * l;
  Tile<VB> s;
  s.k = reinterpret_cast<uint32_t *>(smem);
  s.v = reinterpret_cast<V *>(smem + ((tile * 4 + 15) & ~int64_t(15)));
  const GLOBAL_AS uint32_t *gk = as_global(kin);
  const GLOBAL_AS V *gv = as_global(static_cast<const V *>(vin));
  for (int64_t e = t; e < valid; e += nt) {
    s.k[e] = gk[base + e];
    if constexpr (VB != 0) s.v[e] = gv[base + e];
  }
  // entries past the last pair take the largest key: they stay in place
  for (int64_t e = valid + t; e < tile; e += nt) s.k[e] = 0xffffffffu;
  __syncthreads();
  // source of the final store (the ranking merge writes elsewhere)
  const uint32_t *ok = s.k;
  const V *ov = s.v;

  if constexpr (ALG == SPGEMM_MERGE_RANKING) {
    uint32_t *rk = reinterpret_cast<uint32_t *>(
        smem + ((tile * 4 + 15) & ~int64_t(15)) + (VB ? ((tile * VB + 15) & ~int64_t(15)) : 0));
    V *rv = reinterpret_cast<V *>(reinterpret_cast<unsigned char *>(rk) +
                                  ((tile * 4 + 15) & ~int64_t(15)));
    for (int64_t e = t; e < tile; e += nt) {
      const int64_t p0 = e / two_l * two_l, q = e - p0;
      const uint32_t x = s.k[e];
      int64_t o;
      if (q < l)
        o = q + bound(s.k + p0 + l, l, x, false);
      else
        o = (q - l) + bound(s.k + p0, l, x, true);
      rk[p0 + o] = x;
      if constexpr (VB != 0) rv[p0 + o] = s.v[e];
    }
    __syncthreads();
    ok = rk;
    ov = rv;
  } else if constexpr (ALG == SPGEMM_MERGE_PATH) {
    const int64_t per = tile / nt;  // outputs of this thread (<= MERGE_PATH_EMAX)
    const int64_t d0 = t * per;
    const int64_t p0 = d0 / two_l * two_l, d = d0 - p0;
    const uint32_t *a = s.k + p0, *b = s.k + p0 + l;
    // split of diagonal d: ai entries of a and d - ai of b come first
    int64_t lo = d > l ? d - l : 0, hi = d < l ? d : l;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (a[mid] <= b[d - 1 - mid])
        lo = mid + 1;
      else
        hi = mid;
    }
    int64_t ai = lo, bi = d - lo;
    uint32_t rk[MERGE_PATH_EMAX];
    V rv[MERGE_PATH_EMAX];
#pragma unroll
    for (int x = 0; x < MERGE_PATH_EMAX; ++x) {
      if (x < per) {
        const bool take_a = bi >= l || (ai < l && a[ai] <= b[bi]);
        const int64_t src = take_a ? p0 + ai : p0 + l + bi;
        rk[x] = s.k[src];
        if constexpr (VB != 0) rv[x] = s.v[src];
        ai += take_a ? 1 : 0;
        bi += take_a ? 0 : 1;
      }
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < MERGE_PATH_EMAX; ++x) {
      if (x < per) {
        s.k[d0 + x] = rk[x];
        if constexpr (VB != 0) s.v[d0 + x] = rv[x];
      }
    }
    __syncthreads();
  } else if constexpr (ALG == SPGEMM_MERGE_ODDEVEN) {
    const int64_t ncmp = tile / 2;  // l comparators per pair and stage
    for (int64_t c = t; c < ncmp; c += nt) {
      const int64_t p0 = c / l * two_l, i = c % l;
      s.swap_if(p0 + i, p0 + i + l);
    }
    for (int64_t k = l / 2; k >= 1; k /= 2) {
      __syncthreads();
      for (int64_t c = t; c < ncmp; c += nt) {
        const int64_t p0 = c / l * two_l, ci = c % l;
        if (ci < l - k) {
          const int64_t lo = k + 2 * k * (ci / k) + ci % k;
          s.swap_if(p0 + lo, p0 + lo + k);
        }
      }
    }
    __syncthreads();
  } else {  // bitonic, plain or register-local
    const int64_t ncmp = tile / 2;
    for (int64_t c = t; c < ncmp; c += nt) {
      const int64_t p0 = c / l * two_l, i = c % l;
      s.swap_if(p0 + i, p0 + two_l - 1 - i);
    }
    int64_t k = l / 2;
    if constexpr (ALG == SPGEMM_MERGE_BITONIC_ADV) {
      // groups of three stages (strides k, k/2, k/4) on 8 entries per thread
      for (; k >= 4; k /= 8) {
        __syncthreads();
        const int64_t q = k / 4;  // smallest stride of the group
        for (int64_t g = t; g < tile / 8; g += nt) {
          // insert three zero bits at the stride bits of g
          const int64_t low = g % q, high = g / q;
          const int64_t e0 = high * (8 * q) + low;
          uint32_t kk[8];
          V vv[8];
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            kk[m] = s.k[e0 + m * q];
            if constexpr (VB != 0) vv[m] = s.v[e0 + m * q];
          }
#pragma unroll
          for (int st = 4; st >= 1; st /= 2) {
#pragma unroll
            for (int m = 0; m < 8; ++m) {
              if ((m & st) == 0 && kk[m + st] < kk[m]) {
                const uint32_t tk = kk[m];
                kk[m] = kk[m + st];
                kk[m + st] = tk;
                if constexpr (VB != 0) {
                  const V tv = vv[m];
                  vv[m] = vv[m + st];
                  vv[m + st] = tv;
                }
              }
            }
          }
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            s.k[e0 + m * q] = kk[m];
            if constexpr (VB != 0) s.v[e0 + m * q] = vv[m];
          }
        }
      }
    }
    for (; k >= 1; k /= 2) {
      __syncthreads();
      for (int64_t c = t; c < ncmp; c += nt) {
        const int64_t lo = (c / k) * 2 * k + c % k;
        s.swap_if(lo, lo + k);
      }
    }
    __syncthreads();
  }

  GLOBAL_AS uint32_t *gko = as_global_mut(kout);
  GLOBAL_AS V *gvo = as_global_mut(static_cast<V *>(vout));
  for (int64_t e = t; e < valid; e += nt) {
    gko[base + e] = ok[e];
    if constexpr (VB != 0) gvo[base + e] = ov[e];
  }
}

namespace {

size_t merge_lds_bytes(int alg, int vb, int64_t tile) {
  const size_t one = ((static_cast<size_t>(tile) * 4 + 15) & ~size_t(15)) +
                     (vb ? ((static_cast<size_t>(tile) * vb + 15) & ~size_t(15)) : 0);
  return alg == SPGEMM_MERGE_RANKING ? 2 * one : one;
}

template <int ALG, int VB>
hipError_t launch_merge(const uint32_t *kin, const void *vin, uint32_t *kout, void *vout,
                        int64_t l, int64_t pairs, int nt, int64_t tile, size_t lds,
                        hipStream_t s) {
  const auto fn = k_merge<ALG, VB>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds));
  if (e != hipSuccess) return e;
  const int64_t total = 2 * l * pairs;
  const int64_t nb = (total + tile - 1) / tile;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(nb)), dim3(nt), lds, s, kin, vin, kout, vout,
                     l, total, tile);
  return hipGetLastError();
}

template <int ALG>
hipError_t launch_vb(int vb, const uint32_t *kin, const void *vin, uint32_t *kout, void *vout,
                     int64_t l, int64_t pairs, int nt, int64_t tile, size_t lds, hipStream_t s) {
  switch (vb) {
    case 0: return launch_merge<ALG, 0>(kin, vin, kout, vout, l, pairs, nt, tile, lds, s);
    case 4: return launch_merge<ALG, 4>(kin, vin, kout, vout, l, pairs, nt, tile, lds, s);
    default: return launch_merge<ALG, 8>(kin, vin, kout, vout, l, pairs, nt, tile, lds, s);
  }
}

}  // namespace
}  // namespace spg

extern "C" int spgemm_merge_pairs(int algorithm, int value_bytes, int64_t l, int64_t pairs,
                                  int threads, const uint32_t *keys_in, const void *vals_in,
                                  uint32_t *keys_out, void *vals_out, void *stream) {
  using namespace spg;
  if (algorithm < SPGEMM_MERGE_RANKING || algorithm > SPGEMM_MERGE_BITONIC_ADV) {
    set_last_error("unknown merge algorithm");
    return SPGEMM_EINVAL;
  }
  if (value_bytes != 0 && value_bytes != 4 && value_bytes != 8) {
    set_last_error("value_bytes must be 0, 4 or 8");
    return SPGEMM_EINVAL;
  }
  if (l < 1 || l > (int64_t(1) << 20) || (l & (l - 1)) != 0 || pairs < 0) {
    set_last_error("l must be a power of two in [1, 2^20] and pairs >= 0");
    return SPGEMM_EINVAL;
  }
  if (threads < 64 || threads > 1024 || (threads & (threads - 1)) != 0) {
    set_last_error("threads must be a power of two in [64, 1024]");
    return SPGEMM_EINVAL;
  }
  if (pairs == 0) return SPGEMM_OK;
  if (!keys_in || !keys_out || (value_bytes && (!vals_in || !vals_out))) {
    set_last_error("NULL array");
    return SPGEMM_EINVAL;
  }
  if (2 * l * pairs >= (int64_t(1) << 40)) {
    set_last_error("too many entries");
    return SPGEMM_EOVERFLOW;
  }
  const int64_t tile = 2 * l > 2 * threads ? 2 * l : 2 * static_cast<int64_t>(threads);
  if ((2 * l * pairs + tile - 1) / tile > INT32_MAX) {
    set_last_error("too many work-groups for one launch");
    return SPGEMM_EOVERFLOW;
  }
  if (algorithm == SPGEMM_MERGE_PATH && tile / threads > MERGE_PATH_EMAX) {
    set_last_error("merge path holds at most 32 outputs per thread: use more threads");
    return SPGEMM_EINVAL;
  }
  const size_t lds = merge_lds_bytes(algorithm, value_bytes, tile);
  if (lds > 160 * 1024) {
    set_last_error("the tile does not fit in LDS (160 KB)");
    return SPGEMM_EINVAL;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  switch (algorithm) {
    case SPGEMM_MERGE_RANKING:
      e = launch_vb<SPGEMM_MERGE_RANKING>(value_bytes, keys_in, vals_in, keys_out, vals_out, l,
                                          pairs, threads, tile, lds, s);
      break;
    case SPGEMM_MERGE_PATH:
      e = launch_vb<SPGEMM_MERGE_PATH>(value_bytes, keys_in, vals_in, keys_out, vals_out, l,
                                       pairs, threads, tile, lds, s);
      break;
    case SPGEMM_MERGE_ODDEVEN:
      e = launch_vb<SPGEMM_MERGE_ODDEVEN>(value_bytes, keys_in, vals_in, keys_out, vals_out, l,
                                          pairs, threads, tile, lds, s);
      break;
    case SPGEMM_MERGE_BITONIC:
      e = launch_vb<SPGEMM_MERGE_BITONIC>(value_bytes, keys_in, vals_in, keys_out, vals_out, l,
                                          pairs, threads, tile, lds, s);
      break;
    default:
      e = launch_vb<SPGEMM_MERGE_BITONIC_ADV>(value_bytes, keys_in, vals_in, keys_out, vals_out,
                                              l, pairs, threads, tile, lds, s);
      break;
  }
  if (e != hipSuccess) {
    set_last_error(std::string("merge launch: ") + hipGetErrorString(e));
    return SPGEMM_EHIP;
  }
  return SPGEMM_OK;
}
