// Device building blocks shared by the SpGEMM kernels: wavefront and
// work-group scans, cross-lane exchange, and bitonic sorting networks laid
// out for 64-wide wavefronts (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEVI __device__ __forceinline__

namespace spg {

constexpr int WAVE = 64;

DEVI int lane() { return static_cast<int>(__lane_id()); }

// Orders the LDS accesses of one wavefront (no work-group barrier): for
// data that only the lanes of one wavefront share.
DEVI void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A pointer known to address global memory (one read back from memory or
// LDS is generic, and generic loads are also counted with the LDS
// operations, which makes later LDS reads wait for them).
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T> DEVI const GLOBAL_AS T *as_global(const T *p) {
  return (const GLOBAL_AS T *)p;
}
template <typename T> DEVI GLOBAL_AS T *as_global_mut(T *p) { return (GLOBAL_AS T *)p; }

// Work-groups are dealt to the 8 XCDs (each with its own L2) in turn.  This
// maps the hardware order to a logical one in which every XCD receives runs
// of C consecutive logical ids (the runs themselves dealt in turn), so that
// neighbouring work, which shares cache lines, stays in one L2 while uneven
// work is still spread over all XCDs.  A bijection on [0, gridDim.x): the
// last partial round of 8 C work-groups keeps the hardware order.
constexpr int kNumXcd = 8;
template <int C> DEVI int64_t xcd_block_id() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t full = nb / (kNumXcd * C) * (kNumXcd * C);
  if (b >= full) return b;
  const int64_t x = b % kNumXcd, i = b / kNumXcd;
  return (i / C) * (kNumXcd * C) + x * C + (i % C);
}

// ---------------------------------------------------------------- shuffles

// Value of lane (lane ^ m).  With m known at compile time, masks 1, 2, 3, 7,
// 8 and 15 are DPP moves inside the VALU (quad permutations, the mirror of
// each half row of 8 and of each row of 16 lanes, a rotation of each row by
// 8), 4, 16 and 31 are LDS-unit swizzles inside groups of 32 lanes (no
// address operand), others go through ds_bpermute.
DEVI uint32_t shfl_xor_u32(uint32_t v, int m) {
  const int x = static_cast<int>(v);
  switch (m) {
    case 1: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));
    case 2: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));
    case 3: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x1B, 0xF, 0xF, false));
    case 7: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false));
    case 8: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false));
    case 15: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false));
    case 4: return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(x, 0x1F | (4 << 10)));
    case 16: return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(x, 0x1F | (16 << 10)));
    case 31: return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(x, 0x1F | (31 << 10)));
    default: return static_cast<uint32_t>(__shfl_xor(x, m, WAVE));
  }
}
DEVI uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = shfl_xor_u32(static_cast<uint32_t>(v), m);
  const uint32_t hi = shfl_xor_u32(static_cast<uint32_t>(v >> 32), m);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}
template <typename K> DEVI K shfl_xor_key(K v, int m);
template <> DEVI uint32_t shfl_xor_key<uint32_t>(uint32_t v, int m) { return shfl_xor_u32(v, m); }
template <> DEVI uint64_t shfl_xor_key<uint64_t>(uint64_t v, int m) { return shfl_xor_u64(v, m); }

template <typename K> DEVI K shfl_key(K v, int src);
template <> DEVI uint32_t shfl_key<uint32_t>(uint32_t v, int src) {
  return static_cast<uint32_t>(__shfl(static_cast<int>(v), src, WAVE));
}
template <> DEVI uint64_t shfl_key<uint64_t>(uint64_t v, int src) {
  return static_cast<uint64_t>(__shfl(static_cast<long long>(v), src, WAVE));
}

// DPP move of a 32- or 64-bit value: lanes whose source is outside the
// pattern, and lanes of rows left out by ROWMASK, receive `id`.
template <int CTRL, int ROWMASK, typename V> DEVI V dpp_move(V x, V id) {
  static_assert(sizeof(V) == 4 || sizeof(V) == 8, "32- or 64-bit values");
  if constexpr (sizeof(V) == 4) {
    return __builtin_bit_cast(V, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, id),
                                                             __builtin_bit_cast(int, x), CTRL,
                                                             ROWMASK, 0xF, false));
  } else {
    const uint64_t ux = __builtin_bit_cast(uint64_t, x), ui = __builtin_bit_cast(uint64_t, id);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
        static_cast<int>(ui), static_cast<int>(ux), CTRL, ROWMASK, 0xF, false));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
        static_cast<int>(ui >> 32), static_cast<int>(ux >> 32), CTRL, ROWMASK, 0xF, false));
    return __builtin_bit_cast(V, (static_cast<uint64_t>(hi) << 32) | lo);
  }
}
constexpr int DPP_ROW_SHR = 0x110;      // + n: lane i of a row of 16 reads lane i - n
constexpr int DPP_WAVE_SHR1 = 0x138;    // lane i reads lane i - 1 of the wavefront
constexpr int DPP_ROW_BCAST15 = 0x142;  // last lane of each row to the next row
constexpr int DPP_ROW_BCAST31 = 0x143;  // lane 31 to rows 2 and 3

constexpr int DPP_WAVE_SHL1 = 0x130;    // lane i reads lane i + 1 of the wavefront

// Value of lane (lane - 1); lane 0 receives `id`.
template <typename V> DEVI V wave_shr1(V x, V id) { return dpp_move<DPP_WAVE_SHR1, 0xF>(x, id); }
// Value of lane (lane + 1); lane 63 receives `id`.
template <typename V> DEVI V wave_shl1(V x, V id) { return dpp_move<DPP_WAVE_SHL1, 0xF>(x, id); }

template <typename K> DEVI K shfl_up_key(K v, int d) {
  if (d == 1) return wave_shr1<K>(v, K(0));
  if constexpr (sizeof(K) == 4)
    return static_cast<K>(__shfl_up(static_cast<int>(v), d, WAVE));
  else
    return static_cast<K>(__shfl_up(static_cast<long long>(v), d, WAVE));
}

// ------------------------------------------------------------- group scans
// Scans over aligned groups of G consecutive lanes (G a power of two <= 64),
// as DPP shifts inside rows of 16 lanes and broadcasts across rows.

template <int G, typename V, typename Op> DEVI V group_incl_scan(V x, V id, Op op) {
  const int lg = lane() & (G - 1);
  if constexpr (G >= 2) {
    const V y = dpp_move<DPP_ROW_SHR + 1, 0xF>(x, id);
    x = op(x, (G >= 16 || lg >= 1) ? y : id);
  }
  if constexpr (G >= 4) {
    const V y = dpp_move<DPP_ROW_SHR + 2, 0xF>(x, id);
    x = op(x, (G >= 16 || lg >= 2) ? y : id);
  }
  if constexpr (G >= 8) {
    const V y = dpp_move<DPP_ROW_SHR + 4, 0xF>(x, id);
    x = op(x, (G >= 16 || lg >= 4) ? y : id);
  }
  if constexpr (G >= 16) x = op(x, dpp_move<DPP_ROW_SHR + 8, 0xF>(x, id));
  if constexpr (G >= 32) x = op(x, dpp_move<DPP_ROW_BCAST15, 0xA>(x, id));
  if constexpr (G >= 64) x = op(x, dpp_move<DPP_ROW_BCAST31, 0xC>(x, id));
  return x;
}

template <int G, typename V> DEVI V group_incl_sum(V x) {
  return group_incl_scan<G, V>(x, V(0), [](V a, V b) { return a + b; });
}

template <int G> DEVI int group_incl_max(int x) {
  return group_incl_scan<G, int>(x, INT32_MIN, [](int a, int b) { return a > b ? a : b; });
}

// Value held by the last lane of the group.
template <int G, typename V> DEVI V group_last(V x) {
  return __shfl(x, (lane() & ~(G - 1)) + G - 1, WAVE);
}

// Work-group exclusive sum of one value per thread.  `smem` holds NT/64 + 1
// entries.  Returns the exclusive prefix; `total` receives the block sum.
// Contains barriers: every thread of the block must call it.
template <int NT, typename V> DEVI V block_excl_sum(V x, V *smem, V &total) {
  constexpr int NW = NT / WAVE;
  V inc = group_incl_sum<WAVE>(x);
  const int w = threadIdx.x / WAVE;
  if (lane() == WAVE - 1) smem[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    V run = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      V t = smem[i];
      smem[i] = run;
      run += t;
    }
    smem[NW] = run;
  }
  __syncthreads();
  V res = smem[w] + inc - x;
  total = smem[NW];
  __syncthreads();
  return res;
}

// Work-group inclusive max of one int per thread (same contract).
template <int NT> DEVI int block_incl_max(int x, int *smem) {
  constexpr int NW = NT / WAVE;
  int inc = group_incl_max<WAVE>(x);
  const int w = threadIdx.x / WAVE;
  if (lane() == WAVE - 1) smem[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = -1;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      int t = smem[i];
      smem[i] = run;
      run = max(run, t);
    }
  }
  __syncthreads();
  int res = max(smem[w], inc);
  __syncthreads();
  return res;
}

// Work-group exclusive max of one int per thread: max over threads < t, or
// -1 for thread 0.  `smem` holds NT/64 ints.  Contains barriers.
template <int NT> DEVI int block_excl_max(int x, int *smem) {
  constexpr int NW = NT / WAVE;
  const int inc = group_incl_max<WAVE>(x);
  const int w = threadIdx.x / WAVE;
  if (lane() == WAVE - 1) smem[w] = inc;
  int prev = wave_shr1(inc, -1);
  if (lane() == 0) prev = -1;
  __syncthreads();
  int before = -1;
#pragma unroll
  for (int i = 0; i < NW; ++i)
    if (i < w) before = max(before, smem[i]);
  __syncthreads();
  return max(before, prev);
}

// ------------------------------------------------------------ bitonic sort
// Keys are held K per lane in "blocked" order: lane position p (0..G-1 in its
// group, or the thread index for the work-group version) holds elements
// p*K .. p*K+K-1.  Sorting is ascending.  Strides below K are exchanged in
// registers, strides up to K*G through cross-lane shuffles.

template <typename Key> DEVI void cas_pair(Key &a, Key &b, bool asc) {
  Key lo = a < b ? a : b;
  Key hi = a < b ? b : a;
  a = asc ? lo : hi;
  b = asc ? hi : lo;
}

// One bitonic stage (size, stride) on register-resident keys, strides < K.
template <int K, typename Key>
DEVI void stage_regs(Key (&k)[K], int pos, int size, int stride) {
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int p = kk ^ stride;
    if (p > kk) {
      const int i = pos * K + kk;
      cas_pair(k[kk], k[p], (i & size) == 0);
    }
  }
}

// One stage with stride >= K: partner lane differs by stride/K.
template <int K, typename Key>
DEVI void stage_lanes(Key (&k)[K], int pos, int size, int stride) {
  const int pm = stride / K;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int i = pos * K + kk;
    Key other = shfl_xor_key<Key>(k[kk], pm);
    const bool asc = (i & size) == 0;
    const bool lower = (i & stride) == 0;
    const bool take_min = (asc == lower);
    Key mn = k[kk] < other ? k[kk] : other;
    Key mx = k[kk] < other ? other : k[kk];
    k[kk] = take_min ? mn : mx;
  }
}

// The same network with every comparison ascending: each merge of two
// sorted halves of a block of `size` starts by comparing element i with its
// mirror i ^ (size - 1) (which leaves two bitonic halves, every key of the
// first at most every key of the second), then halves them with strides
// size/4 .. 1.  No comparison depends on a lane's block direction, so the
// register stages need no selects and the lane stages one per key.
template <int K, typename Key> DEVI void cas_asc(Key &a, Key &b) {
  const Key lo = a < b ? a : b;
  const Key hi = a < b ? b : a;
  a = lo;
  b = hi;
}

// Partner kk ^ M in registers (M < K), the lower index keeping the minimum.
template <int K, int M, typename Key> DEVI void flip_regs(Key (&k)[K]) {
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int p = kk ^ M;
    if (p > kk) cas_asc<K, Key>(k[kk], k[p]);
  }
}

// The key a lane keeps from (own, partner's): the minimum in the lower lane,
// the maximum in the upper.  For 32-bit keys that is the median of the two
// and a per-lane bound (0 in the lower lane, all ones in the upper), one
// VALU instruction instead of min, max and a select.
template <typename Key> DEVI Key keep_of(Key own, Key other, bool lower, Key bound) {
  if constexpr (sizeof(Key) == 4) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(own), "v"(other), "v"(bound));
    return r;
  } else {
    const Key mn = own < other ? own : other;
    const Key mx = own < other ? other : own;
    return lower ? mn : mx;
  }
}

// STRIDE >= K: partner lane pos ^ (STRIDE / K), same register.
template <int K, int STRIDE, typename Key> DEVI void half_lanes(Key (&k)[K], int pos) {
  constexpr int PM = STRIDE / K;
  const bool lower = (pos & PM) == 0;
  const Key bound = lower ? Key(0) : ~Key(0);
#pragma unroll
  for (int kk = 0; kk < K; ++kk)
    k[kk] = keep_of<Key>(k[kk], shfl_xor_key<Key>(k[kk], PM), lower, bound);
}

// Mirror of a block of SIZE >= 2K: partner lane pos ^ (SIZE / K - 1),
// register K - 1 - kk.
template <int K, int SIZE, typename Key> DEVI void mirror_lanes(Key (&k)[K], int pos) {
  constexpr int PM = SIZE / K - 1;
  const bool lower = (pos & (SIZE / (2 * K))) == 0;
  const Key bound = lower ? Key(0) : ~Key(0);
  if constexpr (K == 1) {  // the register is its own mirror
    k[0] = keep_of<Key>(k[0], shfl_xor_key<Key>(k[0], PM), lower, bound);
    return;
  }
  // registers kk and K - 1 - kk trade partners: two at a time, so that only
  // two received keys are live at once
#pragma unroll
  for (int kk = 0; kk < K / 2; ++kk) {
    const Key oa = shfl_xor_key<Key>(k[K - 1 - kk], PM);
    const Key ob = shfl_xor_key<Key>(k[kk], PM);
    k[kk] = keep_of<Key>(k[kk], oa, lower, bound);
    k[K - 1 - kk] = keep_of<Key>(k[K - 1 - kk], ob, lower, bound);
  }
}

// The halving stages STRIDE, STRIDE / 2, .. 1 of one merge.
template <int K, int STRIDE, typename Key> DEVI void half_stages(Key (&k)[K], int pos) {
  if constexpr (STRIDE > 0) {
    if constexpr (STRIDE < K)
      flip_regs<K, STRIDE, Key>(k);
    else
      half_lanes<K, STRIDE, Key>(k, pos);
    half_stages<K, STRIDE / 2, Key>(k, pos);
  }
}

// Merges of blocks of SIZE, 2 SIZE, .. N (each instantiated, so that every
// stride and partner is a constant).
template <int N, int K, int SIZE, typename Key> DEVI void merges_from(Key (&k)[K], int pos) {
  if constexpr (SIZE <= N) {
    if constexpr (SIZE <= K)
      flip_regs<K, SIZE - 1, Key>(k);
    else
      mirror_lanes<K, SIZE, Key>(k, pos);
    half_stages<K, SIZE / 4, Key>(k, pos);
    merges_from<N, K, SIZE * 2, Key>(k, pos);
  }
}

// Sort G*K keys held by an aligned group of G lanes (G <= 64).
template <int G, int K, typename Key> DEVI void group_bitonic_sort(Key (&k)[K]) {
  merges_from<G * K, K, 2, Key>(k, lane() & (G - 1));
}

// Sort NT*K keys held by a work-group of NT threads.  Strides that cross
// wavefronts go through `lds` (NT*K keys, layout [kk][thread] so that the
// exchange is bank-conflict free).  Contains barriers.
template <int NT, int K, typename Key> DEVI void block_bitonic_sort(Key (&k)[K], Key *lds) {
  constexpr int N = NT * K;
  const int t = threadIdx.x;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride < K) {
        stage_regs<K, Key>(k, t, size, stride);
      } else if (stride < K * WAVE) {
        stage_lanes<K, Key>(k, t, size, stride);
      } else {
        const int pt = t ^ (stride / K);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < K; ++kk) lds[kk * NT + t] = k[kk];
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
          const int i = t * K + kk;
          Key other = lds[kk * NT + pt];
          const bool asc = (i & size) == 0;
          const bool lower = (i & stride) == 0;
          const bool take_min = (asc == lower);
          Key mn = k[kk] < other ? k[kk] : other;
          Key mx = k[kk] < other ? other : k[kk];
          k[kk] = take_min ? mn : mx;
        }
      }
    }
  }
  __syncthreads();
}

template <typename T> struct KeyMax;
template <> struct KeyMax<uint32_t> { static constexpr uint32_t v = 0xffffffffu; };
template <> struct KeyMax<uint64_t> { static constexpr uint64_t v = 0xffffffffffffffffull; };

template <int B> struct Log2 { static constexpr int v = 1 + Log2<B / 2>::v; };
template <> struct Log2<1> { static constexpr int v = 0; };

// Folds a tile sorted on (column, stream index) and held by an aligned group
// of G lanes: rank pos*K + kk (pos = lane in the group) is key[kk], the
// product of stream index s is pv[s].  Every run of equal
// columns is summed in rank order from +0.0 -- the sequential sum of
// Gustavson's method -- in registers; a run that crosses into the next lane
// continues from that lane's left neighbour's running sum.  The results go,
// in column order, to the LDS staging arrays sc (column + cbase) and sv,
// which may overlap the key buffer and pv; returns their number.  Only
// wavefront-level ordering is used.
template <typename T, int G, int K, typename Key>
DEVI int fold_runs(const Key (&key)[K], const int tn, const T *pv, int32_t *sc, T *sv,
                   const int32_t cbase) {
  constexpr int U = G * K;
  constexpr int LOGU = Log2<U>::v;
  constexpr Key KMAX = KeyMax<Key>::v;
  const int pos = lane() & (G - 1);
  const Key pk = shfl_up_key<Key>(key[K - 1], 1);  // rank pos*K - 1
  const Key nk = wave_shl1<Key>(key[0], KMAX);     // rank pos*K + K
  uint32_t hmask = 0, tmask = 0;
  int nt = 0;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int l = pos * K + kk;
    const Key c = key[kk] >> LOGU;
    const Key before = kk > 0 ? key[kk - 1] : pk;
    const Key after = kk + 1 < K ? key[kk + 1] : nk;
    const bool valid = l < tn;
    const bool head = valid && (l == 0 || (before >> LOGU) != c);
    const bool tail = valid && (l + 1 == tn || (after >> LOGU) != c);
    hmask |= head ? (1u << kk) : 0u;
    tmask |= tail ? (1u << kk) : 0u;
    nt += tail ? 1 : 0;
  }
  // running sum over this lane's ranks, restarting at every head, from cin
  auto run_from = [&](T run) {
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const T v = pv[static_cast<int>(key[kk] & (U - 1))];
      run = (hmask & (1u << kk)) ? T(0) + v : run + v;
    }
    return run;
  };
  // a lane whose first rank continues a run starts from the left
  // neighbour's final running sum: that is final once the neighbour has a
  // head of its own or has received its start (rank 0 always starts a run,
  // so this ends; values shifted in from another group are never used)
  const bool cont0 = pos * K < tn && !(hmask & 1u);
  T last = run_from(T(0));
  T cin = T(0);
  bool have = !cont0;
  bool last_ok = have || hmask != 0u;
  while (__any(!have)) {
    const T left = wave_shr1<T>(last, T(0));
    const int left_ok = wave_shr1<int>(last_ok ? 1 : 0, 1);
    if (!have && left_ok) {
      cin = left;
      last = run_from(cin);
      have = true;
      last_ok = true;
    }
  }
  const int incl_t = group_incl_sum<G>(nt);
  const int r = group_last<G>(incl_t);
  // final pass: tails take their run's sum (all pv reads precede the
  // staging writes, which may overwrite pv)
  T tv[K];
  {
    T run = cin;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const T v = pv[static_cast<int>(key[kk] & (U - 1))];
      run = (hmask & (1u << kk)) ? T(0) + v : run + v;
      tv[kk] = run;
    }
  }
  wave_sync();
  int o = incl_t - nt;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    if (tmask & (1u << kk)) {
      sc[o] = cbase + static_cast<int32_t>(key[kk] >> LOGU);
      sv[o] = tv[kk];
      ++o;
    }
  }
  wave_sync();
  return r;
}

// Values are summed without fused multiply-add (the library is compiled with
// -ffp-contract=off), products first rounded, then added in sequence order.

}  // namespace spg
