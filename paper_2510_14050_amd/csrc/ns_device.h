// Device-side building blocks shared by the libns kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ns {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Decoupled look-back words: status in the top two bits, value in the low 62.
// A tile first publishes its own aggregate (AGG), then, once it knows the sum
// of everything before it, its inclusive prefix (INC). Readers spin on a word
// until its status is non-zero. Status and value share one 64-bit word, so a
// relaxed agent-scope atomic is enough: no other data hangs on the flag.
// Tiles are handed out by an atomic ticket, so every tile a reader waits on
// belongs to a workgroup that is already running.
// ---------------------------------------------------------------------------
constexpr uint64_t kLbAgg = 1ull << 62;
constexpr uint64_t kLbInc = 2ull << 62;
constexpr uint64_t kLbVal = (1ull << 62) - 1;

template <typename T>
__device__ __forceinline__ void lb_store(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T lb_load(const T *p) {
  return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The radix passes' per-digit words come in two widths. 64-bit: status in the
// top two bits as above. 32-bit, for passes over fewer than 2^31 - 1 keys
// (half the look-back traffic): 0 = not yet published, bit 31 = inclusive,
// bits 0..30 = value + 1.
template <typename W>
struct LbWord {
  static __device__ __forceinline__ W agg(uint64_t v) { return kLbAgg | v; }
  static __device__ __forceinline__ W inc(uint64_t v) { return kLbInc | v; }
  static __device__ __forceinline__ bool ready(W w) { return (w >> 62) != 0; }
  static __device__ __forceinline__ bool inclusive(W w) { return (w >> 62) == 2; }
  static __device__ __forceinline__ uint64_t value(W w) { return w & kLbVal; }
};
template <>
struct LbWord<uint32_t> {
  static __device__ __forceinline__ uint32_t agg(uint64_t v) { return (uint32_t)v + 1u; }
  static __device__ __forceinline__ uint32_t inc(uint64_t v) { return 0x80000000u | ((uint32_t)v + 1u); }
  static __device__ __forceinline__ bool ready(uint32_t w) { return w != 0; }
  static __device__ __forceinline__ bool inclusive(uint32_t w) { return (w >> 31) != 0; }
  static __device__ __forceinline__ uint64_t value(uint32_t w) { return (w & 0x7FFFFFFFu) - 1u; }
};

// ---------------------------------------------------------------------------
// wave / block helpers
// Scans and reductions over the 64 lanes use DPP, which moves values between
// lanes inside the VALU (no LDS round trip): row shifts by 1, 2, 4 and 8 scan
// each row of 16 lanes, then the last lane of row 0 is broadcast into row 1
// and of row 2 into row 3 (row_bcast:15), and lane 31 into rows 2 and 3
// (row_bcast:31). Lanes whose source is outside the row, and rows left out by
// the row mask, read 0. Every caller has all 64 lanes active.
// ---------------------------------------------------------------------------
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, true);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
  const uint32_t lo = dpp32<CTRL, ROW_MASK>((uint32_t)x);
  const uint32_t hi = dpp32<CTRL, ROW_MASK>((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp_mv(T v) {
  if constexpr (sizeof(T) == 8) return dpp64<CTRL, ROW_MASK>(v);
  else return dpp32<CTRL, ROW_MASK>(v);
}

// inclusive scan of x over lanes 0..lane with an associative op whose
// identity is 0 (sum, max of unsigned values)
template <typename T, typename Op>
__device__ __forceinline__ T wave_scan_dpp(T x, Op op) {
  x = op(x, dpp_mv<kDppRowShr1, 0xf>(x));
  x = op(x, dpp_mv<kDppRowShr2, 0xf>(x));
  x = op(x, dpp_mv<kDppRowShr4, 0xf>(x));
  x = op(x, dpp_mv<kDppRowShr8, 0xf>(x));
  x = op(x, dpp_mv<kDppRowBcast15, 0xa>(x));
  x = op(x, dpp_mv<kDppRowBcast31, 0xc>(x));
  return x;
}

__device__ __forceinline__ uint64_t lane63(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
  return wave_scan_dpp<uint64_t>(x, [](uint64_t a, uint64_t b) { return a + b; });
}

__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t x) {
  return wave_scan_dpp<uint32_t>(x, [](uint32_t a, uint32_t b) { return a + b; });
}

// sum / maximum over the wave, returned in every lane
__device__ __forceinline__ uint64_t wave_sum(uint64_t x) { return lane63(wave_incl_scan(x)); }

__device__ __forceinline__ uint64_t wave_max(uint64_t x) {
  return lane63(wave_scan_dpp<uint64_t>(x, [](uint64_t a, uint64_t b) { return a > b ? a : b; }));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// number of set bits of m in lanes below this one
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Block-wide exclusive scan of one u64 per thread. s_tmp holds BLOCK/64
// entries. Returns the thread's exclusive prefix; *total = block sum.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *s_tmp, uint64_t *total) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const uint64_t x = wave_incl_scan(v);
  if (lane == kWave - 1) s_tmp[wv] = x;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < BLOCK / kWave; ++q) {
    const uint64_t s = s_tmp[q];
    pre += (q < wv) ? s : 0;
    tot += s;
  }
  *total = tot;
  __syncthreads();
  return pre + x - v;
}

// Load of a table that no kernel of the current launch writes (segment and
// tile offsets), through the constant address space: with a uniform address
// the compiler issues a scalar load, which completes on its own counter
// instead of waiting behind the wave's outstanding vector loads and stores.
__device__ __forceinline__ uint64_t ld_const(const uint64_t *p) {
  return *(const __attribute__((address_space(4))) uint64_t *)(p);
}

// Index of the segment that owns tile t: the last w with off[w] <= t (empty
// segments own no tiles, so this is never an empty one). Binary search; with t
// uniform (in scalar registers) its loads are scalar and mostly hit the scalar
// cache.
__device__ __forceinline__ uint32_t find_owner(const uint64_t *off, uint32_t W, uint64_t t) {
  uint32_t lo = 0, hi = W;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (ld_const(off + mid) <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// The same owner, searched from the proportional guess t*W/total (total =
// off[W] > t): galloping out from the guess brackets the answer, then a
// binary search narrows the bracket. Segments of about equal length take two
// loads; a guess d segments off takes about 2 log2 d.
__device__ __forceinline__ uint32_t find_owner_near(const uint64_t *off, uint32_t W, uint64_t total,
                                                    uint64_t t) {
  uint64_t lo, hi;  // off[lo] <= t < off[hi] (hi == W stands for +infinity)
  uint64_t g = t * W / total;
  if (g >= W) g = W - 1;
  if (ld_const(off + g) <= t) {
    lo = g;
    for (uint64_t s = 1;; s <<= 1) {
      const uint64_t c = lo + s;
      if (c >= W) { hi = W; break; }
      if (ld_const(off + c) > t) { hi = c; break; }
      lo = c;
    }
  } else {
    hi = g;  // off[0] == 0 <= t, so this ends
    for (uint64_t s = 1;; s <<= 1) {
      const uint64_t c = hi > s ? hi - s : 0;
      if (ld_const(off + c) <= t) { lo = c; break; }
      hi = c;
    }
  }
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (ld_const(off + mid) <= t) lo = mid; else hi = mid;
  }
  return (uint32_t)lo;
}

// The same owner, searched by a whole wave (all 64 lanes active, t uniform)
// where t is not known to be uniform: each round probes 64 evenly spaced
// entries of the remaining range, so W segments take ceil(log64 W) dependent
// loads instead of log2 W. off is nondecreasing, so the probes with
// off[p] <= t form a prefix of the lanes (lane 0, at the low end, always
// belongs to it).
__device__ __forceinline__ uint32_t find_owner_wave(const uint64_t *off, uint32_t W, uint64_t t) {
  const uint64_t lane = threadIdx.x & (kWave - 1);
  uint64_t lo = 0, hi = W;  // answer in [lo, hi), off[lo] <= t
  while (hi - lo > 1) {
    const uint64_t step = (hi - lo + kWave - 1) / kWave;
    const uint64_t p = lo + step * lane;
    const uint64_t m = ballot64(p < hi && off[p] <= t);
    const uint64_t f = 63 - __clzll((long long)m);  // highest probe at or below t
    hi = min(lo + step * (f + 1), hi);
    lo += step * f;
  }
  return (uint32_t)lo;
}

// Exclusive prefix of channel `chan` for tile t: the sum of the values of
// tiles t-1, t-2, ... back to and including the nearest one that published
// an inclusive prefix (tile `first` always does). `stride` is the number of
// channels per tile. Up to P predecessor words are in flight per round trip
// (each thread issues the loads of tiles j, j-1, ..., j-P+1 together).
template <int P, typename W = uint64_t>
__device__ __forceinline__ uint64_t lb_walkn(const W *lb, uint32_t stride, uint32_t chan,
                                             uint32_t t, uint32_t first) {
  using L = LbWord<W>;
  uint64_t excl = 0;
  int64_t j = (int64_t)t - 1;
  while (j >= (int64_t)first) {
    W v[P];
#pragma unroll
    for (int q = 0; q < P; ++q)
      v[q] = (j - q >= (int64_t)first) ? lb_load(lb + (uint64_t)(j - q) * stride + chan) : W(0);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      if (j - q < (int64_t)first) return excl;
      const W *p = lb + (uint64_t)(j - q) * stride + chan;
      while (!L::ready(v[q])) {
        __builtin_amdgcn_s_sleep(1);
        v[q] = lb_load(p);
      }
      excl += L::value(v[q]);
      if (L::inclusive(v[q])) return excl;
    }
    j -= P;
  }
  return excl;
}

// Wave-parallel look-back over a single chain (all tiles 0..t-1): the 64 lanes
// of the calling wave inspect 64 predecessors at once, wait until every tile
// up to the nearest inclusive prefix has published, and add them up. One round
// trip covers 64 tiles instead of one. Every lane returns the same value; the
// whole wave must call it.
__device__ __forceinline__ uint64_t lb_walk_wave(const uint64_t *lb, uint32_t stride,
                                                 uint32_t chan, uint32_t t) {
  const int lane = threadIdx.x & 63;
  uint64_t excl = 0;
  int64_t top = (int64_t)t - 1;
  while (top >= 0) {
    const int64_t j = top - lane;
    const uint64_t *p = lb + (j >= 0 ? (uint64_t)j * stride + chan : 0);
    uint64_t v = (j >= 0) ? lb_load(p) : (2ull << 62);  // before tile 0: inclusive 0
    int first_inc;
    for (;;) {
      const uint64_t inc = __ballot((v >> 62) == 2);
      const uint64_t empty = __ballot((v >> 62) == 0);
      first_inc = inc ? __ffsll((long long)inc) - 1 : 64;
      const uint64_t need = first_inc >= 63 ? ~0ull : ((2ull << first_inc) - 1);
      if ((empty & need) == 0) break;
      if ((v >> 62) == 0) {
        __builtin_amdgcn_s_sleep(1);
        v = lb_load(p);
      }
    }
    excl += wave_sum(lane <= first_inc ? (v & kLbVal) : 0);
    if (first_inc < 64) break;
    top -= 64;
  }
  return excl;
}

__device__ __forceinline__ uint64_t pack_key(uint32_t s, uint32_t d) {
  return ((uint64_t)s << 32) | (uint64_t)d;
}

}  // namespace ns
