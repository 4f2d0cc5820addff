// HIP kernels of libns (gfx950, wave64): radix sort of packed (src,dst) keys,
// run-length encoding into a sorted COO traffic matrix, row and column run
// reductions for the eight quantities, and merge-path union-add.
//
// Every kernel that walks a data-dependent number of tiles is persistent: the
// grid is sized to what fits on the device, tiles are handed out by an atomic
// ticket, and the tile count is read from device memory. That makes the whole
// sequence capturable in one HIP graph and keeps the look-back waits safe
// (a waited-on tile always belongs to a running workgroup).
#include <hip/hip_ext.h>

#include <type_traits>

#include "ns_device.h"
#include "ns_launch.h"

#ifndef NS_LAYER_MAX_W
#define NS_LAYER_MAX_W 256  // most segments for layered ticket order
#endif
#ifndef NS_HIST_BLOCK
#define NS_HIST_BLOCK 512  // threads of a histogram workgroup
#endif
constexpr int kHistBlock = NS_HIST_BLOCK;
#ifndef NS_LB_DEPTH
#define NS_LB_DEPTH 4  // look-back words in flight per thread and round trip
#endif
// Debug builds (NS_BOUNDS_CHECK=1) check the index of every scatter and gather
// of the radix passes and run scans against its array's bound; an index
// outside raises bit 3 of the device error word and the access is skipped.
#ifndef NS_BOUNDS_CHECK
#define NS_BOUNDS_CHECK 0
#endif

namespace ns {

__device__ int g_status;  // bit 0: subtraction below zero; bit 1: a capacity (hash table, merge output) is exceeded; bit 2: an input breaks its stated order; bit 3: an index outside its array (debug builds)

// true when i < n; in debug builds, otherwise raises bit 3 of the error word
__device__ __forceinline__ bool in_bounds(uint64_t i, uint64_t n) {
#if NS_BOUNDS_CHECK
  if (i < n) return true;
  atomicOr(&g_status, 8);
  return false;
#else
  (void)i;
  (void)n;
  return true;
#endif
}

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__global__ void k_fill64(uint64_t *p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill32(uint32_t *p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_copy64(uint64_t *dst, const uint64_t *src, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Several fills in one launch (each region written with its own value).
__global__ void k_fill_multi(FillList f) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint32_t q = 0; q < f.count; ++q) {
    const FillEntry e = f.e[q];
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < e.n; i += stride) {
      if (e.wide) static_cast<uint64_t *>(e.p)[i] = e.v;
      else static_cast<uint32_t *>(e.p)[i] = (uint32_t)e.v;
    }
  }
}

// seg = {0, n}, with n read from the device when n_dev is given and clamped to
// the host-known bound `n` (a device count never drives accesses past it)
__global__ void k_seg1(uint64_t *seg, const uint64_t *n_dev, uint64_t n) {
  if (threadIdx.x == 0) {
    seg[0] = 0;
    seg[1] = n_dev ? min(*n_dev, n) : n;
  }
}

// Tile prefix per segment for up to three tile sizes, one workgroup.
__global__ __launch_bounds__(1024) void k_tiles(const uint64_t *seg_off, uint32_t W, uint32_t ta,
                                                uint64_t *oa, uint32_t tb, uint64_t *ob,
                                                uint32_t tc, uint64_t *oc) {
  __shared__ uint64_t s_tmp[16];
  __shared__ uint64_t s_max[16];
  uint64_t ca = 0, cb = 0, cc = 0, mx = 0;
  for (uint32_t base = 0; base < W; base += 1024) {
    const uint32_t w = base + threadIdx.x;
    const uint64_t len = (w < W) ? seg_off[w + 1] - seg_off[w] : 0;
    uint64_t tot;
    if (oa) {
      const uint64_t nt = (len + ta - 1) / ta;
      mx = mx > nt ? mx : nt;
      const uint64_t x = block_excl_scan<1024>(nt, s_tmp, &tot);
      if (w < W) oa[w] = ca + x;
      ca += tot;
    }
    if (ob) {
      const uint64_t x = block_excl_scan<1024>((len + tb - 1) / tb, s_tmp, &tot);
      if (w < W) ob[w] = cb + x;
      cb += tot;
    }
    if (oc) {
      const uint64_t x = block_excl_scan<1024>((len + tc - 1) / tc, s_tmp, &tot);
      if (w < W) oc[w] = cc + x;
      cc += tot;
    }
  }
  mx = wave_max(mx);
  if ((threadIdx.x & (kWave - 1)) == 0) s_max[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < 16; ++q) mx = mx > s_max[q] ? mx : s_max[q];
    if (oa) {
      oa[W] = ca;
      // layered ticket order (see pass_ticket) for a few segments of similar
      // length: at most a quarter of the tickets go to absent tiles. With many
      // segments, tile order keeps each segment's writes close in time, which
      // the memory-side cache merges into whole lines; 0 selects tile order.
      oa[W + 1] = (W > 1 && W <= NS_LAYER_MAX_W && (uint64_t)W * mx <= ca + ca / 4) ? mx : 0;
    }
    if (ob) ob[W] = cb;
    if (oc) oc[W] = cc;
  }
}

// ---------------------------------------------------------------------------
// Radix sort, step 1: byte-digit histograms of every key, per segment.
// Packets: digit p of key src<<32|dst is bits [8p, 8p+8): p<4 come from dst,
// p>=4 from src. Column items dst<<32|count: the 4 digits of dst. One launch
// counts the four digits of one 32-bit array (dst, src, or the items' high
// halves) into rows d0..d0+3 of each segment's histogram, so packets take two
// launches that each read one array (16-byte loads where the range allows).
// Each workgroup takes a contiguous range of tiles and counts into LDS; the
// counters go to the segment's global histogram (one atomic per non-zero bin)
// when the range crosses into the next segment, at its end, and every
// kHistFlushTiles tiles. The counters are the 16-bit halves of LDS words (the
// two digits 2j and 2j+1 share word j) in 32 copies, and lane l updates copy
// l % 32: whatever the digits, the 64 lanes of a wave hit every LDS bank
// exactly twice, so a heavy-tailed digit costs no more than a uniform one.
// Counting is bound by these LDS updates (four per value), not by the loads.
// ---------------------------------------------------------------------------
template <int BLOCK>
struct HistShape {
  static constexpr int kCopies = 32;
  static constexpr int kRows = 4 * kBins / 2;  // counter words per copy
  // most values one thread counts in a tile: its share of the 16-byte body,
  // plus one value of the unaligned head and one of the tail
  static constexpr uint32_t kPerThread = kHistTile / BLOCK + 2;
  // most increments of one half-word per tile: two lanes per wave use a copy
  static constexpr uint32_t kPerTile = 2 * (BLOCK / kWave) * kPerThread;
  static constexpr uint32_t kFlushTiles = 65535 / kPerTile;
  static_assert(kFlushTiles >= 1, "a tile could overflow a 16-bit counter");
};

template <int BLOCK, bool ITEMS64>
__global__ __launch_bounds__(BLOCK) void k_hist(const uint32_t *__restrict__ vals,
                                                const uint64_t *__restrict__ items,
                                                const uint64_t *seg_off, const uint64_t *tile_off,
                                                uint32_t W, uint32_t *hist, uint32_t row_stride,
                                                uint32_t d0) {
  using H = HistShape<BLOCK>;
  constexpr int C = H::kCopies, ROWS = H::kRows;
  __shared__ uint32_t s_h[ROWS * C];
  const uint64_t total = ld_const(tile_off + W);
  const uint64_t per = (total + gridDim.x - 1) / gridDim.x;
  const uint64_t t0 = (uint64_t)blockIdx.x * per, t1 = min(total, t0 + per);
  const uint32_t cp = threadIdx.x & (C - 1);
  for (int i = threadIdx.x; i < ROWS * C; i += BLOCK) s_h[i] = 0;
  __syncthreads();
  auto count = [&](uint32_t x) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t d = (x >> (8 * q)) & 255;
      atomicAdd(&s_h[(q * (kBins / 2) + (d >> 1)) * C + cp], 1u << (16 * (d & 1)));
    }
  };
  // workgroups start their flush at different rows, so the ones that finish
  // together do not queue on the same global counters
  const uint32_t rot = (blockIdx.x * 97u) % ROWS;
  auto flush = [&](uint32_t w) {
    uint32_t *g = hist + (uint64_t)w * row_stride + (uint64_t)d0 * kBins;
    for (int r0 = threadIdx.x; r0 < ROWS; r0 += BLOCK) {
      const int r = (r0 + rot) % ROWS;
      uint32_t lo = 0, hi = 0;
#pragma unroll 8
      for (int k = 0; k < C; ++k) {
        const int c = (k + r0) & (C - 1);  // neighbouring threads read different banks
        const uint32_t x = s_h[r * C + c];
        s_h[r * C + c] = 0;
        lo += x & 0xFFFFu;
        hi += x >> 16;
      }
      const int q = r / (kBins / 2), j = r % (kBins / 2);
      if (lo) atomicAdd(&g[q * kBins + 2 * j], lo);
      if (hi) atomicAdd(&g[q * kBins + 2 * j + 1], hi);
    }
  };
  uint32_t cur = t0 < t1 ? find_owner_wave(tile_off, W, t0) : 0, since = 0;
  for (uint64_t t = t0; t < t1; ++t) {
    uint32_t w = cur;  // tiles come in order: step over finished (and empty) segments
    while (ld_const(tile_off + w + 1) <= t) ++w;
    if (w != cur || since == H::kFlushTiles) {  // uniform: every thread sees the same tile
      __syncthreads();
      flush(cur);
      __syncthreads();
      cur = w;
      since = 0;
    }
    ++since;
    const uint64_t start = ld_const(seg_off + w) + (t - ld_const(tile_off + w)) * (uint64_t)kHistTile;
    const uint64_t end = min(start + (uint64_t)kHistTile, ld_const(seg_off + w + 1));
    if constexpr (ITEMS64) {
      constexpr int R = 8;  // values per thread per round, loads issued together
      for (uint64_t i0 = start + threadIdx.x; i0 < end; i0 += (uint64_t)R * BLOCK) {
        uint32_t v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const uint64_t i = i0 + (uint64_t)k * BLOCK;
          v[k] = i < end ? (uint32_t)(items[i] >> 32) : 0;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
          if (i0 + (uint64_t)k * BLOCK >= end) break;
          count(v[k]);
        }
      }
    } else {
      // [a, b): the 16-byte aligned body; at most three values before and after
      const uint64_t a =
          min(end, start + ((4 - ((reinterpret_cast<uintptr_t>(vals + start) >> 2) & 3)) & 3));
      const uint64_t b = a + ((end - a) & ~3ull);
      if (threadIdx.x < a - start) count(vals[start + threadIdx.x]);
      if (threadIdx.x < end - b) count(vals[b + threadIdx.x]);
      const uint4 *v4 = reinterpret_cast<const uint4 *>(vals + a);
      const uint64_t n4 = (b - a) / 4;
      constexpr int R = kHistTile / (4 * BLOCK) > 0 ? kHistTile / (4 * BLOCK) : 1;
      for (uint64_t j0 = threadIdx.x; j0 < n4; j0 += (uint64_t)R * BLOCK) {
        uint4 x[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const uint64_t j = j0 + (uint64_t)k * BLOCK;
          x[k] = j < n4 ? v4[j] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
          if (j0 + (uint64_t)k * BLOCK >= n4) break;
          count(x[k].x);
          count(x[k].y);
          count(x[k].z);
          count(x[k].w);
        }
      }
    }
  }
  __syncthreads();
  if (t0 < t1) flush(cur);
}

// Radix sort, step 2: exclusive scan of each 256-bin row (one wave per row).
__global__ __launch_bounds__(256) void k_hist_scan(const uint32_t *hist, uint32_t *base,
                                                   uint64_t rows) {
  const uint64_t row = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= rows) return;  // whole wave leaves together
  const uint32_t *h = hist + row * kBins;
  const uint32_t v0 = h[lane * 4 + 0], v1 = h[lane * 4 + 1], v2 = h[lane * 4 + 2],
                 v3 = h[lane * 4 + 3];
  const uint64_t mine = (uint64_t)v0 + v1 + v2 + v3;
  const uint64_t x = wave_incl_scan(mine) - mine;
  uint32_t *b = base + row * kBins;
  b[lane * 4 + 0] = (uint32_t)x;
  b[lane * 4 + 1] = (uint32_t)(x + v0);
  b[lane * 4 + 2] = (uint32_t)(x + v0 + v1);
  b[lane * 4 + 3] = (uint32_t)(x + v0 + v1 + v2);
}

// ---------------------------------------------------------------------------
// Radix sort, step 3: one stable counting pass on one byte digit, segment by
// segment (each key moves only within its own segment).
//
// A tile of BLOCK*ITEMS keys is loaded wave-striped (coalesced). Each wave
// ranks its keys stably with ballot peer masks: lanes holding the same digit
// find each other with 8 ballots, and the lowest such lane updates the wave's
// LDS counter for that digit, so a hot (Zipf) digit costs one LDS update per
// wave, not per lane. Per-wave counts are combined into the tile's digit
// totals, which are published for decoupled look-back; each of 256 threads
// then resolves the prefix of one digit from the preceding tiles of the same
// segment. Keys are scattered into LDS in digit order and written out from
// there, so consecutive threads write consecutive addresses within a digit.
// ---------------------------------------------------------------------------
// Bit B of d spread over all 32 bits (all ones where it is set). Written as
// v_bfe_i32 so that the compiler keeps one instruction per bit instead of
// rebuilding the mask from shifts.
template <int B>
__device__ __forceinline__ uint32_t bit_mask(uint32_t d) {
  uint32_t e;
  asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(e) : "v"(d), "i"(B));
  return e;
}

// One digit bit of the peer search: keep the lanes whose bit B equals this
// lane's. v_bitop3 truth table 0x90 (index p*4 + m*2 + e) = p & ~(m ^ e), so
// each 32-lane half costs one instruction.
template <int B>
__device__ __forceinline__ void peer_bit(uint32_t d, uint32_t &plo, uint32_t &phi) {
  const uint32_t e = bit_mask<B>(d);
  const uint64_t m = ballot64(e != 0);
  plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)m, e, 0x90);
  phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(m >> 32), e, 0x90);
}

// Peer search over digit bits Bit .. R-1 (see peer_bit).
template <int Bit, int R>
__device__ __forceinline__ void peer_bits(uint32_t d, uint32_t &plo, uint32_t &phi) {
  if constexpr (Bit < R) {
    peer_bit<Bit>(d, plo, phi);
    peer_bits<Bit + 1, R>(d, plo, phi);
  }
}

// Stable rank of each key among the wave's keys with the same digit, in
// (item, lane) order = original order; wcnt[d] holds the wave's running count
// of digit d. The peer mask (lanes holding the same digit) is the intersection
// over the R digit bits of the ballot where this lane's bit is set and its
// complement where it is clear. The lowest lane of each group of equal digits
// updates the counter, so a hot digit costs one LDS update per wave, not per
// lane. FULL: every lane holds a key; otherwise digit 2^R marks a missing
// key, which is left out of every peer mask and not ranked. CT is the
// counter type (a wave's count of one digit is at most 64 * ITEMS).
// ANY_ORDER: keys of one digit may take their ranks in any order within an
// item (the first pass of a sort, whose input order carries nothing): one LDS
// atomic per key on the wave's counter replaces the peer search.
template <int ITEMS, bool FULL, int R = 8, typename CT = uint32_t, bool ANY_ORDER = false>
__device__ __forceinline__ void wave_rank(const uint32_t (&dig)[ITEMS], uint32_t (&rank)[ITEMS],
                                          CT *wcnt) {
  constexpr uint32_t B = 1u << R;
  if constexpr (ANY_ORDER) {
    static_assert(std::is_same_v<CT, uint32_t>, "32-bit counters");
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t d = dig[k];
      if (FULL || d < B) rank[k] = atomicAdd(&wcnt[d], 1u);
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t d = dig[k];
    uint32_t plo = ~0u, phi = ~0u;
    if (!FULL) {
      const uint64_t vm = ballot64(d < B);
      plo = (uint32_t)vm;
      phi = (uint32_t)(vm >> 32);
    }
    peer_bits<0, R>(d, plo, phi);
    const uint64_t peers = ((uint64_t)phi << 32) | plo;
    if (FULL || d < B) {
      const uint32_t below = count_below(peers);
      const uint32_t old = wcnt[d];
      rank[k] = old + below;
      if (below == 0) wcnt[d] = (CT)(old + (uint32_t)__popcll(peers));
    }
  }
}

// Digits of a wave-striped tile (2^R for positions at or past n) and their
// ranks within the wave (stable unless ANY_ORDER).
template <int ITEMS, bool FULL, int R = 8, typename CT = uint32_t, bool ANY_ORDER = false>
__device__ __forceinline__ void rank_tile(const uint64_t (&key)[ITEMS], uint32_t shift, uint32_t n,
                                          uint32_t wbase, int lane, uint32_t (&dig)[ITEMS],
                                          uint32_t (&rank)[ITEMS], CT *wcnt) {
  constexpr uint32_t B = 1u << R;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t d = (uint32_t)(key[k] >> shift) & (B - 1);
    dig[k] = (FULL || wbase + k * kWave + lane < n) ? d : B;
  }
  wave_rank<ITEMS, FULL, R, CT, ANY_ORDER>(dig, rank, wcnt);
}

// Tile positions from the per-wave digit counts, on all BLOCK threads between
// two barriers of the caller. Thread d < kBins sums digit d over the waves
// (*tot, handed to publish() at once for the look-back), the 256 totals are
// scanned across the first four waves, and s_wcnt[q][d] becomes the tile
// position of wave q's first key with digit d, *lstart that of the tile's
// first key with digit d. Ends with a barrier.
template <int NW, typename Publish>
__device__ __forceinline__ void tile_offsets(uint32_t (*s_wcnt)[kBins], uint32_t *s_part, int tid,
                                             uint32_t *tot, uint32_t *lstart, Publish publish) {
  const int lane = tid & (kWave - 1), wv = tid / kWave;
  uint32_t run[NW];
  uint32_t sum = 0, incl = 0;
  if (tid < kBins) {
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      run[q] = sum;
      sum += s_wcnt[q][tid];
    }
    publish(sum);
    incl = wave_incl_scan32(sum);
    if (lane == kWave - 1) s_part[wv] = incl;
  }
  __syncthreads();
  if (tid < kBins) {
    uint32_t base = incl - sum;
#pragma unroll
    for (int q = 0; q < kBins / kWave; ++q) base += q < wv ? s_part[q] : 0u;
#pragma unroll
    for (int q = 0; q < NW; ++q) s_wcnt[q][tid] = base + run[q];
    *tot = sum;
    *lstart = base;
  }
  __syncthreads();
}

// Keys into the tile's LDS buffer in digit order.
template <int ITEMS, bool FULL, int R = 8, typename CT = uint32_t>
__device__ __forceinline__ void place_tile(const uint64_t (&key)[ITEMS], const uint32_t (&dig)[ITEMS],
                                           const uint32_t (&rank)[ITEMS], const CT *wpos,
                                           uint64_t *s_keys) {
  constexpr uint32_t B = 1u << R;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t d = dig[k];
    if (FULL || d < B) s_keys[wpos[d] + rank[k]] = key[k];
  }
}

// The tile's keys from LDS (digit order) to their output positions:
// out[s_gdel[d] + i] for the key at LDS position i with digit d. A full tile
// goes in unrolled batches so that each batch's LDS reads are in flight
// together; a partial tile loops.
template <int BLOCK, int ITEMS, int R = 8>
__device__ __forceinline__ void write_tile(const uint64_t *s_keys, const uint64_t *s_gdel,
                                           uint32_t n, uint32_t shift, int tid, uint64_t *out,
                                           uint64_t lim) {
  constexpr uint32_t M = (1u << R) - 1;
  if (n == (uint32_t)(BLOCK * ITEMS)) {
    // opaque copy of the thread index: keeps the compiler from hoisting one
    // 64-bit address per item out of the tile loop (registers it lacks)
    uint32_t tb = tid;
    asm volatile("" : "+v"(tb));
    constexpr int U = ITEMS < 8 ? ITEMS : 8;  // keys per unrolled batch
#pragma unroll
    for (int q0 = 0; q0 < ITEMS; q0 += U) {
      uint64_t x[U], g[U];
#pragma unroll
      for (int q = 0; q < U; ++q) x[q] = s_keys[tb + (q0 + q) * BLOCK];
#pragma unroll
      for (int q = 0; q < U; ++q) g[q] = s_gdel[(uint32_t)(x[q] >> shift) & M] + tb;
#pragma unroll
      for (int q = 0; q < U; ++q)
        if (in_bounds(g[q] + (q0 + q) * BLOCK, lim)) out[g[q] + (q0 + q) * BLOCK] = x[q];
    }
  } else {
    for (uint32_t i = tid; i < n; i += BLOCK) {
      const uint64_t x = s_keys[i];
      const uint64_t g = s_gdel[(uint32_t)(x >> shift) & M] + i;
      if (in_bounds(g, lim)) out[g] = x;
    }
  }
}

// Next tile of a radix pass. With several segments of similar length, tickets
// go layer by layer: ticket k is tile k / W of segment k % W (tickets of absent
// tiles are skipped), so a tile's predecessor in its segment holds a ticket W
// smaller and has usually finished. Otherwise tickets follow tile order. Either
// way every predecessor holds a smaller ticket, so look-back waits always end.
// Returns ~0u when the pass is exhausted; *seg receives the tile's segment.
// Called by a whole wave; every lane returns the same ticket.
__device__ __forceinline__ uint32_t pass_ticket(const PassArgs &a, uint64_t layers,
                                                uint64_t tickets, uint32_t *seg) {
  const int lane = threadIdx.x & (kWave - 1);
  for (;;) {
    uint32_t k0 = 0;
    if (lane == 0) k0 = atomicAdd(a.ticket, 1u);
    const uint64_t k = (uint32_t)__builtin_amdgcn_readfirstlane(k0);
    if (k >= tickets) return 0xFFFFFFFFu;
    if (!layers) {
      // plain (vector) loads here: with thousands of windows, the scalar-cache
      // search handed out tiles measurably faster and the passes ran slower
      uint32_t lo = 0, hi = a.W;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.tile_off[mid] <= k) lo = mid; else hi = mid;
      }
      *seg = lo;
      return (uint32_t)k;
    }
    const uint32_t w = (uint32_t)(k % a.W);
    const uint64_t j = k / a.W;
    const uint64_t f = ld_const(a.tile_off + w);
    if (f + j < ld_const(a.tile_off + w + 1)) {
      *seg = w;
      return (uint32_t)(f + j);
    }
  }
}

// Load one tile wave-striped: item k of lane l of wave v is key
// start + v*64*ITEMS + k*64 + l. Missing keys get digit kBins.
template <int ITEMS, bool PACKETS>
__device__ __forceinline__ void pass_load(const PassArgs &a, uint64_t start, uint32_t n,
                                          uint32_t wbase, int lane, uint32_t full,
                                          uint64_t (&key)[ITEMS]) {
  if (n == full) {  // full tile: unpredicated loads
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t i = start + wbase + k * kWave + lane;
      key[k] = !in_bounds(i, a.lim) ? 0 : PACKETS ? pack_key(a.src[i], a.dst[i]) : a.in[i];
    }
  } else {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t li = wbase + k * kWave + lane;
      uint64_t x = 0;
      if (li < n && in_bounds(start + li, a.lim)) {
        if (PACKETS) x = pack_key(a.src[start + li], a.dst[start + li]);
        else x = a.in[start + li];
      }
      key[k] = x;
    }
  }
}

template <int BLOCK, int ITEMS, bool PACKETS, bool W32>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_pass(PassArgs a) {
  using LW = std::conditional_t<W32, uint32_t, uint64_t>;  // look-back word width
  using L = LbWord<LW>;
  LW *const lbw = reinterpret_cast<LW *>(a.lb);
  LW *const lbn = reinterpret_cast<LW *>(a.lb_next);
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  static_assert(BLOCK >= kBins, "one thread per digit");
  __shared__ uint64_t s_keys[TILE];
  __shared__ uint32_t s_wcnt[NW][kBins];
  __shared__ uint32_t s_part[kBins / kWave];
  __shared__ uint64_t s_gdel[kBins];  // output position of digit d's keys minus their tile position
  __shared__ uint32_t s_tile, s_seg;

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t shift = a.shift;
  const uint64_t layers = ld_const(a.tile_off + a.W + 1);
  const uint64_t tickets = layers ? (uint64_t)a.W * layers : ld_const(a.tile_off + a.W);
  const uint32_t wbase = wv * (kWave * ITEMS);
  // Several segments: the keys of the next tile are requested before this
  // tile's look-back, so their memory latency overlaps the wait. One segment:
  // the next ticket is drawn only after the scatter, since a tile held while
  // another one finishes would delay its own published counts and lengthen
  // every later tile's look-back.
  const bool pipe = a.W > 1;

  for (int i = tid; i < NW * kBins; i += BLOCK) (&s_wcnt[0][0])[i] = 0;
  if (tid < kWave) {
    uint32_t w = 0;
    const uint32_t tk = pass_ticket(a, layers, tickets, &w);
    if (tid == 0) {
      s_tile = tk;
      s_seg = w;
    }
  }
  __syncthreads();
  uint32_t t = __builtin_amdgcn_readfirstlane(s_tile), w = __builtin_amdgcn_readfirstlane(s_seg);
  uint64_t seg_lo = 0;
  uint32_t first = 0, n = 0;
  uint64_t key[ITEMS];
  if (t != 0xFFFFFFFFu) {
    first = (uint32_t)ld_const(a.tile_off + w);
    seg_lo = ld_const(a.seg_off + w);
    const uint64_t start = seg_lo + (uint64_t)(t - first) * TILE;
    n = (uint32_t)min((uint64_t)TILE, ld_const(a.seg_off + w + 1) - start);
    pass_load<ITEMS, PACKETS>(a, start, n, wbase, lane, TILE, key);
  }

  while (t != 0xFFFFFFFFu) {
    uint32_t dig[ITEMS];
    uint32_t rank[ITEMS];
    const bool full = n == TILE;
    if (full) rank_tile<ITEMS, true>(key, shift, n, wbase, lane, dig, rank, s_wcnt[wv]);
    else rank_tile<ITEMS, false>(key, shift, n, wbase, lane, dig, rank, s_wcnt[wv]);
    __syncthreads();
    uint32_t tot = 0, lstart = 0;
    // publish this tile's digit counts as early as possible
    tile_offsets<NW>(s_wcnt, s_part, tid, &tot, &lstart, [&](uint32_t sum) {
      lb_store(lbw + (uint64_t)t * kBins + tid, t == first ? L::inc(sum) : L::agg(sum));
    });
    // local counting sort of the tile into LDS; the key registers are free after
    if (full) place_tile<ITEMS, true>(key, dig, rank, s_wcnt[wv], s_keys);
    else place_tile<ITEMS, false>(key, dig, rank, s_wcnt[wv], s_keys);
    if (pipe && tid < kWave) {
      uint32_t nw = 0;
      const uint32_t tk = pass_ticket(a, layers, tickets, &nw);
      if (tid == 0) {
        s_tile = tk;
        s_seg = nw;
      }
    }
    __syncthreads();
    for (int i = tid; i < NW * kBins; i += BLOCK) (&s_wcnt[0][0])[i] = 0;
    uint32_t t2 = 0xFFFFFFFFu, w2 = 0;
    uint64_t seg_lo2 = 0;
    uint32_t first2 = 0, n2 = 0;
    if (pipe) {
      t2 = __builtin_amdgcn_readfirstlane(s_tile);
      w2 = __builtin_amdgcn_readfirstlane(s_seg);
      if (t2 != 0xFFFFFFFFu) {  // prefetch the next tile
        first2 = (uint32_t)ld_const(a.tile_off + w2);
        seg_lo2 = ld_const(a.seg_off + w2);
        const uint64_t start2 = seg_lo2 + (uint64_t)(t2 - first2) * TILE;
        n2 = (uint32_t)min((uint64_t)TILE, ld_const(a.seg_off + w2 + 1) - start2);
        pass_load<ITEMS, PACKETS>(a, start2, n2, wbase, lane, TILE, key);
      }
    }
    if (tid < kBins) {
      uint64_t excl = 0;
      if (t != first) {
        excl = lb_walkn<NS_LB_DEPTH>(lbw, kBins, tid, t, first);
        lb_store(lbw + (uint64_t)t * kBins + tid, L::inc(excl + tot));
      }
      s_gdel[tid] = seg_lo + a.base[(uint64_t)w * a.base_stride + tid] + excl - lstart;
      lbn[(uint64_t)t * kBins + tid] = 0;
    }
    __syncthreads();
    write_tile<BLOCK, ITEMS>(s_keys, s_gdel, n, shift, tid, a.out, a.lim);
    if (!pipe && tid < kWave) {
      uint32_t nw = 0;
      const uint32_t tk = pass_ticket(a, layers, tickets, &nw);
      if (tid == 0) {
        s_tile = tk;
        s_seg = nw;
      }
    }
    __syncthreads();
    if (!pipe) {
      t2 = __builtin_amdgcn_readfirstlane(s_tile);
      w2 = __builtin_amdgcn_readfirstlane(s_seg);
      if (t2 != 0xFFFFFFFFu) {
        first2 = (uint32_t)ld_const(a.tile_off + w2);
        seg_lo2 = ld_const(a.seg_off + w2);
        const uint64_t start2 = seg_lo2 + (uint64_t)(t2 - first2) * TILE;
        n2 = (uint32_t)min((uint64_t)TILE, ld_const(a.seg_off + w2 + 1) - start2);
        pass_load<ITEMS, PACKETS>(a, start2, n2, wbase, lane, TILE, key);
      }
    }
    t = t2;
    w = w2;
    first = first2;
    seg_lo = seg_lo2;
    n = n2;
  }
}

// ---------------------------------------------------------------------------
// Radix pass over a single segment with the next tile ranked early.
//
// On one segment every tile's look-back goes back to the tile before it, so
// a tile's counts must be published as soon as possible after its ticket is
// drawn. k_pass either draws the next ticket after the scatter (its keys then
// arrive while nothing else happens) or early (its counts then wait behind the
// whole scatter). Here a workgroup draws the next ticket before the current
// tile's look-back, requests its keys, and ranks it and publishes its counts
// right after that look-back, before it scatters the current tile: the key
// loads overlap the look-back, waves without a digit to resolve rank at once,
// and the held tile's counts are out one ranking after its keys arrive. The
// held tile's key positions in the tile wait in registers until the current
// tile's keys have left LDS. A held ticket is still safe: its holder has
// published the counts of its current tile and resolves that tile's prefix
// from smaller tickets only.
// ---------------------------------------------------------------------------
template <int BLOCK, int ITEMS, bool PACKETS, bool W32>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_pass1(PassArgs a) {
  using LW = std::conditional_t<W32, uint32_t, uint64_t>;  // look-back word width
  using L = LbWord<LW>;
  LW *const lbw = reinterpret_cast<LW *>(a.lb);
  LW *const lbn = reinterpret_cast<LW *>(a.lb_next);
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  static_assert(BLOCK >= kBins, "one thread per digit");
  __shared__ uint64_t s_keys[TILE];
  __shared__ uint32_t s_wcnt[NW][kBins];
  __shared__ uint32_t s_part[kBins / kWave];
  __shared__ uint64_t s_gdel[kBins];
  __shared__ uint32_t s_tile;

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t shift = a.shift;
  const uint64_t seg_lo = ld_const(a.seg_off), seg_hi = ld_const(a.seg_off + 1);
  const uint64_t tiles = (seg_hi - seg_lo + TILE - 1) / TILE;
  const uint32_t wbase = wv * (kWave * ITEMS);

  auto draw = [&]() {
    if (tid == 0) {
      const uint32_t k = atomicAdd(a.ticket, 1u);
      s_tile = k < tiles ? k : 0xFFFFFFFFu;
    }
  };
  auto tile_keys = [&](uint32_t t) {
    const uint64_t start = seg_lo + (uint64_t)t * TILE;
    return (uint32_t)min((uint64_t)TILE, seg_hi - start);
  };
  // rank the tile held in `key`, publish its digit counts, and turn the ranks
  // into LDS positions, two 16-bit positions per register (0xFFFF: no key)
  static_assert(TILE < 0xFFFF && ITEMS % 2 == 0, "16-bit tile positions");
  uint64_t key[ITEMS];
  uint32_t pos[ITEMS / 2];
  auto rank_and_publish = [&](uint32_t t, uint32_t n, uint32_t *tot, uint32_t *lstart) {
    uint32_t dig[ITEMS], rank[ITEMS];
    const bool full = n == TILE;
    // the first pass (packets in arrival order) needs no order among equal
    // digits: LDS atomics rank it (2^30 keys: 4.45 vs 4.65 ms; on 8192 windows,
    // in k_pass, the peer search was faster: 3.96 vs 4.04 ms)
    if (full) rank_tile<ITEMS, true, 8, uint32_t, PACKETS>(key, shift, n, wbase, lane, dig, rank, s_wcnt[wv]);
    else rank_tile<ITEMS, false, 8, uint32_t, PACKETS>(key, shift, n, wbase, lane, dig, rank, s_wcnt[wv]);
    __syncthreads();
    tile_offsets<NW>(s_wcnt, s_part, tid, tot, lstart, [&](uint32_t sum) {
      lb_store(lbw + (uint64_t)t * kBins + tid, t == 0 ? L::inc(sum) : L::agg(sum));
    });
#pragma unroll
    for (int k = 0; k < ITEMS; k += 2) {
      const uint32_t p0 = dig[k] < kBins ? s_wcnt[wv][dig[k]] + rank[k] : 0xFFFFu;
      const uint32_t p1 = dig[k + 1] < kBins ? s_wcnt[wv][dig[k + 1]] + rank[k + 1] : 0xFFFFu;
      pos[k / 2] = p0 | (p1 << 16);
    }
  };
  // the held tile's keys into LDS, counters cleared for the next ranking
  // (after a barrier that ends every read of s_keys and s_wcnt)
  auto place = [&]() {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t p = (pos[k / 2] >> (16 * (k & 1))) & 0xFFFFu;
      if (p != 0xFFFFu) s_keys[p] = key[k];
    }
    for (int i = tid; i < NW * kBins; i += BLOCK) (&s_wcnt[0][0])[i] = 0;
  };

  for (int i = tid; i < NW * kBins; i += BLOCK) (&s_wcnt[0][0])[i] = 0;
  draw();
  __syncthreads();
  uint32_t t = __builtin_amdgcn_readfirstlane(s_tile);
  if (t == 0xFFFFFFFFu) return;
  uint32_t n = tile_keys(t);
  pass_load<ITEMS, PACKETS>(a, seg_lo + (uint64_t)t * TILE, n, wbase, lane, TILE, key);
  uint32_t tot = 0, lstart = 0;
  rank_and_publish(t, n, &tot, &lstart);
  __syncthreads();
  place();

  for (;;) {
    draw();
    __syncthreads();  // the ticket; tile t in LDS; counters clear
    const uint32_t t2 = __builtin_amdgcn_readfirstlane(s_tile);
    uint32_t n2 = 0;
    if (t2 != 0xFFFFFFFFu) {
      n2 = tile_keys(t2);
      pass_load<ITEMS, PACKETS>(a, seg_lo + (uint64_t)t2 * TILE, n2, wbase, lane, TILE, key);
    }
    if (tid < kBins) {
      uint64_t excl = 0;
      if (t != 0) {
        excl = lb_walkn<NS_LB_DEPTH>(lbw, kBins, tid, t, 0);
        lb_store(lbw + (uint64_t)t * kBins + tid, L::inc(excl + tot));
      }
      s_gdel[tid] = seg_lo + a.base[tid] + excl - lstart;
      lbn[(uint64_t)t * kBins + tid] = 0;
    }
    uint32_t tot2 = 0, lstart2 = 0;
    if (t2 != 0xFFFFFFFFu) rank_and_publish(t2, n2, &tot2, &lstart2);  // ends with a barrier
    else __syncthreads();
    write_tile<BLOCK, ITEMS>(s_keys, s_gdel, n, shift, tid, a.out, a.lim);
    if (t2 == 0xFFFFFFFFu) break;
    __syncthreads();
    place();
    t = t2;
    n = n2;
    tot = tot2;
    lstart = lstart2;
  }
}

// ---------------------------------------------------------------------------
// Radix pass over one large segment without look-back (reduce, scan, scatter).
//
// With a single segment, every tile's look-back walks a long chain of tiles
// still in flight, and each step is a round trip to memory. Here the segment
// is cut into short chunks of whole tiles instead (kChunkTiles each, within the
// rows of the chunk tables): k_chunk_hist counts each chunk's digits, the
// chunk scan sums them over earlier chunks per digit, and k_pass_chunked sorts
// each chunk's tiles in order, starting from those positions (plus the start
// of the digit's bucket) and carrying its own running offsets from tile to
// tile. The keys are read twice, but nothing ever waits. Chunks are taken by
// ticket, so the ones in flight are neighbours and their writes to each digit's
// bucket stay close together. The tile count, the chunk length and the chunk
// count follow from the segment length on the device, so a launch sized for n
// keys serves any length up to n.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void chunk_geometry(const ChunkArgs &c, uint32_t tile, uint64_t *lo,
                                               uint64_t *n, uint64_t *tiles, uint64_t *per) {
  *lo = ld_const(c.seg_off);
  *n = ld_const(c.seg_off + 1) - *lo;
  *tiles = (*n + tile - 1) / tile;
  const uint64_t p = (*tiles + c.chunks - 1) / c.chunks;
  *per = p ? p : 1;
}

template <int BLOCK, bool PACKETS, int R>
__global__ __launch_bounds__(BLOCK) void k_chunk_hist(PassArgs a, ChunkArgs c, uint32_t tile) {
  constexpr int C = 4;  // counter copies chosen by lane: a hot digit spreads over four
  constexpr uint32_t B = 1u << R;
  __shared__ uint32_t s_h[B * C];
  uint64_t lo, n, tiles, per;
  chunk_geometry(c, tile, &lo, &n, &tiles, &per);
  const uint32_t cp = threadIdx.x & (C - 1);
  for (uint32_t ch = blockIdx.x; ch < c.chunks; ch += gridDim.x) {
    for (int i = threadIdx.x; i < (int)(B * C); i += BLOCK) s_h[i] = 0;
    __syncthreads();
    const uint64_t b = min(n, (uint64_t)ch * per * tile), e = min(n, b + per * tile);
    constexpr int U = 8;
    for (uint64_t i0 = lo + b + threadIdx.x; i0 < lo + e; i0 += (uint64_t)U * BLOCK) {
      uint64_t k[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const uint64_t i = i0 + (uint64_t)q * BLOCK;
        k[q] = i < lo + e ? (PACKETS ? pack_key(a.src[i], a.dst[i]) : a.in[i]) : 0;
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (i0 + (uint64_t)q * BLOCK >= lo + e) break;
        atomicAdd(&s_h[(((uint32_t)(k[q] >> a.shift)) & (B - 1)) * C + cp], 1u);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (int)B; i += BLOCK) {
      uint32_t v = 0;
#pragma unroll
      for (int q = 0; q < C; ++q) v += s_h[i * C + q];
      c.count[(uint64_t)ch * B + i] = v;
    }
    __syncthreads();
  }
}

// The chunk scan: prefix[ch][d] = keys with digit d in chunks before ch, and
// total[d] = keys with digit d, in three coalesced steps over the row-major
// count table (a row is the c.bins counts of one chunk): each workgroup sums
// the rows of one block of consecutive chunks, the block sums are scanned per
// digit, and each block then writes its chunks' prefixes from its own start.
// Thread x of a workgroup with blockIdx.y = g owns digit d = 256 g + x, so a
// row is read in coalesced 1 KiB pieces.
__global__ __launch_bounds__(256) void k_chunk_sums(ChunkArgs c, uint32_t rows) {
  const uint32_t r0 = blockIdx.x * rows, r1 = min(c.chunks, r0 + rows);
  const uint32_t d = blockIdx.y * 256 + threadIdx.x;
  uint64_t s = 0;
  for (uint32_t r = r0; r < r1; ++r) s += c.count[(uint64_t)r * c.bins + d];
  c.bsum[(uint64_t)blockIdx.x * c.bins + d] = s;
}

// One workgroup per digit; thread i scans blocks [i*per, (i+1)*per).
__global__ __launch_bounds__(256) void k_chunk_bscan(ChunkArgs c, uint32_t blocks) {
  __shared__ uint64_t s_tmp[4];
  constexpr int kMaxPer = kChunkBlocks / 256;
  const uint32_t d = blockIdx.x;
  const uint32_t per = (blocks + 255) / 256;
  const uint32_t b0 = threadIdx.x * per;
  uint64_t v[kMaxPer];
  uint64_t sum = 0;
#pragma unroll
  for (int q = 0; q < kMaxPer; ++q) {
    const uint32_t b = b0 + q;
    v[q] = (q < (int)per && b < blocks) ? c.bsum[(uint64_t)b * c.bins + d] : 0;
    sum += v[q];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan<256>(sum, s_tmp, &tot);
#pragma unroll
  for (int q = 0; q < kMaxPer; ++q) {
    const uint32_t b = b0 + q;
    if (q < (int)per && b < blocks) c.bsum[(uint64_t)b * c.bins + d] = run;
    run += v[q];
  }
  if (threadIdx.x == 0) c.total[d] = tot;
}

__global__ __launch_bounds__(256) void k_chunk_prefix(ChunkArgs c, uint32_t rows) {
  const uint32_t r0 = blockIdx.x * rows, r1 = min(c.chunks, r0 + rows);
  const uint32_t d = blockIdx.y * 256 + threadIdx.x;
  uint64_t run = c.bsum[(uint64_t)blockIdx.x * c.bins + d];
  for (uint32_t r = r0; r < r1; ++r) {
    c.prefix[(uint64_t)r * c.bins + d] = run;
    run += c.count[(uint64_t)r * c.bins + d];
  }
}

template <int BLOCK, int ITEMS, bool PACKETS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_pass_chunked(PassArgs a, ChunkArgs c) {
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  static_assert(BLOCK >= kBins, "one thread per digit");
  __shared__ uint64_t s_keys[TILE];
  __shared__ uint32_t s_wcnt[NW][kBins];
  __shared__ uint32_t s_part[kBins / kWave];
  __shared__ uint64_t s_gdel[kBins];  // output position of digit d's keys minus their tile position
  __shared__ uint32_t s_chunk;

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t shift = a.shift;
  const uint32_t wbase = wv * (kWave * ITEMS);
  __shared__ uint64_t s_dbase[kBins];
  __shared__ uint64_t s_tmp[NW];
  uint64_t lo, nk, tiles, per;
  chunk_geometry(c, TILE, &lo, &nk, &tiles, &per);
  {  // start of each digit's bucket: segment start + keys with a smaller digit
    uint64_t tot;
    const uint64_t x = block_excl_scan<BLOCK>(tid < kBins ? c.total[tid] : 0, s_tmp, &tot);
    if (tid < kBins) s_dbase[tid] = lo + x;
  }

  for (;;) {
    if (tid == 0) s_chunk = atomicAdd(a.ticket, 1u);
    for (int i = tid; i < NW * kBins; i += BLOCK) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    const uint32_t ch = s_chunk;
    if (ch >= c.chunks) break;
    const uint64_t t0 = min(tiles, (uint64_t)ch * per), t1 = min(tiles, t0 + per);
    // thread d < kBins: output position of the chunk's next key with digit d
    uint64_t gbase = tid < kBins ? s_dbase[tid] + c.prefix[(uint64_t)ch * kBins + tid] : 0;
    uint64_t key[ITEMS];
    uint32_t n = 0;
    if (t0 < t1) {
      const uint64_t start = lo + t0 * TILE;
      n = (uint32_t)min((uint64_t)TILE, lo + nk - start);
      pass_load<ITEMS, PACKETS>(a, start, n, wbase, lane, TILE, key);
    }
    for (uint64_t t = t0; t < t1; ++t) {
      uint32_t dig[ITEMS];
      uint32_t rank[ITEMS];
      const bool full = n == TILE;
      if (full) rank_tile<ITEMS, true>(key, shift, n, wbase, lane, dig, rank, s_wcnt[wv]);
      else rank_tile<ITEMS, false>(key, shift, n, wbase, lane, dig, rank, s_wcnt[wv]);
      __syncthreads();
      uint32_t tot = 0, lstart = 0;
      tile_offsets<NW>(s_wcnt, s_part, tid, &tot, &lstart, [](uint32_t) {});
      if (tid < kBins) s_gdel[tid] = gbase - lstart;
      if (full) place_tile<ITEMS, true>(key, dig, rank, s_wcnt[wv], s_keys);
      else place_tile<ITEMS, false>(key, dig, rank, s_wcnt[wv], s_keys);
      __syncthreads();
      for (int i = tid; i < NW * kBins; i += BLOCK) (&s_wcnt[0][0])[i] = 0;
      const uint32_t n_cur = n;
      if (t + 1 < t1) {  // the next tile's keys load while this one is written
        const uint64_t start = lo + (t + 1) * TILE;
        n = (uint32_t)min((uint64_t)TILE, lo + nk - start);
        pass_load<ITEMS, PACKETS>(a, start, n, wbase, lane, TILE, key);
      }
      write_tile<BLOCK, ITEMS>(s_keys, s_gdel, n_cur, shift, tid, a.out, a.lim);
      __syncthreads();
      gbase += tot;
    }
    __syncthreads();
  }
}

// The chunked pass on 11-bit digits (2048 bins): 64-bit keys sort in 6
// passes instead of 8, 32-bit column keys in 3 instead of 4. The tile flow is
// that of k_pass_chunked; what changes with 2048 digits:
// * per-wave digit counters are 16-bit (a wave counts at most 64 * ITEMS keys
//   of a digit, and tile positions stay below 2^16), so the counters of a
//   512-thread tile take 32 KiB of LDS;
// * each thread owns DPT = 2048 / BLOCK consecutive digits: it sums them over
//   the waves, a block scan of the threads' sums gives the tile positions, and
//   it keeps its digits' running output positions in registers.
template <int BLOCK, int ITEMS>
constexpr int wide_waves() {
  // occupancy the LDS allows: keys + 16-bit counters + output deltas
  return (160 * 1024) / (BLOCK * ITEMS * 8 + (BLOCK / kWave) * kMaxBins * 2 + kMaxBins * 8) *
         (BLOCK / kWave) / 4;
}

template <int BLOCK, int ITEMS, bool PACKETS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(wide_waves<BLOCK, ITEMS>())))
void k_pass_chunked_wide(PassArgs a, ChunkArgs c) {
  constexpr int R = kWideBits;
  constexpr int B = 1 << R;
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int NW = BLOCK / kWave;
  constexpr int DPT = B / BLOCK;  // consecutive digits owned by each thread
  static_assert(B % BLOCK == 0 && TILE < 65536, "16-bit tile positions");
  __shared__ uint64_t s_keys[TILE];
  __shared__ uint16_t s_wcnt[NW][B];
  __shared__ uint64_t s_gdel[B];  // output position of digit d's keys minus their tile position
  __shared__ uint64_t s_tmp[NW];
  __shared__ uint32_t s_chunk;

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t shift = a.shift;
  const uint32_t wbase = wv * (kWave * ITEMS);
  const uint32_t d0 = tid * DPT;
  uint64_t lo, nk, tiles, per;
  chunk_geometry(c, TILE, &lo, &nk, &tiles, &per);
  uint64_t dbase[DPT];  // start of each owned digit's bucket
  {
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      dbase[j] = sum;
      sum += c.total[d0 + j];
    }
    uint64_t tot;
    const uint64_t x = block_excl_scan<BLOCK>(sum, s_tmp, &tot);
#pragma unroll
    for (int j = 0; j < DPT; ++j) dbase[j] += lo + x;
  }

  for (;;) {
    if (tid == 0) s_chunk = atomicAdd(a.ticket, 1u);
    for (int i = tid; i < NW * B / 2; i += BLOCK) reinterpret_cast<uint32_t *>(&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    const uint32_t ch = s_chunk;
    if (ch >= c.chunks) break;
    const uint64_t t0 = min(tiles, (uint64_t)ch * per), t1 = min(tiles, t0 + per);
    uint64_t gbase[DPT];  // output position of the chunk's next key with each owned digit
#pragma unroll
    for (int j = 0; j < DPT; ++j) gbase[j] = dbase[j] + c.prefix[(uint64_t)ch * B + d0 + j];
    uint64_t key[ITEMS];
    uint32_t n = 0;
    if (t0 < t1) {
      const uint64_t start = lo + t0 * TILE;
      n = (uint32_t)min((uint64_t)TILE, lo + nk - start);
      pass_load<ITEMS, PACKETS>(a, start, n, wbase, lane, TILE, key);
    }
    for (uint64_t t = t0; t < t1; ++t) {
      uint32_t dig[ITEMS];
      uint32_t rank[ITEMS];
      const bool full = n == TILE;
      if (full) rank_tile<ITEMS, true, R, uint16_t>(key, shift, n, wbase, lane, dig, rank, s_wcnt[wv]);
      else rank_tile<ITEMS, false, R, uint16_t>(key, shift, n, wbase, lane, dig, rank, s_wcnt[wv]);
      __syncthreads();
      // tile positions: thread sums of its digits over the waves, block scan
      uint32_t run[NW][DPT], tot[DPT];
      uint32_t sum = 0;
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        uint32_t r = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
          run[q][j] = r;
          r += s_wcnt[q][d0 + j];
        }
        tot[j] = r;
        sum += r;
      }
      uint64_t all;
      uint32_t pos = (uint32_t)block_excl_scan<BLOCK>(sum, s_tmp, &all);
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
#pragma unroll
        for (int q = 0; q < NW; ++q) s_wcnt[q][d0 + j] = (uint16_t)(pos + run[q][j]);
        s_gdel[d0 + j] = gbase[j] - pos;
        gbase[j] += tot[j];
        pos += tot[j];
      }
      __syncthreads();
      if (full) place_tile<ITEMS, true, R, uint16_t>(key, dig, rank, s_wcnt[wv], s_keys);
      else place_tile<ITEMS, false, R, uint16_t>(key, dig, rank, s_wcnt[wv], s_keys);
      __syncthreads();
      for (int i = tid; i < NW * B / 2; i += BLOCK) reinterpret_cast<uint32_t *>(&s_wcnt[0][0])[i] = 0;
      const uint32_t n_cur = n;
      if (t + 1 < t1) {  // the next tile's keys load while this one is written
        const uint64_t start = lo + (t + 1) * TILE;
        n = (uint32_t)min((uint64_t)TILE, lo + nk - start);
        pass_load<ITEMS, PACKETS>(a, start, n, wbase, lane, TILE, key);
      }
      write_tile<BLOCK, ITEMS, R>(s_keys, s_gdel, n_cur, shift, tid, a.out, a.lim);
      __syncthreads();
    }
    __syncthreads();
  }
}

// LDS index with one pad word after every 8: a thread that owns 8 consecutive
// positions then reads them without bank conflicts (consecutive lanes land 9
// words apart instead of 8).
__device__ __forceinline__ constexpr uint32_t pd(uint32_t j) { return j + (j >> 3); }

// ---------------------------------------------------------------------------
// First index in (lo, hi] whose key differs from K, given keys[lo] == K in a
// sorted array (hi if none). The whole calling wave searches together: 64
// probes per round trip (the next 64 positions, then 64 exponentially spaced
// ones, then 64-way subdivision), so even a run of 2^30 equal keys takes a
// handful of dependent loads. Every lane returns the same value.
// ---------------------------------------------------------------------------
__device__ uint64_t run_end_wave(const uint64_t *keys, uint64_t lo, uint64_t hi, uint64_t K) {
  const int lane = threadIdx.x & (kWave - 1);
  {
    const uint64_t p = lo + 1 + lane;
    const uint64_t m = ballot64(p >= hi ? true : keys[p] != K);
    if (m) return min(lo + 1 + (uint64_t)(__ffsll((long long)m) - 1), hi);
  }
  uint64_t L = lo + 64, R;  // keys[L] == K
  {
    const uint64_t p = L + (64ull << min(lane, 40));
    const uint64_t m = ballot64(p >= hi ? true : keys[p] != K);
    const int f = __ffsll((long long)m) - 1;  // some lane reaches hi
    R = min(L + (64ull << f), hi);
    if (f > 0) L += 64ull << (f - 1);
  }
  while (R - L > 1) {
    const uint64_t step = (R - L + 63) / 64;
    const uint64_t p = L + step * (uint64_t)(lane + 1);
    const uint64_t m = ballot64(p >= R ? true : keys[p] != K);
    const int f = __ffsll((long long)m) - 1;
    const uint64_t nR = min(L + step * (uint64_t)(f + 1), R);
    L = L + step * (uint64_t)f;
    R = nR;
  }
  return R;
}

// ---------------------------------------------------------------------------
// Tiles of the run scans (k_rle, k_runs), handed out by ticket one tile ahead:
// while a workgroup resolves tile t, its fourth wave claims the next ticket and
// finds its segment, and once t's offsets are known the next tile's keys are
// requested, so their latency overlaps t's writes. Tickets still reach every
// workgroup in increasing order and each finishes its current tile before it
// starts the claimed one, so every look-back wait ends.
// ---------------------------------------------------------------------------
struct ScanTile {
  uint32_t t, w, first, n;   // ticket (= tile), segment, its first tile, keys in the tile
  uint64_t seg_lo, seg_hi, start;
};

// Claim the next ticket and its segment; called by one whole wave, lane 0
// stores them.
__device__ __forceinline__ void claim_tile(uint32_t *ticket, const uint64_t *tile_off, uint32_t W,
                                           uint64_t total, uint32_t *s_t, uint32_t *s_w) {
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t k0 = 0;
  if (lane == 0) k0 = atomicAdd(ticket, 1u);
  const uint32_t k = __builtin_amdgcn_readfirstlane(k0);
  const uint32_t w = k < total ? find_owner_near(tile_off, W, total, k) : 0u;
  if (lane == 0) {
    *s_t = k;
    *s_w = w;
  }
}

__device__ __forceinline__ ScanTile scan_tile(const uint64_t *tile_off, const uint64_t *seg_off,
                                              uint32_t t_lds, uint32_t w_lds, uint64_t total,
                                              uint32_t tile) {
  ScanTile g;
  g.t = __builtin_amdgcn_readfirstlane(t_lds);
  g.w = __builtin_amdgcn_readfirstlane(w_lds);
  g.first = 0;
  g.n = 0;
  g.seg_lo = g.seg_hi = g.start = 0;
  if (g.t < total) {
    g.first = (uint32_t)ld_const(tile_off + g.w);
    g.seg_lo = ld_const(seg_off + g.w);
    g.seg_hi = ld_const(seg_off + g.w + 1);
    g.start = g.seg_lo + (uint64_t)(g.t - g.first) * tile;
    g.n = (uint32_t)min((uint64_t)tile, g.seg_hi - g.start);
  }
  return g;
}

// Striped loads of a tile (thread i holds positions i, i+BLOCK, ...), the key
// before it (thread 0; only inside the segment) and the key after it (wave 2,
// which searches past the tile end; only inside the segment).
template <int BLOCK, int ITEMS>
__device__ __forceinline__ void scan_load(const uint64_t *keys, const ScanTile &g, uint64_t (&kr)[ITEMS],
                                          uint64_t &kprev, uint64_t &knext, uint64_t lim) {
  const int tid = threadIdx.x;
  // opaque copy of the thread index: keeps the compiler from hoisting one
  // 64-bit address per item out of the tile loop (registers it lacks)
  uint32_t tb = tid;
  asm volatile("" : "+v"(tb));
  const uint64_t *base = keys + g.start;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t i = tb + k * BLOCK;
    kr[k] = i < g.n && in_bounds(g.start + i, lim) ? base[i] : 0;
  }
  if (tid == 0 && g.n && g.start > g.seg_lo && in_bounds(g.start - 1, lim)) kprev = keys[g.start - 1];
  if (tid / kWave == 2 && g.n && g.start + g.n < g.seg_hi && in_bounds(g.start + g.n, lim))
    knext = keys[g.start + g.n];
}

// ---------------------------------------------------------------------------
// Run-length encoding of sorted packet keys, with row heads.
// A link head is a position whose key differs from its predecessor in the
// segment (Table I: unique links = nonzeros of A); a row head is one whose
// source differs (unique sources). Link and row heads are compacted over the
// whole launch with a decoupled look-back over both counts (one word per tile
// holding both below 2^31 keys, else a channel each), so every window's links
// land at [link_off[w], link_off[w+1]). Each link's count is the distance to
// the next link head (in the tile, or found by a galloping search past the tile
// end for the last run). Each row head records its packet position and link
// index; differences of consecutive row heads give per-source packets and
// fan-out. May run in place (ukeys == keys): a tile finishes every read beyond
// its end before it publishes, and later tiles write only after that; a tile
// writes only at or below its own last position, so keys requested ahead for a
// later tile are never overwritten first (the one position just below a tile
// that an earlier tile may rewrite gets the same key back).
// ---------------------------------------------------------------------------
// Waves per SIMD that the register allocation of a run scan must allow: the
// occupancy its LDS allows (a workgroup of 256 threads holds about KIB KiB per
// item per thread, of 160 KiB per CU, and puts one wave on each SIMD), but no
// more than 6, above which the keys held for the next tile would spill.
template <int ITEMS, int KIB>
constexpr int scan_waves() {
  return 160 / (KIB * ITEMS) < 6 ? 160 / (KIB * ITEMS) : 6;
}

// ROWS_LDS: row heads are staged in LDS and written by consecutive threads
// (coalesced; for segments with many sources). Without it each thread writes
// its own row heads straight from registers, which frees 4 B of LDS per key:
// at 16 keys per thread a third workgroup fits on a CU, for one large segment
// (where rows are few and the look-back's wait is what more workgroups hide).
template <int ITEMS, bool ROWS_LDS = true>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(scan_waves<ITEMS, ROWS_LDS || ITEMS < 16 ? 4 : 3>())))
void k_rle(RleArgs a) {
  constexpr int BLOCK = 256;
  constexpr int TILE = BLOCK * ITEMS;
  static_assert(ITEMS <= 32, "head masks are 32-bit");
  static_assert(TILE <= 65536, "tile positions are 16-bit");
  __shared__ uint64_t s_k[pd(TILE) + 1];  // s_k[pd(1 + i)] = key i of the tile
  __shared__ uint16_t s_hpos[TILE];   // link head positions in the tile
  __shared__ uint16_t s_rpos[ROWS_LDS ? TILE : 1];  // row head positions
  __shared__ uint16_t s_rlr[ROWS_LDS ? TILE : 1];   // tile-local link rank of each row head
  __shared__ uint32_t s_ch[ROWS_LDS ? 1 : kColDigits * kBins];  // column digit counts
  __shared__ uint64_t s_tmp[BLOCK / kWave];
  __shared__ uint64_t s_L0, s_R0, s_trail, s_base;
  __shared__ uint32_t s_next, s_next_w;

  const int tid = threadIdx.x, wv = tid / kWave;
  const uint64_t total = ld_const(a.tile_off + a.W);
  const bool in_place = a.ukeys == a.keys;
  const bool packed = a.lim < (1ull << 31);  // one look-back word per tile
  const bool col_hist = !ROWS_LDS && a.col_hist;
  if (col_hist)
    for (int i = tid; i < kColDigits * kBins; i += BLOCK) s_ch[i] = 0;
  if (wv == 3) claim_tile(a.ticket, a.tile_off, a.W, total, &s_next, &s_next_w);
  __syncthreads();
  ScanTile g = scan_tile(a.tile_off, a.seg_off, s_next, s_next_w, total, TILE);
  uint64_t kr[ITEMS], kprev = 0, knext = 0;
  scan_load<BLOCK, ITEMS>(a.keys, g, kr, kprev, knext, a.lim);

  while (g.t < total) {
    const uint32_t t = g.t, w = g.w, first = g.first, n = g.n;
    const uint64_t seg_lo = g.seg_lo, seg_hi = g.seg_hi, start = g.start;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t i = tid + k * BLOCK;
      if (i < n) s_k[pd(1 + i)] = kr[k];
    }
    if (tid == 0) {
      // predecessor of the tile's first key; at a segment start, a value that
      // differs from it in both halves so that position is a link and row head
      s_k[pd(0)] = start > seg_lo ? kprev : (kr[0] ^ 0xFFFFFFFF00000001ull);
    }
    __syncthreads();

    uint32_t lmask = 0, rmask = 0;
    const uint32_t p0 = tid * ITEMS;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t p = p0 + k;
      if (p < n) {
        const uint64_t cur = s_k[pd(1 + p)], prev = s_k[pd(p)];
        lmask |= (uint32_t)(cur != prev) << k;
        rmask |= (uint32_t)((cur >> 32) != (prev >> 32)) << k;
      }
    }
    uint64_t tot;
    const uint64_t x = block_excl_scan<BLOCK>(((uint64_t)__popc(rmask) << 32) | __popc(lmask),
                                              s_tmp, &tot);
    const uint32_t xl = (uint32_t)x, xr = (uint32_t)(x >> 32);
    const uint32_t TL = (uint32_t)tot, TR = (uint32_t)(tot >> 32);
    {
      uint32_t jl = xl, jr = xr;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (ROWS_LDS && (rmask & (1u << k))) {
          s_rpos[jr] = (uint16_t)(p0 + k);
          s_rlr[jr] = (uint16_t)jl;  // a row head is also a link head: its link rank
          ++jr;
        }
        if (lmask & (1u << k)) s_hpos[jl++] = (uint16_t)(p0 + k);
      }
    }
    // end of the tile's last run, searched past the tile by wave 2; in place, the
    // search must finish before this tile publishes (later tiles then write)
    if (wv == 2) {
      uint64_t e = start + n;
      if (TL > 0 && e < seg_hi) {
        const uint64_t K = s_k[pd(n)];
        if (knext == K) e = run_end_wave(a.keys, e, seg_hi, K);
      }
      if ((tid & (kWave - 1)) == 0) s_trail = e;
    }
    if (in_place) __syncthreads();
    if (packed) {
      // fewer than 2^31 keys in the launch: links and rows share one word
      // (rows << 31 | links; neither sum reaches 2^31), walked by one wave
      // (2^30 keys in one segment: 4.58 vs 4.72 ms with two channels)
      constexpr uint64_t M31 = (1ull << 31) - 1;
      const uint64_t mine = ((uint64_t)TR << 31) | TL;
      if (tid == 0) lb_store(a.lb + t, (t == 0 ? kLbInc : kLbAgg) | mine);
      if (wv == 0) {
        uint64_t excl = 0;
        if (t > 0) {
          excl = lb_walk_wave(a.lb, 1, 0, t);
          if (tid == 0) lb_store(a.lb + t, kLbInc | (excl + mine));
        }
        if (tid == 0) {
          s_L0 = excl & M31;
          s_R0 = excl >> 31;
        }
      }
    } else {
      if (tid < 2) lb_store(a.lb + 2ull * t + tid, (t == 0 ? kLbInc : kLbAgg) | (tid == 0 ? TL : TR));
      if (wv < 2) {  // wave 0 resolves the link channel, wave 1 the row channel
        const uint32_t ch = wv;
        uint64_t excl = 0;
        if (t > 0) {
          excl = lb_walk_wave(a.lb, 2, ch, t);
          if ((tid & (kWave - 1)) == 0) lb_store(a.lb + 2ull * t + ch, kLbInc | (excl + (ch ? TR : TL)));
        }
        if ((tid & (kWave - 1)) == 0) {
          if (ch == 0) s_L0 = excl; else s_R0 = excl;
        }
      }
    }
    __syncthreads();
    if (wv == 3) claim_tile(a.ticket, a.tile_off, a.W, total, &s_next, &s_next_w);
    __syncthreads();
    const uint64_t L0 = s_L0, R0 = s_R0, trail = s_trail;
    g = scan_tile(a.tile_off, a.seg_off, s_next, s_next_w, total, TILE);
    scan_load<BLOCK, ITEMS>(a.keys, g, kr, kprev, knext, a.lim);  // next tile, in flight below
    // positional per-segment output: global link index at this segment's start,
    // published by the segment's first tile (an earlier ticket, so it arrives)
    if (a.win_keys && tid == 0) {
      if (t == first) {
        lb_store(a.seg_base + w, kLbInc | L0);
        s_base = L0;
      } else {
        uint64_t v = lb_load(a.seg_base + w);
        while ((v >> 62) == 0) {
          __builtin_amdgcn_s_sleep(1);
          v = lb_load(a.seg_base + w);
        }
        s_base = v & kLbVal;
      }
      if (t + 1 == (uint32_t)a.tile_off[w + 1]) a.win_nnz[w] = L0 + TL - s_base;
    }
    if (tid == 0) {
      if (t == first) {
        a.link_off[w] = L0;
        a.row_off[w] = R0;
        for (int64_t v = (int64_t)w - 1; v >= 0 && a.seg_off[v] == a.seg_off[v + 1]; --v) {
          a.link_off[v] = L0;
          a.row_off[v] = R0;
        }
      }
      if (t == total - 1) {
        const uint64_t Le = L0 + TL, Re = R0 + TR;
        for (uint32_t v = w + 1; v <= a.W; ++v) {
          a.link_off[v] = Le;
          a.row_off[v] = Re;
        }
        if (a.rpos && in_bounds(Re, a.lim + 2)) {
          a.rpos[Re] = a.seg_off[a.W];
          a.rlink[Re] = Le;
        }
        if (a.nnz_out) *a.nnz_out = Le;
      }
    }
    if (a.win_keys) __syncthreads();  // s_base
    const uint64_t wpos = a.win_keys ? seg_lo + L0 - s_base : 0;
    for (uint32_t r = tid; r < TL; r += BLOCK) {
      const uint32_t p = s_hpos[r];
      const uint64_t K = s_k[pd(1 + p)];
      const uint64_t e = (r + 1 < TL) ? start + s_hpos[r + 1] : trail;
      const uint64_t cnt = e - (start + p);
      const uint64_t L = L0 + r;
      if (!in_bounds(L, a.lim)) continue;
      if (a.ukeys) a.ukeys[L] = K;
      if (a.counts) a.counts[L] = cnt;
      if (a.win_keys && in_bounds(wpos + r, a.lim)) {
        a.win_keys[wpos + r] = K;
        a.win_counts[wpos + r] = cnt;
      }
      if (a.items) a.items[L] = (K << 32) | cnt;
      if (col_hist) {  // the item's destination digits, for the column sort
#pragma unroll
        for (int q = 0; q < kColDigits; ++q)
          atomicAdd(&s_ch[q * kBins + (((uint32_t)K >> (8 * q)) & 255)], 1u);
      }
    }
    if (ROWS_LDS && a.rpos) {
      for (uint32_t q = tid; q < TR; q += BLOCK) {
        if (!in_bounds(R0 + q, a.lim + 2)) continue;
        a.rpos[R0 + q] = start + s_rpos[q];
        a.rlink[R0 + q] = L0 + s_rlr[q];
      }
    }
    if (!ROWS_LDS && a.rpos && rmask) {  // each thread writes its own row heads
      uint32_t q = xr;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (rmask & (1u << k)) {
          if (in_bounds(R0 + q, a.lim + 2)) {
            a.rpos[R0 + q] = start + p0 + k;
            // a row head is also a link head: its link index
            a.rlink[R0 + q] = L0 + xl + __popc(lmask & ((1u << k) - 1u));
          }
          ++q;
        }
      }
    }
    __syncthreads();
  }
  if (col_hist) {  // after the loop's last barrier: this workgroup's counts
    for (int i = tid; i < kColDigits * kBins; i += BLOCK)
      if (s_ch[i]) atomicAdd(&a.col_hist[i], s_ch[i]);
  }
}

// ---------------------------------------------------------------------------
// Run reduction over a sorted array with explicit values.
// mode 0 (rows of a matrix): group = source, value = A(i,j); every link also
//   emits its column item dst<<32|count.
// mode 1 (columns): group = destination of a sorted column item, value = the
//   item's count.
// Heads are compacted with a two-channel look-back (heads, value prefix); each
// head stores its position and the exclusive value prefix, so consecutive
// heads give run length (fan-out / fan-in) and run sum (packets). Tiles come
// one ahead as in k_rle.
// WIDE (matrices of 2^32 packets or more, whose counts and run sums need 64
// bits): values and their tile sums are 64-bit, a column item carries the
// link's index in the matrix instead of its count (dst<<32 | link index, so
// the matrix has fewer than 2^32 links), and the column runs read the count
// of each item's link from `gather` (the matrix counts).
// ---------------------------------------------------------------------------
template <int ITEMS, int MODE, bool WIDE = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(scan_waves<ITEMS, WIDE ? 7 : 5>())))
void k_runs(RunArgs a) {
  constexpr int BLOCK = 256;
  constexpr int TILE = BLOCK * ITEMS;
  static_assert(TILE <= 65536, "tile positions are 16-bit");
  using V = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
  __shared__ uint64_t s_g[pd(TILE) + 1];  // s_g[pd(1 + i)]: group key (a 32-bit address; 2^32 marks "none")
  __shared__ V s_v[pd(TILE)];             // s_v[pd(i)]: value (< 2^32 unless WIDE)
  __shared__ uint16_t s_hp[TILE];      // head local positions
  __shared__ V s_hv[TILE];             // tile-local exclusive value prefix at head
  __shared__ uint64_t s_tmp[BLOCK / kWave];
  __shared__ uint64_t s_H0, s_V0;
  __shared__ uint32_t s_next, s_next_w;

  const int tid = threadIdx.x, wv = tid / kWave;
  const uint64_t total = ld_const(a.tile_off + a.W);
  // heads and values in one look-back word per tile when both sums stay below 2^31
  const bool packed = !WIDE && a.lim < (1ull << 31) && a.vlim && a.vlim < (1ull << 31);
  if (wv == 3) claim_tile(a.ticket, a.tile_off, a.W, total, &s_next, &s_next_w);
  __syncthreads();
  ScanTile g = scan_tile(a.tile_off, a.seg_off, s_next, s_next_w, total, TILE);
  uint64_t kr[ITEMS], cr[ITEMS], kprev = 0, knext = 0;
  auto load = [&]() {
    scan_load<BLOCK, ITEMS>(a.keys, g, kr, kprev, knext, a.lim);
    if (MODE == 0) {
      uint32_t tb = tid;
      asm volatile("" : "+v"(tb));
      const uint64_t *base = a.counts + g.start;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t i = tb + k * BLOCK;
        cr[k] = i < g.n && in_bounds(g.start + i, a.lim) ? base[i] : 0;
      }
    }
  };
  load();

  while (g.t < total) {
    const uint32_t t = g.t, w = g.w, first = g.first, n = g.n;
    const uint64_t seg_lo = g.seg_lo, start = g.start;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t i = tid + k * BLOCK;
      if (i < n) {
        s_g[pd(1 + i)] = kr[k] >> 32;
        if (MODE == 0) {
          s_v[pd(i)] = (V)cr[k];
          if (a.items && in_bounds(start + i, a.lim))
            a.items[start + i] = (kr[k] << 32) | (WIDE ? start + i : cr[k]);
        } else if (WIDE) {
          s_v[pd(i)] = in_bounds((uint32_t)kr[k], a.lim) ? a.gather[(uint32_t)kr[k]] : 0;
        } else {
          s_v[pd(i)] = (uint32_t)kr[k];
        }
      }
    }
    if (tid == 0) s_g[pd(0)] = start > seg_lo ? (kprev >> 32) : ~0ull;
    __syncthreads();

    uint32_t hmask = 0;
    V vsum = 0;
    const uint32_t p0 = tid * ITEMS;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t p = p0 + k;
      if (p < n) {
        hmask |= (uint32_t)(s_g[pd(1 + p)] != s_g[pd(p)]) << k;
        vsum += s_v[pd(p)];
      }
    }
    V xv, TV;
    uint32_t xh, TH;
    if constexpr (WIDE) {  // heads and 64-bit values in two scans
      uint64_t th, tv;
      xh = (uint32_t)block_excl_scan<BLOCK>(__popc(hmask), s_tmp, &th);
      xv = block_excl_scan<BLOCK>(vsum, s_tmp, &tv);
      TH = (uint32_t)th;
      TV = tv;
    } else {  // both in one 64-bit scan: heads in the high half, values in the low
      uint64_t tot;
      const uint64_t x = block_excl_scan<BLOCK>(((uint64_t)__popc(hmask) << 32) | vsum, s_tmp, &tot);
      xv = (uint32_t)x;
      xh = (uint32_t)(x >> 32);
      TV = (uint32_t)tot;
      TH = (uint32_t)(tot >> 32);
    }
    {
      uint32_t jh = xh;
      V run = xv;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t p = p0 + k;
        if (hmask & (1u << k)) {
          s_hp[jh] = (uint16_t)p;
          s_hv[jh] = run;
          ++jh;
        }
        if (p < n) run += s_v[pd(p)];
      }
    }
    if (packed) {  // values << 31 | heads, walked by one wave
      constexpr uint64_t M31 = (1ull << 31) - 1;
      const uint64_t mine = ((uint64_t)TV << 31) | TH;
      if (tid == 0) lb_store(a.lb + t, (t == 0 ? kLbInc : kLbAgg) | mine);
      if (wv == 0) {
        uint64_t excl = 0;
        if (t > 0) {
          excl = lb_walk_wave(a.lb, 1, 0, t);
          if (tid == 0) lb_store(a.lb + t, kLbInc | (excl + mine));
        }
        if (tid == 0) {
          s_H0 = excl & M31;
          s_V0 = excl >> 31;
        }
      }
    } else {
      if (tid < 2) lb_store(a.lb + 2ull * t + tid, (t == 0 ? kLbInc : kLbAgg) | (tid == 0 ? TH : TV));
      if (wv < 2) {  // wave 0: head channel, wave 1: value channel
        const uint32_t ch = wv;
        uint64_t excl = 0;
        if (t > 0) {
          excl = lb_walk_wave(a.lb, 2, ch, t);
          if ((tid & (kWave - 1)) == 0) lb_store(a.lb + 2ull * t + ch, kLbInc | (excl + (ch ? TV : TH)));
        }
        if ((tid & (kWave - 1)) == 0) {
          if (ch == 0) s_H0 = excl; else s_V0 = excl;
        }
      }
    }
    __syncthreads();
    if (wv == 3) claim_tile(a.ticket, a.tile_off, a.W, total, &s_next, &s_next_w);
    __syncthreads();
    const uint64_t H0 = s_H0, V0 = s_V0;
    g = scan_tile(a.tile_off, a.seg_off, s_next, s_next_w, total, TILE);
    load();  // next tile, in flight below
    if (tid == 0) {
      if (t == first) {
        a.head_off[w] = H0;
        for (int64_t v = (int64_t)w - 1; v >= 0 && a.seg_off[v] == a.seg_off[v + 1]; --v)
          a.head_off[v] = H0;
      }
      if (t == total - 1) {
        const uint64_t He = H0 + TH;
        for (uint32_t v = w + 1; v <= a.W; ++v) a.head_off[v] = He;
        if (in_bounds(He, a.lim + 2)) {
          a.hpos[He] = a.seg_off[a.W];
          a.hval[He] = V0 + TV;
        }
      }
    }
    for (uint32_t h = tid; h < TH; h += BLOCK) {
      if (!in_bounds(H0 + h, a.lim + 2)) continue;
      a.hpos[H0 + h] = start + s_hp[h];
      a.hval[H0 + h] = V0 + s_hv[h];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Batches of at most kSmallMax packets in total: each window goes through the
// whole per-window pipeline inside one workgroup and its LDS, in one launch
// (the multi-kernel pipeline spends most of such a batch starting and
// draining some twenty-five launches). Steps, all on LDS: the stable LSD
// radix sort of the packed keys (8 byte-digit passes with the same wave
// ranking as the radix passes, keys in registers between passes, the LDS
// array as the scatter target); link and row heads by comparing neighbours
// in the sorted keys, ranked by a block scan; each link's count (distance to
// the next link head) and key, written as the window's matrix at its packet
// offset; row maxima from consecutive row heads; the column items
// destination << 32 | count sorted by destination (4 passes); column heads,
// and per column the packet sum and link count accumulated in LDS (both
// below 2^16 here, so one 32-bit word holds the pair); then the eight
// quantities of Table I and Sec. IV. Windows go to workgroups round robin.
// ---------------------------------------------------------------------------
template <int ITEMS, int NW>
__device__ __forceinline__ void small_sort(uint64_t (&key)[ITEMS], uint32_t n, uint32_t shift0,
                                           int passes, uint64_t *s_keys,
                                           uint32_t (*s_wcnt)[kBins], uint32_t *s_part) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t wbase = wv * (kWave * ITEMS);
  for (int p = 0; p < passes; ++p) {
    uint32_t dig[ITEMS], rank[ITEMS];
    rank_tile<ITEMS, false>(key, shift0 + 8 * p, n, wbase, lane, dig, rank, s_wcnt[wv]);
    __syncthreads();
    uint32_t tot, lstart;
    tile_offsets<NW>(s_wcnt, s_part, tid, &tot, &lstart, [](uint32_t) {});
    place_tile<ITEMS, false>(key, dig, rank, s_wcnt[wv], s_keys);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t i = wbase + k * kWave + lane;
      key[k] = i < n ? s_keys[i] : 0;
    }
    for (int i = tid; i < NW * kBins; i += NW * kWave) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
  }
}

template <int NW>
__device__ __forceinline__ uint64_t block_max(uint64_t v, uint64_t *s_tmp) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  v = wave_max(v);
  if (lane == 0) s_tmp[wv] = v;
  __syncthreads();
  uint64_t m = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) m = s_tmp[q] > m ? s_tmp[q] : m;
  __syncthreads();
  return m;
}

__global__ __launch_bounds__(kSmallBlock) void k_small(const uint32_t *src, const uint32_t *dst,
                                                       const uint64_t *off, uint32_t W,
                                                       uint64_t *stats, uint64_t *win_keys,
                                                       uint64_t *win_counts, uint64_t *win_nnz) {
  constexpr int BLOCK = kSmallBlock, ITEMS = kSmallMax / kSmallBlock, NW = BLOCK / kWave;
  constexpr uint32_t TILE = kSmallMax;
  static_assert(BLOCK >= kBins && ITEMS <= 32, "tile layout");
  __shared__ uint64_t s_keys[TILE];        // sort target; then the column items
  __shared__ uint32_t s_wcnt[NW][kBins];
  __shared__ uint32_t s_part[kBins / kWave];
  __shared__ uint16_t s_hpos[TILE];        // link head positions
  __shared__ uint32_t s_aux[TILE];         // row heads (position << 16 | link rank), then columns
  __shared__ uint64_t s_tmp[NW];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t wbase = wv * (kWave * ITEMS);
  for (int i = tid; i < NW * kBins; i += BLOCK) (&s_wcnt[0][0])[i] = 0;
  __syncthreads();
  for (uint32_t w = blockIdx.x; w < W; w += gridDim.x) {
    const uint64_t lo = off[w];
    const uint64_t n64 = off[w + 1] - lo;
    if (n64 > TILE) {  // the host sends only batches that fit
      if (tid == 0) atomicOr(&g_status, 2);
      continue;
    }
    const uint32_t n = (uint32_t)n64;
    // 1. keys, sorted
    uint64_t key[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t i = wbase + k * kWave + lane;
      key[k] = i < n ? pack_key(src[lo + i], dst[lo + i]) : 0;
    }
    small_sort<ITEMS, NW>(key, n, 0, 8, s_keys, s_wcnt, s_part);
    // 2. link and row heads (each thread: ITEMS consecutive positions)
    const uint32_t p0 = tid * ITEMS;
    uint32_t lmask = 0, rmask = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t p = p0 + k;
      if (p < n) {
        const uint64_t cur = s_keys[p];
        const uint64_t prev = p ? s_keys[p - 1] : cur ^ 0xFFFFFFFF00000001ull;
        lmask |= (uint32_t)(cur != prev) << k;
        rmask |= (uint32_t)((cur >> 32) != (prev >> 32)) << k;
      }
    }
    uint64_t tot;
    const uint64_t x = block_excl_scan<BLOCK>(((uint64_t)__popc(rmask) << 32) | __popc(lmask),
                                              s_tmp, &tot);
    const uint32_t TL = (uint32_t)tot, TR = (uint32_t)(tot >> 32);
    {
      uint32_t jl = (uint32_t)x, jr = (uint32_t)(x >> 32);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (rmask & (1u << k)) s_aux[jr++] = ((p0 + k) << 16) | jl;
        if (lmask & (1u << k)) s_hpos[jl++] = (uint16_t)(p0 + k);
      }
    }
    __syncthreads();
    // 3. links: the window's matrix and its column items (kept in registers)
    uint64_t item[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t r = tid + j * BLOCK;
      item[j] = 0;
      if (r < TL) {
        const uint32_t pos = s_hpos[r];
        const uint32_t e = r + 1 < TL ? s_hpos[r + 1] : n;
        const uint64_t K = s_keys[pos];
        const uint32_t cnt = e - pos;
        if (win_keys) {
          win_keys[lo + r] = K;
          win_counts[lo + r] = cnt;
        }
        item[j] = (K << 32) | cnt;
      }
    }
    // 4. rows: packets and links between consecutive row heads
    uint64_t mpk = 0, mfan = 0;
    for (uint32_t q = tid; q < TR; q += BLOCK) {
      const uint32_t a = s_aux[q];
      const uint32_t b = q + 1 < TR ? s_aux[q + 1] : (n << 16) | TL;
      const uint64_t pk = (b >> 16) - (a >> 16), fan = (b & 0xFFFFu) - (a & 0xFFFFu);
      mpk = pk > mpk ? pk : mpk;
      mfan = fan > mfan ? fan : mfan;
    }
    __syncthreads();  // s_keys, s_hpos and s_aux are free
    // 5. column items sorted by destination
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t r = tid + j * BLOCK;
      if (r < TL) s_keys[r] = item[j];
    }
    for (uint32_t i = tid; i < TL; i += BLOCK) s_aux[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t i = wbase + k * kWave + lane;
      key[k] = i < TL ? s_keys[i] : 0;
    }
    small_sort<ITEMS, NW>(key, TL, 32, 4, s_keys, s_wcnt, s_part);
    // 6. columns: heads ranked by a block scan, packet sum and link count per
    // column accumulated in LDS (sum << 16 | count, each below 2^16)
    uint32_t cmask = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t p = p0 + k;
      if (p < TL) cmask |= (uint32_t)(p == 0 || (s_keys[p] >> 32) != (s_keys[p - 1] >> 32)) << k;
    }
    uint64_t ctot;
    const uint32_t xc = (uint32_t)block_excl_scan<BLOCK>((uint64_t)__popc(cmask), s_tmp, &ctot);
    const uint32_t TC = (uint32_t)ctot;
    {
      int64_t c = (int64_t)xc - 1;  // a thread's first item continues the column before it
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t p = p0 + k;
        if (p < TL) {
          c += (cmask >> k) & 1;
          atomicAdd(&s_aux[c], (uint32_t)((s_keys[p] & 0xFFFFFFFFu) << 16) | 1u);
        }
      }
    }
    __syncthreads();
    uint64_t mdp = 0, mfi = 0;
    for (uint32_t c = tid; c < TC; c += BLOCK) {
      const uint32_t v = s_aux[c];
      mdp = (v >> 16) > mdp ? (v >> 16) : mdp;
      mfi = (v & 0xFFFFu) > mfi ? (v & 0xFFFFu) : mfi;
    }
    mpk = block_max<NW>(mpk, s_tmp);
    mfan = block_max<NW>(mfan, s_tmp);
    mdp = block_max<NW>(mdp, s_tmp);
    mfi = block_max<NW>(mfi, s_tmp);
    if (tid == 0) {
      if (stats) {
        uint64_t *o = stats + (uint64_t)w * 8;
        o[0] = n;
        o[1] = TL;
        o[2] = TR;
        o[3] = TC;
        o[4] = mpk;
        o[5] = mfan;
        o[6] = mdp;
        o[7] = mfi;
      }
      if (win_nnz) win_nnz[w] = TL;
    }
    __syncthreads();  // LDS reused by the next window
  }
}

// ---------------------------------------------------------------------------
// Hypersparse CSR to sorted COO (Sec. IV, "Data Representation": the
// challenge's matrices come as CSR; the statistics here read the flat
// entries). Row r (source address rows[r]) holds entries [row_ptr[r],
// row_ptr[r+1]) of cols (destination addresses) and vals (A(i,j)); entry e
// becomes key rows[r] << 32 | cols[e] with count vals[e]. Each thread expands
// ITEMS consecutive entries: it bisects row_ptr for the row of its first
// entry and then steps through the rows; every read stays inside the arrays
// whatever their contents. Keys must increase strictly over the whole matrix,
// values must lie in [1, 2^32) (the column items hold a count in 32 bits; with
// fewer than 2^32 entries their sum then cannot wrap) and row_ptr must run
// from 0 to nnz without decreasing (every row pointer is also compared with
// the next one, in a grid-stride sweep over the rows): a violation raises
// the device status (invalid argument).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_csr_expand(const uint32_t *rows, const uint64_t *row_ptr,
                                                    uint64_t nrows, const uint32_t *cols,
                                                    const uint64_t *vals, uint64_t nnz,
                                                    uint64_t *keys, uint64_t *counts,
                                                    uint64_t *nnz_out) {
  constexpr int ITEMS = 8;
  const uint64_t e0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * ITEMS;
  bool bad = false;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *nnz_out = nnz;
    bad = row_ptr[0] != 0 || row_ptr[nrows] != nnz;
  }
  if (e0 < nnz) {
    uint64_t lo = 0, hi = nrows;  // row of e0: the last r < nrows with row_ptr[r] <= e0
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (row_ptr[mid] <= e0) lo = mid; else hi = mid;
    }
    uint64_t r = lo, prev = 0;
    bool has_prev = false;
    if (e0 > 0) {  // the entry before this thread's first, for the order check
      uint64_t rp = r;
      while (rp > 0 && row_ptr[rp] > e0 - 1) --rp;
      prev = ((uint64_t)rows[rp] << 32) | cols[e0 - 1];
      has_prev = true;
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint64_t e = e0 + k;
      if (e >= nnz) break;
      while (r + 1 < nrows && row_ptr[r + 1] <= e) ++r;
      const uint64_t key = ((uint64_t)rows[r] << 32) | cols[e], c = vals[e];
      bad |= c == 0 || (c >> 32) != 0 || (has_prev && key <= prev);
      prev = key;
      has_prev = true;
      keys[e] = key;
      counts[e] = c;
    }
  }
  for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < nrows;
       r += (uint64_t)gridDim.x * 256)
    bad |= row_ptr[r] > row_ptr[r + 1];
  if (bad) atomicOr(&g_status, 4);
}

// The packet total of a CSR input (its valid packets, stats[0], the sum of
// the values) against the caller's bound on it: a larger sum raises the device
// status (invalid argument).
__global__ void k_check_total(const uint64_t *stats, uint64_t packets) {
  if (threadIdx.x == 0 && stats[0] > packets) atomicOr(&g_status, 4);
}

// ---------------------------------------------------------------------------
// Largest link count per window (Sec. IV, "Analytics and Operations": maximum
// link counts). Window w's counts sit at [off[w], off[w] + nnz[w]) (the
// positional layout of the batched per-window matrices); with off == nullptr
// there is one window at [0, nnz[0]). Each workgroup reduces one contiguous
// range of positions, window by window, and raises out[w] with one atomic
// per window it touches; out must start at zero.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_max_counts(const uint64_t *counts, const uint64_t *off,
                                                    const uint64_t *nnz, uint32_t W,
                                                    uint64_t total, uint64_t *out) {
  __shared__ uint64_t s_m[4];
  const uint64_t per = (total + gridDim.x - 1) / gridDim.x;
  const uint64_t p0 = (uint64_t)blockIdx.x * per, p1 = min(total, p0 + per);
  if (p0 >= p1) return;  // the whole workgroup leaves together
  uint32_t w = off ? find_owner_wave(off, W, p0) : 0;
  for (; w < W; ++w) {
    const uint64_t lo = off ? off[w] : 0;
    if (lo >= p1) break;
    const uint64_t hi = lo + nnz[w];
    const uint64_t a = max(lo, p0), b = min(hi, p1);
    uint64_t m = 0;
    for (uint64_t p = a + threadIdx.x; p < b; p += 256) m = max(m, counts[p]);
    m = wave_max(m);
    if ((threadIdx.x & (kWave - 1)) == 0) s_m[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint64_t v = max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
      if (v > lb_load(out + w)) atomicMax(reinterpret_cast<unsigned long long *>(out + w), (unsigned long long)v);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-segment maxima of consecutive-head differences. Each workgroup takes one
// contiguous range of heads, splits it at segment boundaries (usually none or
// one), reduces each piece with wave and LDS maxima and issues one 64-bit
// atomic per piece and field.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_segmax(const uint64_t *a, const uint64_t *b,
                                                const uint64_t *head_off, uint32_t W,
                                                uint64_t *stats, int fa, int fb) {
  __shared__ uint64_t s_ma[4], s_mb[4];
  const uint64_t total = head_off[W];
  const uint64_t chunk = (total + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = blockIdx.x * chunk, hi = min(lo + chunk, total);
  if (lo >= hi) return;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t w0 = find_owner_wave(head_off, W, lo), w1 = find_owner_wave(head_off, W, hi - 1);
  for (uint32_t w = w0; w <= w1; ++w) {
    const uint64_t plo = max(lo, head_off[w]), phi = min(hi, head_off[w + 1]);
    if (plo >= phi) continue;  // uniform: every thread sees the same bounds
    uint64_t ma = 0, mb = 0;
    constexpr int R = 4;  // rounds of loads issued together
    for (uint64_t r0 = plo + tid; r0 < phi; r0 += R * 256) {
      uint64_t a0[R], a1[R], b0[R], b1[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const uint64_t r = r0 + q * 256;
        const bool in = r < phi;
        a0[q] = in ? a[r] : 0;
        a1[q] = in ? a[r + 1] : 0;
        b0[q] = in ? b[r] : 0;
        b1[q] = in ? b[r + 1] : 0;
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const uint64_t da = a1[q] - a0[q], db = b1[q] - b0[q];
        ma = ma > da ? ma : da;
        mb = mb > db ? mb : db;
      }
    }
    ma = wave_max(ma);
    mb = wave_max(mb);
    if (lane == 0) {
      s_ma[wv] = ma;
      s_mb[wv] = mb;
    }
    __syncthreads();
    if (tid == 0) {
      for (int q = 1; q < 4; ++q) {
        ma = ma > s_ma[q] ? ma : s_ma[q];
        mb = mb > s_mb[q] ? mb : s_mb[q];
      }
      // With many workgroups per window their atomics would queue on the same
      // two words; maxima only grow, so a value not above the one already there
      // (even a stale read of it) needs none, and few workgroups issue one.
      uint64_t *pa = &stats[(uint64_t)w * 8 + fa], *pb = &stats[(uint64_t)w * 8 + fb];
      const bool crowded = gridDim.x > 8ull * W;
      if (!crowded || ma > lb_load(pa)) atomicMax((unsigned long long *)pa, (unsigned long long)ma);
      if (!crowded || mb > lb_load(pb)) atomicMax((unsigned long long *)pb, (unsigned long long)mb);
    }
    __syncthreads();
  }
}

__global__ void k_finalize(const uint64_t *seg_off, const uint64_t *link_off,
                           const uint64_t *row_off, const uint64_t *col_off, uint32_t W,
                           uint64_t *stats) {
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < W; w += gridDim.x * blockDim.x) {
    uint64_t *s = stats + (uint64_t)w * 8;
    s[0] = seg_off[w + 1] - seg_off[w];
    s[1] = link_off[w + 1] - link_off[w];
    s[2] = row_off[w + 1] - row_off[w];
    s[3] = col_off[w + 1] - col_off[w];
  }
}

// Matrix totals: with row_hval, valid packets (the row pass's value sentinel =
// sum of all counts), unique links and unique sources; with col_off, unique
// destinations.
__global__ void k_finalize_matrix(const uint64_t *row_hval, const uint64_t *row_off,
                                  const uint64_t *col_off, const uint64_t *nnz, uint64_t *stats) {
  if (threadIdx.x == 0) {
    if (row_hval) {
      stats[0] = row_hval[row_off[1]];
      stats[1] = *nnz;
      stats[2] = row_off[1];
    }
    if (col_off) stats[3] = col_off[1];
  }
}

// ---------------------------------------------------------------------------
// Union-add / subtract of two sorted COO matrices by merge path.
// Merged order puts A's entry before B's on equal keys, so equal keys are
// adjacent: the A entry absorbs B's count (plus or minus) and the B entry is
// dropped; for subtraction, entries that reach zero are dropped and a B entry
// without a matching, large-enough A entry raises the device error word.
// Kept entries are compacted with a one-channel look-back.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t merge_split(const uint64_t *A, uint64_t na, const uint64_t *B,
                                                uint64_t nb, uint64_t d) {
  uint64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (A[mid] <= B[d - mid - 1]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_merge(MergeArgs a) {
  constexpr int BLOCK = 256, ITEMS = 8, TILE = BLOCK * ITEMS;
  __shared__ uint64_t s_k[TILE];
  __shared__ uint64_t s_c[TILE];
  __shared__ uint64_t s_tmp[BLOCK / kWave];
  __shared__ uint64_t s_i0, s_i1, s_L0;
  __shared__ uint64_t s_prevA, s_nextB, s_nextBc;
  __shared__ int s_hasPrevA, s_hasNextB;
  __shared__ uint32_t s_tile;

  const int tid = threadIdx.x;
  const uint64_t na = min(*a.na, a.na_max), nb = min(*a.nb, a.nb_max), ntot = na + nb;
  const uint64_t tiles = (ntot + TILE - 1) / TILE;
  if (ntot == 0) {
    if (blockIdx.x == 0 && tid == 0) *a.nc = 0;
    return;
  }
  for (;;) {
    if (tid == 0) s_tile = atomicAdd(a.ticket, 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    if (t >= tiles) break;
    const uint64_t d0 = (uint64_t)t * TILE, d1 = min(d0 + TILE, ntot);
    if (tid == 0) s_i0 = merge_split(a.ka, na, a.kb, nb, d0);
    if (tid == kWave) s_i1 = merge_split(a.ka, na, a.kb, nb, d1);
    __syncthreads();
    const uint64_t i0 = s_i0, i1 = s_i1, j0 = d0 - i0, j1 = d1 - i1;
    const uint32_t la = (uint32_t)(i1 - i0), lb = (uint32_t)(j1 - j0);
    for (uint32_t i = tid; i < la; i += BLOCK) {
      s_k[i] = a.ka[i0 + i];
      s_c[i] = a.ca[i0 + i];
    }
    for (uint32_t i = tid; i < lb; i += BLOCK) {
      s_k[la + i] = a.kb[j0 + i];
      s_c[la + i] = a.cb[j0 + i];
    }
    if (tid == 0) {
      s_hasPrevA = i0 > 0;
      s_prevA = i0 > 0 ? a.ka[i0 - 1] : 0;
      s_hasNextB = j1 < nb;
      s_nextB = j1 < nb ? a.kb[j1] : 0;
      s_nextBc = j1 < nb ? a.cb[j1] : 0;
    }
    __syncthreads();
    const uint64_t *sa = s_k, *sca = s_c, *sb = s_k + la, *scb = s_c + la;
    // this thread's share of the tile's merged positions
    const uint32_t dd0 = min((uint32_t)(tid * ITEMS), la + lb);
    const uint32_t dd1 = min((uint32_t)((tid + 1) * ITEMS), la + lb);
    uint32_t ia;
    {
      uint32_t lo = dd0 > lb ? dd0 - lb : 0, hi = dd0 < la ? dd0 : la;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sa[mid] <= sb[dd0 - mid - 1]) lo = mid + 1; else hi = mid;
      }
      ia = lo;
    }
    uint32_t ib = dd0 - ia;
    uint64_t ok[ITEMS], oc[ITEMS];
    uint32_t kmask = 0;
    bool underflow = false;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      ok[k] = 0;
      oc[k] = 0;
      if (dd0 + k < dd1) {
        const bool takeA = ib >= lb || (ia < la && sa[ia] <= sb[ib]);
        if (takeA) {
          const uint64_t key = sa[ia], c = sca[ia];
          bool hasB;
          uint64_t bk, bc;
          if (ib < lb) {
            hasB = true;
            bk = sb[ib];
            bc = scb[ib];
          } else {
            hasB = s_hasNextB;
            bk = s_nextB;
            bc = s_nextBc;
          }
          const bool matched = hasB && bk == key;
          uint64_t out = c;
          if (matched) {
            if (a.sign > 0) {
              out = c + bc;
            } else if (bc > c) {
              underflow = true;
              out = 0;
            } else {
              out = c - bc;
            }
          }
          if (out != 0) {
            ok[k] = key;
            oc[k] = out;
            kmask |= 1u << k;
          }
          ++ia;
        } else {
          const uint64_t key = sb[ib], c = scb[ib];
          const bool hasA = ia > 0 || s_hasPrevA;
          const uint64_t ak = ia > 0 ? sa[ia - 1] : s_prevA;
          if (!(hasA && ak == key)) {  // unmatched B entry
            if (a.sign > 0) {
              ok[k] = key;
              oc[k] = c;
              kmask |= 1u << k;
            } else {
              underflow = true;
            }
          }
          ++ib;
        }
      }
    }
    const uint32_t keep = __popc(kmask);
    if (underflow) atomicOr(&g_status, 1);
    uint64_t tot;
    const uint64_t x = block_excl_scan<BLOCK>(keep, s_tmp, &tot);
    if (tid == 0) lb_store(a.lb + t, (t == 0 ? kLbInc : kLbAgg) | tot);
    if (tid < kWave) {
      uint64_t excl = 0;
      if (t > 0) {
        excl = lb_walk_wave(a.lb, 1, 0, t);
        if (tid == 0) lb_store(a.lb + t, kLbInc | (excl + tot));
      }
      if (tid == 0) {
        s_L0 = excl;
        if (t == tiles - 1) {
          // a union larger than the output's capacity keeps its first entries
          // and raises the device status (capacity)
          const uint64_t nc = excl + tot;
          if (nc > a.nc_max) atomicOr(&g_status, 2);
          *a.nc = min(nc, a.nc_max);
        }
      }
    }
    __syncthreads();  // everyone is done reading s_k / s_c
    {
      uint32_t pos = (uint32_t)x;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (kmask & (1u << k)) {
          s_k[pos] = ok[k];
          s_c[pos] = oc[k];
          ++pos;
        }
      }
    }
    __syncthreads();
    const uint64_t L0 = s_L0;
    const uint32_t room = L0 < a.nc_max ? (uint32_t)min((uint64_t)tot, a.nc_max - L0) : 0u;
    for (uint32_t i = tid; i < room; i += BLOCK) {
      a.kc[L0 + i] = s_k[i];
      a.cc[L0 + i] = s_c[i];
    }
    __syncthreads();
  }
}

// ===========================================================================
// host launchers
// ===========================================================================
thread_local int tl_timing_kind = -1;

// Launch, with start/stop events taken by the dispatch itself when timing is on
// (hipExtLaunchKernelGGL), so a recorded duration is the kernel's own.
#define NS_LAUNCH(kernel, grid, block, stream, ...)                                        \
  do {                                                                                     \
    hipEvent_t e0_ = nullptr, e1_ = nullptr;                                               \
    if (tl_timing_kind >= 0 && hipEventCreate(&e0_) == hipSuccess &&                        \
        hipEventCreate(&e1_) == hipSuccess) {                                              \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, e0_, e1_, 0, __VA_ARGS__);      \
      record_timing(tl_timing_kind, e0_, e1_);                                             \
    } else {                                                                               \
      hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);                     \
    }                                                                                      \
  } while (0)

namespace {

int device_id() {
  int d = 0;
  hipGetDevice(&d);
  return d;
}

int cu_count() {
  static int cus[64] = {0};
  const int d = device_id();
  if (d < 64 && cus[d]) return cus[d];
  int v = 0;
  hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d);
  if (v <= 0) v = 256;
  if (d < 64) cus[d] = v;
  return v;
}

// resident workgroups of `fn` at `block` threads on the current device
template <typename F>
uint64_t resident(F fn, int block) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, block, 0) != hipSuccess || per <= 0)
    per = 1;
  return (uint64_t)per * cu_count();
}

uint32_t clamp_grid(uint64_t want, uint64_t cap) {
  uint64_t g = want < cap ? want : cap;
  if (g == 0) g = 1;
  return (uint32_t)g;
}

}  // namespace

hipError_t launch_fill64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t g = clamp_grid((n + 255) / 256, 4096);
  NS_LAUNCH(k_fill64, dim3(g), dim3(256), s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_copy64(uint64_t *dst, const uint64_t *src, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  NS_LAUNCH(k_copy64, dim3(clamp_grid((n + 255) / 256, 4096)), dim3(256), s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_fill_multi(const FillList &f, hipStream_t s) {
  uint64_t most = 0;
  for (uint32_t q = 0; q < f.count; ++q) most = f.e[q].n > most ? f.e[q].n : most;
  if (most == 0) return hipSuccess;
  NS_LAUNCH(k_fill_multi, dim3(clamp_grid((most + 255) / 256, 4096)), dim3(256), s, f);
  return hipGetLastError();
}

hipError_t launch_max_counts(const uint64_t *counts, const uint64_t *off, const uint64_t *nnz,
                             uint32_t W, uint64_t total, uint64_t *out, hipStream_t s) {
  hipError_t e = launch_fill64(out, W, 0, s);
  if (e != hipSuccess || total == 0) return e;
  NS_LAUNCH(k_max_counts, dim3(clamp_grid((total + 4095) / 4096, 2048)), dim3(256), s, counts,
            off, nnz, W, total, out);
  return hipGetLastError();
}

hipError_t launch_fill32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t g = clamp_grid((n + 255) / 256, 4096);
  NS_LAUNCH(k_fill32, dim3(g), dim3(256), s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_seg1(uint64_t *seg, const uint64_t *n_dev, uint64_t n, hipStream_t s) {
  NS_LAUNCH(k_seg1, dim3(1), dim3(64), s, seg, n_dev, n);
  return hipGetLastError();
}

hipError_t launch_tiles(const uint64_t *seg_off, uint32_t W, uint32_t ta, uint64_t *oa,
                        uint32_t tb, uint64_t *ob, uint32_t tc, uint64_t *oc, hipStream_t s) {
  NS_LAUNCH(k_tiles, dim3(1), dim3(1024), s, seg_off, W, ta, oa, tb, ob, tc, oc);
  return hipGetLastError();
}

// Histogram workgroups: four tiles each, since every flush of a workgroup's
// counters costs one global atomic per bin and fewer, longer ranges cost fewer
// atomics; but at least one tile each up to 64 workgroups, so that a small
// batch is not counted by a handful of workgroups.
static uint64_t hist_blocks(uint64_t tiles) {
  const uint64_t four = (tiles + 3) / 4, floor = tiles < 64 ? tiles : 64;
  return four > floor ? four : floor;
}

hipError_t launch_hist_packets(const uint32_t *src, const uint32_t *dst, const uint64_t *seg_off,
                               const uint64_t *tile_off, uint32_t W, uint64_t max_tiles,
                               uint32_t *hist, hipStream_t s) {
  static uint64_t cap[64];
  const int d = device_id();
  if (!cap[d]) cap[d] = resident(k_hist<kHistBlock, false>, kHistBlock);
  const dim3 grid(clamp_grid(hist_blocks(max_tiles), cap[d]));
  const uint32_t stride = kKeyDigits * kBins;
  NS_LAUNCH((k_hist<kHistBlock, false>), grid, dim3(kHistBlock), s, dst, nullptr, seg_off, tile_off, W,
            hist, stride, 0u);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  NS_LAUNCH((k_hist<kHistBlock, false>), grid, dim3(kHistBlock), s, src, nullptr, seg_off, tile_off, W,
            hist, stride, 4u);
  return hipGetLastError();
}

hipError_t launch_hist_items(const uint64_t *items, const uint64_t *seg_off,
                             const uint64_t *tile_off, uint32_t W, uint64_t max_tiles,
                             uint32_t *hist, hipStream_t s) {
  static uint64_t cap[64];
  const int d = device_id();
  if (!cap[d]) cap[d] = resident(k_hist<kHistBlock, true>, kHistBlock);
  NS_LAUNCH((k_hist<kHistBlock, true>), dim3(clamp_grid(hist_blocks(max_tiles), cap[d])), dim3(kHistBlock), s, nullptr,
            items, seg_off, tile_off, W, hist, (uint32_t)(kColDigits * kBins), 0u);
  return hipGetLastError();
}

hipError_t launch_hist_scan(const uint32_t *hist, uint32_t *base, uint64_t rows, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  const uint64_t blocks = (rows + 3) / 4;  // 4 waves per block
  NS_LAUNCH(k_hist_scan, dim3((uint32_t)blocks), dim3(256), s, hist, base, rows);
  return hipGetLastError();
}

// 32-bit look-back words while every count + 1 fits in 31 bits
constexpr uint64_t kLbNarrowMax = (1ull << 31) - 2;

template <int B, int I, bool P>
static hipError_t pass_impl(const PassArgs &a, uint64_t max_tiles, hipStream_t s) {
  static uint64_t cap[64];
  const int d = device_id();
  if (!cap[d]) cap[d] = resident(k_pass<B, I, P, true>, B);
  if (a.lim <= kLbNarrowMax)
    NS_LAUNCH((k_pass<B, I, P, true>), dim3(clamp_grid(max_tiles, cap[d])), dim3(B), s, a);
  else
    NS_LAUNCH((k_pass<B, I, P, false>), dim3(clamp_grid(max_tiles, cap[d])), dim3(B), s, a);
  return hipGetLastError();
}

template <int B, int I, bool P>
static hipError_t pass1_impl(const PassArgs &a, uint64_t max_tiles, hipStream_t s) {
  static uint64_t cap[64];
  const int d = device_id();
  if (!cap[d]) cap[d] = resident(k_pass1<B, I, P, true>, B);
  if (a.lim <= kLbNarrowMax)
    NS_LAUNCH((k_pass1<B, I, P, true>), dim3(clamp_grid(max_tiles, cap[d])), dim3(B), s, a);
  else
    NS_LAUNCH((k_pass1<B, I, P, false>), dim3(clamp_grid(max_tiles, cap[d])), dim3(B), s, a);
  return hipGetLastError();
}

hipError_t launch_pass(const SortShape &sh, const PassArgs &a, uint64_t max_tiles, hipStream_t s) {
  const bool P = a.src != nullptr;
  // one segment of at least 2^28 keys: the early-ranking pass (2^30 keys:
  // 46.5 vs 47.7 ms per aggregate step; below 2^28 it was slower, 6.32 vs
  // 6.23 ms at 2^27 and 1.06 vs 1.02 ms at 2^24)
  if (a.W == 1 && a.lim >= (1ull << 28)) {
    if (sh.block == 256 && sh.items == 8) return P ? pass1_impl<256, 8, true>(a, max_tiles, s) : pass1_impl<256, 8, false>(a, max_tiles, s);
    if (sh.block == 256 && sh.items == 16) return P ? pass1_impl<256, 16, true>(a, max_tiles, s) : pass1_impl<256, 16, false>(a, max_tiles, s);
    if (sh.block == 512 && sh.items == 8) return P ? pass1_impl<512, 8, true>(a, max_tiles, s) : pass1_impl<512, 8, false>(a, max_tiles, s);
    if (sh.block == 512 && sh.items == 16) return P ? pass1_impl<512, 16, true>(a, max_tiles, s) : pass1_impl<512, 16, false>(a, max_tiles, s);
    return hipErrorInvalidValue;
  }
  if (sh.block == 256 && sh.items == 8) return P ? pass_impl<256, 8, true>(a, max_tiles, s) : pass_impl<256, 8, false>(a, max_tiles, s);
  if (sh.block == 256 && sh.items == 16) return P ? pass_impl<256, 16, true>(a, max_tiles, s) : pass_impl<256, 16, false>(a, max_tiles, s);
  if (sh.block == 512 && sh.items == 8) return P ? pass_impl<512, 8, true>(a, max_tiles, s) : pass_impl<512, 8, false>(a, max_tiles, s);
  if (sh.block == 512 && sh.items == 16) return P ? pass_impl<512, 16, true>(a, max_tiles, s) : pass_impl<512, 16, false>(a, max_tiles, s);
  return hipErrorInvalidValue;
}

template <int B, int I, bool P, int BITS>
static hipError_t pass_chunked_impl(const PassArgs &a, ChunkArgs c, uint64_t max_keys,
                                    int count_kind, hipStream_t s) {
  static uint64_t cap[64], hcap[64];
  const int d = device_id();
  if (!cap[d]) {
    if constexpr (BITS == 8) cap[d] = resident(k_pass_chunked<B, I, P>, B);
    else cap[d] = resident(k_pass_chunked_wide<B, I, P>, B);
  }
  if (!hcap[d]) hcap[d] = resident(k_chunk_hist<256, P, BITS>, 256);
  // short chunks of kChunkTiles tiles, taken in order by the resident
  // workgroups: the chunks in flight at any time are neighbours, so each
  // digit's writes land in one narrow band of its bucket
  uint64_t ch = chunk_rows(max_keys, (uint64_t)B * I);
  if (ch > c.max_chunks) ch = c.max_chunks;
  c.chunks = (uint32_t)ch;
  c.bins = 1u << BITS;
  const uint32_t blocks = (uint32_t)(ch < kChunkBlocks ? ch : kChunkBlocks);
  const uint32_t rows = (uint32_t)((ch + blocks - 1) / blocks);
  const uint32_t nb = (uint32_t)((ch + rows - 1) / rows);
  const int kind = tl_timing_kind;
  if (kind >= 0) tl_timing_kind = count_kind;
  NS_LAUNCH((k_chunk_hist<256, P, BITS>), dim3(clamp_grid(ch, hcap[d])), dim3(256), s, a, c, (uint32_t)(B * I));
  NS_LAUNCH(k_chunk_sums, dim3(nb, c.bins / 256), dim3(256), s, c, rows);
  NS_LAUNCH(k_chunk_bscan, dim3(c.bins), dim3(256), s, c, nb);
  NS_LAUNCH(k_chunk_prefix, dim3(nb, c.bins / 256), dim3(256), s, c, rows);
  tl_timing_kind = kind;
  if constexpr (BITS == 8) {
    NS_LAUNCH((k_pass_chunked<B, I, P>), dim3(clamp_grid(ch, cap[d])), dim3(B), s, a, c);
  } else {
    NS_LAUNCH((k_pass_chunked_wide<B, I, P>), dim3(clamp_grid(ch, cap[d])), dim3(B), s, a, c);
  }
  return hipGetLastError();
}

template <int BITS>
static hipError_t pass_chunked_bits(const SortShape &sh, const PassArgs &a, const ChunkArgs &c,
                                    uint64_t max_keys, int count_kind, hipStream_t s) {
  const bool P = a.src != nullptr;
  if (sh.block == 256 && sh.items == 8) return P ? pass_chunked_impl<256, 8, true, BITS>(a, c, max_keys, count_kind, s) : pass_chunked_impl<256, 8, false, BITS>(a, c, max_keys, count_kind, s);
  if (sh.block == 256 && sh.items == 16) return P ? pass_chunked_impl<256, 16, true, BITS>(a, c, max_keys, count_kind, s) : pass_chunked_impl<256, 16, false, BITS>(a, c, max_keys, count_kind, s);
  if (sh.block == 512 && sh.items == 8) return P ? pass_chunked_impl<512, 8, true, BITS>(a, c, max_keys, count_kind, s) : pass_chunked_impl<512, 8, false, BITS>(a, c, max_keys, count_kind, s);
  if (sh.block == 512 && sh.items == 16) return P ? pass_chunked_impl<512, 16, true, BITS>(a, c, max_keys, count_kind, s) : pass_chunked_impl<512, 16, false, BITS>(a, c, max_keys, count_kind, s);
  return hipErrorInvalidValue;
}

hipError_t launch_pass_chunked(const SortShape &sh, const PassArgs &a, const ChunkArgs &c,
                               uint64_t max_keys, int bits, int count_kind, hipStream_t s) {
  if (bits == 8) return pass_chunked_bits<8>(sh, a, c, max_keys, count_kind, s);
  if (bits == kWideBits) return pass_chunked_bits<kWideBits>(sh, a, c, max_keys, count_kind, s);
  return hipErrorInvalidValue;
}

template <int I, bool ROWS_LDS = true>
static hipError_t rle_impl(const RleArgs &a, uint64_t max_tiles, hipStream_t s) {
  static uint64_t cap[64];
  const int d = device_id();
  if (!cap[d]) cap[d] = resident(k_rle<I, ROWS_LDS>, 256);
  NS_LAUNCH((k_rle<I, ROWS_LDS>), dim3(clamp_grid(max_tiles, cap[d])), dim3(256), s, a);
  return hipGetLastError();
}

// one segment of 2^24 keys or more: 3 workgroups per CU, rows from registers
// (2^30 keys: 4.77 vs 4.98 ms; 8192 windows of 2^17 keys lose, 7.5 vs 6.0 ms)
bool rle_one_large_segment(const ScanShape &sh, uint32_t W, uint64_t max_tiles, uint64_t lim) {
  return sh.items == 16 && W == 1 && max_tiles * 256 * 16 >= (1ull << 24) && lim < (1ull << 31);
}

hipError_t launch_rle(const ScanShape &sh, const RleArgs &a, uint64_t max_tiles, hipStream_t s) {
  if (sh.items == 4) return rle_impl<4>(a, max_tiles, s);
  if (sh.items == 8) return rle_impl<8>(a, max_tiles, s);
  if (sh.items == 16) {
    if (rle_one_large_segment(sh, a.W, max_tiles, a.lim)) return rle_impl<16, false>(a, max_tiles, s);
    return rle_impl<16>(a, max_tiles, s);
  }
  return hipErrorInvalidValue;
}

template <int I, int M, bool WIDE = false>
static hipError_t runs_impl(const RunArgs &a, uint64_t max_tiles, hipStream_t s) {
  static uint64_t cap[64];
  const int d = device_id();
  if (!cap[d]) cap[d] = resident(k_runs<I, M, WIDE>, 256);
  NS_LAUNCH((k_runs<I, M, WIDE>), dim3(clamp_grid(max_tiles, cap[d])), dim3(256), s, a);
  return hipGetLastError();
}

hipError_t launch_runs(const ScanShape &sh, int mode, const RunArgs &a, uint64_t max_tiles,
                       hipStream_t s) {
  if (a.wide)  // matrices of 2^32 packets or more: one tile shape (256 x 8)
    return mode == 0 ? runs_impl<8, 0, true>(a, max_tiles, s) : runs_impl<8, 1, true>(a, max_tiles, s);
  if (sh.items == 4) return mode == 0 ? runs_impl<4, 0>(a, max_tiles, s) : runs_impl<4, 1>(a, max_tiles, s);
  if (sh.items == 8) return mode == 0 ? runs_impl<8, 0>(a, max_tiles, s) : runs_impl<8, 1>(a, max_tiles, s);
  if (sh.items == 16) return mode == 0 ? runs_impl<16, 0>(a, max_tiles, s) : runs_impl<16, 1>(a, max_tiles, s);
  return hipErrorInvalidValue;
}

hipError_t launch_small(const uint32_t *src, const uint32_t *dst, const uint64_t *off, uint32_t W,
                        uint64_t *stats, uint64_t *win_keys, uint64_t *win_counts,
                        uint64_t *win_nnz, hipStream_t s) {
  if (W == 0) return hipSuccess;
  const uint32_t grid = W < 2048u ? W : 2048u;
  NS_LAUNCH(k_small, dim3(grid), dim3(kSmallBlock), s, src, dst, off, W, stats, win_keys,
            win_counts, win_nnz);
  return hipGetLastError();
}

hipError_t launch_segmax(const uint64_t *a, const uint64_t *b, const uint64_t *head_off,
                         uint32_t W, uint64_t max_heads, uint64_t *stats, int fa, int fb,
                         hipStream_t s) {
  const uint32_t g = clamp_grid((max_heads + 1023) / 1024, 4ull * cu_count());
  NS_LAUNCH(k_segmax, dim3(g), dim3(256), s, a, b, head_off, W, stats, fa, fb);
  return hipGetLastError();
}

hipError_t launch_finalize(const uint64_t *seg_off, const uint64_t *link_off,
                           const uint64_t *row_off, const uint64_t *col_off, uint32_t W,
                           uint64_t *stats, hipStream_t s) {
  if (W == 0) return hipSuccess;
  const uint32_t g = clamp_grid((W + 255) / 256, 1024);
  NS_LAUNCH(k_finalize, dim3(g), dim3(256), s, seg_off, link_off, row_off, col_off, W,
                     stats);
  return hipGetLastError();
}

hipError_t launch_finalize_matrix(const uint64_t *row_hval, const uint64_t *row_off,
                                  const uint64_t *col_off, const uint64_t *nnz, uint64_t *stats,
                                  hipStream_t s) {
  NS_LAUNCH(k_finalize_matrix, dim3(1), dim3(64), s, row_hval, row_off, col_off, nnz,
                     stats);
  return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs &a, uint64_t max_tiles, hipStream_t s) {
  static uint64_t cap[64];
  const int d = device_id();
  if (!cap[d]) cap[d] = resident(k_merge, 256);
  NS_LAUNCH(k_merge, dim3(clamp_grid(max_tiles, cap[d])), dim3(256), s, a);
  return hipGetLastError();
}

hipError_t launch_csr_expand(const uint32_t *rows, const uint64_t *row_ptr, uint64_t nrows,
                             const uint32_t *cols, const uint64_t *vals, uint64_t nnz,
                             uint64_t *keys, uint64_t *counts, uint64_t *nnz_out, hipStream_t s) {
  const uint64_t per = 256ull * 8;
  const uint64_t blocks = nnz ? (nnz + per - 1) / per : 1;
  if (blocks > 0xFFFFFFFFull) return hipErrorInvalidValue;
  NS_LAUNCH(k_csr_expand, dim3((uint32_t)blocks), dim3(256), s, rows, row_ptr, nrows, cols, vals,
            nnz, keys, counts, nnz_out);
  return hipGetLastError();
}

hipError_t launch_check_total(const uint64_t *stats, uint64_t packets, hipStream_t s) {
  NS_LAUNCH(k_check_total, dim3(1), dim3(kWave), s, stats, packets);
  return hipGetLastError();
}

hipError_t read_and_clear_status(int *host_status) {
  int v = 0;
  hipError_t e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_status), sizeof(int), 0,
                                     hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  const int zero = 0;
  e = hipMemcpyToSymbol(HIP_SYMBOL(g_status), &zero, sizeof(int), 0, hipMemcpyHostToDevice);
  *host_status = (v & 8) ? -7 : (v & 1) ? -5 : (v & 2) ? -2 : (v & 4) ? -1 : 0;
  return e;
}

}  // namespace ns

// the rolling-aggregate kernels share this translation unit (and g_status)
#include "ns_rolling.hip"
