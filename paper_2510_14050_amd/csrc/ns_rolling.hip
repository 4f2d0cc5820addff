// Rolling aggregate for serving: A <- A + W_new - W_old kept in device hash
// tables, so one update costs O(entries of W_new and W_old) instead of
// O(entries of A).
//
// State (one caller-owned device buffer):
//   header                      live counts, special-key counter, scan scratch
//   link table  [link_cap]      key = src<<32|dst (u64, EMPTY = all ones), count (u32)
//   source table [addr_cap]     key = src + 1 (u64, EMPTY = 0), packets (u32), fan-out (u32)
//   destination table [addr_cap] key = dst + 1, packets, fan-in
// Open addressing with linear probing; keys are never removed (an entry whose
// count drops to zero stays as a tombstone that only its own key reuses), so a
// lookup never meets an empty slot before its key. Compaction into a fresh
// state drops the tombstones. The header counts the slots taken in each table
// since the last clear or compaction (live entries plus tombstones), which is
// what decides when to compact.
//
// The eight quantities follow from the tables: a link appears when its count
// leaves zero and disappears when it returns to zero (unique links, fan-out of
// its source, fan-in of its destination); a source or destination is present
// while its packet count is non-zero. Maxima are taken by a scan over the
// source and destination tables after each update. All counters change by
// atomics whose sums commute, so adds and removes of one update may run in any
// order. Every count stays below 2^32 (the state holds fewer than 2^32
// packets); an add that wraps a link or address packet count raises the
// device status (capacity).
// Included at the end of ns_kernels.hip, whose device error word it sets.
#include "ns_device.h"
#include "ns_launch.h"

namespace ns {

constexpr uint64_t kEmptyLink = ~0ull;
constexpr uint32_t kProbeLimit = 1u << 16;

// MurmurHash3's 64-bit finaliser (Appleby, public domain)
__device__ __forceinline__ uint64_t fmix64(uint64_t z) {
  z ^= z >> 33;
  z *= 0xff51afd7ed558ccdull;
  z ^= z >> 33;
  z *= 0xc4ceb9fe1a85ec53ull;
  z ^= z >> 33;
  return z;
}

__device__ __forceinline__ uint64_t ld64(const uint64_t *p) { return lb_load(p); }

// slot of `key` in a table of `cap` (power of two) u64 keys, inserting it if
// absent; `empty` marks a free slot; *took is set when this call took a free
// slot. Returns cap on overflow.
__device__ uint64_t find_or_insert(uint64_t *keys, uint64_t cap, uint64_t key, uint64_t empty,
                                   bool insert, bool *took) {
  uint64_t i = fmix64(key) & (cap - 1);
  for (uint32_t probe = 0; probe < kProbeLimit; ++probe) {
    const uint64_t cur = ld64(keys + i);
    if (cur == key) return i;
    if (cur == empty) {
      if (!insert) return cap;
      const uint64_t prev = atomicCAS((unsigned long long *)(keys + i), (unsigned long long)empty,
                                      (unsigned long long)key);
      if (prev == empty) *took = true;
      if (prev == empty || prev == key) return i;
    }
    i = (i + 1) & (cap - 1);
  }
  return cap;
}

__device__ __forceinline__ void flag_status(int bit) { atomicOr(&g_status, bit); }

// one address side (source or destination): packets +-c, fan +-1 on link
// appearance / disappearance; presence transitions update the live count.
// Returns 1 when the address took a free slot.
__device__ uint32_t address_update(const RollTables &t, bool src_side, uint32_t addr, uint32_t dp,
                                   bool plus, int dfan) {
  uint64_t *keys = src_side ? t.src_keys : t.dst_keys;
  uint32_t *pk = src_side ? t.src_pk : t.dst_pk;
  uint32_t *fan = src_side ? t.src_fan : t.dst_fan;
  unsigned long long *live = (unsigned long long *)(src_side ? &t.hdr->sources : &t.hdr->dests);
  bool took = false;
  const uint64_t s = find_or_insert(keys, t.addr_cap, (uint64_t)addr + 1, 0, plus, &took);
  if (s == t.addr_cap) {
    flag_status(plus ? 2 : 1);
    return 0;
  }
  if (plus) {
    const uint32_t old = atomicAdd(pk + s, dp);
    if (old + dp < old) flag_status(2);  // the 32-bit packet count wrapped
    if (old == 0 && dp) atomicAdd(live, 1ull);
  } else {
    const uint32_t old = atomicSub(pk + s, dp);
    if (old < dp) flag_status(1);
    else if (old == dp && dp) atomicAdd(live, ~0ull);
  }
  if (dfan > 0) atomicAdd(fan + s, 1u);
  if (dfan < 0) atomicSub(fan + s, 1u);
  return took ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_roll_update(RollTables t, RollDelta d) {
  const uint64_t na = d.add_nnz ? min(*d.add_nnz, d.add_cap) : 0;
  const uint64_t nr = d.rem_nnz ? min(*d.rem_nnz, d.rem_cap) : 0;
  if (blockIdx.x == 0 && threadIdx.x < 4) t.hdr->scan[threadIdx.x] = 0;  // for the scan that follows
  uint32_t took[3] = {0, 0, 0};  // slots this thread took (links, sources, destinations)
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < na + nr;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const bool plus = i < na;
    const uint64_t key = plus ? d.add_keys[i] : d.rem_keys[i - na];
    const uint32_t c = (uint32_t)(plus ? d.add_counts[i] : d.rem_counts[i - na]);
    uint32_t *cnt;
    if (key == kEmptyLink) {
      cnt = &t.hdr->special_count;
    } else {
      bool tk = false;
      const uint64_t s = find_or_insert(t.link_keys, t.link_cap, key, kEmptyLink, plus, &tk);
      if (s == t.link_cap) {
        flag_status(plus ? 2 : 1);
        continue;
      }
      took[0] += tk;
      cnt = t.link_cnt + s;
    }
    int dfan = 0;
    if (plus) {
      const uint32_t old = atomicAdd(cnt, c);
      if (old + c < old) flag_status(2);  // the 32-bit link count wrapped
      atomicAdd((unsigned long long *)&t.hdr->packets, (unsigned long long)c);
      if (old == 0) {
        atomicAdd((unsigned long long *)&t.hdr->links, 1ull);
        dfan = 1;
      }
    } else {
      const uint32_t old = atomicSub(cnt, c);
      atomicAdd((unsigned long long *)&t.hdr->packets, (unsigned long long)(0ull - c));
      if (old < c) {
        flag_status(1);
        continue;
      }
      if (old == c) {
        atomicAdd((unsigned long long *)&t.hdr->links, ~0ull);
        dfan = -1;
      }
    }
    took[1] += address_update(t, true, (uint32_t)(key >> 32), c, plus, dfan);
    took[2] += address_update(t, false, (uint32_t)key, c, plus, dfan);
  }
  // one counter update per wave and table (a counter hit by every insert
  // would serialise them)
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const uint64_t w = wave_sum((uint64_t)took[q]);
    if ((threadIdx.x & (kWave - 1)) == 0 && w) atomicAdd((unsigned long long *)&t.hdr->used[q], w);
  }
}

// maxima of packets and fan over the source and destination tables
__global__ __launch_bounds__(256) void k_roll_scan(RollTables t) {
  __shared__ uint64_t s_m[4][4];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  uint64_t m[4] = {0, 0, 0, 0};  // src packets, src fan-out, dst packets, dst fan-in
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + tid; i < t.addr_cap;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t a = t.src_pk[i], b = t.src_fan[i], c = t.dst_pk[i], e = t.dst_fan[i];
    m[0] = m[0] > a ? m[0] : a;
    m[1] = m[1] > b ? m[1] : b;
    m[2] = m[2] > c ? m[2] : c;
    m[3] = m[3] > e ? m[3] : e;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    m[q] = wave_max(m[q]);
    if (lane == 0) s_m[wv][q] = m[q];
  }
  __syncthreads();
  if (tid < 4) {
    uint64_t v = 0;
    for (int w = 0; w < 4; ++w) v = v > s_m[w][tid] ? v : s_m[w][tid];
    atomicMax((unsigned long long *)&t.hdr->scan[tid], (unsigned long long)v);
  }
}

__global__ void k_roll_finalize(RollTables t, uint64_t *out) {
  if (threadIdx.x == 0) {
    out[0] = t.hdr->packets;
    out[1] = t.hdr->links;
    out[2] = t.hdr->sources;
    out[3] = t.hdr->dests;
    out[4] = t.hdr->scan[0];
    out[5] = t.hdr->scan[1];
    out[6] = t.hdr->scan[2];
    out[7] = t.hdr->scan[3];
  }
}

__global__ __launch_bounds__(256) void k_roll_clear(RollTables t) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  for (uint64_t i = i0; i < t.link_cap; i += stride) {
    t.link_keys[i] = kEmptyLink;
    t.link_cnt[i] = 0;
  }
  for (uint64_t i = i0; i < t.addr_cap; i += stride) {
    t.src_keys[i] = 0;
    t.src_pk[i] = 0;
    t.src_fan[i] = 0;
    t.dst_keys[i] = 0;
    t.dst_pk[i] = 0;
    t.dst_fan[i] = 0;
  }
  if (i0 == 0) {
    RollHeader *h = t.hdr;
    h->links = h->sources = h->dests = h->packets = 0;
    h->special_count = 0;
    for (int q = 0; q < 4; ++q) h->scan[q] = 0;
    for (int q = 0; q < 3; ++q) h->used[q] = 0;
  }
}

// copy the live entries of `from` into the cleared state `to`
__global__ __launch_bounds__(256) void k_roll_compact(RollTables from, RollTables to) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  for (uint64_t i = i0; i < from.link_cap; i += stride) {
    const uint32_t c = from.link_cnt[i];
    if (!c) continue;
    bool tk = false;  // not needed here: the live counts give the slots taken
    const uint64_t s = find_or_insert(to.link_keys, to.link_cap, from.link_keys[i], kEmptyLink, true, &tk);
    if (s == to.link_cap) flag_status(2);
    else to.link_cnt[s] = c;
  }
  for (uint64_t i = i0; i < from.addr_cap; i += stride) {
    if (from.src_pk[i]) {
      bool tk = false;
      const uint64_t s = find_or_insert(to.src_keys, to.addr_cap, from.src_keys[i], 0, true, &tk);
      if (s == to.addr_cap) flag_status(2);
      else {
        to.src_pk[s] = from.src_pk[i];
        to.src_fan[s] = from.src_fan[i];
      }
    }
    if (from.dst_pk[i]) {
      bool tk = false;
      const uint64_t s = find_or_insert(to.dst_keys, to.addr_cap, from.dst_keys[i], 0, true, &tk);
      if (s == to.addr_cap) flag_status(2);
      else {
        to.dst_pk[s] = from.dst_pk[i];
        to.dst_fan[s] = from.dst_fan[i];
      }
    }
  }
  if (i0 == 0) {
    to.hdr->links = from.hdr->links;
    to.hdr->sources = from.hdr->sources;
    to.hdr->dests = from.hdr->dests;
    to.hdr->packets = from.hdr->packets;
    to.hdr->special_count = from.hdr->special_count;
    // the new tables hold the live entries only (the all-ones link lives outside)
    to.hdr->used[0] = from.hdr->links - (from.hdr->special_count ? 1 : 0);
    to.hdr->used[1] = from.hdr->sources;
    to.hdr->used[2] = from.hdr->dests;
  }
}

// slots taken in the link, source and destination tables since the last
// clear or compaction
__global__ void k_roll_used(RollTables t, uint64_t *out) {
  if (threadIdx.x < 3) out[threadIdx.x] = t.hdr->used[threadIdx.x];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {
uint64_t up256(uint64_t x) { return (x + 255) / 256 * 256; }
uint32_t grid_for(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return (uint32_t)(g ? g : 1);
}
}  // namespace

uint64_t roll_bytes(uint64_t link_cap, uint64_t addr_cap) {
  return up256(sizeof(RollHeader)) + up256(link_cap * 8) + up256(link_cap * 4) +
         2 * (up256(addr_cap * 8) + 2 * up256(addr_cap * 4));
}

RollTables roll_tables(void *mem, uint64_t link_cap, uint64_t addr_cap) {
  uint8_t *p = static_cast<uint8_t *>(mem);
  RollTables t{};
  t.link_cap = link_cap;
  t.addr_cap = addr_cap;
  t.hdr = reinterpret_cast<RollHeader *>(p);
  p += up256(sizeof(RollHeader));
  t.link_keys = reinterpret_cast<uint64_t *>(p);
  p += up256(link_cap * 8);
  t.link_cnt = reinterpret_cast<uint32_t *>(p);
  p += up256(link_cap * 4);
  t.src_keys = reinterpret_cast<uint64_t *>(p);
  p += up256(addr_cap * 8);
  t.src_pk = reinterpret_cast<uint32_t *>(p);
  p += up256(addr_cap * 4);
  t.src_fan = reinterpret_cast<uint32_t *>(p);
  p += up256(addr_cap * 4);
  t.dst_keys = reinterpret_cast<uint64_t *>(p);
  p += up256(addr_cap * 8);
  t.dst_pk = reinterpret_cast<uint32_t *>(p);
  p += up256(addr_cap * 4);
  t.dst_fan = reinterpret_cast<uint32_t *>(p);
  return t;
}

hipError_t launch_roll_clear(const RollTables &t, hipStream_t s) {
  hipLaunchKernelGGL(k_roll_clear, dim3(grid_for(t.link_cap)), dim3(256), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_roll_update(const RollTables &t, const RollDelta &d, uint64_t max_items,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_roll_update, dim3(grid_for(max_items)), dim3(256), 0, s, t, d);
  return hipGetLastError();
}

hipError_t launch_roll_stats(const RollTables &t, uint64_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_roll_scan, dim3(grid_for(t.addr_cap / 4)), dim3(256), 0, s, t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_roll_finalize, dim3(1), dim3(64), 0, s, t, out);
  return hipGetLastError();
}

hipError_t launch_roll_compact(const RollTables &from, const RollTables &to, hipStream_t s) {
  hipError_t e = launch_roll_clear(to, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_roll_compact, dim3(grid_for(from.link_cap)), dim3(256), 0, s, from, to);
  return hipGetLastError();
}

hipError_t launch_roll_used(const RollTables &t, uint64_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_roll_used, dim3(1), dim3(64), 0, s, t, out);
  return hipGetLastError();
}

}  // namespace ns
