// C ABI of libns (declared in include/ns.h): argument checks, workspace
// layout, the kernel sequence of each entry point, and the HIP-graph cache of
// the batched path.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ns.h"
#include "ns_launch.h"

using namespace ns;

namespace {

constexpr uint64_t kAlign = 256;
constexpr int kMaxTickets = 64;
// A single segment of at least this many keys is sorted by chunked passes
// (reduce, scan, scatter) instead of passes with look-back. The autotuner
// chooses per size class (on MI355X the passes with look-back were faster for
// single segments of 2^24 .. 2^30 keys).
#ifndef NS_CHUNKED_MIN
#define NS_CHUNKED_MIN (1ull << 24)
#endif
constexpr uint64_t kChunkedMin = NS_CHUNKED_MIN;
// Batches of fewer packets run the aggregate pipeline beside the per-window one.
#ifndef NS_FORK_MAX_PACKETS
#define NS_FORK_MAX_PACKETS (1ull << 27)
#endif
constexpr uint64_t kForkMaxPackets = NS_FORK_MAX_PACKETS;
constexpr uint64_t kMaxPackets32 = 0xFFFFFFFFull;  // packets per window / matrix < 2^32
constexpr int kMinSortTile = 256 * 8;
constexpr int kMinScanTile = 256 * 4;
constexpr int kChunkBlock = 512, kChunkItems = 16;  // launch shape of the chunked passes
constexpr uint64_t kChunkTile = (uint64_t)kChunkBlock * kChunkItems;

uint64_t up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Workspace carve-up for at most N packets / entries and W windows.
struct Layout {
  uint64_t tickets, seg, t_sort, t_hist, t_rle, t_csort, t_run;
  uint64_t link_off, row_off, col_off, seg_base;
  uint64_t hist, base, chist, cbase;
  uint64_t lb0, lb1, lbs;
  uint64_t ccount, cprefix, cbsum;
  uint64_t chunk_rows;
  uint64_t KA, KB, HA, HB;
  uint64_t total;
  uint64_t sort_tiles, scan_tiles;
};

Layout plan(uint64_t N, uint32_t W) {
  Layout L{};
  const uint64_t W1 = (uint64_t)W + 1 > 2 ? (uint64_t)W + 1 : 2;
  const uint64_t Wd = W > 1 ? W : 1;
  L.sort_tiles = N / kMinSortTile + Wd + 1;
  L.scan_tiles = N / kMinScanTile + Wd + 1;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { const uint64_t at = o; o += up(bytes); return at; };
  L.tickets = take(kMaxTickets * 4);
  L.seg = take(W1 * 8);
  L.t_sort = take((W1 + 1) * 8);
  L.t_hist = take((W1 + 1) * 8);
  L.t_rle = take((W1 + 1) * 8);
  L.t_csort = take((W1 + 1) * 8);
  L.t_run = take((W1 + 1) * 8);
  L.link_off = take(W1 * 8);
  L.row_off = take(W1 * 8);
  L.col_off = take(W1 * 8);
  L.seg_base = take(W1 * 8);
  L.hist = take(Wd * kKeyDigits * kBins * 4);
  L.base = take(Wd * kKeyDigits * kBins * 4);
  L.chist = take(Wd * kColDigits * kBins * 4);
  L.cbase = take(Wd * kColDigits * kBins * 4);
  L.lb0 = take(L.sort_tiles * kBins * 8);
  L.lb1 = take(L.sort_tiles * kBins * 8);
  L.lbs = take(L.scan_tiles * 2 * 8);
  // chunk tables sized for the widest digit (2048 bins); byte digits use the
  // first 256 entries of each row
  L.chunk_rows = chunk_rows(N, kChunkTile);
  L.ccount = take(L.chunk_rows * kMaxBins * 4);
  L.cprefix = take((L.chunk_rows + 1) * kMaxBins * 8);  // + digit totals
  L.cbsum = take((L.chunk_rows < kChunkBlocks ? L.chunk_rows : kChunkBlocks) * kMaxBins * 8);
  L.KA = take((N + 1) * 8);
  L.KB = take((N + 1) * 8);
  L.HA = take((N + 2) * 8);
  L.HB = take((N + 2) * 8);
  L.total = o;
  return L;
}

// Pointers into a caller workspace.
struct Ws {
  Layout L;
  uint8_t *base;
  int next_ticket = 0;
  template <typename T>
  T *at(uint64_t off) const { return reinterpret_cast<T *>(base + off); }
  uint32_t *ticket() { return at<uint32_t>(L.tickets) + (next_ticket++ % kMaxTickets); }
};

// Chunk tables of a chunked pass over the segment [seg_off[0], seg_off[1]).
ChunkArgs chunk_args(const Ws &ws, const uint64_t *seg_off) {
  ChunkArgs c{};
  c.seg_off = seg_off;
  c.max_chunks = (uint32_t)ws.L.chunk_rows;
  c.count = ws.at<uint32_t>(ws.L.ccount);
  c.prefix = ws.at<uint64_t>(ws.L.cprefix);
  c.total = ws.at<uint64_t>(ws.L.cprefix) + ws.L.chunk_rows * kMaxBins;
  c.bsum = ws.at<uint64_t>(ws.L.cbsum);
  return c;
}

// Workspace of the streamed build: the build workspace of one sub-partition,
// two staging buffers of its packets, the sub-partition's own matrix, a second
// aggregate of `capacity` entries (the union-add alternates between it and
// the output) and the merge's look-back words.
struct StreamLayout {
  uint64_t inner, stage, bkeys, bcounts, bnnz, akeys, acounts, annz, mlb, merge_tiles, total;
};

StreamLayout stream_plan(uint64_t batch, uint64_t capacity) {
  StreamLayout L{};
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) { const uint64_t at = o; o += up(bytes); return at; };
  L.inner = take(plan(batch, 1).total);
  L.stage = take(4 * batch * 4);  // src and dst of two sub-partitions
  L.bkeys = take(batch * 8);
  L.bcounts = take(batch * 8);
  L.bnnz = take(8);
  L.akeys = take(capacity * 8);
  L.acounts = take(capacity * 8);
  L.annz = take(8);
  L.merge_tiles = (capacity + batch) / kMergeTile + 2;
  L.mlb = take(L.merge_tiles * 8);
  L.total = o;
  return L;
}

// Workspace of a union-add of at most n entries: the merge tiles' ticket,
// then one look-back word per merge tile.
struct MergeLayout {
  uint64_t lbs, tiles, total;
};

MergeLayout merge_plan(uint64_t n) {
  MergeLayout L{};
  L.tiles = n / kMergeTile + 2;
  L.lbs = up(4);
  L.total = L.lbs + up(L.tiles * 8);
  return L;
}

#define HIP_TRY(expr)                           \
  do {                                          \
    if ((expr) != hipSuccess) return NS_ERR_HIP; \
  } while (0)

// Optional per-kernel timing: HIP events recorded on the launching stream
// around every launch of the eager paths (never inside a captured graph).
enum Kind { K_FILL, K_TILES, K_HIST, K_HSCAN, K_PASS0, K_PASS, K_CPASS, K_RLE, K_RUNS, K_SEGMAX,
            K_FINAL, K_MERGE, K_CHUNK_COUNT, K_PASS0_CHUNKED, K_PASS_CHUNKED, K_CPASS_CHUNKED,
            K_SMALL, K_COUNT };

struct Profiler {
  std::mutex mu;
  bool on = false;
  struct Mark { int kind; hipEvent_t a, b; };
  std::vector<Mark> marks;
};

Profiler &prof() {
  static Profiler *p = new Profiler();
  return *p;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

// Runs `launch` (returning hipError_t) with kernel timing of the given kind
// switched on for this thread when profiling is enabled and the stream is not
// being captured: each kernel it launches records its own start/stop events.
template <typename F>
hipError_t timed(int kind, hipStream_t s, F launch, int = 1) {
  Profiler &p = prof();
  if (!p.on || capturing(s)) return launch();
  tl_timing_kind = kind;
  const hipError_t e = launch();
  tl_timing_kind = -1;
  return e;
}

int check_ws(void *ws, uint64_t ws_bytes, uint64_t N, uint32_t W, Ws *out) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return NS_ERR_WORKSPACE;
  out->L = plan(N, W);
  if (ws_bytes < out->L.total) return NS_ERR_WORKSPACE;
  out->base = static_cast<uint8_t *>(ws);
  return NS_OK;
}

struct Shapes {
  SortShape sort;
  ScanShape scan;
  uint64_t chunked_min = kChunkedMin;
  int digit_bits = 8;  // digit width of the chunked passes (8 or kWideBits)
  // chunked passes: the largest tile measured fastest (fewest tiles per chunk
  // boundary, most keys per digit run)
  SortShape chunk = {kChunkBlock, kChunkItems};
};

int resolve_tuning(const ns_tuning_t *t, Shapes *sh) {
  sh->sort = {256, 16};
  sh->scan = {8};
  sh->chunked_min = kChunkedMin;
  sh->digit_bits = 8;
  if (!t) return NS_OK;
  if (t->digit_bits && t->digit_bits != 8 && t->digit_bits != kWideBits) return NS_ERR_INVALID_ARG;
  if (t->digit_bits) sh->digit_bits = (int)t->digit_bits;
  if (t->sort_block) {
    if (t->sort_block != 256 && t->sort_block != 512) return NS_ERR_INVALID_ARG;
    sh->sort.block = (int)t->sort_block;
  }
  if (t->sort_items) {
    if (t->sort_items != 8 && t->sort_items != 16) return NS_ERR_INVALID_ARG;
    sh->sort.items = (int)t->sort_items;
  }
  if (t->scan_items) {
    if (t->scan_items != 4 && t->scan_items != 8 && t->scan_items != 16) return NS_ERR_INVALID_ARG;
    sh->scan.items = (int)t->scan_items;
  }
  if (t->chunked_min) sh->chunked_min = t->chunked_min;
  return NS_OK;
}

// Column pass shared by every statistics path: items dst<<32|count of each
// link segment (segments [link_off[w], link_off[w+1]) in items_in) are
// radix-sorted by destination, then destination runs give unique
// destinations, max fan-in and max destination packets.
// On return the sorted items are in `tmp` (4 passes: in -> tmp -> in -> tmp -> in
// ... ends in items_in).
int enqueue_columns(Ws &ws, const Shapes &sh, uint64_t *items, uint64_t *tmp,
                    const uint64_t *link_off, uint32_t W, uint64_t max_items, uint64_t *stats,
                    hipStream_t s, const uint64_t *gather = nullptr, uint64_t packets = 0,
                    bool hist_ready = false) {
  const Layout &L = ws.L;
  uint64_t *t_csort = ws.at<uint64_t>(L.t_csort), *t_run = ws.at<uint64_t>(L.t_run);
  uint32_t *chist = ws.at<uint32_t>(L.chist), *cbase = ws.at<uint32_t>(L.cbase);
  const bool chunked = W == 1 && max_items >= sh.chunked_min;
  uint64_t *t_chist = ws.at<uint64_t>(L.t_hist);  // free again once the key histograms are done
  HIP_TRY(timed(K_TILES, s, [&] { return launch_tiles(link_off, W, sh.sort.tile(), t_csort, sh.scan.tile(), t_run, kHistTile, t_chist, s); }));
  uint64_t *lbs = ws.at<uint64_t>(L.lbs);
  uint64_t *hpos = ws.at<uint64_t>(L.HA), *hval = ws.at<uint64_t>(L.HB);
  uint64_t *col_off = ws.at<uint64_t>(L.col_off);
  const uint64_t run_tiles = max_items / sh.scan.tile() + W + 1;
  {
    FillList f;
    if (!chunked && !hist_ready) f.add32(chist, (uint64_t)W * kColDigits * kBins);
    f.add64(lbs, run_tiles * 2);
    f.add64(col_off, (uint64_t)W + 1);
    f.add64(hpos, 1);
    f.add64(hval, 1);
    HIP_TRY(launch_fill_multi(f, s));
  }
  if (!chunked) {
    // (hist_ready: the run-length pass counted the items' digits as it wrote them)
    const uint64_t hist_tiles = max_items / kHistTile + W + 1;
    if (!hist_ready)
      HIP_TRY(timed(K_HIST, s, [&] { return launch_hist_items(items, link_off, t_chist, W, hist_tiles, chist, s); }));
    HIP_TRY(timed(K_HSCAN, s, [&] { return launch_hist_scan(chist, cbase, (uint64_t)W * kColDigits, s); }));
  }
  const uint64_t sort_tiles = max_items / sh.sort.tile() + W + 1;
  uint64_t *lb[2] = {ws.at<uint64_t>(L.lb0), ws.at<uint64_t>(L.lb1)};
  uint64_t *buf[2] = {items, tmp};
  // the 32-bit destination in digits of `bits` bits, least significant first
  const int bits = chunked ? sh.digit_bits : 8;
  const int passes = (32 + bits - 1) / bits;
  HIP_TRY(timed(chunked ? K_CPASS_CHUNKED : K_CPASS, s, [&] {
    for (int q = 0; q < passes; ++q) {
      PassArgs a{};
      a.in = buf[q & 1];
      a.out = buf[(q + 1) & 1];
      a.shift = 32 + bits * q;
      a.ticket = ws.ticket();
      a.lim = max_items;
      if (chunked) {
        const ChunkArgs c = chunk_args(ws, link_off);
        const hipError_t e = launch_pass_chunked(sh.chunk, a, c, max_items, bits, K_CHUNK_COUNT, s);
        if (e != hipSuccess) return e;
        continue;
      }
      a.seg_off = link_off;
      a.tile_off = t_csort;
      a.W = W;
      a.base = cbase + q * kBins;
      a.base_stride = kColDigits * kBins;
      a.lb = lb[q & 1];
      a.lb_next = lb[(q + 1) & 1];
      const hipError_t e = launch_pass(sh.sort, a, sort_tiles, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }, passes));
  // an even number of passes leaves the sorted items in `items`, an odd one in `tmp`
  RunArgs r{};
  r.keys = buf[passes & 1];
  r.seg_off = link_off;
  r.tile_off = t_run;
  r.W = W;
  r.hpos = hpos;
  r.hval = hval;
  r.head_off = col_off;
  r.lb = lbs;
  r.ticket = ws.ticket();
  r.wide = gather != nullptr;  // items carry link indices; counts come from `gather`
  r.gather = gather;
  r.lim = max_items;
  r.vlim = packets;  // the items' counts sum to the packets
  HIP_TRY(timed(K_RUNS, s, [&] { return launch_runs(sh.scan, 1, r, run_tiles, s); }));
  // fan-in = run length, destination packets = run sum
  HIP_TRY(timed(K_SEGMAX, s, [&] { return launch_segmax(hpos, hval, col_off, W, max_items, stats, 7, 6, s); }));
  return NS_OK;
}

// Full pipeline from packets: radix sort of the packed keys of W segments,
// run-length encoding, and (optionally) the eight quantities per segment.
struct PacketOut {
  uint64_t *stats;         // [W][8] or null
  uint64_t *ukeys;         // matrix keys (may be the in-place sorted buffer) or null
  uint64_t *counts;        // matrix counts or null
  uint64_t *nnz;           // total links (device scalar) or null
  uint64_t *win_keys;      // positional per-window matrices (or null)
  uint64_t *win_counts;
  uint64_t *win_nnz;       // [W]
  uint64_t *sort_a;        // sort ping-pong buffers (capacity >= N each); the sorted
  uint64_t *sort_b;        // keys end in sort_b
};

int enqueue_packets(Ws &ws, const Shapes &sh, const uint32_t *src, const uint32_t *dst,
                    const uint64_t *seg_off, uint32_t W, uint64_t N, const PacketOut &o,
                    hipStream_t s) {
  const Layout &L = ws.L;
  uint64_t *t_sort = ws.at<uint64_t>(L.t_sort), *t_hist = ws.at<uint64_t>(L.t_hist),
           *t_rle = ws.at<uint64_t>(L.t_rle);
  uint32_t *hist = ws.at<uint32_t>(L.hist), *base = ws.at<uint32_t>(L.base);
  uint64_t *link_off = ws.at<uint64_t>(L.link_off);
  uint64_t *row_off = ws.at<uint64_t>(L.row_off);
  uint64_t *lb[2] = {ws.at<uint64_t>(L.lb0), ws.at<uint64_t>(L.lb1)};
  const uint64_t sort_tiles = N / sh.sort.tile() + W + 1;
  const uint64_t rle_tiles = N / sh.scan.tile() + W + 1;
  const uint64_t hist_tiles = N / kHistTile + W + 1;
  const bool want_stats = o.stats != nullptr;
  // one large segment: chunked passes, which need neither the digit
  // histograms nor the look-back words (the column passes follow suit)
  const bool chunked = W == 1 && N >= sh.chunked_min;

  {
    FillList f;
    if (!chunked) f.add32(hist, (uint64_t)W * kKeyDigits * kBins);
    if (want_stats) f.add64(o.stats, (uint64_t)W * 8);
    if (!chunked) f.add64(lb[0], sort_tiles * kBins);
    f.add64(link_off, (uint64_t)W + 1);
    f.add64(row_off, (uint64_t)W + 1);
    if (o.nnz) f.add64(o.nnz, 1);
    if (o.win_keys) {
      f.add64(o.win_nnz, W);
      f.add64(ws.at<uint64_t>(L.seg_base), W);
    }
    HIP_TRY(launch_fill_multi(f, s));
  }
  HIP_TRY(launch_tiles(seg_off, W, sh.sort.tile(), t_sort, kHistTile, t_hist, sh.scan.tile(),
                       t_rle, s));
  if (!chunked) {
    HIP_TRY(timed(K_HIST, s, [&] { return launch_hist_packets(src, dst, seg_off, t_hist, W, hist_tiles, hist, s); }));
    HIP_TRY(timed(K_HSCAN, s, [&] { return launch_hist_scan(hist, base, (uint64_t)W * kKeyDigits, s); }));
  }
  // stable passes over digits of `bits` bits, least significant first (8 byte
  // digits, or 6 of 11 bits for a chunked single segment); pass p writes buf[p & 1]
  uint64_t *buf[2] = {o.sort_a, o.sort_b};
  const int bits = chunked ? sh.digit_bits : 8;
  const int passes = (64 + bits - 1) / bits;
  auto pass = [&](int p) {
    PassArgs a{};
    if (p == 0) {
      a.src = src;
      a.dst = dst;
    } else {
      a.in = buf[(p - 1) & 1];
    }
    a.out = buf[p & 1];
    a.shift = bits * p;
    a.ticket = ws.ticket();
    a.lim = N;
    if (chunked) {
      const ChunkArgs c = chunk_args(ws, seg_off);
      return launch_pass_chunked(sh.chunk, a, c, N, bits, K_CHUNK_COUNT, s);
    }
    a.seg_off = seg_off;
    a.tile_off = t_sort;
    a.W = W;
    a.base = base + p * kBins;
    a.base_stride = kKeyDigits * kBins;
    a.lb = lb[p & 1];
    a.lb_next = lb[(p + 1) & 1];
    return launch_pass(sh.sort, a, sort_tiles, s);
  };
  HIP_TRY(timed(chunked ? K_PASS0_CHUNKED : K_PASS0, s, [&] { return pass(0); }));
  HIP_TRY(timed(chunked ? K_PASS_CHUNKED : K_PASS, s, [&] {
    for (int p = 1; p < passes; ++p) {
      const hipError_t e = pass(p);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }, passes - 1));
  uint64_t *sorted = buf[(passes - 1) & 1];  // == sort_b (8 or 6 passes)
  // run-length encoding (+ rows and column items when statistics are wanted)
  uint64_t *lbs = ws.at<uint64_t>(L.lbs);
  uint64_t *items = nullptr, *rpos = nullptr, *rlink = nullptr;
  // one large segment whose sorts are not chunked (the column sort takes the
  // same path as the key sort): the run-length pass also counts the column
  // items' digits
  const bool col_hist = want_stats && !chunked && rle_one_large_segment(sh.scan, W, rle_tiles, N);
  {
    FillList f;
    f.add64(lbs, rle_tiles * 2);
    if (col_hist) f.add32(ws.at<uint32_t>(L.chist), (uint64_t)kColDigits * kBins);
    if (want_stats) {
      items = ws.at<uint64_t>(L.KA) == sorted ? ws.at<uint64_t>(L.KB) : ws.at<uint64_t>(L.KA);
      rpos = ws.at<uint64_t>(L.HA);
      rlink = ws.at<uint64_t>(L.HB);
      f.add64(rpos, 1);
      f.add64(rlink, 1);
    }
    HIP_TRY(launch_fill_multi(f, s));
  }
  RleArgs r{};
  r.keys = sorted;
  r.seg_off = seg_off;
  r.tile_off = t_rle;
  r.W = W;
  r.ukeys = o.ukeys;
  r.counts = o.counts;
  r.items = items;
  r.win_keys = o.win_keys;
  r.win_counts = o.win_counts;
  r.win_nnz = o.win_nnz;
  r.seg_base = ws.at<uint64_t>(L.seg_base);
  r.rpos = rpos;
  r.rlink = rlink;
  r.link_off = link_off;
  r.row_off = row_off;
  r.nnz_out = o.nnz;
  r.lb = lbs;
  r.ticket = ws.ticket();
  r.lim = N;
  r.col_hist = col_hist ? ws.at<uint32_t>(L.chist) : nullptr;
  HIP_TRY(timed(K_RLE, s, [&] { return launch_rle(sh.scan, r, rle_tiles, s); }));
  if (!want_stats) return NS_OK;
  // rows: packets = distance between row heads, fan-out = links between them
  HIP_TRY(timed(K_SEGMAX, s, [&] { return launch_segmax(rpos, rlink, row_off, W, N, o.stats, 4, 5, s); }));
  // columns: items are sorted in place (ping-pong with the other sort buffer)
  uint64_t *tmp = (items == ws.at<uint64_t>(L.KA)) ? ws.at<uint64_t>(L.KB) : ws.at<uint64_t>(L.KA);
  int rc = enqueue_columns(ws, sh, items, tmp, link_off, W, N, o.stats, s, nullptr, N, col_hist);
  if (rc) return rc;
  HIP_TRY(timed(K_FINAL, s, [&] { return launch_finalize(seg_off, link_off, row_off, ws.at<uint64_t>(L.col_off), W, o.stats, s); }));
  return NS_OK;
}

// The eight quantities of a sorted COO matrix. A matrix of 2^32 packets or
// more (fewer than 2^32 links) takes the 64-bit run reductions.
int enqueue_matrix_stats(Ws &ws, const Shapes &sh, const ns_matrix_t *m, uint64_t *stats,
                         hipStream_t s) {
  const Layout &L = ws.L;
  const uint64_t cap = m->capacity < m->packets ? m->capacity : m->packets;
  const bool wide = m->packets > kMaxPackets32;
  uint64_t *seg = ws.at<uint64_t>(L.seg);
  uint64_t *t_run = ws.at<uint64_t>(L.t_run);
  uint64_t *link_off = ws.at<uint64_t>(L.link_off);
  uint64_t *row_off = ws.at<uint64_t>(L.row_off);
  uint64_t *items = ws.at<uint64_t>(L.KA), *tmp = ws.at<uint64_t>(L.KB);
  uint64_t *hpos = ws.at<uint64_t>(L.HA), *hval = ws.at<uint64_t>(L.HB);
  uint64_t *lbs = ws.at<uint64_t>(L.lbs);
  const uint64_t run_tiles = cap / sh.scan.tile() + 2;

  {
    FillList f;
    f.add64(stats, 8);
    f.add64(ws.at<uint64_t>(L.lb0), (cap / sh.sort.tile() + 2) * kBins);
    f.add64(lbs, run_tiles * 2);
    f.add64(row_off, 2);
    f.add64(hpos, 1);
    f.add64(hval, 1);
    HIP_TRY(launch_fill_multi(f, s));
  }
  HIP_TRY(launch_seg1(seg, m->nnz, cap, s));
  HIP_TRY(launch_seg1(link_off, m->nnz, cap, s));
  HIP_TRY(timed(K_TILES, s, [&] { return launch_tiles(seg, 1, sh.scan.tile(), t_run, 1, nullptr, 1, nullptr, s); }));
  RunArgs r{};
  r.keys = m->keys;
  r.counts = m->counts;
  r.seg_off = seg;
  r.tile_off = t_run;
  r.W = 1;
  r.hpos = hpos;
  r.hval = hval;
  r.head_off = row_off;
  r.items = items;
  r.lb = lbs;
  r.ticket = ws.ticket();
  r.wide = wide;
  r.lim = cap;
  r.vlim = m->packets;
  HIP_TRY(timed(K_RUNS, s, [&] { return launch_runs(sh.scan, 0, r, run_tiles, s); }));
  // fan-out = run length, source packets = run sum
  HIP_TRY(timed(K_SEGMAX, s, [&] { return launch_segmax(hpos, hval, row_off, 1, cap, stats, 5, 4, s); }));
  // valid packets = value sentinel, read before the column pass reuses hpos/hval
  HIP_TRY(timed(K_FINAL, s, [&] { return launch_finalize_matrix(hval, row_off, nullptr, m->nnz, stats, s); }));
  int rc = enqueue_columns(ws, sh, items, tmp, link_off, 1, cap, stats, s,
                           wide ? m->counts : nullptr, m->packets);
  if (rc) return rc;
  HIP_TRY(timed(K_FINAL, s, [&] { return launch_finalize_matrix(nullptr, nullptr, ws.at<uint64_t>(L.col_off), nullptr, stats, s); }));
  return NS_OK;
}

}  // namespace

namespace ns {
void record_timing(int kind, hipEvent_t start, hipEvent_t stop) {
  Profiler &p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  p.marks.push_back(Profiler::Mark{kind, start, stop});
}
}  // namespace ns

// ===========================================================================
// graph cache for the batched path
// ===========================================================================
namespace {

struct GraphCache {
  std::mutex mu;
  std::unordered_map<std::string, hipGraphExec_t> execs;
  hipStream_t capture[64] = {};   // capture streams per device (the second carries
  hipStream_t capture2[64] = {};  // the aggregate pipeline inside the graph)
  hipEvent_t fork[64] = {};
  hipEvent_t join[64] = {};
};

GraphCache &cache() {
  static GraphCache *c = new GraphCache();  // never destroyed: graphs may outlive statics
  return *c;
}

struct BatchArgs {
  const uint32_t *src, *dst;
  const uint64_t *offsets;
  uint32_t W;
  uint64_t N;
  ns_stats_t *out;
  ns_matrix_t *agg;
  ns_stats_t *agg_stats;
  ns_batch_matrices_t *win;
  Shapes sh;
};

// Per-window pipeline on `s` with workspace `ws`; the aggregate pipeline on
// `s2` with workspace `ws2` (its own tickets, histograms, look-back words and
// buffers). With s2 != s the aggregate forks off `s` through an event and joins
// back, so the two independent pipelines overlap (also inside a captured graph).
int enqueue_batch(const BatchArgs &b, Ws &ws, Ws &ws2, hipStream_t s, hipStream_t s2,
                  hipEvent_t fork, hipEvent_t join) {
  HIP_TRY(launch_fill32(ws.at<uint32_t>(ws.L.tickets), kMaxTickets, 0, s));
  if (b.agg && (b.W == 1 || !b.out)) {
    // one window: its matrix is the aggregate, so one pipeline writes both
    // (and the window's quantities are copied to the aggregate's); no
    // per-window output: the aggregate's pipeline alone, over all packets
    PacketOut o{};
    uint64_t *seg = ws.at<uint64_t>(ws.L.seg);
    const uint64_t *off = b.offsets;
    if (!b.out) {
      HIP_TRY(launch_seg1(seg, nullptr, b.N, s));
      off = seg;
    }
    o.stats = reinterpret_cast<uint64_t *>(b.out ? b.out : b.agg_stats);
    o.ukeys = b.agg->keys;
    o.counts = b.agg->counts;
    o.nnz = b.agg->nnz;
    o.sort_a = ws.at<uint64_t>(ws.L.KA);
    o.sort_b = ws.at<uint64_t>(ws.L.KB);
    if (b.win) {
      o.win_keys = b.win->keys;
      o.win_counts = b.win->counts;
      o.win_nnz = b.win->nnz;
    }
    int rc = enqueue_packets(ws, b.sh, b.src, b.dst, off, 1, b.N, o, s);
    if (rc) return rc;
    if (b.agg_stats && b.out)
      HIP_TRY(launch_copy64(reinterpret_cast<uint64_t *>(b.agg_stats),
                            reinterpret_cast<const uint64_t *>(b.out), 8, s));
    return NS_OK;
  }
  // Both pipelines are latency-bound on small batches, where running them side
  // by side fills each other's ramps and tails; on large ones each saturates
  // HBM alone and sharing the GPU only adds interference.
  const bool split = b.agg && s2 != s && b.N < kForkMaxPackets;
  if (split) {
    HIP_TRY(hipEventRecord(fork, s));
    HIP_TRY(hipStreamWaitEvent(s2, fork, 0));
  }
  if (b.agg) {
    hipStream_t sa = split ? s2 : s;
    HIP_TRY(launch_fill32(ws2.at<uint32_t>(ws2.L.tickets), kMaxTickets, 0, sa));
    uint64_t *seg = ws2.at<uint64_t>(ws2.L.seg);
    HIP_TRY(launch_seg1(seg, nullptr, b.N, sa));
    PacketOut o{};
    o.stats = reinterpret_cast<uint64_t *>(b.agg_stats);
    o.ukeys = b.agg->keys;
    o.counts = b.agg->counts;
    o.nnz = b.agg->nnz;
    // sorting in the workspace keeps the run-length pass out of place, so a
    // tile publishes its counts without first finishing its run-end search
    o.sort_a = ws2.at<uint64_t>(ws2.L.KA);
    o.sort_b = ws2.at<uint64_t>(ws2.L.KB);
    int rc = enqueue_packets(ws2, b.sh, b.src, b.dst, seg, 1, b.N, o, sa);
    if (rc) return rc;
    if (split) HIP_TRY(hipEventRecord(join, s2));
  }
  if (b.W > 0 && b.N <= kSmallMax) {
    // a small batch: every window's whole pipeline in one workgroup, one launch
    HIP_TRY(timed(K_SMALL, s, [&] {
      return launch_small(b.src, b.dst, b.offsets, b.W, reinterpret_cast<uint64_t *>(b.out),
                          b.win ? b.win->keys : nullptr, b.win ? b.win->counts : nullptr,
                          b.win ? b.win->nnz : nullptr, s);
    }));
  } else if (b.W > 0) {
    PacketOut o{};
    o.stats = reinterpret_cast<uint64_t *>(b.out);
    o.sort_a = ws.at<uint64_t>(ws.L.KA);
    o.sort_b = ws.at<uint64_t>(ws.L.KB);
    if (b.win) {
      o.win_keys = b.win->keys;
      o.win_counts = b.win->counts;
      o.win_nnz = b.win->nnz;
    }
    int rc = enqueue_packets(ws, b.sh, b.src, b.dst, b.offsets, b.W, b.N, o, s);
    if (rc) return rc;
  }
  if (split) HIP_TRY(hipStreamWaitEvent(s, join, 0));
  return NS_OK;
}

int batch_checks(const uint32_t *src, const uint32_t *dst, const uint64_t *offsets, uint32_t W,
                 uint64_t N, ns_stats_t *out, ns_matrix_t *agg, ns_stats_t *agg_stats,
                 ns_batch_matrices_t *win, const ns_tuning_t *tune, void *ws, uint64_t ws_bytes,
                 BatchArgs *b, Ws *w, Ws *w2) {
  if (N > 0 && (!src || !dst)) return NS_ERR_INVALID_ARG;
  if (W > 0 && !offsets) return NS_ERR_INVALID_ARG;
  if (W > 0 && !out && !agg) return NS_ERR_INVALID_ARG;  // nothing to compute
  if (W == 0 && N > 0) return NS_ERR_INVALID_ARG;
  if (!out && win) return NS_ERR_INVALID_ARG;  // window matrices come from the per-window pipeline
  if (N > kMaxPackets32) return NS_ERR_UNSUPPORTED;
  if (agg_stats && !agg) return NS_ERR_INVALID_ARG;
  if (agg) {
    if (!agg->keys || !agg->counts || !agg->nnz) return NS_ERR_INVALID_ARG;
    if (agg->capacity < N) return NS_ERR_CAPACITY;
  }
  if (win) {
    if (!win->keys || !win->counts || !win->nnz) return NS_ERR_INVALID_ARG;
    if (win->capacity < N) return NS_ERR_CAPACITY;
  }
  b->sh = Shapes{};
  int rc = resolve_tuning(tune, &b->sh);
  if (rc) return rc;
  // the workspace holds the per-window layout, then the aggregate's layout
  rc = check_ws(ws, ws_bytes, N, W, w);
  if (rc) return rc;
  const uint64_t first = up(w->L.total);
  if (agg) {
    if (ws_bytes < first) return NS_ERR_WORKSPACE;
    rc = check_ws(static_cast<uint8_t *>(ws) + first, ws_bytes - first, N, 1, w2);
    if (rc) return rc;
  }
  b->src = src;
  b->dst = dst;
  b->offsets = offsets;
  b->W = W;
  b->N = N;
  b->out = out;
  b->agg = agg;
  b->agg_stats = agg_stats;
  b->win = win;
  return NS_OK;
}

std::string batch_key(int dev, const BatchArgs &b, void *ws, uint64_t ws_bytes) {
  char buf[512];
  snprintf(buf, sizeof buf, "%d|%p|%p|%p|%u|%llu|%p|%p|%p|%p|%llu|%p|%p|%p|%p|%p|%llu|%d,%d,%d,%llu|%p|%llu",
           dev, (const void *)b.src, (const void *)b.dst, (const void *)b.offsets, b.W,
           (unsigned long long)b.N, (void *)b.out, b.agg ? (void *)b.agg->keys : nullptr,
           b.agg ? (void *)b.agg->counts : nullptr, b.agg ? (void *)b.agg->nnz : nullptr,
           (unsigned long long)(b.agg ? b.agg->capacity : 0), (void *)b.agg_stats,
           b.win ? (void *)b.win->keys : nullptr, b.win ? (void *)b.win->counts : nullptr,
           b.win ? (void *)b.win->nnz : nullptr, (void *)nullptr,
           (unsigned long long)(b.win ? b.win->capacity : 0), b.sh.sort.block, b.sh.sort.items,
           b.sh.scan.items * 100 + b.sh.digit_bits,
           (unsigned long long)b.sh.chunked_min, ws,
           (unsigned long long)ws_bytes);
  return std::string(buf);
}

// Library-owned scratch of ns_accumulate_noalloc: the merge's ticket and
// look-back words for up to NS_ACCUMULATE_NOALLOC_MAX_ENTRIES merged entries,
// in a file-scope device array (each device holds its own copy for the life
// of the process). Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
// Same carve-up as merge_plan: the ticket in the first 256 bytes, then the
// look-back words rounded up to 256 bytes.
constexpr uint64_t kScratchBytes =
    kAlign + ((NS_ACCUMULATE_NOALLOC_MAX_ENTRIES / kMergeTile + 2) * 8 + kAlign - 1) / kAlign * kAlign;

}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

int scratch_address(void **out) {
  static std::mutex mu;
  static void *addr[64] = {};
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return NS_ERR_HIP;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % kAlign) return NS_ERR_HIP;
    addr[dev] = p;
  }
  *out = addr[dev];
  return NS_OK;
}

// Union-add / subtract of two sorted COO matrices into acc_out (the checks
// and kernel sequence of ns_accumulate) with the merge's ticket and look-back
// words in the caller's `ws`, or, with `noalloc`, in the library's scratch
// array (its address is taken only after the host-side checks passed).
int accumulate_into(const ns_matrix_t *acc_in, const ns_matrix_t *win, int sign,
                    ns_matrix_t *acc_out, void *ws, uint64_t ws_bytes, hipStream_t s,
                    bool noalloc) {
  if (!acc_in || !win || !acc_out) return NS_ERR_INVALID_ARG;
  if (sign != 1 && sign != -1) return NS_ERR_INVALID_ARG;
  const ns_matrix_t *ins[2] = {acc_in, win};
  for (const ns_matrix_t *m : ins) {
    if (!m->keys || !m->counts || !m->nnz) return NS_ERR_INVALID_ARG;
    if (m->keys == acc_out->keys || m->counts == acc_out->counts || m->nnz == acc_out->nnz ||
        m->keys == acc_out->counts || m->counts == acc_out->keys)
      return NS_ERR_INVALID_ARG;
  }
  if (!acc_out->keys || !acc_out->counts || !acc_out->nnz) return NS_ERR_INVALID_ARG;
  const uint64_t na = acc_in->capacity < acc_in->packets ? acc_in->capacity : acc_in->packets;
  const uint64_t nb = win->capacity < win->packets ? win->capacity : win->packets;
  if (sign < 0 && win->packets > acc_in->packets) return NS_ERR_UNDERFLOW;
  const uint64_t need = sign > 0 ? na + nb : na;
  if (acc_out->capacity < need) return NS_ERR_CAPACITY;
  const MergeLayout ML = merge_plan(na + nb);
  if (noalloc) {
    if (na + nb > NS_ACCUMULATE_NOALLOC_MAX_ENTRIES || ML.total > kScratchBytes)
      return NS_ERR_UNSUPPORTED;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    ws_bytes = kScratchBytes;
  }
  if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign) return NS_ERR_WORKSPACE;
  if (ws_bytes < ML.total) return NS_ERR_WORKSPACE;
  const uint64_t tiles = ML.tiles;
  uint32_t *ticket = static_cast<uint32_t *>(ws);
  uint64_t *lbs = reinterpret_cast<uint64_t *>(static_cast<uint8_t *>(ws) + ML.lbs);
  // ticket and look-back words start at zero (fill kernels: no memset nodes
  // if the caller captures the call into a graph)
  HIP_TRY(launch_fill32(ticket, 1, 0, s));
  HIP_TRY(launch_fill64(lbs, tiles, 0, s));
  MergeArgs a{};
  a.ka = acc_in->keys;
  a.ca = acc_in->counts;
  a.na = acc_in->nnz;
  a.kb = win->keys;
  a.cb = win->counts;
  a.nb = win->nnz;
  a.na_max = na;
  a.nb_max = nb;
  a.kc = acc_out->keys;
  a.cc = acc_out->counts;
  a.nc = acc_out->nnz;
  a.nc_max = acc_out->capacity;
  a.sign = sign;
  a.lb = lbs;
  a.ticket = ticket;
  if (noalloc) HIP_TRY(launch_merge(a, tiles, s));  // no timing events either
  else HIP_TRY(timed(K_MERGE, s, [&] { return launch_merge(a, tiles, s); }));
  acc_out->packets = sign > 0 ? acc_in->packets + win->packets : acc_in->packets - win->packets;
  return NS_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *ns_version(void) { return "libns 1.0 (gfx950)"; }

const char *ns_error_string(int code) {
  switch (code) {
    case NS_OK: return "ok";
    case NS_ERR_INVALID_ARG: return "invalid argument";
    case NS_ERR_CAPACITY: return "output capacity below the a-priori bound";
    case NS_ERR_WORKSPACE: return "workspace too small or not 256-byte aligned";
    case NS_ERR_HIP: return "HIP runtime error";
    case NS_ERR_UNDERFLOW: return "subtraction below zero";
    case NS_ERR_UNSUPPORTED: return "size beyond the supported range";
    case NS_ERR_BOUNDS: return "an index outside its array (bounds-checked build)";
    default: return "unknown error";
  }
}

int ns_workspace_size(uint64_t max_packets, uint32_t num_windows, uint64_t *bytes) {
  if (!bytes) return NS_ERR_INVALID_ARG;
  // a batched call with an aggregate uses a second, single-window layout
  *bytes = up(plan(max_packets, num_windows).total) + plan(max_packets, 1).total;
  return NS_OK;
}

int ns_build_matrix(const uint32_t *src, const uint32_t *dst, uint64_t n, ns_matrix_t *out,
                    void *ws, uint64_t ws_bytes, void *stream) {
  if (!out || !out->keys || !out->counts || !out->nnz) return NS_ERR_INVALID_ARG;
  if (n > 0 && (!src || !dst)) return NS_ERR_INVALID_ARG;
  if (n > kMaxPackets32) return NS_ERR_UNSUPPORTED;
  if (out->capacity < n) return NS_ERR_CAPACITY;
  Ws w;
  int rc = check_ws(ws, ws_bytes, n, 1, &w);
  if (rc) return rc;
  Shapes sh;
  resolve_tuning(nullptr, &sh);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_fill32(w.at<uint32_t>(w.L.tickets), kMaxTickets, 0, s));
  uint64_t *seg = w.at<uint64_t>(w.L.seg);
  HIP_TRY(launch_seg1(seg, nullptr, n, s));
  PacketOut o{};
  o.ukeys = out->keys;
  o.counts = out->counts;
  o.nnz = out->nnz;
  o.sort_a = w.at<uint64_t>(w.L.KA);  // out of place (see the aggregate in enqueue_batch)
  o.sort_b = w.at<uint64_t>(w.L.KB);
  rc = enqueue_packets(w, sh, src, dst, seg, 1, n, o, s);
  if (rc) return rc;
  out->packets = n;
  return NS_OK;
}

int ns_stats(const ns_matrix_t *m, ns_stats_t *out, void *ws, uint64_t ws_bytes, void *stream) {
  if (!m || !out || !m->keys || !m->counts || !m->nnz) return NS_ERR_INVALID_ARG;
  const uint64_t cap = m->capacity < m->packets ? m->capacity : m->packets;
  // 2^32 packets or more: column items carry 32-bit link indices
  if (m->packets > kMaxPackets32 && cap > kMaxPackets32 + 1) return NS_ERR_UNSUPPORTED;
  Ws w;
  int rc = check_ws(ws, ws_bytes, cap, 1, &w);
  if (rc) return rc;
  Shapes sh;
  resolve_tuning(nullptr, &sh);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_fill32(w.at<uint32_t>(w.L.tickets), kMaxTickets, 0, s));
  return enqueue_matrix_stats(w, sh, m, reinterpret_cast<uint64_t *>(out), s);
}

int ns_stats_csr_workspace_size(uint64_t nnz, uint64_t *bytes) {
  if (!bytes) return NS_ERR_INVALID_ARG;
  // the flat entries (keys, counts, nnz word), then the statistics' workspace
  *bytes = up((2 * nnz + 1) * 8) + plan(nnz, 1).total;
  return NS_OK;
}

int ns_stats_csr(const uint32_t *rows, const uint64_t *row_ptr, uint64_t nrows,
                 const uint32_t *cols, const uint64_t *vals, uint64_t nnz, uint64_t packets,
                 ns_stats_t *out, void *ws, uint64_t ws_bytes, void *stream) {
  if (!out || !row_ptr) return NS_ERR_INVALID_ARG;
  if (nnz > 0 && (!rows || !cols || !vals || nrows == 0)) return NS_ERR_INVALID_ARG;
  if (packets < nnz) return NS_ERR_INVALID_ARG;  // every entry holds at least one packet
  if (packets > kMaxPackets32) return NS_ERR_UNSUPPORTED;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign) return NS_ERR_WORKSPACE;
  const uint64_t flat = up((2 * nnz + 1) * 8);
  if (ws_bytes < flat) return NS_ERR_WORKSPACE;
  Ws w;
  int rc = check_ws(static_cast<uint8_t *>(ws) + flat, ws_bytes - flat, nnz, 1, &w);
  if (rc) return rc;
  uint64_t *keys = static_cast<uint64_t *>(ws);
  ns_matrix_t m{keys, keys + nnz, keys + 2 * nnz, nnz, packets};
  Shapes sh;
  resolve_tuning(nullptr, &sh);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_csr_expand(rows, row_ptr, nrows, cols, vals, nnz, m.keys, m.counts, m.nnz, s));
  HIP_TRY(launch_fill32(w.at<uint32_t>(w.L.tickets), kMaxTickets, 0, s));
  rc = enqueue_matrix_stats(w, sh, &m, reinterpret_cast<uint64_t *>(out), s);
  if (rc) return rc;
  // the values' sum (valid packets) may not pass the caller's bound
  HIP_TRY(launch_check_total(reinterpret_cast<const uint64_t *>(out), packets, s));
  return NS_OK;
}

int ns_max_link_packets(const ns_matrix_t *m, uint64_t *out, void *stream) {
  if (!m || !out || !m->counts || !m->nnz) return NS_ERR_INVALID_ARG;
  const uint64_t cap = m->capacity < m->packets ? m->capacity : m->packets;
  HIP_TRY(launch_max_counts(m->counts, nullptr, m->nnz, 1, cap, out,
                            static_cast<hipStream_t>(stream)));
  return NS_OK;
}

int ns_batch_max_link_packets(const ns_batch_matrices_t *win, const uint64_t *offsets,
                              uint32_t num_windows, uint64_t total_packets, uint64_t *out,
                              void *stream) {
  if (!win || !offsets || !out || !win->counts || !win->nnz) return NS_ERR_INVALID_ARG;
  if (num_windows == 0) return NS_OK;
  if (win->capacity < total_packets) return NS_ERR_CAPACITY;
  HIP_TRY(launch_max_counts(win->counts, offsets, win->nnz, num_windows, total_packets, out,
                            static_cast<hipStream_t>(stream)));
  return NS_OK;
}

int ns_accumulate_workspace_size(uint64_t na, uint64_t nb, uint64_t *bytes) {
  if (!bytes) return NS_ERR_INVALID_ARG;
  *bytes = merge_plan(na + nb).total;
  return NS_OK;
}

int ns_accumulate(const ns_matrix_t *acc_in, const ns_matrix_t *win, int sign,
                  ns_matrix_t *acc_out, void *ws, uint64_t ws_bytes, void *stream) {
  return accumulate_into(acc_in, win, sign, acc_out, ws, ws_bytes,
                         static_cast<hipStream_t>(stream), false);
}

int ns_accumulate_noalloc(const ns_matrix_t *acc_in, const ns_matrix_t *win, int sign,
                          ns_matrix_t *acc_out, void *stream) {
  return accumulate_into(acc_in, win, sign, acc_out, nullptr, 0,
                         static_cast<hipStream_t>(stream), true);
}

// True when [p, p + n) is page-locked host memory known to the runtime
// (hipHostMalloc, or torch's pin_memory). A pointer the runtime does not know
// (pageable memory) makes the query fail; its error is consumed here so that
// it does not surface from a later call.
static bool page_locked(const uint32_t *p, uint64_t n) {
  const uint32_t *ends[2] = {p, p + (n - 1)};
  for (const uint32_t *q : ends) {
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, q) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    if (attr.type != hipMemoryTypeHost) return false;
  }
  return true;
}

int ns_stream_workspace_size(uint64_t batch, uint64_t capacity, uint64_t *bytes) {
  if (!bytes || batch == 0) return NS_ERR_INVALID_ARG;
  *bytes = stream_plan(batch, capacity).total;
  return NS_OK;
}

int ns_build_matrix_streamed(const uint32_t *src, const uint32_t *dst, uint64_t n, uint64_t batch,
                             ns_matrix_t *out, void *ws, uint64_t ws_bytes, void *stream,
                             void *copy_stream) {
  if (!out || !out->keys || !out->counts || !out->nnz) return NS_ERR_INVALID_ARG;
  if (n > 0 && (!src || !dst)) return NS_ERR_INVALID_ARG;
  if (batch == 0) return NS_ERR_INVALID_ARG;
  if (batch > kMaxPackets32) return NS_ERR_UNSUPPORTED;
  const uint64_t first = n < batch ? n : batch;
  if (out->capacity < first) return NS_ERR_CAPACITY;
  if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign) return NS_ERR_WORKSPACE;
  const StreamLayout SL = stream_plan(batch, out->capacity);
  if (ws_bytes < SL.total) return NS_ERR_WORKSPACE;
  // the packets must be page-locked host memory: an asynchronous copy of a
  // large pageable range makes the runtime lock the existing pages in place,
  // which hosts may refuse (and the failure then surfaces on the device)
  if (n > 0 && !(page_locked(src, n) && page_locked(dst, n))) return NS_ERR_INVALID_ARG;
  uint8_t *base = static_cast<uint8_t *>(ws);
  Ws w;
  int rc = check_ws(base + SL.inner, ws_bytes - SL.inner, batch, 1, &w);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStream_t cs = copy_stream ? static_cast<hipStream_t>(copy_stream) : s;
  const uint64_t C = out->capacity;
  const uint64_t nb = (n + batch - 1) / batch;  // b_n sub-partitions
  if (nb == 0) {
    HIP_TRY(launch_fill64(out->nnz, 1, 0, s));
    out->packets = 0;
    return NS_OK;
  }
  auto at64 = [&](uint64_t off) { return reinterpret_cast<uint64_t *>(base + off); };
  uint32_t *stage = reinterpret_cast<uint32_t *>(base + SL.stage);
  uint32_t *st_src[2] = {stage, stage + 2 * batch};
  uint32_t *st_dst[2] = {stage + batch, stage + 3 * batch};
  ns_matrix_t bm{at64(SL.bkeys), at64(SL.bcounts), at64(SL.bnnz), batch, 0};
  ns_matrix_t am{at64(SL.akeys), at64(SL.acounts), at64(SL.annz), C, 0};
  // the aggregate after sub-partition k lives in `out` when nb-1-k is even, so
  // the last one lands there
  auto agg = [&](uint64_t k) -> ns_matrix_t * { return ((nb - 1 - k) & 1) == 0 ? out : &am; };
  Shapes sh;
  resolve_tuning(nullptr, &sh);
  hipEvent_t copied[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr}, entry = nullptr;
  int status = NS_OK;
  for (int b = 0; b < 2 && status == NS_OK; ++b) {
    if (hipEventCreateWithFlags(&copied[b], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&freed[b], hipEventDisableTiming) != hipSuccess)
      status = NS_ERR_HIP;
  }
  // work enqueued earlier on `stream` (an earlier call's builds) may still read
  // the staging buffers: the first copies wait for it
  if (status == NS_OK && cs != s &&
      (hipEventCreateWithFlags(&entry, hipEventDisableTiming) != hipSuccess ||
       hipEventRecord(entry, s) != hipSuccess || hipStreamWaitEvent(cs, entry, 0) != hipSuccess))
    status = NS_ERR_HIP;
  // sub-partition k goes to staging buffer k&1 once the build of k-2 has read it
  auto copy_in = [&](uint64_t k) -> int {
    const int b = (int)(k & 1);
    const uint64_t off = k * batch, len = n - off < batch ? n - off : batch;
    if (k >= 2) HIP_TRY(hipStreamWaitEvent(cs, freed[b], 0));
    HIP_TRY(hipMemcpyAsync(st_src[b], src + off, len * 4, hipMemcpyHostToDevice, cs));
    HIP_TRY(hipMemcpyAsync(st_dst[b], dst + off, len * 4, hipMemcpyHostToDevice, cs));
    HIP_TRY(hipEventRecord(copied[b], cs));
    return NS_OK;
  };
  if (status == NS_OK) status = copy_in(0);
  for (uint64_t k = 0; k < nb && status == NS_OK; ++k) {
    // the next sub-partition crosses the bus while this one is built
    if (k + 1 < nb && (status = copy_in(k + 1)) != NS_OK) break;
    const int b = (int)(k & 1);
    const uint64_t len = n - k * batch < batch ? n - k * batch : batch;
    if (hipStreamWaitEvent(s, copied[b], 0) != hipSuccess) { status = NS_ERR_HIP; break; }
    ns_matrix_t *dest = k == 0 ? agg(0) : &bm;
    if (launch_fill32(w.at<uint32_t>(w.L.tickets), kMaxTickets, 0, s) != hipSuccess) { status = NS_ERR_HIP; break; }
    uint64_t *seg = w.at<uint64_t>(w.L.seg);
    if (launch_seg1(seg, nullptr, len, s) != hipSuccess) { status = NS_ERR_HIP; break; }
    PacketOut o{};
    o.ukeys = dest->keys;
    o.counts = dest->counts;
    o.nnz = dest->nnz;
    o.sort_a = w.at<uint64_t>(w.L.KA);
    o.sort_b = w.at<uint64_t>(w.L.KB);
    if ((status = enqueue_packets(w, sh, st_src[b], st_dst[b], seg, 1, len, o, s)) != NS_OK) break;
    if (hipEventRecord(freed[b], s) != hipSuccess) { status = NS_ERR_HIP; break; }
    if (k == 0) continue;
    // union-add into the other aggregate buffer (Fig. 2: load and aggregate)
    const ns_matrix_t *prev = agg(k - 1);
    ns_matrix_t *next = agg(k);
    uint64_t *lbs = at64(SL.mlb);
    const uint64_t na_max = k * batch < C ? k * batch : C;
    if (launch_fill64(lbs, SL.merge_tiles, 0, s) != hipSuccess) { status = NS_ERR_HIP; break; }
    MergeArgs a{};
    a.ka = prev->keys;
    a.ca = prev->counts;
    a.na = prev->nnz;
    a.kb = bm.keys;
    a.cb = bm.counts;
    a.nb = bm.nnz;
    a.na_max = na_max;
    a.nb_max = len;
    a.kc = next->keys;
    a.cc = next->counts;
    a.nc = next->nnz;
    a.nc_max = C;
    a.sign = 1;
    a.lb = lbs;
    a.ticket = w.ticket();
    if (launch_merge(a, (na_max + len) / kMergeTile + 2, s) != hipSuccess) { status = NS_ERR_HIP; break; }
  }
  // destruction of a recorded event waits for nothing; it is released once
  // its work completes
  for (int b = 0; b < 2; ++b) {
    if (copied[b]) hipEventDestroy(copied[b]);
    if (freed[b]) hipEventDestroy(freed[b]);
  }
  if (entry) hipEventDestroy(entry);
  if (status != NS_OK) return status;
  out->packets = n;
  return NS_OK;
}

int ns_batch_stats_eager(const uint32_t *src, const uint32_t *dst, const uint64_t *offsets,
                         uint32_t num_windows, uint64_t total_packets, ns_stats_t *out,
                         ns_matrix_t *agg_out, ns_stats_t *agg_stats,
                         ns_batch_matrices_t *win_out, const ns_tuning_t *tune, void *ws,
                         uint64_t ws_bytes, void *stream) {
  BatchArgs b;
  Ws w, w2;
  int rc = batch_checks(src, dst, offsets, num_windows, total_packets, out, agg_out, agg_stats,
                        win_out, tune, ws, ws_bytes, &b, &w, &w2);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = enqueue_batch(b, w, w2, s, s, nullptr, nullptr);
  if (rc) return rc;
  if (agg_out) agg_out->packets = total_packets;
  return NS_OK;
}

int ns_batch_stats(const uint32_t *src, const uint32_t *dst, const uint64_t *offsets,
                   uint32_t num_windows, uint64_t total_packets, ns_stats_t *out,
                   ns_matrix_t *agg_out, ns_stats_t *agg_stats, ns_batch_matrices_t *win_out,
                   const ns_tuning_t *tune, void *ws, uint64_t ws_bytes, void *stream) {
  BatchArgs b;
  Ws w, w2;
  int rc = batch_checks(src, dst, offsets, num_windows, total_packets, out, agg_out, agg_stats,
                        win_out, tune, ws, ws_bytes, &b, &w, &w2);
  if (rc) return rc;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return NS_ERR_HIP;
  const std::string key = batch_key(dev, b, ws, ws_bytes);
  GraphCache &c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  auto it = c.execs.find(key);
  hipGraphExec_t exec = nullptr;
  if (it != c.execs.end()) {
    exec = it->second;
  } else {
    if (!c.capture[dev]) {
      HIP_TRY(hipStreamCreateWithFlags(&c.capture[dev], hipStreamNonBlocking));
      HIP_TRY(hipStreamCreateWithFlags(&c.capture2[dev], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&c.fork[dev], hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&c.join[dev], hipEventDisableTiming));
    }
    hipStream_t cs = c.capture[dev];
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    rc = enqueue_batch(b, w, w2, cs, c.capture2[dev], c.fork[dev], c.join[dev]);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc || e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return rc ? rc : NS_ERR_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) return NS_ERR_HIP;
    if (c.execs.size() >= 64) {
      for (auto &kv : c.execs) hipGraphExecDestroy(kv.second);
      c.execs.clear();
    }
    c.execs.emplace(key, exec);
  }
  HIP_TRY(hipGraphLaunch(exec, static_cast<hipStream_t>(stream)));
  if (agg_out) agg_out->packets = total_packets;
  return NS_OK;
}

int ns_rolling_size(uint64_t link_slots, uint64_t address_slots, uint64_t *bytes) {
  if (!bytes) return NS_ERR_INVALID_ARG;
  *bytes = roll_bytes(link_slots, address_slots);
  return NS_OK;
}

static int rolling_check(const ns_rolling_t *r) {
  if (!r || !r->mem || (reinterpret_cast<uintptr_t>(r->mem) % kAlign) != 0) return NS_ERR_INVALID_ARG;
  const uint64_t l = r->link_slots, a = r->address_slots;
  if (l < 64 || a < 64 || (l & (l - 1)) || (a & (a - 1))) return NS_ERR_INVALID_ARG;
  if (r->bytes < roll_bytes(l, a)) return NS_ERR_WORKSPACE;
  return NS_OK;
}

int ns_rolling_init(const ns_rolling_t *r, void *stream) {
  int rc = rolling_check(r);
  if (rc) return rc;
  const RollTables t = roll_tables(r->mem, r->link_slots, r->address_slots);
  HIP_TRY(launch_roll_clear(t, static_cast<hipStream_t>(stream)));
  return NS_OK;
}

int ns_rolling_update(const ns_rolling_t *r, const ns_matrix_t *add, const ns_matrix_t *remove,
                      ns_stats_t *out, void *stream) {
  int rc = rolling_check(r);
  if (rc) return rc;
  if (!out) return NS_ERR_INVALID_ARG;
  const ns_matrix_t *ms[2] = {add, remove};
  for (const ns_matrix_t *m : ms)
    if (m && (!m->keys || !m->counts || !m->nnz)) return NS_ERR_INVALID_ARG;
  const RollTables t = roll_tables(r->mem, r->link_slots, r->address_slots);
  RollDelta d{};
  uint64_t items = 0;
  if (add) {
    d.add_keys = add->keys;
    d.add_counts = add->counts;
    d.add_nnz = add->nnz;
    d.add_cap = add->capacity < add->packets ? add->capacity : add->packets;
    items += d.add_cap;
  }
  if (remove) {
    d.rem_keys = remove->keys;
    d.rem_counts = remove->counts;
    d.rem_nnz = remove->nnz;
    d.rem_cap = remove->capacity < remove->packets ? remove->capacity : remove->packets;
    items += d.rem_cap;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(timed(K_MERGE, s, [&] { return launch_roll_update(t, d, items, s); }));
  HIP_TRY(timed(K_SEGMAX, s, [&] { return launch_roll_stats(t, reinterpret_cast<uint64_t *>(out), s); }));
  return NS_OK;
}

int ns_rolling_compact(const ns_rolling_t *from, const ns_rolling_t *to, void *stream) {
  int rc = rolling_check(from);
  if (rc) return rc;
  rc = rolling_check(to);
  if (rc) return rc;
  if (from->link_slots != to->link_slots || from->address_slots != to->address_slots ||
      from->mem == to->mem)
    return NS_ERR_INVALID_ARG;
  const RollTables a = roll_tables(from->mem, from->link_slots, from->address_slots);
  const RollTables b = roll_tables(to->mem, to->link_slots, to->address_slots);
  HIP_TRY(launch_roll_compact(a, b, static_cast<hipStream_t>(stream)));
  return NS_OK;
}

int ns_rolling_occupancy(const ns_rolling_t *r, uint64_t *slots_used, void *stream) {
  int rc = rolling_check(r);
  if (rc) return rc;
  if (!slots_used) return NS_ERR_INVALID_ARG;
  const RollTables t = roll_tables(r->mem, r->link_slots, r->address_slots);
  HIP_TRY(launch_roll_used(t, slots_used, static_cast<hipStream_t>(stream)));
  return NS_OK;
}

int ns_device_status(void *stream, int *status) {
  if (!status) return NS_ERR_INVALID_ARG;
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  HIP_TRY(read_and_clear_status(status));
  return NS_OK;
}

int ns_timing_enable(int on) {
  Profiler &p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  p.on = on != 0;
  return NS_OK;
}

int ns_timing_reset(void) {
  Profiler &p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  for (auto &m : p.marks) {
    hipEventDestroy(m.a);
    hipEventDestroy(m.b);
  }
  p.marks.clear();
  return NS_OK;
}

int ns_timing_read(uint32_t kind, double *total_ms, uint64_t *launches) {
  if (!total_ms || !launches || kind >= K_COUNT) return NS_ERR_INVALID_ARG;
  Profiler &p = prof();
  std::lock_guard<std::mutex> lock(p.mu);
  double t = 0;
  uint64_t n = 0;
  for (auto &m : p.marks) {
    if ((uint32_t)m.kind != kind) continue;
    HIP_TRY(hipEventSynchronize(m.b));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, m.a, m.b));
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return NS_OK;
}

int ns_release_graphs(void) {
  GraphCache &c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  for (auto &kv : c.execs) hipGraphExecDestroy(kv.second);
  c.execs.clear();
  return NS_OK;
}

}  // extern "C"
