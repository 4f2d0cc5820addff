// Host-side launchers of the libns kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ns {

// Byte digits of the packed key src<<32|dst: digit p covers bits [8p, 8p+8).
constexpr int kKeyDigits = 8;
constexpr int kColDigits = 4;  // digits 4..7 of a column item dst<<32|count
constexpr int kBins = 256;

struct SortShape {
  int block;  // 256 or 512
  int items;  // 8 or 16
  int tile() const { return block * items; }
};

struct ScanShape {
  int items;  // 4, 8 or 16 positions per thread (block is 256)
  int tile() const { return 256 * items; }
};

constexpr int kHistTile = 256 * 32;   // packets per histogram tile
constexpr int kMergeTile = 256 * 8;   // merged positions per merge tile

// --- generic -----------------------------------------------------------------
hipError_t launch_fill64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
// up to kFillMax regions of 32- or 64-bit words, each set to its value, in one launch
constexpr int kFillMax = 12;
struct FillEntry {
  void *p;
  uint64_t n;      // words
  uint64_t v;
  uint32_t wide;   // 1: 64-bit words, 0: 32-bit words
};
struct FillList {
  FillEntry e[kFillMax];
  uint32_t count = 0;
  void add64(uint64_t *p, uint64_t n, uint64_t v = 0) { e[count++] = {p, n, v, 1}; }
  void add32(uint32_t *p, uint64_t n, uint32_t v = 0) { e[count++] = {p, n, v, 0}; }
};
hipError_t launch_fill_multi(const FillList &f, hipStream_t s);
hipError_t launch_copy64(uint64_t *dst, const uint64_t *src, uint64_t n, hipStream_t s);
// seg[0] = 0, seg[1] = min(*n_dev, n) if n_dev else n
hipError_t launch_seg1(uint64_t *seg, const uint64_t *n_dev, uint64_t n, hipStream_t s);
// per-segment tile prefix for up to three tile sizes (null outputs skipped);
// oa[W+1] receives the layer count for layered ticket order, or 0 (oa needs
// W+2 entries)
hipError_t launch_tiles(const uint64_t *seg_off, uint32_t W, uint32_t ta, uint64_t *oa,
                        uint32_t tb, uint64_t *ob, uint32_t tc, uint64_t *oc, hipStream_t s);

// --- radix sort ----------------------------------------------------------------
hipError_t launch_hist_packets(const uint32_t *src, const uint32_t *dst, const uint64_t *seg_off,
                               const uint64_t *tile_off, uint32_t W, uint64_t max_tiles,
                               uint32_t *hist, hipStream_t s);
// digit histograms (4 digits of dst) of column items dst<<32|count, per segment
hipError_t launch_hist_items(const uint64_t *items, const uint64_t *seg_off,
                             const uint64_t *tile_off, uint32_t W, uint64_t max_tiles,
                             uint32_t *hist, hipStream_t s);
// exclusive scan of rows of 256 bins
hipError_t launch_hist_scan(const uint32_t *hist, uint32_t *base, uint64_t rows, hipStream_t s);

struct PassArgs {
  const uint32_t *src;       // packets input (first key pass) or null
  const uint32_t *dst;
  const uint64_t *in;        // u64 input otherwise
  uint64_t *out;
  const uint64_t *seg_off;   // [W+1]
  const uint64_t *tile_off;  // [W+2] tile prefix of this sort's tile size, [W+1] = layers
  uint32_t W;
  uint32_t shift;            // digit = (key >> shift) & 255
  const uint32_t *base;      // bucket starts of this digit: base[w*base_stride + bin]
  uint32_t base_stride;
  uint64_t *lb;              // look-back words of this pass [tiles][256]
  uint64_t *lb_next;         // cleared for the next pass
  uint32_t *ticket;
  uint64_t lim;              // entries of the input and output arrays (bounds checks)
};
hipError_t launch_pass(const SortShape &sh, const PassArgs &a, uint64_t max_tiles, hipStream_t s);

// --- batches of at most kSmallMax packets: the per-window pipeline of each
// window inside one workgroup's LDS (quantities [W][8] and/or the positional
// window matrices; null outputs are skipped) ---
constexpr int kSmallBlock = 1024;
constexpr uint32_t kSmallMax = 8192;  // packets per batch (so per window)
hipError_t launch_small(const uint32_t *src, const uint32_t *dst, const uint64_t *off, uint32_t W,
                        uint64_t *stats, uint64_t *win_keys, uint64_t *win_counts,
                        uint64_t *win_nnz, hipStream_t s);

// --- radix pass over one large segment: reduce, scan, scatter (no look-back) ---
#ifndef NS_CHUNK_TILES
#define NS_CHUNK_TILES 4
#endif
constexpr uint32_t kChunkTiles = NS_CHUNK_TILES;  // tiles per chunk
constexpr uint32_t kChunkBlocks = 1024;            // most row blocks of the chunk scan
// rows of the chunk tables for a segment of n keys in tiles of `tile` keys
inline uint64_t chunk_rows(uint64_t n, uint64_t tile) {
  const uint64_t r = (n + tile * kChunkTiles - 1) / (tile * kChunkTiles);
  return r ? r : 1;
}
// Digit widths of the chunked passes: byte digits, or 11-bit digits (2048
// bins) that sort 64-bit keys in 6 passes and 32-bit column keys in 3.
constexpr int kWideBits = 11;
constexpr int kMaxBins = 1 << kWideBits;
struct ChunkArgs {
  const uint64_t *seg_off;  // [2]: the segment is [seg_off[0], seg_off[1])
  uint32_t chunks;          // set by the launcher (<= max_chunks)
  uint32_t max_chunks;      // rows of count and prefix
  uint32_t bins;            // set by the launcher: 2^(digit bits), the row length
  uint32_t *count;          // [max_chunks][bins] digit counts per chunk
  uint64_t *prefix;         // [max_chunks][bins] keys of the digit in earlier chunks
  uint64_t *bsum;           // [blocks][bins] per row block: sum, then exclusive prefix
  uint64_t *total;          // [bins] keys per digit
};
// Sorts at most max_keys keys on the digit of `bits` bits (8 or kWideBits) at
// a.shift. a.seg_off / tile_off / W / base / lb are unused; a.ticket must
// start at zero. When kernel timing is on, the counting and scan kernels are
// recorded under count_kind.
hipError_t launch_pass_chunked(const SortShape &sh, const PassArgs &a, const ChunkArgs &c,
                               uint64_t max_keys, int bits, int count_kind, hipStream_t s);

// --- run-length encoding of sorted packet keys ------------------------------------
struct RleArgs {
  const uint64_t *keys;
  const uint64_t *seg_off;
  const uint64_t *tile_off;
  uint32_t W;
  uint64_t *ukeys;     // nullable; may equal keys (in place)
  uint64_t *counts;    // nullable
  uint64_t *items;     // nullable: dst<<32 | count per link
  uint64_t *win_keys;  // nullable: positional per-segment matrices (segment w's links
  uint64_t *win_counts;//   start at seg_off[w]); then seg_base and win_nnz are used
  uint64_t *win_nnz;   // [W] links per segment
  uint64_t *seg_base;  // [W] flagged words: global link index at each segment start
  uint64_t *rpos;      // nullable: packet position of each row head (+ sentinel)
  uint64_t *rlink;     // link index of each row head (+ sentinel)
  uint64_t *link_off;  // [W+1]
  uint64_t *row_off;   // [W+1]
  uint64_t *nnz_out;   // nullable: total links
  uint64_t *lb;        // [tiles][2]
  uint32_t *ticket;
  uint64_t lim;        // positions (and so links) of the input; head arrays hold lim + 2
  uint32_t *col_hist;  // nullable, with rle_one_large_segment only: the column items'
                       // destination-digit counts [4][256] are added here (zeroed by the caller)
};
hipError_t launch_rle(const ScanShape &sh, const RleArgs &a, uint64_t max_tiles, hipStream_t s);
// whether launch_rle takes its single-large-segment variant (rows from
// registers, one look-back word per tile, column histogram on the way)
bool rle_one_large_segment(const ScanShape &sh, uint32_t W, uint64_t max_tiles, uint64_t lim);

// --- run reduction over a sorted array with explicit values -----------------------
// mode 0: rows of a matrix (group = key>>32, value = counts[p]); also emits
//         column items.
// mode 1: columns of sorted items (group = item>>32, value = item & 0xffffffff,
//         or with `wide`, gather[item & 0xffffffff]).
// wide: 64-bit values (matrices of 2^32 packets or more): column items carry
//       the link index instead of the count, and tile sums are 64-bit.
struct RunArgs {
  const uint64_t *keys;
  const uint64_t *counts;    // mode 0
  const uint64_t *seg_off;
  const uint64_t *tile_off;
  uint32_t W;
  uint64_t *hpos;            // head position (+ sentinel)
  uint64_t *hval;            // exclusive value prefix at head (+ sentinel)
  uint64_t *head_off;        // [W+1]
  uint64_t *items;           // mode 0, nullable
  uint64_t *lb;              // [tiles][2]
  uint32_t *ticket;
  uint32_t wide;             // 0 or 1 (see above)
  const uint64_t *gather;    // mode 1 with wide: the matrix counts
  uint64_t lim;              // entries of keys / items / gather; head arrays hold lim + 2
  uint64_t vlim;             // bound on the sum of all values (packets); 0 = unknown
};
hipError_t launch_runs(const ScanShape &sh, int mode, const RunArgs &a, uint64_t max_tiles,
                       hipStream_t s);

// out[w] = max over counts[off[w] .. off[w]+nnz[w]) (0 if empty); off == nullptr:
// one window at [0, nnz[0]). Positions scanned: [0, total).
hipError_t launch_max_counts(const uint64_t *counts, const uint64_t *off, const uint64_t *nnz,
                             uint32_t W, uint64_t total, uint64_t *out, hipStream_t s);

// per segment: stats[w][fa] = max(a[r+1]-a[r]), stats[w][fb] = max(b[r+1]-b[r])
// over the heads r of segment w (heads [head_off[w], head_off[w+1]))
hipError_t launch_segmax(const uint64_t *a, const uint64_t *b, const uint64_t *head_off,
                         uint32_t W, uint64_t max_heads, uint64_t *stats, int fa, int fb,
                         hipStream_t s);

// stats[w][0..3] from segment, link, row and column offsets
hipError_t launch_finalize(const uint64_t *seg_off, const uint64_t *link_off,
                           const uint64_t *row_off, const uint64_t *col_off, uint32_t W,
                           uint64_t *stats, hipStream_t s);
// matrix stats[0..3]: valid = rows value sentinel, links = *nnz, rows, cols
hipError_t launch_finalize_matrix(const uint64_t *row_hval, const uint64_t *row_off,
                                  const uint64_t *col_off, const uint64_t *nnz,
                                  uint64_t *stats, hipStream_t s);

// --- union-add / subtract ---------------------------------------------------------
struct MergeArgs {
  const uint64_t *ka, *ca, *na;
  const uint64_t *kb, *cb, *nb;
  uint64_t na_max, nb_max;  // host bounds on *na, *nb
  uint64_t *kc, *cc, *nc;
  uint64_t nc_max;  // capacity of kc / cc: entries past it are dropped and flagged
  int sign;
  uint64_t *lb;   // [tiles]
  uint32_t *ticket;
};
hipError_t launch_merge(const MergeArgs &a, uint64_t max_tiles, hipStream_t s);

// --- hypersparse CSR -> sorted COO (keys, counts); *nnz_out = nnz ---------------
hipError_t launch_csr_expand(const uint32_t *rows, const uint64_t *row_ptr, uint64_t nrows,
                             const uint32_t *cols, const uint64_t *vals, uint64_t nnz,
                             uint64_t *keys, uint64_t *counts, uint64_t *nnz_out, hipStream_t s);
// Raises the device status when stats[0] (valid packets) exceeds `packets`.
hipError_t launch_check_total(const uint64_t *stats, uint64_t packets, hipStream_t s);

// --- rolling aggregate (serving) ----------------------------------------------------
struct RollHeader {
  uint64_t links, sources, dests, packets;  // live counts
  uint64_t scan[4];                         // maxima found by the last scan
  uint64_t used[3];                         // slots taken since the last clear or compaction
                                            // (link, source, destination tables)
  uint32_t special_count;                   // count of the link key 0xFFFFFFFFFFFFFFFF
  uint32_t pad;
};
struct RollTables {
  RollHeader *hdr;
  uint64_t link_cap, addr_cap;  // slots, powers of two
  uint64_t *link_keys;
  uint32_t *link_cnt;
  uint64_t *src_keys;
  uint32_t *src_pk, *src_fan;
  uint64_t *dst_keys;
  uint32_t *dst_pk, *dst_fan;
};
struct RollDelta {
  const uint64_t *add_keys, *add_counts, *add_nnz;
  uint64_t add_cap;
  const uint64_t *rem_keys, *rem_counts, *rem_nnz;
  uint64_t rem_cap;
};
uint64_t roll_bytes(uint64_t link_cap, uint64_t addr_cap);
RollTables roll_tables(void *mem, uint64_t link_cap, uint64_t addr_cap);
hipError_t launch_roll_clear(const RollTables &t, hipStream_t s);
hipError_t launch_roll_update(const RollTables &t, const RollDelta &d, uint64_t max_items,
                              hipStream_t s);
hipError_t launch_roll_stats(const RollTables &t, uint64_t *out, hipStream_t s);
hipError_t launch_roll_compact(const RollTables &from, const RollTables &to, hipStream_t s);
hipError_t launch_roll_used(const RollTables &t, uint64_t *out, hipStream_t s);

// device error word: bit 0 underflow, bit 1 capacity (hash table full), bit 2
// invalid input, bit 3 an index outside its array (bounds-checked builds)
hipError_t read_and_clear_status(int *host_status);

// Kernel timing: while tl_timing_kind >= 0, every launch on this thread takes
// start/stop events in its dispatch and hands them to record_timing (defined by
// the API layer, which owns the events).
extern thread_local int tl_timing_kind;
void record_timing(int kind, hipEvent_t start, hipEvent_t stop);

}  // namespace ns
