/*
 * ns.h -- C ABI of libns.so: anonymized network sensing on MI355X (gfx950).
 *
 * A window is a multiset of packets, each a (source, destination) pair of
 * 32-bit anonymized IPv4 addresses. Its traffic matrix A has A(i,j) = number
 * of packets from source i to destination j (Table I caption). The library
 * builds A as a hypersparse 2^32 x 2^32 matrix in sorted COO form and reduces
 * it to the eight quantities of ns_stats_t.
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless marked "host". Buffers are owned by
 *     the caller (the library never allocates device memory); the library only
 *     reads inputs and writes outputs and the caller's workspace.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the default
 *     stream). Results are valid once the stream reaches the call.
 *   - Return 0 (NS_OK) or a negative NS_ERR_* code. Argument and capacity
 *     errors are found on the host before anything is enqueued; then outputs
 *     are untouched. No device-to-host synchronisation happens on any hot path:
 *     capacities are checked against host-known bounds (packet counts), and
 *     sizes produced on the device (nnz) stay on the device.
 *   - Packets per window and per batched call must be below 2^32; a matrix
 *     given to ns_stats may hold more (with fewer than 2^32 + 1 entries).
 *   - `ws` is caller workspace of at least ns_workspace_size() bytes, 256-byte
 *     aligned. Calls that share one workspace must be ordered on one stream.
 */
#ifndef NS_H_
#define NS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NS_OK = 0,
  NS_ERR_INVALID_ARG = -1,  /* null pointer, bad size, aliasing, bad sign */
  NS_ERR_CAPACITY = -2,     /* an output's capacity is below the a-priori bound */
  NS_ERR_WORKSPACE = -3,    /* ws too small or misaligned */
  NS_ERR_HIP = -4,          /* a HIP runtime call failed */
  NS_ERR_UNDERFLOW = -5,    /* subtraction below zero (host-detected, or via ns_device_status) */
  NS_ERR_UNSUPPORTED = -6,  /* size beyond the supported range (>= 2^32 packets) */
  NS_ERR_BOUNDS = -7        /* an index outside its array (libns_debug.so only, via ns_device_status) */
};

/* The eight quantities, all exact uint64, in this fixed order (64 bytes).
 *   valid_packets        sum_i sum_j A(i,j)                         Table I
 *   unique_links         number of (i,j) with A(i,j) > 0            Table I
 *   unique_sources       number of rows i with sum_j A(i,j) > 0     Table I
 *   unique_destinations  number of columns j with sum_i A(i,j) > 0  Table I
 *   max_source_packets   max_i sum_j A(i,j)        (row sums, Sec. IV data representation)
 *   max_source_fanout    max_i #{j : A(i,j) > 0}   (Table I, read as the row's nonzero count)
 *   max_destination_packets  max_j sum_i A(i,j)    (column sums, Sec. IV)
 *   max_destination_fanin    max_j #{i : A(i,j) > 0} (Table I, column nonzero count)
 * An empty window has all eight equal to 0. */
typedef struct {
  uint64_t valid_packets;
  uint64_t unique_links;
  uint64_t unique_sources;
  uint64_t unique_destinations;
  uint64_t max_source_packets;
  uint64_t max_source_fanout;
  uint64_t max_destination_packets;
  uint64_t max_destination_fanin;
} ns_stats_t;

/* A traffic matrix in sorted COO form: a NON-OWNING view of caller buffers.
 *   keys[k]   = (uint64)source << 32 | destination, strictly increasing on [0, *nnz)
 *   counts[k] = A(source, destination) >= 1
 *   nnz       device scalar, written by the library
 *   capacity  host: entries allocated in keys and in counts
 *   packets   host: exact number of packets the matrix represents (= sum of
 *             counts); set by the library on every output matrix. */
typedef struct {
  uint64_t *keys;
  uint64_t *counts;
  uint64_t *nnz;
  uint64_t capacity;
  uint64_t packets;
} ns_matrix_t;

/* Launch shape of the batched path. 0 in any field selects the built-in
 * default; the autotuner in the Python package fills these from its cache.
 *   sort_block   workgroup size of the radix passes (256 or 512)
 *   sort_items   keys per thread in a radix pass (8 or 16): tile = block*items
 *   digit_bits   radix digit width of the chunked passes (8 or 11): a single
 *                segment on chunked passes sorts its 64-bit keys in 8 passes of
 *                byte digits or 6 of 11-bit digits (2048 bins), and its 32-bit
 *                column keys in 4 or 3; passes with look-back (several segments)
 *                always use byte digits (their per-segment histograms and
 *                per-tile look-back words grow with the bin count)
 *   scan_items   positions per thread in the run-length / run-reduce passes (4, 8 or 16)
 *   chunked_min  a single segment (one window, or the aggregate of all windows)
 *                of at least this many keys is sorted by chunked passes (count,
 *                scan, scatter) rather than passes with look-back; 0 = 2^24,
 *                UINT64_MAX = never. Results are identical either way. */
typedef struct {
  uint32_t sort_block;
  uint32_t sort_items;
  uint32_t digit_bits;
  uint32_t scan_items;
  uint64_t chunked_min;
} ns_tuning_t;

/* Per-window matrices of a batch, laid out by packet offset: window w's
 * sorted COO occupies keys/counts[offsets[w] .. offsets[w] + nnz[w]) where
 * offsets are the batch's packet offsets (so a caller that knows them can
 * address any window's matrix without reading the device), and nnz is a device
 * array of num_windows entries written by the library. capacity (host) must be
 * >= the batch's total packets. */
typedef struct {
  uint64_t *keys;
  uint64_t *counts;
  uint64_t *nnz;
  uint64_t capacity;
} ns_batch_matrices_t;

/* Bytes of workspace sufficient for every entry point called with at most
 * `max_packets` packets (or matrix entries / capacity) in total and at most
 * `num_windows` windows. Host-only; writes *bytes (host). */
int ns_workspace_size(uint64_t max_packets, uint32_t num_windows, uint64_t *bytes);

/* Build the traffic matrix of one window (Table I caption: A(i,j) counts the
 * packets from i to j). src/dst: n uint32 each. out->keys and out->counts must
 * hold at least n entries;
 * out->packets is set to n; *out->nnz is written on the device. n = 0 gives an
 * empty matrix. */
int ns_build_matrix(const uint32_t *src, const uint32_t *dst, uint64_t n, ns_matrix_t *out,
                    void *ws, uint64_t ws_bytes, void *stream);

/* Union-add (sign = +1) or subtract (sign = -1) of two matrices: acc_out(i,j)
 * = acc_in(i,j) + sign*win(i,j), structure = union, entries that reach zero
 * are dropped ("load and aggregate", Fig. 2 caption; subtraction is its exact
 * inverse and serves rolling windows). acc_out must not alias either input.
 * Capacity: acc_out->capacity >= min(acc_in cap, acc_in packets) + min(win
 * cap, win packets) for add, >= min(acc_in cap, acc_in packets) for subtract.
 * Subtracting more packets than acc_in holds is rejected on the host; an
 * entry of win that is absent from or larger than acc_in is detected on the
 * device and reported by ns_device_status (acc_out is then undefined).
 * Workspace: ns_accumulate_workspace_size(na, nb) bytes, 256-byte aligned,
 * with na = min(acc_in cap, acc_in packets) and nb = min(win cap, win
 * packets) (a few bytes per thousand entries; a workspace of
 * ns_workspace_size(na + nb, 1) bytes is also large enough). */
int ns_accumulate_workspace_size(uint64_t na, uint64_t nb, uint64_t *bytes);
int ns_accumulate(const ns_matrix_t *acc_in, const ns_matrix_t *win, int sign,
                  ns_matrix_t *acc_out, void *ws, uint64_t ws_bytes, void *stream);

/* ns_accumulate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same union-add / subtract with the same arguments and results, but the
 * merge's ticket and look-back words live in a scratch array the library
 * holds in device memory (one per device, about 4 MiB, kept until the process
 * ends) instead of a caller workspace. No call allocates or frees memory.
 * Supports na + nb <= NS_ACCUMULATE_NOALLOC_MAX_ENTRIES (na, nb as for
 * ns_accumulate); larger inputs return NS_ERR_UNSUPPORTED before anything is
 * enqueued. Every call on a device uses that device's one scratch array (it
 * is cleared by kernels at the start of each call): calls that may overlap on
 * one device, such as calls on different streams without ordering between
 * them, race and give undefined results. */
#define NS_ACCUMULATE_NOALLOC_MAX_ENTRIES (1ull << 30)
int ns_accumulate_noalloc(const ns_matrix_t *acc_in, const ns_matrix_t *win, int sign,
                          ns_matrix_t *acc_out, void *stream);

/* Out-of-core build (Sec. III-C "Concurrent Batching", Fig. 3: input data
 * held on the host is cut into b_n batches that are moved to the GPU one
 * after the other during the computation). The n packets in PAGE-LOCKED HOST
 * memory (src, dst: n uint32 each, allocated with hipHostMalloc or torch's
 * pin_memory; pageable memory is rejected with NS_ERR_INVALID_ARG, since an
 * asynchronous copy of a large pageable range would have the runtime lock the
 * existing pages, which hosts may refuse) are taken in
 * b_n = ceil(n / batch) sub-partitions of `batch`
 * packets: sub-partition k+1 is copied to the device on `copy_stream` while
 * sub-partition k is built into its matrix on `stream` (as ns_build_matrix),
 * which is then union-added into the running aggregate (as ns_accumulate).
 * On return (asynchronously) `out` holds the matrix of all n packets, exactly
 * as ns_build_matrix would build it: the result does not depend on `batch`.
 *   batch        packets per sub-partition, 1 .. 2^32-1
 *   out          device matrix; out->capacity bounds the links of the
 *                aggregate (it must be >= min(n, batch)); out->packets = n.
 *                If the links exceed it, the first out->capacity links are
 *                kept, *out->nnz = out->capacity, and ns_device_status
 *                reports NS_ERR_CAPACITY.
 *   ws, ws_bytes device workspace of ns_stream_workspace_size(batch,
 *                out->capacity) bytes (256-byte aligned)
 *   copy_stream  stream of the host-to-device copies (NULL: `stream`); the
 *                first copies wait for the work already enqueued on `stream`,
 *                so calls sharing a workspace may be issued back to back; the
 *                host memory must stay valid until `stream` has completed
 * Not capturable into a graph (it orders two streams with events). */
int ns_stream_workspace_size(uint64_t batch, uint64_t capacity, uint64_t *bytes);
int ns_build_matrix_streamed(const uint32_t *src, const uint32_t *dst, uint64_t n, uint64_t batch,
                             ns_matrix_t *out, void *ws, uint64_t ws_bytes, void *stream,
                             void *copy_stream);

/* The eight quantities of a matrix (Table I with the row/column-sum maxima)
 * into *out (device). A matrix of 2^32 packets or more (such as the aggregate
 * of an out-of-core build) is reduced with 64-bit run sums; it must then hold
 * at most 2^32 entries (min(capacity, packets) <= 2^32), else
 * NS_ERR_UNSUPPORTED. */
int ns_stats(const ns_matrix_t *m, ns_stats_t *out, void *ws, uint64_t ws_bytes, void *stream);

/* The eight quantities of a matrix given in hypersparse CSR form, the form
 * of the challenge's matrices (Sec. IV "Data Representation": the CSR is
 * read as flat containers of its entries). All arrays are device memory:
 *   rows     [nrows] source address of each stored row
 *   row_ptr  [nrows+1] row r's entries are [row_ptr[r], row_ptr[r+1]);
 *            row_ptr[0] = 0, row_ptr[nrows] = nnz
 *   cols     [nnz] destination addresses, vals [nnz] A(i,j), 1 <= A(i,j) < 2^32
 *   nnz      entries (host); packets = sum of vals (host bound, < 2^32)
 * The keys rows[r]<<32 | cols[e] must increase strictly in entry order (rows
 * ascending, columns ascending within a row); stored rows may be empty. An
 * input that breaks this, holds a value outside [1, 2^32), whose values sum
 * to more than `packets`, or whose row_ptr does not run from 0 to nnz is
 * reported by ns_device_status (NS_ERR_INVALID_ARG) and gives undefined
 * quantities; every read stays inside the arrays. Workspace:
 * ns_stats_csr_workspace_size(nnz) bytes (it holds the flat entries). */
int ns_stats_csr_workspace_size(uint64_t nnz, uint64_t *bytes);
int ns_stats_csr(const uint32_t *rows, const uint64_t *row_ptr, uint64_t nrows,
                 const uint32_t *cols, const uint64_t *vals, uint64_t nnz, uint64_t packets,
                 ns_stats_t *out, void *ws, uint64_t ws_bytes, void *stream);

/* Batched path: the eight quantities of each of num_windows windows in one
 * submission (captured once as a HIP graph and replayed; sizes are read from
 * device memory, so the graph holds for any window sizes within the bounds).
 *   src, dst      concatenated packets of all windows (total_packets each)
 *   offsets       device [num_windows+1], offsets[0] = 0, non-decreasing,
 *                 offsets[num_windows] = total_packets; window w = [offsets[w], offsets[w+1])
 *   total_packets host bound, equal to offsets[num_windows]; below 2^32
 *                 (NS_ERR_UNSUPPORTED otherwise)
 *   out           device [num_windows] results; nullable when agg_out is given:
 *                 then only the aggregate (the union-add of all windows, Fig. 2
 *                 "load and aggregate") and its quantities are computed
 *   agg_out       nullable: union-add of all windows (capacity >= total_packets)
 *   agg_stats     nullable: device ns_stats_t of agg_out (requires agg_out)
 *   win_out       nullable: every window's own matrix (batched COO; requires out)
 *   tune          nullable: launch shape (NULL = defaults)
 * Windows may be empty. */
int ns_batch_stats(const uint32_t *src, const uint32_t *dst, const uint64_t *offsets,
                   uint32_t num_windows, uint64_t total_packets, ns_stats_t *out,
                   ns_matrix_t *agg_out, ns_stats_t *agg_stats, ns_batch_matrices_t *win_out,
                   const ns_tuning_t *tune, void *ws, uint64_t ws_bytes, void *stream);

/* Same computation as ns_batch_stats, enqueued kernel by kernel without a
 * graph (used to compare graph and eager submission). */
int ns_batch_stats_eager(const uint32_t *src, const uint32_t *dst, const uint64_t *offsets,
                         uint32_t num_windows, uint64_t total_packets, ns_stats_t *out,
                         ns_matrix_t *agg_out, ns_stats_t *agg_stats,
                         ns_batch_matrices_t *win_out, const ns_tuning_t *tune, void *ws,
                         uint64_t ws_bytes, void *stream);

/* Rolling aggregate for serving (the running union-add of the windows added
 * minus the windows removed), kept in device hash tables so that an update
 * costs time proportional to the entries of the windows involved plus one
 * scan of the source and destination tables (16 bytes per address slot, for
 * the four maxima), not to the links of the aggregate. Layout: one
 * caller-owned device buffer `mem` of `bytes` >= ns_rolling_size(...);
 * link_slots and address_slots are powers of two (hash slots for distinct
 * links and for distinct sources / destinations; keep live entries plus those
 * added since the last compaction below ~60% of them). The state holds fewer
 * than 2^32 packets: an add that would wrap a link's or an address's 32-bit
 * packet count is reported by ns_device_status (NS_ERR_CAPACITY). */
typedef struct {
  void *mem;
  uint64_t bytes;
  uint64_t link_slots;
  uint64_t address_slots;
} ns_rolling_t;

/* Bytes of state for the given slot counts (host only). */
int ns_rolling_size(uint64_t link_slots, uint64_t address_slots, uint64_t *bytes);
/* Clears the state to the empty aggregate. */
int ns_rolling_init(const ns_rolling_t *r, void *stream);
/* Applies A <- A + add - remove (either may be NULL; remove must be part of
 * A, as a window that entered earlier) and writes the eight quantities of the
 * new A to *out (device), all exactly as ns_stats would compute them on the
 * matrix A. A full table or a remove that is not part of A is reported by
 * ns_device_status (NS_ERR_CAPACITY / NS_ERR_UNDERFLOW). */
int ns_rolling_update(const ns_rolling_t *r, const ns_matrix_t *add, const ns_matrix_t *remove,
                      ns_stats_t *out, void *stream);
/* Copies the live entries of `from` into `to` (same slot counts), dropping the
 * tombstones of links, sources and destinations whose counts returned to 0. */
int ns_rolling_compact(const ns_rolling_t *from, const ns_rolling_t *to, void *stream);
/* Writes to slots_used[0..2] (device, 3 x uint64) the slots taken in the link,
 * source and destination tables since the last ns_rolling_init or since the
 * state was filled by ns_rolling_compact: live entries plus tombstones, the
 * occupancy that decides when to compact (the link key 0xFFFFFFFFFFFFFFFF is
 * kept outside the table and not counted). Enqueued on `stream` after the
 * state's earlier calls. */
int ns_rolling_occupancy(const ns_rolling_t *r, uint64_t *slots_used, void *stream);

/* Synchronises `stream`, then reads and clears the current device's error
 * word: *status (host) = NS_OK, NS_ERR_BOUNDS (an index outside its array; the
 * bounds-checked build libns_debug.so only), NS_ERR_UNDERFLOW,
 * NS_ERR_CAPACITY or NS_ERR_INVALID_ARG (a CSR input out of order), in that
 * priority. */
int ns_device_status(void *stream, int *status);

/* Largest link count max_ij A(i,j) of a matrix: the "maximum link counts"
 * among the analytics of Sec. IV ("Analytics and Operations"), the maximum
 * over the matrix's counts. out: device uint64, written with the maximum (0
 * for an empty matrix). Reads m->counts[0 .. *m->nnz), bounded by
 * min(m->capacity, m->packets). No workspace. */
int ns_max_link_packets(const ns_matrix_t *m, uint64_t *out, void *stream);

/* Per-window largest link count of the per-window matrices that
 * ns_batch_stats wrote into `win` (window w's entries start at offsets[w]).
 * offsets: device [num_windows+1], the same as given to ns_batch_stats;
 * total_packets: host bound >= offsets[num_windows] (positions scanned); out:
 * device [num_windows] uint64 (0 for an empty window). NS_ERR_CAPACITY if
 * win->capacity < total_packets. */
int ns_batch_max_link_packets(const ns_batch_matrices_t *win, const uint64_t *offsets,
                              uint32_t num_windows, uint64_t total_packets, uint64_t *out,
                              void *stream);

/* Destroys every cached HIP graph (call before freeing buffers a cached graph
 * refers to, or to bound memory). */
int ns_release_graphs(void);

/* Kernel timing for measurement (not on any hot path). While enabled, the
 * eager entry points (all but ns_batch_stats, whose graph is left untouched)
 * record a pair of HIP events on the launching stream around every kernel
 * launch. ns_timing_read synchronises those events and returns, for one
 * kernel kind, the summed duration (host *total_ms) and the number of
 * launches (host *launches). Kinds: 0 fill, 1 tile setup, 2 digit histogram,
 * 3 histogram scan, 4 first radix pass (packs keys), 5 other key radix passes,
 * 6 column radix passes, 7 run-length encoding, 8 run reduction,
 * 9 segment maxima, 10 finalize, 11 merge, 12 digit counts and scans of the
 * chunked passes, 13 first radix pass (chunked), 14 other key radix passes
 * (chunked), 15 column radix passes (chunked). ns_timing_reset destroys the
 * recorded events. */
int ns_timing_enable(int on);
int ns_timing_reset(void);
int ns_timing_read(uint32_t kind, double *total_ms, uint64_t *launches);

/* Static description of an error code. */
const char *ns_error_string(int code);

/* Library version string. */
const char *ns_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NS_H_ */
