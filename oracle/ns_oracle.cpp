// CPU oracle for the anonymized network sensing statistics.
//
// TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or call
// this file: only the tests, the smoke check and the benchmark's CPU-baseline
// leg use it. It shares no code, header, table or helper with the HIP library.
//
// What it computes (all integer, uint64, exact):
//   Traffic matrix A(i,j) = number of packets from source i to destination j
//   in a window (Table I caption). Each input pair is one packet.
//   The eight quantities, in this fixed order:
//     0 valid packets        N_V = sum_i sum_j A(i,j)                (Table I)
//     1 unique links         sum_i sum_j |A(i,j)|_0                  (Table I)
//     2 unique sources       sum_i |sum_j A(i,j)|_0                  (Table I)
//     3 unique destinations  sum_j |sum_i A(i,j)|_0                  (Table I)
//     4 max source packets   max_i sum_j A(i,j)     (row sums, Sec. IV "Data
//                                                    Representation"; source
//                                                    packet counts, "Analytics")
//     5 max source fan-out   max_i sum_j |A(i,j)|_0 (Table I; the printed
//                                                    |sum_j A|_0 is read as the
//                                                    row's nonzero count, i.e.
//                                                    the "degrees" it names)
//     6 max destination packets  max_j sum_i A(i,j) (column sums, same passages)
//     7 max destination fan-in   max_j sum_i |A(i,j)|_0  (Table I, same reading)
//   Empty input: all eight are 0.
//   Aggregation ("load and aggregate", Fig. 2 caption): A = A_1 + A_2 elementwise,
//   structure = union; subtraction is its inverse and drops entries that reach 0.
//
// Two independent routes:
//   * map route (oracle_stats_map): std::map from (i,j) to A(i,j), then per-row
//     and per-column maps, straight from the definitions above.
//   * sort route (oracle_build / oracle_stats_matrix): keys (i<<32|j) sorted with
//     std::sort, equal keys counted, rows scanned in key order, columns scanned
//     after a std::sort of (j, A(i,j)) pairs. This is the timed CPU baseline.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

namespace {

struct Tally {            // per-row or per-column state: packets and nonzeros
  uint64_t packets = 0;
  uint64_t nonzeros = 0;
};

void clear8(uint64_t out[8]) { std::memset(out, 0, 8 * sizeof(uint64_t)); }

}  // namespace

extern "C" {

// Map route, straight from the definitions. Suitable up to ~2^20 packets.
void oracle_stats_map(const uint32_t *src, const uint32_t *dst, uint64_t n, uint64_t out[8]) {
  clear8(out);
  std::map<std::pair<uint32_t, uint32_t>, uint64_t> A;
  for (uint64_t k = 0; k < n; ++k) A[{src[k], dst[k]}] += 1;
  std::map<uint32_t, Tally> rows, cols;
  uint64_t valid = 0;
  for (const auto &e : A) {
    const uint32_t i = e.first.first, j = e.first.second;
    const uint64_t a = e.second;
    valid += a;
    rows[i].packets += a;
    rows[i].nonzeros += 1;
    cols[j].packets += a;
    cols[j].nonzeros += 1;
  }
  out[0] = valid;
  out[1] = A.size();
  out[2] = rows.size();
  out[3] = cols.size();
  for (const auto &r : rows) {
    out[4] = std::max(out[4], r.second.packets);
    out[5] = std::max(out[5], r.second.nonzeros);
  }
  for (const auto &c : cols) {
    out[6] = std::max(out[6], c.second.packets);
    out[7] = std::max(out[7], c.second.nonzeros);
  }
}

// Sort route: the sorted COO of A. keys[k] = i<<32|j strictly increasing,
// counts[k] = A(i,j) >= 1. Returns nnz. keys/counts must hold n entries.
uint64_t oracle_build(const uint32_t *src, const uint32_t *dst, uint64_t n,
                      uint64_t *keys, uint64_t *counts) {
  std::vector<uint64_t> k(n);
  for (uint64_t p = 0; p < n; ++p) k[p] = (uint64_t(src[p]) << 32) | uint64_t(dst[p]);
  std::sort(k.begin(), k.end());
  uint64_t nnz = 0;
  for (uint64_t p = 0; p < n;) {
    uint64_t q = p + 1;
    while (q < n && k[q] == k[p]) ++q;
    keys[nnz] = k[p];
    counts[nnz] = q - p;
    ++nnz;
    p = q;
  }
  return nnz;
}

// The eight quantities of a sorted COO matrix (keys strictly increasing).
void oracle_stats_matrix(const uint64_t *keys, const uint64_t *counts, uint64_t nnz,
                         uint64_t out[8]) {
  clear8(out);
  out[1] = nnz;
  // rows: runs of equal source (high half) in key order
  for (uint64_t p = 0; p < nnz;) {
    const uint64_t i = keys[p] >> 32;
    uint64_t packets = 0, q = p;
    while (q < nnz && (keys[q] >> 32) == i) packets += counts[q++];
    out[0] += packets;
    out[2] += 1;
    out[4] = std::max(out[4], packets);
    out[5] = std::max(out[5], q - p);
    p = q;
  }
  // columns: group (j, A(i,j)) by destination j
  std::vector<std::pair<uint32_t, uint64_t>> col(nnz);
  for (uint64_t p = 0; p < nnz; ++p) col[p] = {uint32_t(keys[p] & 0xFFFFFFFFu), counts[p]};
  std::sort(col.begin(), col.end(),
            [](const std::pair<uint32_t, uint64_t> &a, const std::pair<uint32_t, uint64_t> &b) {
              return a.first < b.first;
            });
  for (uint64_t p = 0; p < nnz;) {
    const uint32_t j = col[p].first;
    uint64_t packets = 0, q = p;
    while (q < nnz && col[q].first == j) packets += col[q++].second;
    out[3] += 1;
    out[6] = std::max(out[6], packets);
    out[7] = std::max(out[7], q - p);
    p = q;
  }
}

// Sort route from packets: build, then the quantities of the built matrix.
void oracle_stats_packets(const uint32_t *src, const uint32_t *dst, uint64_t n, uint64_t out[8]) {
  std::vector<uint64_t> keys(n), counts(n);
  const uint64_t nnz = oracle_build(src, dst, n, keys.data(), counts.data());
  oracle_stats_matrix(keys.data(), counts.data(), nnz, out);
}

// Per-window quantities of W windows stored back to back; window w holds
// packets [offsets[w], offsets[w+1]). out holds 8*W values.
void oracle_stats_windows(const uint32_t *src, const uint32_t *dst, const uint64_t *offsets,
                          uint64_t num_windows, uint64_t *out) {
  for (uint64_t w = 0; w < num_windows; ++w) {
    const uint64_t a = offsets[w], b = offsets[w + 1];
    oracle_stats_packets(src + a, dst + a, b - a, out + 8 * w);
  }
}

// Union-add (sign=+1) or subtract (sign=-1) of two sorted COO matrices:
// C(i,j) = A(i,j) + sign*B(i,j), structure = union, zero entries dropped.
// Returns nnz of C, or -1 when subtraction would go below zero (C undefined).
// keys_c/counts_c must hold nnz_a + nnz_b entries.
int64_t oracle_accumulate(const uint64_t *keys_a, const uint64_t *counts_a, uint64_t nnz_a,
                          const uint64_t *keys_b, const uint64_t *counts_b, uint64_t nnz_b,
                          int sign, uint64_t *keys_c, uint64_t *counts_c) {
  std::map<uint64_t, uint64_t> C;
  for (uint64_t p = 0; p < nnz_a; ++p) C[keys_a[p]] += counts_a[p];
  for (uint64_t p = 0; p < nnz_b; ++p) {
    if (sign > 0) {
      C[keys_b[p]] += counts_b[p];
    } else {
      auto it = C.find(keys_b[p]);
      if (it == C.end() || it->second < counts_b[p]) return -1;
      it->second -= counts_b[p];
      if (it->second == 0) C.erase(it);
    }
  }
  int64_t nnz = 0;
  for (const auto &e : C) {
    keys_c[nnz] = e.first;
    counts_c[nnz] = e.second;
    ++nnz;
  }
  return nnz;
}

}  // extern "C"
