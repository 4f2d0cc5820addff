// Sanitizer run of the CPU oracle (test infrastructure only).
//
// Built with g++ -fsanitize=address,undefined together with ns_oracle.cpp and
// run by tests/test_oracle_sanitized.py on the CPU: every oracle entry point is
// exercised on empty, tiny and colliding inputs, edge addresses (0 and
// 2^32-1), and the results are checked against each other and against closed
// forms, so that an out-of-bounds access, an overflow the sanitizers know or a
// disagreement ends the run with a non-zero status.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
void oracle_stats_map(const uint32_t *src, const uint32_t *dst, uint64_t n, uint64_t out[8]);
uint64_t oracle_build(const uint32_t *src, const uint32_t *dst, uint64_t n, uint64_t *keys,
                      uint64_t *counts);
void oracle_stats_matrix(const uint64_t *keys, const uint64_t *counts, uint64_t nnz,
                         uint64_t out[8]);
void oracle_stats_packets(const uint32_t *src, const uint32_t *dst, uint64_t n, uint64_t out[8]);
void oracle_stats_windows(const uint32_t *src, const uint32_t *dst, const uint64_t *offsets,
                          uint64_t num_windows, uint64_t *out);
int64_t oracle_accumulate(const uint64_t *keys_a, const uint64_t *counts_a, uint64_t nnz_a,
                          const uint64_t *keys_b, const uint64_t *counts_b, uint64_t nnz_b,
                          int sign, uint64_t *keys_c, uint64_t *counts_c);
}

namespace {

int failures = 0;

void expect(bool ok, const char *what, uint64_t a = 0, uint64_t b = 0) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s (%llu vs %llu)\n", what, (unsigned long long)a,
                 (unsigned long long)b);
    ++failures;
  }
}

// SplitMix64 (Steele, Lea, Flood): a seeded stream of test inputs
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

struct Matrix {
  std::vector<uint64_t> keys, counts;
};

Matrix build(const std::vector<uint32_t> &s, const std::vector<uint32_t> &d) {
  Matrix m;
  const size_t n = s.size();
  m.keys.resize(n ? n : 1);
  m.counts.resize(n ? n : 1);
  const uint64_t nnz = oracle_build(s.data(), d.data(), n, m.keys.data(), m.counts.data());
  m.keys.resize(nnz);
  m.counts.resize(nnz);
  return m;
}

void same8(const uint64_t *a, const uint64_t *b, const char *what) {
  for (int q = 0; q < 8; ++q) expect(a[q] == b[q], what, a[q], b[q]);
}

}  // namespace

int main() {
  Rng rng{20251014};
  // tiny windows: the map route and the sort route agree, per window and for
  // the stats of the built matrix; the per-window entry agrees with them
  for (int trial = 0; trial < 400; ++trial) {
    const uint64_t n = rng.next() % 257;
    const uint32_t pool = 1 + (uint32_t)(rng.next() % 8);
    std::vector<uint32_t> addr(pool);
    for (auto &a : addr) {
      const uint64_t r = rng.next() % 4;
      a = r == 0 ? 0u : r == 1 ? 0xFFFFFFFFu : (uint32_t)rng.next();
    }
    std::vector<uint32_t> s(n), d(n);
    for (uint64_t k = 0; k < n; ++k) {
      s[k] = addr[rng.next() % pool];
      d[k] = addr[rng.next() % pool];
    }
    uint64_t a[8], b[8], c[8];
    oracle_stats_map(s.data(), d.data(), n, a);
    oracle_stats_packets(s.data(), d.data(), n, b);
    same8(a, b, "map vs sort route");
    const Matrix m = build(s, d);
    oracle_stats_matrix(m.keys.data(), m.counts.data(), m.keys.size(), c);
    same8(a, c, "map route vs stats of the built matrix");
    expect(a[0] == n, "valid packets = n", a[0], n);
    // split into up to three windows
    const uint64_t cut1 = n ? rng.next() % (n + 1) : 0, cut2 = cut1 + (n - cut1) / 2;
    const uint64_t off[4] = {0, cut1, cut2, n};
    uint64_t per[24];
    oracle_stats_windows(s.data(), d.data(), off, 3, per);
    for (int w = 0; w < 3; ++w) {
      uint64_t x[8];
      oracle_stats_map(s.data() + off[w], d.data() + off[w], off[w + 1] - off[w], x);
      same8(per + 8 * w, x, "per-window entry vs map route");
    }
    // union-add of the first and second halves is the whole; subtracting the
    // second gives the first back
    const uint64_t h = n / 2;
    const Matrix A = build({s.begin(), s.begin() + h}, {d.begin(), d.begin() + h});
    const Matrix B = build({s.begin() + h, s.end()}, {d.begin() + h, d.end()});
    std::vector<uint64_t> kc(A.keys.size() + B.keys.size() + 1), cc(kc.size());
    const int64_t nc = oracle_accumulate(A.keys.data(), A.counts.data(), A.keys.size(),
                                         B.keys.data(), B.counts.data(), B.keys.size(), 1,
                                         kc.data(), cc.data());
    expect(nc == (int64_t)m.keys.size(), "union size", nc, m.keys.size());
    for (int64_t p = 0; p < nc && p < (int64_t)m.keys.size(); ++p) {
      expect(kc[p] == m.keys[p] && cc[p] == m.counts[p], "union entry", kc[p], m.keys[p]);
    }
    std::vector<uint64_t> kd(kc.size()), cd(kc.size());
    const int64_t nd = oracle_accumulate(kc.data(), cc.data(), nc, B.keys.data(),
                                         B.counts.data(), B.keys.size(), -1, kd.data(),
                                         cd.data());
    expect(nd == (int64_t)A.keys.size(), "difference size", nd, A.keys.size());
    for (int64_t p = 0; p < nd && p < (int64_t)A.keys.size(); ++p) {
      expect(kd[p] == A.keys[p] && cd[p] == A.counts[p], "difference entry", kd[p], A.keys[p]);
    }
    if (!B.keys.empty()) {  // B minus (A+B) goes below zero unless A is empty
      std::vector<uint64_t> ke(B.keys.size() + kc.size() + 1), ce(ke.size());
      const int64_t ne = oracle_accumulate(B.keys.data(), B.counts.data(), B.keys.size(),
                                           kc.data(), cc.data(), nc, -1, ke.data(), ce.data());
      expect((ne < 0) == !A.keys.empty(), "underflow detected", ne, A.keys.size());
    }
  }
  // closed forms: a sources x b destinations, each pair r times
  for (uint32_t a = 1; a <= 5; ++a)
    for (uint32_t b = 1; b <= 5; ++b)
      for (uint32_t r = 1; r <= 3; ++r) {
        std::vector<uint32_t> s, d;
        for (uint32_t i = 0; i < a; ++i)
          for (uint32_t j = 0; j < b; ++j)
            for (uint32_t k = 0; k < r; ++k) {
              s.push_back(0xFFFFFFFFu - i);
              d.push_back(j);
            }
        uint64_t x[8];
        oracle_stats_packets(s.data(), d.data(), s.size(), x);
        const uint64_t want[8] = {uint64_t(a) * b * r, uint64_t(a) * b, a, b, uint64_t(b) * r, b,
                                  uint64_t(a) * r, a};
        same8(x, want, "a x b grid repeated r times");
      }
  // empty input: all zeros, nothing read
  uint64_t z[8];
  oracle_stats_packets(nullptr, nullptr, 0, z);
  const uint64_t zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  same8(z, zero, "empty window");
  oracle_stats_matrix(nullptr, nullptr, 0, z);
  same8(z, zero, "empty matrix");
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("oracle sanitizer run: OK\n");
  return 0;
}
