// Seeded synthetic directed graphs standing in for the paper's power-law
// datasets (Section 4, Table 2): R-MAT and Chung-Lu generators.
//
// This module produces inputs only.  It holds none of ExactSim's arithmetic;
// both the CPU oracle and the HIP library consume the edge lists it writes.
//
// Every edge list it returns is a set: exactly m distinct (src, dst) pairs,
// no self-loops, sorted by (src, dst).  The graph is a pure function of its
// parameters and seed, independent of the number of threads.
//
// Candidate edges are drawn from a counter-based hash (splitmix64 finaliser
// over (seed, candidate index, draw index)), so candidate i is the same no
// matter which thread makes it.  Distinct edges are kept in order of first
// appearance in the candidate sequence until m of them exist.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <parallel/algorithm>
#include <vector>

#include <omp.h>

namespace {

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Draw number `draw` of candidate `i` under `seed`.
inline uint64_t hash3(uint64_t seed, uint64_t i, uint64_t draw) {
  return mix64(mix64(seed ^ 0x6A09E667F3BCC909ull) + i * 0x9E3779B97F4A7C15ull +
               (draw + 1) * 0xD1B54A32D192ED03ull);
}

constexpr uint64_t kInvalid = ~0ull;

struct KeyIdx {
  uint64_t key;
  uint64_t idx;
};

// Shared driver: `cand(i)` returns the packed key (src << 32 | dst) of
// candidate i, or kInvalid when the candidate is rejected (self-loop, id
// out of range).  Fills keys_out (sorted, unique) with exactly m keys.
template <class Cand>
int collect_unique(int64_t m, Cand cand, std::vector<uint64_t>& keys_out) {
  keys_out.clear();
  uint64_t next = 0;
  int stalls = 0;
  const uint64_t kMaxBatch = 1ull << 27;
  while ((int64_t)keys_out.size() < m) {
    uint64_t need = (uint64_t)(m - (int64_t)keys_out.size());
    uint64_t batch = std::min<uint64_t>(kMaxBatch, std::max<uint64_t>(need + need / 4, 1u << 16));
    std::vector<KeyIdx> c(batch);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)batch; ++t) {
      uint64_t i = next + (uint64_t)t;
      c[t] = KeyIdx{cand(i), i};
    }
    next += batch;
    // drop rejected candidates
    c.erase(std::remove_if(c.begin(), c.end(), [](const KeyIdx& a) { return a.key == kInvalid; }),
            c.end());
    // unique by key, keeping the first appearance
    __gnu_parallel::sort(c.begin(), c.end(), [](const KeyIdx& a, const KeyIdx& b) {
      return a.key < b.key || (a.key == b.key && a.idx < b.idx);
    });
    c.erase(std::unique(c.begin(), c.end(), [](const KeyIdx& a, const KeyIdx& b) { return a.key == b.key; }),
            c.end());
    // drop keys already kept
    std::vector<char> fresh(c.size());
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)c.size(); ++t)
      fresh[t] = !std::binary_search(keys_out.begin(), keys_out.end(), c[t].key);
    size_t w = 0;
    for (size_t t = 0; t < c.size(); ++t)
      if (fresh[t]) c[w++] = c[t];
    c.resize(w);
    if (c.empty()) {
      if (++stalls > 64) return -1;
      continue;
    }
    stalls = 0;
    // take new keys in candidate order
    __gnu_parallel::sort(c.begin(), c.end(), [](const KeyIdx& a, const KeyIdx& b) { return a.idx < b.idx; });
    if (c.size() > need) c.resize(need);
    std::vector<uint64_t> add(c.size());
    for (size_t t = 0; t < c.size(); ++t) add[t] = c[t].key;
    std::vector<KeyIdx>().swap(c);
    __gnu_parallel::sort(add.begin(), add.end());
    std::vector<uint64_t> merged(keys_out.size() + add.size());
    std::merge(keys_out.begin(), keys_out.end(), add.begin(), add.end(), merged.begin());
    keys_out.swap(merged);
  }
  return 0;
}

void unpack(const std::vector<uint64_t>& keys, int32_t* src, int32_t* dst) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)keys.size(); ++e) {
    src[e] = (int32_t)(keys[e] >> 32);
    dst[e] = (int32_t)(keys[e] & 0xffffffffu);
  }
}

}  // namespace

extern "C" {

// Random permutation of [0, n) by Fisher-Yates over a seeded splitmix stream.
int gg_permutation(int32_t n, uint64_t seed, int32_t* perm) {
  if (n < 0 || !perm) return -1;
  for (int32_t i = 0; i < n; ++i) perm[i] = i;
  for (int64_t i = (int64_t)n - 1; i > 0; --i) {
    uint64_t h = hash3(seed, (uint64_t)i, 77);
    uint64_t j = (uint64_t)(((unsigned __int128)h * (uint64_t)(i + 1)) >> 64);
    std::swap(perm[i], perm[j]);
  }
  return 0;
}

// R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each candidate picks one of the
// four quadrants per level with probabilities (a, b, c, d) over
// scale = ceil(log2 n) levels.  Ids >= n and self-loops are rejected; the
// surviving ids are relabelled by a seeded random permutation so that id
// order carries no locality.  Returns 0, or -1 on bad arguments / stall.
int gg_rmat(int32_t n, int64_t m, double a, double b, double c, double d, uint64_t seed,
            int32_t* src, int32_t* dst) {
  if (n < 2 || m < 0 || !src || !dst) return -1;
  if ((double)m > (double)n * (double)(n - 1)) return -1;
  if (a < 0 || b < 0 || c < 0 || d < 0 || std::fabs(a + b + c + d - 1.0) > 1e-9) return -1;
  int scale = 0;
  while ((1ll << scale) < (int64_t)n) ++scale;
  const double two32 = 4294967296.0;
  const uint64_t ta = (uint64_t)(a * two32);
  const uint64_t tab = (uint64_t)((a + b) * two32);
  const uint64_t tabc = (uint64_t)((a + b + c) * two32);
  std::vector<int32_t> perm(n);
  gg_permutation(n, seed ^ 0x5bd1e995ull, perm.data());
  auto cand = [&](uint64_t i) -> uint64_t {
    uint64_t s = 0, t = 0;
    uint64_t h = 0;
    for (int lvl = 0; lvl < scale; ++lvl) {
      uint64_t u;
      if ((lvl & 1) == 0) {
        h = hash3(seed, i, (uint64_t)(lvl >> 1));
        u = h & 0xffffffffu;
      } else {
        u = h >> 32;
      }
      uint64_t sb, tb;
      if (u < ta) { sb = 0; tb = 0; }
      else if (u < tab) { sb = 0; tb = 1; }
      else if (u < tabc) { sb = 1; tb = 0; }
      else { sb = 1; tb = 1; }
      s = (s << 1) | sb;
      t = (t << 1) | tb;
    }
    if (s >= (uint64_t)n || t >= (uint64_t)n || s == t) return kInvalid;
    return ((uint64_t)(uint32_t)perm[s] << 32) | (uint64_t)(uint32_t)perm[t];
  };
  std::vector<uint64_t> keys;
  if (collect_unique(m, cand, keys) != 0) return -1;
  unpack(keys, src, dst);
  return 0;
}

// Chung-Lu: node i has weight w_i = (i+1)^(-1/(gamma-1)) for both its
// in- and out-side, so node 0 is the largest hub; each candidate draws its
// source and its target independently with probability proportional to w.
// Self-loops and duplicates are rejected.  Returns 0 or -1.
int gg_chung_lu(int32_t n, int64_t m, double gamma, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 2 || m < 0 || !src || !dst || !(gamma > 1.0)) return -1;
  if ((double)m > (double)n * (double)(n - 1)) return -1;
  std::vector<double> cum(n);
  double acc = 0.0;
  const double ex = -1.0 / (gamma - 1.0);
  for (int32_t i = 0; i < n; ++i) {
    acc += std::pow((double)(i + 1), ex);
    cum[i] = acc;
  }
  const double total = acc;
  auto pick = [&](uint64_t h) -> uint64_t {
    double u = (double)(h >> 11) * 0x1.0p-53 * total;
    uint64_t k = (uint64_t)(std::upper_bound(cum.begin(), cum.end(), u) - cum.begin());
    return k < (uint64_t)n ? k : (uint64_t)n - 1;
  };
  auto cand = [&](uint64_t i) -> uint64_t {
    uint64_t s = pick(hash3(seed, i, 0));
    uint64_t t = pick(hash3(seed, i, 1));
    if (s == t) return kInvalid;
    return (s << 32) | t;
  };
  std::vector<uint64_t> keys;
  if (collect_unique(m, cand, keys) != 0) return -1;
  unpack(keys, src, dst);
  return 0;
}

int gg_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
