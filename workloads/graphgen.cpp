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
// matter which thread makes it.  The edge set is the first m distinct edges
// in order of first appearance in the candidate sequence.

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

// Shared driver.  `cand(i)` returns the packed key (src << 32 | dst) of
// candidate i before relabelling, or kInvalid when the candidate is rejected
// (self-loop, id out of range); `relabel(key)` maps a key to its final ids
// by a bijection.  Fills keys_out with the relabelled first m distinct keys
// in order of first appearance among candidates 0, 1, 2, ..., sorted.
//
// The raw keys of candidates 0..N-1 are generated once into one array.
// Distinctness is decided before relabelling (a bijection keeps it): valid
// candidates are spread over buckets by a hash of the key (equal keys share
// a bucket), each bucket sorted and reduced to its distinct keys with their
// first candidate index, and the m distinct keys of smallest first index are
// kept.  The result does not depend on N once N holds m distinct keys, so
// when it does not, the array is extended and the dedup redone.
template <class Cand, class Relabel>
int collect_unique(int64_t m, Cand cand, Relabel relabel, std::vector<uint64_t>& keys_out) {
  keys_out.clear();
  if (m == 0) return 0;
  const int nthreads = omp_get_max_threads();
  const int kBucketBits = 14;
  const uint64_t nbuckets = 1ull << kBucketBits;
  auto bucket_of = [](uint64_t key) -> uint64_t { return mix64(key) >> (64 - kBucketBits); };
  std::vector<uint64_t> raw;
  uint64_t N = (uint64_t)m + (uint64_t)m / 4 + 1024;
  for (int attempt = 0; attempt < 40; ++attempt) {
    // raw keys of candidates [raw.size(), N)
    const uint64_t N0 = raw.size();
    raw.resize(N);
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = (int64_t)N0; i < (int64_t)N; ++i) raw[i] = cand((uint64_t)i);
    // counts per (thread, bucket) over contiguous ranges of candidates
    std::vector<uint64_t> counts((size_t)nthreads * nbuckets, 0);
#pragma omp parallel num_threads(nthreads)
    {
      const int t = omp_get_thread_num();
      const uint64_t lo = N * t / nthreads, hi = N * (t + 1) / nthreads;
      uint64_t* c = counts.data() + (size_t)t * nbuckets;
      for (uint64_t i = lo; i < hi; ++i)
        if (raw[i] != kInvalid) c[bucket_of(raw[i])]++;
    }
    std::vector<uint64_t> off((size_t)nthreads * nbuckets, 0), bstart(nbuckets + 1, 0);
    uint64_t acc = 0;
    for (uint64_t b = 0; b < nbuckets; ++b) {
      bstart[b] = acc;
      for (int t = 0; t < nthreads; ++t) {
        off[(size_t)t * nbuckets + b] = acc;
        acc += counts[(size_t)t * nbuckets + b];
      }
    }
    bstart[nbuckets] = acc;
    std::vector<uint64_t>().swap(counts);
    std::vector<KeyIdx> cands(acc);
#pragma omp parallel num_threads(nthreads)
    {
      const int t = omp_get_thread_num();
      const uint64_t lo = N * t / nthreads, hi = N * (t + 1) / nthreads;
      uint64_t* o = off.data() + (size_t)t * nbuckets;
      for (uint64_t i = lo; i < hi; ++i)
        if (raw[i] != kInvalid) cands[o[bucket_of(raw[i])]++] = KeyIdx{raw[i], i};
    }
    // per bucket: sort by (key, index), keep each key's first appearance
    std::vector<uint64_t> ucount(nbuckets, 0);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t b = 0; b < (int64_t)nbuckets; ++b) {
      KeyIdx* first = cands.data() + bstart[b];
      KeyIdx* last = cands.data() + bstart[b + 1];
      std::sort(first, last, [](const KeyIdx& x, const KeyIdx& y) {
        return x.key < y.key || (x.key == y.key && x.idx < y.idx);
      });
      KeyIdx* e = std::unique(first, last, [](const KeyIdx& x, const KeyIdx& y) { return x.key == y.key; });
      ucount[b] = (uint64_t)(e - first);
    }
    uint64_t U = 0;
    for (uint64_t c : ucount) U += c;
    if (U < (uint64_t)m) {
      // not enough distinct keys yet: more candidates, sized from this yield
      const double grow = 1.15 * (double)m / (double)std::max<uint64_t>(U, 1);
      N = std::max(N + N / 8, (uint64_t)((double)N * std::min(grow, 8.0)));
      continue;
    }
    std::vector<uint64_t>().swap(raw);
    // theta = the m-th smallest first-appearance index: histogram of the
    // indices in 2^20 bins, then an exact selection inside the bin holding it
    const int kBinBits = 20;
    const uint64_t nbins = 1ull << kBinBits;
    const uint64_t binw = (N + nbins - 1) / nbins;
    std::vector<uint64_t> hist(nbins, 0);
#pragma omp parallel num_threads(nthreads)
    {
      std::vector<uint64_t> h(nbins, 0);
#pragma omp for schedule(dynamic, 64)
      for (int64_t b = 0; b < (int64_t)nbuckets; ++b)
        for (uint64_t j = 0; j < ucount[b]; ++j) h[cands[bstart[b] + j].idx / binw]++;
#pragma omp critical
      for (uint64_t k = 0; k < nbins; ++k) hist[k] += h[k];
    }
    uint64_t below = 0, bin = 0;
    while (below + hist[bin] < (uint64_t)m) below += hist[bin++];
    std::vector<uint64_t> inbin;
    inbin.reserve(hist[bin]);
    for (uint64_t b = 0; b < nbuckets; ++b)
      for (uint64_t j = 0; j < ucount[b]; ++j) {
        const uint64_t idx = cands[bstart[b] + j].idx;
        if (idx / binw == bin) inbin.push_back(idx);
      }
    const uint64_t rank = (uint64_t)m - below - 1;
    std::nth_element(inbin.begin(), inbin.begin() + rank, inbin.end());
    const uint64_t theta = inbin[rank];
    // relabelled keys of every distinct key first seen at index <= theta
    std::vector<uint64_t> keep(nbuckets + 1, 0);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
    for (int64_t b = 0; b < (int64_t)nbuckets; ++b) {
      uint64_t k = 0;
      for (uint64_t j = 0; j < ucount[b]; ++j) k += cands[bstart[b] + j].idx <= theta;
      keep[b + 1] = k;
    }
    for (uint64_t b = 0; b < nbuckets; ++b) keep[b + 1] += keep[b];
    if (keep[nbuckets] != (uint64_t)m) return -1;
    keys_out.resize((size_t)m);
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
    for (int64_t b = 0; b < (int64_t)nbuckets; ++b) {
      uint64_t w = keep[b];
      for (uint64_t j = 0; j < ucount[b]; ++j) {
        const KeyIdx& ki = cands[bstart[b] + j];
        if (ki.idx <= theta) keys_out[w++] = relabel(ki.key);
      }
    }
    std::vector<KeyIdx>().swap(cands);
    __gnu_parallel::sort(keys_out.begin(), keys_out.end());
    return 0;
  }
  return -1;
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
      // quadrant: [0, ta) -> (0,0), [ta, tab) -> (0,1), [tab, tabc) -> (1,0),
      // [tabc, 2^32) -> (1,1); branch-free, the draws are unpredictable
      const uint64_t sb = (uint64_t)(u >= tab);
      const uint64_t tb = (uint64_t)(u >= ta) ^ (uint64_t)(u >= tab) ^ (uint64_t)(u >= tabc);
      s = (s << 1) | sb;
      t = (t << 1) | tb;
    }
    if (s >= (uint64_t)n || t >= (uint64_t)n || s == t) return kInvalid;
    return (s << 32) | t;
  };
  auto relabel = [&](uint64_t key) -> uint64_t {
    return ((uint64_t)(uint32_t)perm[key >> 32] << 32) | (uint64_t)(uint32_t)perm[key & 0xffffffffu];
  };
  std::vector<uint64_t> keys;
  if (collect_unique(m, cand, relabel, keys) != 0) return -1;
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
  if (collect_unique(m, cand, [](uint64_t key) { return key; }, keys) != 0) return -1;
  unpack(keys, src, dst);
  return 0;
}

int gg_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
