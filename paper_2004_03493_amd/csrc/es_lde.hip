// Local deterministic exploitation for D(k,k) (Section 3.2, Algorithm 3,
// Lemma 4).
//
// Z_l(k) is the probability that two sqrt(c)-walks from v_k first meet at
// their l-th step; D(k,k) = 1 - sum_l Z_l(k).  Algorithm 3 computes the first
// l(k) terms exactly and estimates the rest with pairs that do not stop
// during their first l(k) steps:
//   D^(k,k) = (1 - sum_{l <= l(k)} Z_l(k)) - c^l(k) M(k) / R'(k).
//
// Level rule.  Algorithm 3 runs rounds l = 0, 1, ...: round l evaluates
// Z_l(k, .) and extends, for l' = 0..l and every node q' reached from v_k in
// exactly l - l' steps, the transition table of q' from step l' to l' + 1,
// counting one edge per in-neighbour of every node in the table's support.
// It stops in the round where the count E_k reaches 2 R(k) / sqrt(c).  With
// S_j(v) the nodes reachable from v in exactly j in-steps (each once) and
// N_j(v) = sum of d_in over S_j(v), round l counts
//   sum_{l'=0..l} sum_{q' in S_{l-l'}(k)} N_{l'}(q'),
// that is d_in(k), 2 N_1(k), 2 N_2(k) + sum_{a in I(k)} N_1(a) and
// 2 N_3(k) + sum_{a in I(k)} N_2(a) + sum_{q in S_2(k)} N_1(q) for rounds
// 0..3.  A round that counts nothing ends the exploitation (no walk survives
// another step, the exact part is all of 1 - D).  The caller's cap bounds
// the level: l(k) = min(l_printed(k), cap); this library evaluates Lemma 4
// up to level 3, so an uncapped query whose rule asks for more is refused.
//
// Lemma 4 summed over the meeting node gives Z_l in terms of collision
// numbers C_m(x) = sum_q (P^T)^m(x, q)^2 (C_1(x) = 1/d_in(x)):
//   Z_1(k) = c C_1(k),
//   Z_2(k) = c^2 (C_2(k) - d_in(k)^-2 sum_{a in I(k)} C_1(a)),
//   Z_3(k) = c^3 (C_3(k) - sum_q (P^T)^2(k, q)^2 C_1(q)
//                 + d_in(k)^-2 sum_{a in I(k)} d_in(a)^-2 sum_{q in I(a)} C_1(q)
//                 - d_in(k)^-2 sum_{a in I(k)} C_2(a)).
//
// GPU design.  A per-graph cache holds N_1(x) and G(x) = sum_{a in I(x)}
// C_1(a).  One kernel settles rounds 0 and 1 of every sampled node (most
// nodes stop there) and lists the rest.  For those, the transition tables
// (P^T)^j(x, .) of every needed origin x are built level by level in one
// hash table whose regions belong to the origins (a region that would need
// n slots or more is a dense array indexed by node): a load-balanced launch
// inserts every (origin, in-neighbour) term, values in 2^-62 fixed point
// (each term rounded once, exact integer sums), keys inserted even for zero
// terms so the supports are exact; a second launch reads each region back
// and adds N_j, sum N_1, C_j and sum_q (P^T)^j(x, q)^2 C_1(q) per origin in
// exact integer arithmetic (128-bit for the squares).  Every result is
// therefore independent of launch shapes and atomics order, and the host
// finishes the rounds and the Z_l in float64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "es_internal.h"

namespace es {
namespace {

constexpr int kMaxLevel = 3;          // Lemma 4 is evaluated up to Z_3
constexpr int kStatWords = 6;         // N, sum N_1, C (lo, hi), Cw (lo, hi) per (origin, level)
constexpr uint64_t kOne = 1ull << 62; // probability 1 in fixed point
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;
constexpr int64_t kSlotBudget = 1ll << 27;  // hash slots per pass (12 bytes each)
constexpr int kInsertThreads = 256;
constexpr int kInsertPer = 16;              // inserts per thread

using u128 = unsigned __int128;

struct Ent {
  int32_t o;   // origin index
  int32_t x;   // node (internal id)
  uint64_t V;  // (P^T)^j(origin, x) in 2^-62 fixed point
};

// ---- per-graph sums --------------------------------------------------------

// One wave per node: N_1(x) = sum_{a in I(x)} d_in(a), G(x) = sum_{a in I(x)} 1/d_in(a).
__global__ void graph_sums_kernel(int32_t n, const int32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx,
                                  const int32_t* __restrict__ din, const double* __restrict__ inv_din,
                                  long long* __restrict__ N1, double* __restrict__ G) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t x = w0; x < n; x += nw) {
    long long s = 0;
    double g = 0.0;
    for (int32_t e = in_off[x] + lane; e < in_off[x + 1]; e += 64) {
      const int32_t a = in_idx[e];
      s += din[a];
      g += inv_din[a];
    }
    for (int m = 32; m > 0; m >>= 1) {
      s += __shfl_xor(s, m, 64);
      g += __shfl_xor(g, m, 64);
    }
    if (lane == 0) {
      N1[x] = s;
      G[x] = g;
    }
  }
}

// ---- rounds 0 and 1 ---------------------------------------------------------

__device__ __forceinline__ uint64_t reduced_count(uint64_t r, int32_t l, int32_t mode, double cl1, double cl2,
                                                  double cl3) {
  if (mode != 2 || r == 0 || l == 0) return r;
  const double cl = l == 1 ? cl1 : (l == 2 ? cl2 : cl3);
  return (uint64_t)ceil((double)r * cl);
}

// l(k) for the nodes whose count reaches the budget in round 0 or 1 (or
// whose rounds run dry, or at cap 1); the others are listed with their
// count after round 1.
__global__ void plan01_kernel(int32_t n, const uint64_t* __restrict__ Rk, const int32_t* __restrict__ din,
                              const long long* __restrict__ N1, double c, double sc, int32_t cap, int32_t mode,
                              double cl1, double cl2, double cl3, int32_t* __restrict__ ell,
                              double* __restrict__ zsum, uint64_t* __restrict__ Rk2, int32_t* __restrict__ ncand,
                              int32_t* __restrict__ cand, long long* __restrict__ candE) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint64_t r = Rk[k];
  int32_t l = 0;
  if (mode != 0 && r > 0) {
    const double T = (2.0 * (double)r) / sc;
    const int32_t d = din[k];
    long long E = d;
    if ((double)E >= T || d == 0) {
      l = 0;
    } else {
      const long long c1 = 2 * N1[k];
      E += c1;
      if ((double)E >= T || c1 == 0 || cap == 1) {
        l = 1;
      } else {
        l = -1;
        const int32_t i = atomicAdd(ncand, 1);
        cand[i] = (int32_t)k;
        candE[i] = E;
      }
    }
  }
  if (l >= 0) {
    ell[k] = l;
    zsum[k] = l == 1 ? c / (double)din[k] : 0.0;
    Rk2[k] = reduced_count(r, l, mode, cl1, cl2, cl3);
  }
}

// One wave per listed node: sum_{a in I(k)} N_1(a) and
// sum_{a in I(k)} d_in(a)^-2 G(a).
__global__ void cand_sums_kernel(int32_t ncand, const int32_t* __restrict__ cand, const int32_t* __restrict__ in_off,
                                 const int32_t* __restrict__ in_idx, const double* __restrict__ inv_din,
                                 const long long* __restrict__ N1, const double* __restrict__ G,
                                 const uint64_t* __restrict__ Rk, long long* __restrict__ sN1,
                                 double* __restrict__ A2, uint64_t* __restrict__ Rc, double* __restrict__ Gc) {
  const int lane = threadIdx.x & 63;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= ncand) return;
  const int32_t k = cand[w];
  long long s = 0;
  double a2 = 0.0;
  for (int32_t e = in_off[k] + lane; e < in_off[k + 1]; e += 64) {
    const int32_t a = in_idx[e];
    const double ia = inv_din[a];
    s += N1[a];
    a2 += (ia * ia) * G[a];
  }
  for (int m = 32; m > 0; m >>= 1) {
    s += __shfl_xor(s, m, 64);
    a2 += __shfl_xor(a2, m, 64);
  }
  if (lane == 0) {
    sN1[w] = s;
    A2[w] = a2;
    Rc[w] = Rk[k];
    Gc[w] = G[k];
  }
}

// rows I(k) of the listed nodes, packed (dst offsets from the host)
__global__ void gather_rows_kernel(int32_t nrows, const int32_t* __restrict__ rows, const long long* __restrict__ dst,
                                   const int32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx,
                                   int32_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= nrows) return;
  const int32_t k = rows[w];
  const int32_t b = in_off[k], len = in_off[k + 1] - b;
  for (int32_t i = lane; i < len; i += 64) out[dst[w] + i] = in_idx[b + i];
}

// ---- exclusive scan of int64 counts ------------------------------------------

__device__ long long block_exclusive(long long v, long long* sh, long long* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long inc = v;
  for (int m = 1; m < 64; m <<= 1) {
    const long long t = __shfl_up(inc, m, 64);
    if (lane >= m) inc += t;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
      const long long t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[kScanThreads / 64] = run;
  }
  __syncthreads();
  const long long out = inc - v + sh[wv];
  *total = sh[kScanThreads / 64];
  __syncthreads();
  return out;
}

// pass 1: tile sums
__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(int64_t ne, const long long* __restrict__ in,
                                                                  long long* __restrict__ tsum) {
  __shared__ long long sh[kScanThreads / 64 + 1];
  const int64_t b = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  long long s = 0;
  for (int i = 0; i < kScanPer; ++i)
    if (b + i < ne) s += in[b + i];
  long long tot;
  (void)block_exclusive(s, sh, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// pass 2 (one workgroup): exclusive scan of the tile sums in place; grand total in tsum[nt]
__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(int32_t nt, long long* __restrict__ tsum) {
  __shared__ long long sh[kScanThreads / 64 + 1];
  long long base = 0;
  for (int32_t t0 = 0; t0 < nt; t0 += kScanThreads) {
    const int32_t t = t0 + threadIdx.x;
    const long long v = t < nt ? tsum[t] : 0;
    long long tot;
    const long long ex = block_exclusive(v, sh, &tot);
    if (t < nt) tsum[t] = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) tsum[nt] = base;
}

// pass 3: out[i] = exclusive prefix, out[ne] = total
__global__ __launch_bounds__(kScanThreads) void scan_write_kernel(int64_t ne, int32_t nt,
                                                                  const long long* __restrict__ in,
                                                                  const long long* __restrict__ tsum,
                                                                  long long* __restrict__ out) {
  __shared__ long long sh[kScanThreads / 64 + 1];
  const int64_t b = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  long long v[kScanPer];
  long long s = 0;
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = b + i < ne ? in[b + i] : 0;
    s += v[i];
  }
  long long tot;
  long long run = block_exclusive(s, sh, &tot) + tsum[blockIdx.x];
  for (int i = 0; i < kScanPer; ++i) {
    if (b + i < ne) out[b + i] = run;
    run += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[ne] = tsum[nt];
}

// ---- transition tables in a hash table --------------------------------------

__device__ __forceinline__ uint32_t slot_hash(uint32_t q) {
  q ^= q >> 16;
  q *= 0x7feb352dU;
  q ^= q >> 15;
  q *= 0x846ca68bU;
  q ^= q >> 16;
  return q;
}

__global__ void fill_slots_kernel(int64_t S, int32_t* __restrict__ keys, unsigned long long* __restrict__ vals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    keys[i] = -1;
    vals[i] = 0ull;
  }
}

// inserts of entry e: d_in(x) if its origin is in [o0, o1), else 0
__global__ void insert_counts_kernel(int64_t ne, const Ent* __restrict__ ents, const int32_t* __restrict__ din,
                                     int32_t o0, int32_t o1, long long* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const Ent t = ents[e];
  cnt[e] = (t.o >= o0 && t.o < o1) ? din[t.x] : 0;
}

// largest e in [lo, hi] with pre[e] <= t (pre ascending, pre[lo] <= t)
__device__ __forceinline__ int64_t find_entry(const long long* __restrict__ pre, int64_t lo, int64_t hi, long long t) {
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Every (entry, in-neighbour) term once: the entry's value divided by d_in(x)
// (rounded to nearest, ties up) added at key q of the origin's region.  A
// block takes kInsertThreads * kInsertPer consecutive terms and each wave a
// contiguous quarter of them, interleaved over its lanes so that neighbouring
// lanes read neighbouring in_idx entries.  A lane's entry index only grows,
// so the next one is found by galloping forward from the current one.  A
// region of at least n slots is dense: key q sits in slot q (no probing, the
// key written by plain stores of the same value).
__global__ __launch_bounds__(kInsertThreads) void insert_kernel(
    long long total, int64_t ne, const Ent* __restrict__ ents, const long long* __restrict__ pre,
    const int32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx, const int32_t* __restrict__ din,
    const long long* __restrict__ reg_off, int32_t o0, int32_t n, int32_t* __restrict__ keys,
    unsigned long long* __restrict__ vals) {
  const long long b0 = (long long)blockIdx.x * kInsertThreads * kInsertPer;
  if (b0 >= total) return;
  const long long b1 = min(total, b0 + (long long)kInsertThreads * kInsertPer);
  __shared__ int64_t range[2];
  if (threadIdx.x == 0) {
    range[0] = find_entry(pre, 0, ne - 1, b0);
    range[1] = find_entry(pre, range[0], ne - 1, b1 - 1);
  }
  __syncthreads();
  const int64_t r0 = range[0], r1 = range[1];
  const long long w0 = b0 + (long long)(threadIdx.x >> 6) * 64 * kInsertPer;
  const long long w1 = min(b1, w0 + 64ll * kInsertPer);
  int64_t last = -1;
  Ent en{};
  unsigned long long term = 0;
  long long base = 0, row = 0, first = 0;
  uint32_t mask = 0;
  bool dense = false;
  for (long long t = w0 + (threadIdx.x & 63); t < w1; t += 64) {
    int64_t e = last;
    if (last < 0) {
      e = find_entry(pre, r0, r1, t);
    } else if (t >= pre[last + 1]) {
      // gallop: pre[lo] <= t throughout, the answer lies in [lo, hi]
      int64_t lo = last + 1, hi = r1, step = 1;
      while (lo + step <= r1) {
        if (pre[lo + step] > t) {
          hi = lo + step - 1;
          break;
        }
        lo += step;
        step <<= 1;
      }
      e = find_entry(pre, lo, hi, t);
    }
    if (e != last) {
      // the entry's term is shared by all its in-neighbours
      last = e;
      en = ents[e];
      const int32_t d = din[en.x];
      term = (en.V + (uint64_t)(d >> 1)) / (uint64_t)d;
      base = reg_off[en.o - o0];
      const long long size = reg_off[en.o - o0 + 1] - base;
      mask = (uint32_t)(size - 1);
      dense = size >= (long long)n;
      row = in_off[en.x];
      first = pre[e];
    }
    const int32_t q = in_idx[row + (t - first)];
    uint32_t h;
    if (dense) {
      h = (uint32_t)q;
      if (keys[base + h] != q) keys[base + h] = q;
    } else {
      h = slot_hash((uint32_t)q) & mask;
      while (true) {
        const int32_t k = keys[base + h];
        if (k == q) break;
        if (k == -1) {
          const int32_t old = atomicCAS(&keys[base + h], -1, q);
          if (old == -1 || old == q) break;
        }
        h = (h + 1) & mask;
      }
    }
    if (term) atomicAdd(&vals[base + h], term);
  }
}

__device__ __forceinline__ void atomic_add_u128(unsigned long long* p, u128 v) {
  const unsigned long long lo = (unsigned long long)v;
  unsigned long long hi = (unsigned long long)(v >> 64);
  const unsigned long long old = atomicAdd(&p[0], lo);
  if (old + lo < old) hi += 1ull;
  if (hi) atomicAdd(&p[1], hi);
}

__device__ __forceinline__ u128 shfl_xor_u128(u128 v, int m) {
  const unsigned long long lo = __shfl_xor((unsigned long long)v, m, 64);
  const unsigned long long hi = __shfl_xor((unsigned long long)(v >> 64), m, 64);
  return ((u128)hi << 64) | lo;
}

// C_1(q) (P^T)^j(x, q)^2 in 2^-120 fixed point, from float64 (per entry, so
// the exact integer sum does not depend on the order).
__device__ __forceinline__ u128 weighted_square(uint64_t V, double inv_d) {
  const double p = (double)V * 0x1p-62;
  const double w = (p * p) * inv_d;                    // < 1
  const double hi_d = floor(w * 0x1p56);
  const unsigned long long hi = (unsigned long long)hi_d;
  const unsigned long long lo = (unsigned long long)((w * 0x1p56 - hi_d) * 0x1p64);
  return ((u128)hi << 64) | lo;
}

// Read back the regions of origins [o0, o1): per origin at level `lev`
//   N = sum d_in(q), SN = sum N_1(q), C = sum V^2 (2^-124), Cw = sum V^2/d_in(q) (2^-120)
// over the distinct keys q, and the entries of origins that go deeper.
// Regions are whole 64-slot pages (at least 64 slots, sizes powers of two),
// so a wave's 64 lanes always share one region; each wave walks a contiguous
// run of pages, keeps its sums in registers while the region stays the same
// and adds them to the region's statistics when it leaves it, and appends
// the entries that go deeper with one counter update per wave.
__global__ void compact_kernel(int64_t S, const long long* __restrict__ reg_off, int32_t nreg, int32_t o0,
                               const int32_t* __restrict__ keys, const unsigned long long* __restrict__ vals,
                               const int32_t* __restrict__ din, const double* __restrict__ inv_din,
                               const long long* __restrict__ N1, const int32_t* __restrict__ depth, int32_t lev,
                               unsigned long long* __restrict__ stats, Ent* __restrict__ out,
                               unsigned long long* __restrict__ nout) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t pages = S >> 6;
  const int64_t per = (pages + nwaves - 1) / nwaves;
  const int64_t p0 = wave * per;
  const int64_t p1 = min(pages, p0 + per);
  if (p0 >= p1) return;  // whole wave
  // region of the first page: the last r with reg_off[r] <= slot
  int32_t r = 0;
  {
    int32_t lo = 0, hi = nreg - 1;
    const long long s0 = p0 << 6;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (reg_off[mid] <= s0) lo = mid;
      else hi = mid - 1;
    }
    r = lo;
  }
  long long rend = reg_off[r + 1];
  bool deeper = depth[o0 + r] > lev;
  unsigned long long nsum = 0, snsum = 0;
  u128 csum = 0, wsum = 0;
  auto flush = [&]() {
    for (int m = 32; m > 0; m >>= 1) {
      nsum += __shfl_xor(nsum, m, 64);
      snsum += __shfl_xor(snsum, m, 64);
      csum += shfl_xor_u128(csum, m);
      wsum += shfl_xor_u128(wsum, m);
    }
    if (lane == 0) {
      unsigned long long* st = stats + ((int64_t)(o0 + r) * (kMaxLevel + 1) + lev) * kStatWords;
      if (nsum) atomicAdd(&st[0], nsum);
      if (snsum) atomicAdd(&st[1], snsum);
      if (csum) atomic_add_u128(&st[2], csum);
      if (wsum) atomic_add_u128(&st[4], wsum);
    }
    nsum = snsum = 0;
    csum = wsum = 0;
  };
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int64_t p = p0; p < p1; ++p) {
    const long long s = (p << 6) + lane;
    if ((p << 6) >= rend) {
      flush();
      do {
        ++r;
        rend = reg_off[r + 1];
      } while ((p << 6) >= rend);
      deeper = depth[o0 + r] > lev;
    }
    const int32_t q = keys[s];
    uint64_t V = 0;
    if (q >= 0) {
      V = vals[s];
      const int32_t d = din[q];
      nsum += (unsigned long long)d;
      snsum += (unsigned long long)N1[q];
      csum += (u128)V * (u128)V;
      if (d > 0) wsum += weighted_square(V, inv_din[q]);
    }
    const unsigned long long go = __ballot(deeper && q >= 0);
    if (go) {
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(nout, (unsigned long long)__popcll(go));
      base = __shfl(base, 0, 64);
      if ((go >> lane) & 1ull) out[base + __popcll(go & below)] = Ent{o0 + r, q, V};
    }
  }
  flush();
}

__global__ void zero_u64_kernel(int64_t n, unsigned long long* __restrict__ p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Final values of the listed nodes.
__global__ void plan_scatter_kernel(int32_t cnt, const int32_t* __restrict__ ids, const int32_t* __restrict__ lv,
                                    const double* __restrict__ zs, const uint64_t* __restrict__ Rk, int32_t mode,
                                    double cl1, double cl2, double cl3, int32_t* __restrict__ ell,
                                    double* __restrict__ zsum, uint64_t* __restrict__ Rk2) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int32_t k = ids[i];
  ell[k] = lv[i];
  zsum[k] = zs[i];
  Rk2[k] = reduced_count(Rk[k], lv[i], mode, cl1, cl2, cl3);
}

__global__ void diag_lde_kernel(int32_t n, const uint64_t* __restrict__ Rk, const uint64_t* __restrict__ M,
                                const int32_t* __restrict__ ell, const double* __restrict__ zsum,
                                const int32_t* __restrict__ din, double one_minus_c, double cl1, double cl2,
                                double cl3, int32_t exact_small_din, double* __restrict__ D) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint64_t r = Rk[k];
  double d = 1.0;
  if (r > 0) {
    const int32_t l = ell[k];
    if (l == 0) {
      d = (double)(r - M[k]) / (double)r;
    } else {
      const double cl = l == 1 ? cl1 : (l == 2 ? cl2 : cl3);
      d = (1.0 - zsum[k]) - cl * ((double)M[k] / (double)r);
    }
  }
  if (exact_small_din) {
    const int32_t dd = din[k];
    if (dd == 0) d = 1.0;
    else if (dd == 1) d = one_minus_c;
  }
  D[k] = d;
}

__global__ void permute_i32_kernel(int32_t n, const int32_t* __restrict__ src, const int32_t* __restrict__ map,
                                   int32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[map[i]];
}

bool valid_c(double c) { return c > 0.0 && c <= 0.99; }

// c^l by repeated multiplication
double c_power(double c, int l) {
  double p = 1.0;
  for (int i = 0; i < l; ++i) p = p * c;
  return p;
}

int64_t pow2_at_least(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

double u128_to_double(uint64_t lo, uint64_t hi, double scale) {
  return ((double)hi * 0x1p64 + (double)lo) * scale;
}

// Per-origin results of a propagation, level j = 1..depth.
struct OriginLevel {
  uint64_t N = 0;    // sum of d_in over the support S_j(x)
  uint64_t SN1 = 0;  // sum of N_1 over S_j(x)
  double C = 0;      // sum_q (P^T)^j(x, q)^2
  double Cw = 0;     // sum_q (P^T)^j(x, q)^2 / d_in(q)
};

es_status ensure_graph_sums(es_ctx* ctx, const es_graph* g) {
  if (g->lde_n1) return ES_OK;
  const int32_t n = g->n;
  ES_CHECK_HIP(ctx, hipMalloc((void**)&g->lde_n1, sizeof(long long) * (size_t)n));
  ES_CHECK_HIP(ctx, hipMalloc((void**)&g->lde_g, sizeof(double) * (size_t)n));
  const int grid = (int)std::min<int64_t>(ceil_div((int64_t)n * 64, 256), (int64_t)ctx->num_cus * 16);
  graph_sums_kernel<<<std::max(grid, 1), 256, 0, ctx->stream>>>(n, g->in_off, g->in_idx, g->din_int, g->inv_din,
                                                                 g->lde_n1, g->lde_g);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

// Build (P^T)^j(x, .) for every origin x = origins[i] up to depth[i] steps and
// return each level's sums.  Origins are independent; they are processed in
// passes of at most kSlotBudget hash slots (a single origin's region never
// exceeds max(64, 2n) slots).
es_status propagate(es_ctx* ctx, const es_graph* g, const std::vector<int32_t>& origins,
                    const std::vector<int32_t>& depth, std::vector<OriginLevel>& res) {
  const int32_t no = (int32_t)origins.size();
  const int32_t n = g->n;
  res.assign((size_t)no * (kMaxLevel + 1), OriginLevel{});
  if (no == 0) return ES_OK;
  es_status st;
  int32_t maxd = 0;
  for (int32_t d : depth) maxd = std::max(maxd, d);
  const int64_t dense_cap = pow2_at_least(std::max<int64_t>(n, 64));
  const size_t nstat = (size_t)no * (kMaxLevel + 1) * kStatWords;
  auto* misc = (unsigned long long*)workspace(ctx, kWsLdeStats, 8 * nstat + 8 * (size_t)no + 64, &st);
  if (!misc) return st;
  unsigned long long* stats = misc;
  auto* dep_d = (int32_t*)(misc + nstat);
  unsigned long long* nout = misc + nstat + (no + 1) / 2 + 1;
  const int tb = 256;
  zero_u64_kernel<<<std::max(1, std::min(ceil_div((int64_t)nstat, tb), 1024)), tb, 0, ctx->stream>>>(
      (int64_t)nstat, stats);
  ES_CHECK_HIP(ctx, hipMemcpyAsync(dep_d, depth.data(), sizeof(int32_t) * no, hipMemcpyHostToDevice, ctx->stream));
  // level 0: one entry per origin
  std::vector<Ent> e0;
  for (int32_t i = 0; i < no; ++i)
    if (depth[i] >= 1) e0.push_back(Ent{i, origins[i], kOne});
  int64_t ne = (int64_t)e0.size();
  std::vector<uint64_t> ins(no, 0);  // inserts of each origin at the current level
  for (int32_t i = 0; i < no; ++i)
    ins[i] = depth[i] >= 1 ? (uint64_t)(g->h_in_off[origins[i] + 1] - g->h_in_off[origins[i]]) : 0;
  auto* ent_cur = (Ent*)workspace(ctx, kWsLdeEnt0, sizeof(Ent) * (size_t)std::max<int64_t>(ne, 1), &st);
  if (!ent_cur) return st;
  ES_CHECK_HIP(ctx, hipMemcpyAsync(ent_cur, e0.data(), sizeof(Ent) * ne, hipMemcpyHostToDevice, ctx->stream));
  int cur_slot = kWsLdeEnt0;
  std::vector<unsigned long long> hstat(nstat);
  for (int32_t j = 0; j < maxd && ne > 0; ++j) {
    // regions and next-level entry capacity
    std::vector<int64_t> cap(no, 0);
    int64_t next_cap = 0;
    for (int32_t i = 0; i < no; ++i) {
      if (depth[i] <= j || ins[i] == 0) continue;
      const int64_t distinct = (int64_t)std::min<uint64_t>(ins[i], (uint64_t)n);
      cap[i] = std::max<int64_t>(64, pow2_at_least(2 * distinct));  // whole 64-slot pages
      // a hash region no smaller than the dense one is replaced by it
      // (regions below n slots are hashed, those of n or more dense)
      cap[i] = std::min(cap[i], dense_cap);
      if (depth[i] > j + 1) next_cap += distinct;
    }
    const int nxt_slot = cur_slot == kWsLdeEnt0 ? kWsLdeEnt1 : kWsLdeEnt0;
    auto* ent_nxt = (Ent*)workspace(ctx, nxt_slot, sizeof(Ent) * (size_t)std::max<int64_t>(next_cap, 1), &st);
    if (!ent_nxt) return st;
    ent_cur = (Ent*)ctx->ws[cur_slot];
    zero_u64_kernel<<<1, 64, 0, ctx->stream>>>(1, nout);
    auto* cnt = (long long*)workspace(ctx, kWsLdeCnt, 8 * ((size_t)ne + 1), &st);
    if (!cnt) return st;
    auto* pre = (long long*)workspace(ctx, kWsLdePre, 8 * ((size_t)ne + 1), &st);
    if (!pre) return st;
    const int32_t nt = ceil_div(ne, kScanTile);
    auto* tsum = (long long*)workspace(ctx, kWsLdeTsum, 8 * ((size_t)nt + 1), &st);
    if (!tsum) return st;
    int32_t o0 = 0;
    while (o0 < no) {
      // a pass: consecutive origins within the slot budget (at least one)
      int64_t S = 0;
      int32_t o1 = o0;
      std::vector<long long> roff(1, 0);
      while (o1 < no && (o1 == o0 || S + cap[o1] <= kSlotBudget)) {
        S += cap[o1];
        roff.push_back(S);
        ++o1;
      }
      if (S > 0) {
        auto* keys = (int32_t*)workspace(ctx, kWsLdeKeys, sizeof(int32_t) * (size_t)S, &st);
        if (!keys) return st;
        auto* vals = (unsigned long long*)workspace(ctx, kWsLdeVals, sizeof(uint64_t) * (size_t)S, &st);
        if (!vals) return st;
        auto* reg = (long long*)workspace(ctx, kWsLdeReg, sizeof(long long) * roff.size(), &st);
        if (!reg) return st;
        ES_CHECK_HIP(ctx, hipMemcpyAsync(reg, roff.data(), sizeof(long long) * roff.size(), hipMemcpyHostToDevice,
                                         ctx->stream));
        const int fgrid = (int)std::min<int64_t>(ceil_div(S, tb), (int64_t)ctx->num_cus * 32);
        fill_slots_kernel<<<fgrid, tb, 0, ctx->stream>>>(S, keys, vals);
        insert_counts_kernel<<<ceil_div(ne, tb), tb, 0, ctx->stream>>>(ne, ent_cur, g->din_int, o0, o1, cnt);
        scan_tiles_kernel<<<nt, kScanThreads, 0, ctx->stream>>>(ne, cnt, tsum);
        scan_sums_kernel<<<1, kScanThreads, 0, ctx->stream>>>(nt, tsum);
        scan_write_kernel<<<nt, kScanThreads, 0, ctx->stream>>>(ne, nt, cnt, tsum, pre);
        ES_CHECK_HIP(ctx, hipGetLastError());
        long long total = 0;
        ES_CHECK_HIP(ctx, hipMemcpyAsync(&total, pre + ne, 8, hipMemcpyDeviceToHost, ctx->stream));
        ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (total > 0) {
          const int64_t ib = (total + (int64_t)kInsertThreads * kInsertPer - 1) / ((int64_t)kInsertThreads * kInsertPer);
          insert_kernel<<<(unsigned)ib, kInsertThreads, 0, ctx->stream>>>(total, ne, ent_cur, pre, g->in_off,
                                                                          g->in_idx, g->din_int, reg, o0, n, keys,
                                                                          vals);
        }
        const int cgrid = (int)std::min<int64_t>(ceil_div(S, tb), (int64_t)ctx->num_cus * 32);
        compact_kernel<<<cgrid, tb, 0, ctx->stream>>>(S, reg, o1 - o0, o0, keys, vals, g->din_int, g->inv_din,
                                                      g->lde_n1, dep_d, j + 1, stats, ent_nxt, nout);
        ES_CHECK_HIP(ctx, hipGetLastError());
      }
      o0 = o1;
    }
    // next level: inserts per origin = N_{j+1}
    unsigned long long cnt_next = 0;
    ES_CHECK_HIP(ctx, hipMemcpyAsync(&cnt_next, nout, 8, hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipMemcpyAsync(hstat.data(), stats, 8 * nstat, hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int32_t i = 0; i < no; ++i)
      ins[i] = depth[i] > j + 1 ? hstat[((size_t)i * (kMaxLevel + 1) + j + 1) * kStatWords] : 0;
    ne = (int64_t)cnt_next;
    cur_slot = nxt_slot;
  }
  for (int32_t i = 0; i < no; ++i)
    for (int32_t j = 1; j <= std::min(depth[i], kMaxLevel); ++j) {
      const unsigned long long* s = &hstat[((size_t)i * (kMaxLevel + 1) + j) * kStatWords];
      OriginLevel& r = res[(size_t)i * (kMaxLevel + 1) + j];
      r.N = s[0];
      r.SN1 = s[1];
      r.C = u128_to_double(s[2], s[3], 0x1p-124);
      r.Cw = u128_to_double(s[4], s[5], 0x1p-120);
    }
  return ES_OK;
}

}  // namespace

es_status launch_lde(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, double c, int32_t mode, int32_t max_level,
                     LdeOut out) {
  const int32_t n = g->n;
  const double sc = std::sqrt(c);
  const bool capped = max_level >= 1 && max_level <= kMaxLevel;
  const int32_t cap = capped ? max_level : kMaxLevel;
  const double cl1 = c_power(c, 1), cl2 = c_power(c, 2), cl3 = c_power(c, 3);
  const int tb = 256;
  es_status st;
  if (mode != 0) ES_TRY(ensure_graph_sums(ctx, g));
  auto* misc = (int32_t*)workspace(ctx, kWsLdeMisc, 64, &st);
  if (!misc) return st;
  auto* cand = (int32_t*)workspace(ctx, kWsLdeCand, sizeof(int32_t) * (size_t)n, &st);
  if (!cand) return st;
  auto* candE = (long long*)workspace(ctx, kWsLdeW, sizeof(long long) * (size_t)n, &st);
  if (!candE) return st;
  zero_u64_kernel<<<1, 64, 0, ctx->stream>>>(1, (unsigned long long*)misc);
  plan01_kernel<<<ceil_div(n, tb), tb, 0, ctx->stream>>>(n, Rk, g->din_int, mode ? g->lde_n1 : nullptr, c, sc, cap,
                                                         mode, cl1, cl2, cl3, out.ell, out.zsum, out.Rk2, misc, cand,
                                                         candE);
  ES_CHECK_HIP(ctx, hipGetLastError());
  if (mode == 0) return ES_OK;
  int32_t ncand = 0;
  ES_CHECK_HIP(ctx, hipMemcpyAsync(&ncand, misc, 4, hipMemcpyDeviceToHost, ctx->stream));
  ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ncand == 0) return ES_OK;
  // the listed nodes (rounds 2, 3), in id order
  std::vector<int32_t> ids(ncand);
  std::vector<long long> E1(ncand);
  ES_CHECK_HIP(ctx, hipMemcpy(ids.data(), cand, 4 * (size_t)ncand, hipMemcpyDeviceToHost));
  ES_CHECK_HIP(ctx, hipMemcpy(E1.data(), candE, 8 * (size_t)ncand, hipMemcpyDeviceToHost));
  {
    std::vector<int32_t> ord(ncand);
    for (int32_t i = 0; i < ncand; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return ids[a] < ids[b]; });
    std::vector<int32_t> i2(ncand);
    std::vector<long long> e2(ncand);
    for (int32_t i = 0; i < ncand; ++i) {
      i2[i] = ids[ord[i]];
      e2[i] = E1[ord[i]];
    }
    ids.swap(i2);
    E1.swap(e2);
  }
  std::vector<uint64_t> R(ncand);
  std::vector<double> Gk(ncand);
  std::vector<long long> sN1(ncand);
  std::vector<double> A2(ncand);
  {
    ES_CHECK_HIP(ctx, hipMemcpy(cand, ids.data(), 4 * (size_t)ncand, hipMemcpyHostToDevice));
    auto* sn = (long long*)workspace(ctx, kWsLdeSums, 32 * (size_t)ncand, &st);
    if (!sn) return st;
    auto* a2 = (double*)(sn + ncand);
    auto* rc = (uint64_t*)(sn + 2 * (size_t)ncand);
    auto* gc = (double*)(sn + 3 * (size_t)ncand);
    cand_sums_kernel<<<ceil_div((int64_t)ncand * 64, tb), tb, 0, ctx->stream>>>(
        ncand, cand, g->in_off, g->in_idx, g->inv_din, g->lde_n1, g->lde_g, Rk, sn, a2, rc, gc);
    ES_CHECK_HIP(ctx, hipGetLastError());
    ES_CHECK_HIP(ctx, hipMemcpyAsync(sN1.data(), sn, 8 * (size_t)ncand, hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipMemcpyAsync(A2.data(), a2, 8 * (size_t)ncand, hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipMemcpyAsync(R.data(), rc, 8 * (size_t)ncand, hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipMemcpyAsync(Gk.data(), gc, 8 * (size_t)ncand, hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  auto din_of = [&](int32_t k) { return g->h_in_off[k + 1] - g->h_in_off[k]; };
  // table sums of the listed nodes: from the graph's cache, else built now
  // (depth 2) and cached
  std::unique_lock<std::mutex> lock(g->lde_mu);
  auto& cache = g->lde_cache;
  auto fill = [&](const std::vector<int32_t>& nodes, const std::vector<int32_t>& dep) -> es_status {
    if (nodes.empty()) return ES_OK;
    std::vector<OriginLevel> r;
    ES_TRY(propagate(ctx, g, nodes, dep, r));
    for (size_t t = 0; t < nodes.size(); ++t) {
      LdeNodeStats& e = cache[nodes[t]];
      const OriginLevel& s2 = r[t * (kMaxLevel + 1) + 2];
      e.has2 = true;
      e.N2 = s2.N;
      e.SN1_2 = s2.SN1;
      e.C2 = s2.C;
      e.Cw2 = s2.Cw;
      if (dep[t] >= 3) {
        const OriginLevel& s3 = r[t * (kMaxLevel + 1) + 3];
        e.has3 = true;
        e.N3 = s3.N;
        e.C3 = s3.C;
      }
    }
    return ES_OK;
  };
  {
    std::vector<int32_t> need;
    for (int32_t k : ids)
      if (!cache[k].has2) need.push_back(k);
    ES_TRY(fill(need, std::vector<int32_t>(need.size(), 2)));
  }
  // round 2
  std::vector<int32_t> lv(ncand, 2);
  std::vector<double> z(ncand, 0.0);
  std::vector<long long> E2(ncand);
  std::vector<int32_t> deep;  // indices of nodes that take (at least) round 3
  for (int32_t i = 0; i < ncand; ++i) {
    const LdeNodeStats& e = cache[ids[i]];
    const double T = (2.0 * (double)R[i]) / sc;
    const long long cost2 = 2 * (long long)e.N2 + sN1[i];
    E2[i] = E1[i] + cost2;
    if ((double)E2[i] >= T || cost2 == 0 || cap == 2) lv[i] = 2;
    else deep.push_back(i);
  }
  // round 3: three-step tables of the deep nodes, two-step tables of their in-neighbours
  if (!deep.empty()) {
    // in-neighbour rows of the deep nodes, packed on the device
    const int32_t nd = (int32_t)deep.size();
    std::vector<int32_t> rows(nd);
    std::vector<long long> dst(nd + 1, 0);
    for (int32_t t = 0; t < nd; ++t) {
      rows[t] = ids[deep[t]];
      dst[t + 1] = dst[t] + din_of(rows[t]);
    }
    auto* rbuf = (int32_t*)workspace(ctx, kWsLdeRows, 4 * (size_t)nd + 8 * (size_t)(nd + 1) + 4 * (size_t)dst[nd] + 16,
                                     &st);
    if (!rbuf) return st;
    auto* dst_d = (long long*)(rbuf + ((nd + 1) & ~1));
    auto* packed = (int32_t*)(dst_d + nd + 1);
    ES_CHECK_HIP(ctx, hipMemcpyAsync(rbuf, rows.data(), 4 * (size_t)nd, hipMemcpyHostToDevice, ctx->stream));
    ES_CHECK_HIP(ctx, hipMemcpyAsync(dst_d, dst.data(), 8 * (size_t)(nd + 1), hipMemcpyHostToDevice, ctx->stream));
    gather_rows_kernel<<<ceil_div((int64_t)nd * 64, tb), tb, 0, ctx->stream>>>(nd, rbuf, dst_d, g->in_off, g->in_idx,
                                                                              packed);
    ES_CHECK_HIP(ctx, hipGetLastError());
    std::vector<int32_t> flat((size_t)dst[nd]);
    ES_CHECK_HIP(ctx, hipMemcpyAsync(flat.data(), packed, 4 * flat.size(), hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<int32_t> need, dep;
    for (int32_t t = 0; t < nd; ++t)
      if (!cache[rows[t]].has3) {
        need.push_back(rows[t]);
        dep.push_back(3);
      }
    std::vector<int32_t> nb(flat);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    for (int32_t a : nb) {
      const LdeNodeStats& e = cache[a];
      if (!e.has2 && std::find(need.begin(), need.end(), a) == need.end()) {
        need.push_back(a);
        dep.push_back(2);
      }
    }
    ES_TRY(fill(need, dep));
    for (int32_t t = 0; t < nd; ++t) {
      const int32_t i = deep[t];
      const LdeNodeStats& e = cache[rows[t]];
      double sc2 = 0.0;
      long long sN2 = 0;
      for (long long p = dst[t]; p < dst[t + 1]; ++p) {
        const LdeNodeStats& a = cache[flat[p]];
        sc2 += a.C2;
        sN2 += (long long)a.N2;
      }
      lv[i] = 3;
      if (!capped) {
        // the printed rule asks for Z_4 unless round 3 reaches the budget or runs dry
        const long long cost3 = 2 * (long long)e.N3 + sN2 + (long long)e.SN1_2;
        const double T = (2.0 * (double)R[i]) / sc;
        if (!((double)(E2[i] + cost3) >= T || cost3 == 0))
          return fail(ctx, ES_EUNSUPPORTED,
                      "Algorithm 3 asks for more than %d exact levels at a node with R(k)=%llu (E_k=%lld after "
                      "round 3, budget %.6g); cap the level with lde_max_level",
                      kMaxLevel, (unsigned long long)R[i], E2[i] + cost3, T);
      }
      const double iu = 1.0 / (double)din_of(rows[t]);
      const double iu2 = iu * iu;
      z[i] = cl3 * (((e.C3 - e.Cw2) + iu2 * A2[i]) - iu2 * sc2);
    }
  }
  // Z_1 + Z_2 (+ Z_3) of every listed node
  for (int32_t i = 0; i < ncand; ++i) {
    const LdeNodeStats& e = cache[ids[i]];
    const double d = (double)din_of(ids[i]);
    const double iu = 1.0 / d;
    const double z1 = c / d;
    const double z2 = cl2 * (e.C2 - (iu * iu) * Gk[i]);
    z[i] = (z1 + z2) + z[i];
  }
  lock.unlock();
  auto* up = (int32_t*)workspace(ctx, kWsLdeSums, 16 * (size_t)ncand, &st);
  if (!up) return st;
  auto* zs = (double*)((char*)up + 8 * (size_t)ncand);
  ES_CHECK_HIP(ctx, hipMemcpyAsync(up, lv.data(), 4 * (size_t)ncand, hipMemcpyHostToDevice, ctx->stream));
  ES_CHECK_HIP(ctx, hipMemcpyAsync(zs, z.data(), 8 * (size_t)ncand, hipMemcpyHostToDevice, ctx->stream));
  plan_scatter_kernel<<<ceil_div(ncand, tb), tb, 0, ctx->stream>>>(ncand, cand, up, zs, Rk, mode, cl1, cl2, cl3,
                                                                   out.ell, out.zsum, out.Rk2);
  ES_CHECK_HIP(ctx, hipGetLastError());
  ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return ES_OK;
}

es_status launch_diag_lde(es_ctx* ctx, int32_t n, const uint64_t* Rk, const uint64_t* M, const int32_t* ell,
                          const double* zsum, const int32_t* din, double c, int32_t exact_small_din, double* D) {
  const int tb = 256;
  diag_lde_kernel<<<ceil_div(n, tb), tb, 0, ctx->stream>>>(n, Rk, M, ell, zsum, din, 1.0 - c, c_power(c, 1),
                                                           c_power(c, 2), c_power(c, 3), exact_small_din, D);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

}  // namespace es

using namespace es;

extern "C" {

es_status es_lde_plan(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, double c, int32_t mode, int32_t max_level,
                      int32_t* ell, double* zsum, uint64_t* Rk_out) {
  if (!ctx || !g || !Rk || !ell || !zsum || !Rk_out) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  if (mode < 0 || mode > 2) return fail(ctx, ES_EINVAL, "exploitation mode %d outside 0..2", mode);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  const int32_t n = g->n;
  es_status st;
  auto* rin = (uint64_t*)workspace(ctx, kWsLdeRin, sizeof(uint64_t) * (size_t)n, &st);
  if (!rin) return st;
  auto* e_int = (int32_t*)workspace(ctx, kWsLdeEll, sizeof(int32_t) * (size_t)n, &st);
  if (!e_int) return st;
  auto* z_int = (double*)workspace(ctx, kWsLdeZ, sizeof(double) * (size_t)n, &st);
  if (!z_int) return st;
  auto* r_int = (uint64_t*)workspace(ctx, kWsLdeR, sizeof(uint64_t) * (size_t)n, &st);
  if (!r_int) return st;
  // caller order -> internal order (sample counts bit for bit)
  ES_TRY(launch_permute_f64(ctx, n, 1, (const double*)Rk, g->ext_of, (double*)rin));
  ES_TRY(launch_lde(ctx, g, rin, c, mode, max_level, LdeOut{e_int, z_int, r_int}));
  const int tb = 256;
  permute_i32_kernel<<<ceil_div(n, tb), tb, 0, ctx->stream>>>(n, e_int, g->int_of, ell);
  ES_CHECK_HIP(ctx, hipGetLastError());
  ES_TRY(launch_permute_f64(ctx, n, 1, z_int, g->int_of, zsum));
  return launch_permute_f64(ctx, n, 1, (const double*)r_int, g->int_of, (double*)Rk_out);
}

es_status es_diag_lde(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, const uint64_t* M, const int32_t* ell,
                      const double* zsum, double c, int32_t exact_small_din, double* D) {
  if (!ctx || !g || !Rk || !M || !ell || !zsum || !D) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  return launch_diag_lde(ctx, g->n, Rk, M, ell, zsum, g->din_ext, c, exact_small_din, D);
}

}  // extern "C"
