// Sample budget, sample-space scan, walk pairs and the diagonal estimate.
//
// Budget (Algorithm 1; Section 3.2): R(k) = ceil(R * pi(k)^2).
// Walk pairs (Algorithm 2): every node's pairs are laid end to end in one
// 64-bit sample space [0, sum_k R(k)); a persistent grid takes fixed-size
// chunks of it from a queue, each lane walking its own run of consecutive
// samples.  Every loop iteration a lane draws exactly one Philox block: the
// lifetime block of its next four pairs, or the movement block of two steps of
// its current pair; pairs whose lifetime is zero end without any block, so
// lanes stay busy while pair lengths vary.
// Diagonal (Algorithm 2; the exact cases that open Algorithm 3): D^(k) = (R(k) - M(k)) / R(k).
#include <cmath>

#include "es_internal.h"

namespace es {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;  // nodes per scan block

constexpr int kWalkThreads = 256;
constexpr uint64_t kWalkMinRun = 16;    // samples per lane per chunk, lower and upper bound
constexpr uint64_t kWalkMaxRun = 1024;
#ifndef ES_LIFE_REGS
#define ES_LIFE_REGS 8
#endif
constexpr int kLifeRegs = ES_LIFE_REGS;  // leading lifetime thresholds passed by value (scalar registers)
static_assert(kLifeRegs >= 1 && kLifeRegs <= 16, "es_ctx keeps 16 leading thresholds");

__global__ void budget_kernel(int32_t n, const double* __restrict__ pi, const int32_t* __restrict__ din_arr,
                              double R, int32_t alloc, int32_t exact_small_din, const float* __restrict__ vhat,
                              double vbar_inv, uint64_t* __restrict__ Rk) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double p = pi[k];
  const int32_t din = din_arr[k];
  double want;
  if (alloc == ES_ALLOC_PI) {
    want = R * p;
  } else if (alloc == ES_ALLOC_LEARNED) {
    // R * pi^2 * (v / vbar), pi^2 term first as in the pi^2 rule
    want = R * (p * p);
    want = want * ((double)vhat[k] * vbar_inv);
  } else {
    want = R * (p * p);
  }
  uint64_t r = (uint64_t)ceil(want);
  if (p == 0.0) r = 0;
  if (exact_small_din && din <= 1) r = 0;
  Rk[k] = r;
}

__device__ __forceinline__ uint64_t sample_count(const uint64_t* r_begin, const uint64_t* r_end, int64_t k) {
  const uint64_t e = r_end[k];
  const uint64_t b = r_begin ? r_begin[k] : 0ull;
  return e > b ? e - b : 0ull;
}

// Block-wide exclusive scan of (flag, value) pairs; returns totals in *tot_*.
__device__ void block_scan2(uint32_t& f, uint64_t& v, uint32_t* tot_f, uint64_t* tot_v, uint32_t* sf,
                            uint64_t* sv, uint32_t* ovf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // inclusive wave scan
  uint32_t fi = f;
  uint64_t vi = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t fo = __shfl_up(fi, d, 64);
    const uint64_t vo = __shfl_up(vi, d, 64);
    if (lane >= d) {
      fi += fo;
      const uint64_t s = vi + vo;
      if (s < vi) *ovf = 1;
      vi = s;
    }
  }
  if (lane == 63) {
    sf[wave] = fi;
    sv[wave] = vi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t af = 0;
    uint64_t av = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
      const uint32_t tf = sf[w];
      const uint64_t tv = sv[w];
      sf[w] = af;
      sv[w] = av;
      af += tf;
      const uint64_t s = av + tv;
      if (s < av) *ovf = 1;
      av = s;
    }
    *tot_f = af;
    *tot_v = av;
  }
  __syncthreads();
  f = fi - f + sf[wave];
  v = vi - v + sv[wave];
}

// The scans lay the count indices out in descending order: with degree-ordered
// internal ids, the many low-degree nodes holding a single sample each then
// open the sample space, and their node switches (a few dependent loads per
// sample) run alongside the hubs' long runs instead of as the kernel's tail.
// A pair's draws depend only on (k, r), so the layout does not change results.
__device__ __forceinline__ int64_t scan_index(int32_t n, int64_t q) { return (int64_t)n - 1 - q; }

// Pass 1: per scan block, the number of nodes with samples and the sample sum.
__global__ __launch_bounds__(kScanThreads) void scan_count_kernel(int32_t n, const uint64_t* __restrict__ r_begin,
                                                                  const uint64_t* __restrict__ r_end,
                                                                  uint32_t* __restrict__ bcnt,
                                                                  uint64_t* __restrict__ bsum,
                                                                  WalkTotals* __restrict__ tot) {
  __shared__ uint32_t sf[kScanThreads / 64];
  __shared__ uint64_t sv[kScanThreads / 64];
  __shared__ uint32_t tf;
  __shared__ uint64_t tv;
  __shared__ uint32_t ovf;
  if (threadIdx.x == 0) ovf = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  uint32_t f = 0;
  uint64_t v = 0;
  for (int t = 0; t < kScanPer; ++t) {
    const int64_t q = base + t;
    if (q < n) {
      const uint64_t c = sample_count(r_begin, r_end, scan_index(n, q));
      f += c > 0;
      const uint64_t s = v + c;
      if (s < v || (s >> 63)) ovf = 1;
      v = s;
    }
  }
  block_scan2(f, v, &tf, &tv, sf, sv, &ovf);
  if (threadIdx.x == 0) {
    bcnt[blockIdx.x] = tf;
    bsum[blockIdx.x] = tv;
    if (ovf) atomicExch(&tot->overflow, 1);
  }
}

// Pass 2 (one workgroup): exclusive scan over the scan blocks; totals.
__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(int32_t nb, uint32_t* __restrict__ bcnt,
                                                                   uint64_t* __restrict__ bsum,
                                                                   WalkTotals* __restrict__ tot) {
  __shared__ uint32_t sf[kScanThreads / 64];
  __shared__ uint64_t sv[kScanThreads / 64];
  __shared__ uint32_t tf;
  __shared__ uint64_t tv;
  __shared__ uint32_t ovf;
  __shared__ uint32_t carry_f;
  __shared__ uint64_t carry_v;
  if (threadIdx.x == 0) {
    ovf = 0;
    carry_f = 0;
    carry_v = 0;
  }
  __syncthreads();
  for (int base = 0; base < nb; base += kScanThreads) {
    const int i = base + threadIdx.x;
    uint32_t f = i < nb ? bcnt[i] : 0;
    uint64_t v = i < nb ? bsum[i] : 0;
    block_scan2(f, v, &tf, &tv, sf, sv, &ovf);
    const uint32_t cf = carry_f;
    const uint64_t cv = carry_v;
    if (i < nb) {
      bcnt[i] = f + cf;
      const uint64_t s = v + cv;
      if (s < v) ovf = 1;
      bsum[i] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      carry_f = cf + tf;
      const uint64_t s = cv + tv;
      if (s < cv) ovf = 1;
      carry_v = s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int32_t prior = tot->overflow;
    const bool bad = ovf || prior || (carry_v >> 63);
    tot->total = bad ? 0ull : carry_v;
    tot->n_active = bad ? 0 : (int32_t)carry_f;
    tot->overflow = bad ? 1 : 0;
    tot->cursor = 0;
  }
}

// Pass 3: active node list and the sample-space prefix over it.
__global__ __launch_bounds__(kScanThreads) void scan_write_kernel(int32_t n, const uint64_t* __restrict__ r_begin,
                                                                  const uint64_t* __restrict__ r_end,
                                                                  const uint32_t* __restrict__ bcnt,
                                                                  const uint64_t* __restrict__ bsum,
                                                                  const WalkTotals* __restrict__ tot,
                                                                  int32_t* __restrict__ active,
                                                                  uint64_t* __restrict__ prefix) {
  __shared__ uint32_t sf[kScanThreads / 64];
  __shared__ uint64_t sv[kScanThreads / 64];
  __shared__ uint32_t tf;
  __shared__ uint64_t tv;
  __shared__ uint32_t ovf;
  if (tot->overflow) return;  // uniform over the grid
  if (threadIdx.x == 0) ovf = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  uint64_t cnt[kScanPer];
  uint32_t f = 0;
  uint64_t v = 0;
  for (int t = 0; t < kScanPer; ++t) {
    const int64_t q = base + t;
    cnt[t] = q < n ? sample_count(r_begin, r_end, scan_index(n, q)) : 0ull;
    f += cnt[t] > 0;
    v += cnt[t];
  }
  block_scan2(f, v, &tf, &tv, sf, sv, &ovf);
  uint32_t pos = bcnt[blockIdx.x] + f;
  uint64_t off = bsum[blockIdx.x] + v;
  for (int t = 0; t < kScanPer; ++t) {
    if (cnt[t] > 0) {
      active[pos] = (int32_t)scan_index(n, base + t);
      prefix[pos] = off;
      ++pos;
      off += cnt[t];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) prefix[tot->n_active] = tot->total;
}

__global__ void zero_u64_kernel(int64_t n, unsigned long long* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void zero_totals_kernel(WalkTotals* tot) {
  tot->total = 0;
  tot->cursor = 0;
  tot->meets = 0;
  tot->blocks = 0;
  tot->steps = 0;
  tot->n_active = 0;
  tot->overflow = 0;
}

// ---- Philox4x64-10 (Salmon et al., SC 2011) --------------------------------

// 64 x 64 -> 128-bit product from four 32 x 32 -> 64 multiply-adds that
// share their partial products (no separate low product; each sum fits in
// 64 bits):
//   t = a1 b0 + hi(a0 b0),  w = a0 b1 + lo(t),
//   hi = a1 b1 + hi(t) + hi(w),  lo = lo(w) 2^32 + lo(a0 b0).
// Fewer instructions than a low product plus a high product; its longer-lived
// temporaries cost the batched and non-stop instantiations a few spilled
// registers, and they still run 1-3% faster with it.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t t = (uint64_t)a1 * b0 + (p00 >> 32);
  const uint64_t w = (uint64_t)a0 * b1 + (uint32_t)t;
  hi = (uint64_t)a1 * b1 + ((t >> 32) + (w >> 32));
  lo = (w << 32) | (uint32_t)p00;
}

struct Words {
  uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                               uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  // an empty asm that "changes" k0 keeps the compiler from hoisting the ten
  // round keys out of the walk loop into scalar registers, which it then
  // spilled to vector-register lanes and read back with v_readlane in every
  // round; recomputing them with scalar adds is free
  asm volatile("" : "+s"(k0));
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return Words{c0, c1, c2, c3};
}

// floor(w * d / 2^64) for d < 2^32
__device__ __forceinline__ uint32_t mulhi_index(uint64_t w, uint32_t d) {
  const uint64_t lo = (uint64_t)(uint32_t)w * d;
  const uint64_t hi = (w >> 32) * d;
  return (uint32_t)((hi + (lo >> 32)) >> 32);
}

struct WalkArgs {
  const int32_t* __restrict__ in_off;
  const int32_t* __restrict__ active;
  const uint64_t* __restrict__ prefix;
  const uint64_t* __restrict__ r_begin;
  const int32_t* __restrict__ to_graph;   // count index -> internal id (NULL: identity)
  const int32_t* __restrict__ to_stream;  // count index -> external id (NULL: identity)
  const uint64_t* __restrict__ thr;
  uint64_t head[kLifeRegs];  // thr[1..kLifeRegs]
  int32_t tmax;
  WalkTotals* tot;
  unsigned long long* __restrict__ M;  // per count index; with buckets: [index * B + bucket]
  const uint64_t* __restrict__ T;      // buckets only: ascending thresholds of each index, stride B
  int32_t B;
  uint64_t seed;
  const int32_t* __restrict__ nonstop;  // non-stop variant only: l(k) per count index
  const WalkEntry* __restrict__ adj;    // in-CSR entries with their own rows
};

// A walk's position: its node's key (row offset, or -1 - id for a node
// without in-neighbours; unique per node) and in-degree.
struct Pos {
  int32_t key, deg;
};

// One step of both walks; returns 1 = met, 0 = moved without meeting, -1 = a
// walk is stuck.  Each walk reads one entry of its current row, which is the
// next node's row.
__device__ __forceinline__ int walk_step(const WalkEntry* __restrict__ adj, Pos& x, Pos& y, uint64_t wx,
                                         uint64_t wy) {
  if (x.deg == 0 || y.deg == 0) return -1;
  const WalkEntry ex = adj[x.key + mulhi_index(wx, (uint32_t)x.deg)];
  const WalkEntry ey = adj[y.key + mulhi_index(wy, (uint32_t)y.deg)];
  x = Pos{ex.key, ex.deg};
  y = Pos{ey.key, ey.deg};
  return x.key == y.key ? 1 : 0;
}

// Sum the per-lane work counters over the wave, one atomic each (wave-uniform call).
__device__ __forceinline__ void flush_work(WalkTotals* tot, uint32_t nblocks, uint32_t nsteps) {
  unsigned long long b = nblocks, s = nsteps;
  for (int m = 32; m > 0; m >>= 1) {
    b += __shfl_xor(b, m, 64);
    s += __shfl_xor(s, m, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&tot->blocks, b);
    atomicAdd(&tot->steps, s);
  }
}

// kBuckets = false: M[k] counts the meeting pairs of node k.
// kBuckets = true (shared samples of a source block): a meeting pair r of node k
// is counted in bucket j = #{b : T[k][b] <= r} of M[k * B + j], where T[k] holds
// the block's per-source sample counts R_b(k) in ascending order; source b then
// owns the meetings of buckets j <= #{b' : R_b'(k) < R_b(k)}, i.e. exactly the
// meetings among its own pairs r < R_b(k).
// kNonstop = true (Algorithm 3): the pairs of count index k take their first
// l = nonstop[k] steps without stopping (lifetime l + T), and a meeting at a
// step t <= l ends the pair without counting.
// Eight waves per SIMD (at most 64 VGPRs) measured faster than the looser
// register budget the compiler picks by itself, so the state a lane carries
// from one iteration to the next is kept small: 32-bit where the range allows.
template <bool kBuckets, bool kNonstop>
__global__ __launch_bounds__(kWalkThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void walk_pairs_kernel(
    WalkArgs a) {
  const int lane = threadIdx.x & 63;
  const uint64_t total = a.tot->total;
  const int32_t nact = a.tot->n_active;
  // samples per lane per chunk: long runs shorten the idle tail at the end of a
  // chunk, bounded so that every wave still takes several chunks
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  uint64_t run = total / (waves * 64ull * 4ull);
  run = run < kWalkMinRun ? kWalkMinRun : (run > kWalkMaxRun ? kWalkMaxRun : run);
  const unsigned long long chunk = 64ull * run;
  // meeting count held for node cnt_node, flushed when the lane moves on (or
  // before the 32-bit count could wrap)
  int32_t cnt_node = -1;
  uint32_t cnt = 0;
  int32_t cnt_bucket = 0;      // buckets only
  uint32_t nblocks = 0, nsteps = 0;  // work counters for the roofline, flushed per chunk
  auto flush_meets = [&]() {
    if (cnt) {
      if constexpr (kBuckets) atomicAdd(&a.M[(int64_t)cnt_node * a.B + cnt_bucket], (unsigned long long)cnt);
      else atomicAdd(&a.M[cnt_node], (unsigned long long)cnt);
      atomicAdd(&a.tot->meets, (unsigned long long)cnt);
    }
  };
  auto lifetime = [&](uint64_t u) -> uint32_t {
    uint32_t T = 0;
#pragma unroll
    for (int q = 1; q <= kLifeRegs; ++q) T += u < a.head[q - 1] ? 1u : 0u;  // thresholds decrease
    if (T == kLifeRegs)
      while ((int32_t)T < a.tmax && u < a.thr[T + 1]) ++T;
    return T;
  };
  for (;;) {
    unsigned long long c0 = 0;
    if (lane == 0) c0 = atomicAdd(&a.tot->cursor, chunk);
    c0 = __shfl(c0, 0, 64);
    if (c0 >= total) break;
    // this lane's run of samples: nleft of them from i
    uint64_t i = c0 + (uint64_t)lane * run;
    uint32_t nleft = i < total ? (uint32_t)(total - i < run ? total - i : run) : 0u;
    // lifetimes of the four pairs of one quad of count index lk, 16 bits each
    // (T <= 4096); cached within the chunk only, so the low 32 bits of the
    // quad index name it
    int32_t lk = -1;
    uint32_t lq = 0;
    uint64_t lt = 0;
    // slot p of the active list: count index pk, its stream id, the pair index
    // of sample s (s + pdelta), its last sample + 1, and its start position
    int32_t p = 0, pk = 0;
    uint32_t pkc = 0;
    int32_t nsl = 0;  // non-stop variant: l(pk), the non-stop steps of pk's pairs
    uint64_t pend = 0, pdelta = 0;
    Pos pstart{0, 0};
    auto load_node = [&](uint64_t pbeg) {
      pk = a.active[p];
      pdelta = (a.r_begin ? a.r_begin[pk] : 0ull) - pbeg;
      const int32_t kg = a.to_graph ? a.to_graph[pk] : pk;
      const int32_t o = a.in_off[kg];
      const int32_t d = a.in_off[kg + 1] - o;
      pstart = Pos{d > 0 ? o : -1 - kg, d};
      pkc = (uint32_t)(a.to_stream ? a.to_stream[pk] : pk);
      if constexpr (kNonstop) nsl = a.nonstop[pk];
    };
    if (nleft) {
      // last active slot whose prefix is <= i
      int32_t lo = 0, hi = nact;  // prefix[lo] <= i < prefix[hi]
      while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (a.prefix[mid] <= i) lo = mid;
        else hi = mid;
      }
      p = lo;
      pend = a.prefix[p + 1];
      load_node(a.prefix[p]);
    }
    bool in_pair = false;
    int32_t t = 0, T = 0;
    Pos x{0, 0}, y{0, 0};
    for (;;) {
      // out of a pair: start the next one; pairs whose cached lifetime is 0
      // end at once, a pair without a cached lifetime needs its lifetime block
      bool need_life = false;
      if (!in_pair) {
        while (nleft) {
          if (i >= pend) {
            uint64_t pbeg;
            do {
              ++p;
              pbeg = pend;
              pend = a.prefix[p + 1];
            } while (i >= pend);
            load_node(pbeg);
          }
          const uint64_t rr = i + pdelta;
          if (pk == lk && (uint32_t)(rr >> 2) == lq) {
            int32_t TT = (int32_t)((lt >> (16 * (rr & 3))) & 0xffffu);
            ++i;
            --nleft;
            if constexpr (kNonstop) TT += nsl;
            if (TT == 0) continue;  // both walks stop at once: no meeting
            T = TT;
            x = pstart;
            y = pstart;
            t = 0;
            in_pair = true;
            break;
          }
          need_life = true;
          break;
        }
      }
      const bool busy = in_pair || need_life;
      if (!__any(busy)) break;
      if (!busy) continue;
      // the pair's index: its sample is i - 1 while it walks (i moved on when
      // it started) and i while its lifetime block is due
      const uint64_t r = i + pdelta - (in_pair ? 1ull : 0ull);
      // one Philox block per lane and iteration: a lifetime block (k, q, 0, 1)
      // or the movement block (k, r, j, 0) of steps 2j+1 and 2j+2
      const uint64_t c1 = need_life ? (r >> 2) : r;
      const uint64_t c2 = need_life ? 0ull : (uint64_t)(t >> 1);
      const uint64_t c3 = need_life ? 1ull : 0ull;
      const Words w = philox4x64_10((uint64_t)pkc, c1, c2, c3, a.seed, 0ull);
      ++nblocks;
      if (need_life) {
        lk = pk;
        lq = (uint32_t)(r >> 2);
        lt = (uint64_t)(lifetime(w.w0) | (lifetime(w.w1) << 16)) |
             ((uint64_t)(lifetime(w.w2) | (lifetime(w.w3) << 16)) << 32);
        continue;  // the pair starts from the cache on the next iteration
      }
      int st = walk_step(a.adj, x, y, w.w0, w.w1);
      t += 1;
      ++nsteps;
      if constexpr (kNonstop) {
        if (st > 0 && t <= nsl) st = -1;  // met during the exact levels: not counted
      }
      if (st == 0 && t < T) {
        st = walk_step(a.adj, x, y, w.w2, w.w3);
        t += 1;
        ++nsteps;
        if constexpr (kNonstop) {
          if (st > 0 && t <= nsl) st = -1;
        }
      }
      const int res = st != 0 ? st : (t >= T ? -1 : 0);  // 1: met, -1: ended, 0: go on
      if (res != 0) {
        in_pair = false;
        if (res > 0) {
          if constexpr (!kBuckets) {
            if (pk == cnt_node && cnt < 0x7fffffffu) {
              ++cnt;
            } else {
              flush_meets();
              cnt_node = pk;
              cnt = 1;
            }
          } else {
            // the cached bucket still holds r while r is below its upper threshold
            // (read again at each meeting rather than kept in a register)
            if (pk == cnt_node && cnt < 0x7fffffffu &&
                (cnt_bucket >= a.B || r < a.T[(int64_t)pk * a.B + cnt_bucket])) {
              ++cnt;
            } else {
              flush_meets();
              const uint64_t* Tk = a.T + (int64_t)pk * a.B;
              int32_t lo = 0, hi = a.B;  // first threshold above r
              while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (Tk[mid] <= r) lo = mid + 1;
                else hi = mid;
              }
              cnt_bucket = lo;
              cnt_node = pk;
              cnt = 1;
            }
          }
        }
      }
    }
    // every lane leaves the pair loop together: flush the 32-bit work counters per chunk
    flush_work(a.tot, nblocks, nsteps);
    nblocks = nsteps = 0;
  }
  flush_meets();
}

__global__ void diag_kernel(int32_t n, const uint64_t* __restrict__ Rk, const uint64_t* __restrict__ M,
                            const int32_t* __restrict__ din_arr, double one_minus_c, int32_t exact_small_din,
                            double* __restrict__ D) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint64_t r = Rk[k];
  double d = 1.0;
  if (r > 0) d = (double)(r - M[k]) / (double)r;
  if (exact_small_din) {
    const int32_t din = din_arr[k];
    if (din == 0) d = 1.0;
    else if (din == 1) d = one_minus_c;
  }
  D[k] = d;
}

}  // namespace

es_status launch_budget(es_ctx* ctx, const es_graph* g, const double* pi, const int32_t* din, double R,
                        int32_t alloc, int32_t exact_small_din, const float* vhat, double vbar_inv, uint64_t* Rk) {
  const int tb = 256;
  budget_kernel<<<ceil_div(g->n, tb), tb, 0, ctx->stream>>>(g->n, pi, din, R, alloc, exact_small_din, vhat,
                                                            vbar_inv, Rk);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

namespace {

es_status walks_core(es_ctx* ctx, const es_graph* g, const uint64_t* r_begin, const uint64_t* r_end, uint64_t seed,
                     double c, unsigned long long* M, int64_t m_len, bool external_counts, const uint64_t* T,
                     int32_t B, const int32_t* nonstop, WalkTotals** totals_out) {
  const int32_t n = g->n;
  es_status st;
  ES_TRY(lifetime_table(ctx, c));
  const int nb = ceil_div(n, kScanBlock);
  auto* tot = (WalkTotals*)workspace(ctx, kWsTotals, sizeof(WalkTotals), &st);
  if (!tot) return st;
  auto* bcnt = (uint32_t*)workspace(ctx, kWsScanCnt, sizeof(uint32_t) * nb, &st);
  if (!bcnt) return st;
  auto* bsum = (uint64_t*)workspace(ctx, kWsScanSum, sizeof(uint64_t) * nb, &st);
  if (!bsum) return st;
  auto* active = (int32_t*)workspace(ctx, kWsActive, sizeof(int32_t) * (size_t)n, &st);
  if (!active) return st;
  auto* prefix = (uint64_t*)workspace(ctx, kWsPrefix, sizeof(uint64_t) * ((size_t)n + 1), &st);
  if (!prefix) return st;
  zero_totals_kernel<<<1, 1, 0, ctx->stream>>>(tot);
  zero_u64_kernel<<<ceil_div(m_len, 256), 256, 0, ctx->stream>>>(m_len, M);
  scan_count_kernel<<<nb, kScanThreads, 0, ctx->stream>>>(n, r_begin, r_end, bcnt, bsum, tot);
  scan_blocks_kernel<<<1, kScanThreads, 0, ctx->stream>>>(nb, bcnt, bsum, tot);
  scan_write_kernel<<<nb, kScanThreads, 0, ctx->stream>>>(n, r_begin, r_end, bcnt, bsum, tot, active, prefix);
  WalkArgs a;
  a.in_off = g->in_off;
  a.active = active;
  a.prefix = prefix;
  a.r_begin = r_begin;
  a.to_graph = external_counts ? g->int_of : nullptr;
  a.to_stream = external_counts ? nullptr : g->ext_of;
  a.thr = ctx->thr;
  for (int q = 0; q < kLifeRegs; ++q) a.head[q] = ctx->thr_head[q];
  a.tmax = ctx->tmax;
  a.tot = tot;
  a.M = M;
  a.T = T;
  a.B = B;
  a.seed = seed;
  a.nonstop = nonstop;
  a.adj = g->walk_adj;
  const int grid = ctx->num_cus * 8;
  if (ctx->ev_walk_begin) ES_CHECK_HIP(ctx, hipEventRecord(ctx->ev_walk_begin, ctx->stream));
  if (T) walk_pairs_kernel<true, false><<<grid, kWalkThreads, 0, ctx->stream>>>(a);
  else if (nonstop) walk_pairs_kernel<false, true><<<grid, kWalkThreads, 0, ctx->stream>>>(a);
  else walk_pairs_kernel<false, false><<<grid, kWalkThreads, 0, ctx->stream>>>(a);
  ES_CHECK_HIP(ctx, hipGetLastError());
  if (totals_out) *totals_out = tot;
  return ES_OK;
}

}  // namespace

es_status launch_walks(es_ctx* ctx, const es_graph* g, const uint64_t* r_begin, const uint64_t* r_end,
                       uint64_t seed, double c, uint64_t* M, bool external_counts, WalkTotals** totals_out,
                       const int32_t* nonstop) {
  return walks_core(ctx, g, r_begin, r_end, seed, c, (unsigned long long*)M, g->n, external_counts, nullptr, 1,
                    nonstop, totals_out);
}

es_status launch_walks_buckets(es_ctx* ctx, const es_graph* g, const uint64_t* Rmax, const uint64_t* T, int32_t B,
                               uint64_t seed, double c, uint64_t* H, WalkTotals** totals_out) {
  return walks_core(ctx, g, nullptr, Rmax, seed, c, (unsigned long long*)H, (int64_t)g->n * B, false, T, B,
                    nullptr, totals_out);
}

es_status launch_diag(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, const uint64_t* M, const int32_t* din,
                      double c, int32_t exact_small_din, double* D) {
  const int tb = 256;
  diag_kernel<<<ceil_div(g->n, tb), tb, 0, ctx->stream>>>(g->n, Rk, M, din, 1.0 - c, exact_small_din, D);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

}  // namespace es
