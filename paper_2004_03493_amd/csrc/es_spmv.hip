// Level passes of a single-source query: the pull-form SpMV over a CSR and,
// for graphs beyond the caches, the binned push form further below.
//
// Forward (Algorithm 1, l-hop PPR):  pi^l(i) = sqrt(c) * sum_{j in O(v_i)} pi^(l-1)(j)/d_in(j),
//   each term pre-rounded to a multiple of 2^-62 and summed exactly in int64, so the
//   result is independent of how rows are split across lanes and workgroups.
// Backward (Algorithm 1, back-accumulation): s^l(j) = sqrt(c) (1/d_in(j)) sum_{i in I(v_j)} s^(l-1)(i)
//   + D(j) pi^(L-l)(j)/(1-sqrt c), float64.
//
// Pull form: the CSR index stream is read once per level and the gathered
// operand (8 bytes per entry) comes through the caches, one request per gather.
// One workgroup of kSpmvThreads (512) lanes per row block: the block's column ids are streamed
// coalesced, the gathered operands staged in LDS, then each row is reduced by a
// group of lanes sized to the block's average row length.
#include <algorithm>
#include <cmath>

#include "es_internal.h"

namespace es {

namespace {

constexpr double kFix = 0x1p62;
constexpr double kFixInv = 0x1p-62;

template <class V>
__device__ __forceinline__ V shfl_xor_v(V v, int m) {
  return __shfl_xor(v, m, 64);
}

// Sum over the g lanes of a group (g a power of two <= 64, groups aligned).
template <class V>
__device__ __forceinline__ V group_sum(V v, int g) {
  for (int m = g >> 1; m > 0; m >>= 1) v += shfl_xor_v(v, m);
  return v;
}

template <class V>
__device__ __forceinline__ V block_sum(V v, V* red) {
  v = group_sum(v, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  V t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kSpmvThreads / 64; ++w) t += red[w];
  return t;  // valid in thread 0
}

template <class V>
__device__ __forceinline__ void store_partial(V* p, V v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class V>
__device__ __forceinline__ V load_partial(const V* p) {
  return __hip_atomic_load(const_cast<V*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct FwdGather {
  const int64_t* __restrict__ q;
  __device__ __forceinline__ int64_t operator()(int32_t j) const { return q[j]; }
};

// Epilogues split into the per-row operands (loaded early, with the column
// ids, so their latency overlaps the gathers) and the arithmetic.
struct FwdEpi {
  struct Row {
    double inv_din;
  };
  double sc;
  const double* __restrict__ inv_din;
  double* __restrict__ pi_l;
  int64_t* __restrict__ q_next;
  __device__ __forceinline__ Row load(int32_t r) const { return Row{inv_din[r]}; }
  __device__ __forceinline__ void apply(int32_t r, int64_t acc, const Row& d) const {
    const double p = sc * ((double)acc * kFixInv);
    pi_l[r] = p;
    q_next[r] = (int64_t)rint((p * d.inv_din) * kFix);
  }
};

struct BackGather {
  const double* __restrict__ s;
  __device__ __forceinline__ double operator()(int32_t j) const { return s[j]; }
};

struct BackEpi {
  struct Row {
    double inv_din, D, pil;
  };
  double sc, a;
  const double* __restrict__ inv_din;
  const double* __restrict__ D;
  const double* __restrict__ pil;
  double* __restrict__ s_next;
  __device__ __forceinline__ Row load(int32_t r) const { return Row{inv_din[r], D[r], pil[r]}; }
  __device__ __forceinline__ void apply(int32_t r, double acc, const Row& d) const {
    s_next[r] = sc * (d.inv_din * acc) + a * (d.D * d.pil);
  }
};

// back pass of sparse linearization: the level term is added afterwards by
// level_scatter_kernel for the stored entries only
struct BackEpiSparse {
  struct Row {
    double inv_din;
  };
  double sc;
  const double* __restrict__ inv_din;
  double* __restrict__ s_next;
  __device__ __forceinline__ Row load(int32_t r) const { return Row{inv_din[r]}; }
  __device__ __forceinline__ void apply(int32_t r, double acc, const Row& d) const {
    s_next[r] = sc * (d.inv_din * acc);
  }
};

template <class V, class Gather, class Epi>
__global__ __launch_bounds__(kSpmvThreads) void spmv_pull_kernel(const BlockDesc* __restrict__ blocks,
                                                                 const int32_t* __restrict__ off,
                                                                 const int32_t* __restrict__ idx, Gather gather,
                                                                 Epi epi, V* __restrict__ partials,
                                                                 const int32_t* __restrict__ long_p0,
                                                                 const int32_t* __restrict__ long_nch,
                                                                 uint32_t* __restrict__ counters) {
  using Row = typename Epi::Row;
  __shared__ V vals[kSpmvNnz];
  __shared__ int32_t roff[kSpmvRows + 1];
  __shared__ Row rdat[kSpmvRows];
  __shared__ V red[kSpmvThreads / 64];
  const BlockDesc b = blocks[blockIdx.x];
  const int tid = threadIdx.x;
  if (b.row1 >= 0) {
    const int nnz = b.e1 - b.e0;
    const int nrows = b.row1 - b.row0;
    constexpr int kPer = kSpmvNnz / kSpmvThreads;
    constexpr int kRowsPer = (kSpmvRows + 1 + kSpmvThreads - 1) / kSpmvThreads;  // rows + 1 offsets
    // 1. everything that depends only on the block: column ids, row offsets, row operands
    int32_t col[kPer];
    if (nnz > 0) {
      // branch-free so that all kPer index loads, then all kPer gathers, are in flight at once;
      // lanes past the end re-read the block's last entry and do not store it
#pragma unroll
      for (int t = 0; t < kPer; ++t) col[t] = idx[b.e0 + min(t * kSpmvThreads + tid, nnz - 1)];
    }
#pragma unroll
    for (int t = 0; t < kRowsPer; ++t) {
      const int rr = t * kSpmvThreads + tid;
      if (rr < nrows) rdat[rr] = epi.load(b.row0 + rr);
      if (rr <= nrows) roff[rr] = off[b.row0 + rr] - b.e0;
    }
    // 2. the gathers
    if (nnz > 0) {
      V v[kPer];
#pragma unroll
      for (int t = 0; t < kPer; ++t) v[t] = gather(col[t]);
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int e = t * kSpmvThreads + tid;
        if (e < nnz) vals[e] = v[t];
      }
    }
    __syncthreads();
    // 3. rows from LDS: lanes per row = the largest power of two <= threads / rows, at most 64
    int g = 1;
    while (g < 64 && g * 2 * nrows <= kSpmvThreads) g *= 2;
    const int lane_in_g = tid & (g - 1);
    const int groups = kSpmvThreads / g;
    // all lanes of a group share rr, so a group's shuffles run with the whole group active
    for (int rr = tid / g; rr < nrows; rr += groups) {
      const int s0 = roff[rr], e = roff[rr + 1];
      V acc = 0;
      for (int k = s0 + lane_in_g; k < e; k += g) acc += vals[k];
      if (g > 1) acc = group_sum(acc, g);
      if (lane_in_g == 0) epi.apply(b.row0 + rr, acc, rdat[rr]);
    }
  } else {
    const int lid = -b.row1 - 1;
    const int r = b.row0;
    V acc = 0;
    constexpr int kUnroll = 8;
    for (int base = b.e0; base < b.e1; base += kUnroll * kSpmvThreads) {
      int32_t col[kUnroll];
#pragma unroll
      for (int t = 0; t < kUnroll; ++t) col[t] = idx[min(base + t * kSpmvThreads + tid, b.e1 - 1)];
      V v[kUnroll];
#pragma unroll
      for (int t = 0; t < kUnroll; ++t) v[t] = gather(col[t]);
#pragma unroll
      for (int t = 0; t < kUnroll; ++t)
        if (base + t * kSpmvThreads + tid < b.e1) acc += v[t];
    }
    acc = block_sum(acc, red);
    if (tid == 0) {
      const int32_t p0 = long_p0[lid];
      const int32_t nch = long_nch[lid];
      const int32_t slot = p0 + (b.e0 - off[r]) / kLongChunk;
      store_partial(&partials[slot], acc);
      const uint32_t prev = __hip_atomic_fetch_add(&counters[lid], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (prev == (uint32_t)(nch - 1)) {
        V tot = 0;
        for (int c = 0; c < nch; ++c) tot += load_partial(&partials[p0 + c]);
        __hip_atomic_store(&counters[lid], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        epi.apply(r, tot, epi.load(r));
      }
    }
  }
}

// ---- binned level pass (push form) ----------------------------------------
//
// Scatter: one workgroup per range of sources stages their values in LDS and
// writes each entry's value to its position in the bin-major array (runs of
// consecutive positions, one per bin the range reaches).  Accumulate: one workgroup
// per item sums its entries into the bin's rows in LDS (int64 forward; 128-bit
// fixed point backward, so the sums are exact and the order of the atomics
// does not matter), then applies the epilogue, or stores partial sums when
// the bin is split over several items; a combine launch adds those in slot
// order.

constexpr int kBinThreads = 1024;

constexpr int kFixBits = 72;  // backward terms as multiples of 2^-72
constexpr double kFixBInv = 0x1p-72;

template <class V>
__global__ __launch_bounds__(kBinThreads) void bin_scatter_kernel(const BinRange* __restrict__ ranges,
                                                                  const uint16_t* __restrict__ src_local,
                                                                  const uint32_t* __restrict__ pos,
                                                                  const V* __restrict__ x, V* __restrict__ vals) {
  __shared__ V xs[kBinSrc];
  const BinRange r = ranges[blockIdx.x];
  const int tid = threadIdx.x;
  for (int t = tid; t < r.j1 - r.j0; t += kBinThreads) xs[t] = x[r.j0 + t];
  __syncthreads();
  constexpr int kU = 4;
  for (int k = r.e0 + tid; k < r.e1; k += kU * kBinThreads) {
    uint32_t sl[kU], ps[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = min(k + u * kBinThreads, r.e1 - 1);
      sl[u] = src_local[q];
      ps[u] = pos[q];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (k + u * kBinThreads < r.e1) vals[ps[u]] = xs[sl[u]];
  }
}

// forward: exact int64 sums of the bin's rows
template <class Epi>
__global__ __launch_bounds__(kBinThreads) void bin_acc_fwd_kernel(const BinItem* __restrict__ items,
                                                                  const uint16_t* __restrict__ row_local,
                                                                  const int64_t* __restrict__ vals, int32_t n,
                                                                  Epi epi, int64_t* __restrict__ partials) {
  constexpr int kRows = 1 << kBinShiftFwd;
  __shared__ unsigned long long acc[kRows];
  const BinItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  for (int t = tid; t < kRows; t += kBinThreads) acc[t] = 0ull;
  __syncthreads();
  constexpr int kU = 4;
  for (int p = it.p0 + tid; p < it.p1; p += kU * kBinThreads) {
    uint32_t rr[kU];
    unsigned long long v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = min(p + u * kBinThreads, it.p1 - 1);
      rr[u] = row_local[q];
      v[u] = (unsigned long long)vals[q];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (p + u * kBinThreads < it.p1) atomicAdd(&acc[rr[u]], v[u]);
  }
  __syncthreads();
  const int32_t r0 = it.bin << kBinShiftFwd;
  const int nr = min(n - r0, kRows);
  if (it.slot < 0) {
    for (int t = tid; t < nr; t += kBinThreads) epi.apply(r0 + t, (int64_t)acc[t], epi.load(r0 + t));
  } else {
    int64_t* dst = partials + (size_t)it.slot * kRows;
    for (int t = tid; t < nr; t += kBinThreads) dst[t] = (int64_t)acc[t];
  }
}

template <class Epi>
__global__ void bin_combine_fwd_kernel(const BinSplit* __restrict__ splits, int32_t n, Epi epi,
                                       const int64_t* __restrict__ partials) {
  constexpr int kRows = 1 << kBinShiftFwd;
  constexpr int kPer = kRows / 256;
  const BinSplit sp = splits[blockIdx.x / kPer];
  const int t = (blockIdx.x % kPer) * 256 + threadIdx.x;
  const int32_t r = (sp.bin << kBinShiftFwd) + t;
  if (r >= n) return;
  int64_t acc = 0;
  for (int q = 0; q < sp.nslot; ++q) acc += partials[(size_t)(sp.slot0 + q) * kRows + t];
  epi.apply(r, acc, epi.load(r));
}

// v as a 128-bit two's-complement multiple of 2^-72, rounded half away from
// zero; zero for |v| < 2^-1022 (never a term above the rounding)
__device__ __forceinline__ void to_fixed(double v, unsigned long long& lo, unsigned long long& hi) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const int e = (int)((bits >> 52) & 0x7ff);
  lo = 0ull;
  hi = 0ull;
  if (e == 0) return;
  const unsigned long long m = (bits & 0xfffffffffffffull) | (1ull << 52);
  const int sh = e - 1075 + kFixBits;
  if (sh >= 64) {
    hi = m << (sh - 64);
  } else if (sh > 0) {
    lo = m << sh;
    hi = m >> (64 - sh);
  } else if (sh == 0) {
    lo = m;
  } else if (sh > -64) {
    lo = (m + (1ull << (-sh - 1))) >> (-sh);
  }
  if (bits >> 63) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
}

__device__ __forceinline__ double from_fixed(unsigned long long lo, unsigned long long hi) {
  const bool neg = (long long)hi < 0;
  if (neg) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  const double d = ((double)hi * 0x1p64 + (double)lo) * kFixBInv;
  return neg ? -d : d;
}

// backward: exact 128-bit sums of the bin's rows (low words with their carries
// passed on to the high words)
template <class Epi>
__global__ __launch_bounds__(kBinThreads) void bin_acc_back_kernel(const BinItem* __restrict__ items,
                                                                   const uint16_t* __restrict__ row_local,
                                                                   const double* __restrict__ vals, int32_t n,
                                                                   Epi epi,
                                                                   unsigned long long* __restrict__ partials) {
  constexpr int kRows = 1 << kBinShiftBack;
  __shared__ unsigned long long alo[kRows];
  __shared__ unsigned long long ahi[kRows];
  const BinItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  for (int t = tid; t < kRows; t += kBinThreads) {
    alo[t] = 0ull;
    ahi[t] = 0ull;
  }
  __syncthreads();
  constexpr int kU = 4;
  for (int p = it.p0 + tid; p < it.p1; p += kU * kBinThreads) {
    uint32_t rr[kU];
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = min(p + u * kBinThreads, it.p1 - 1);
      rr[u] = row_local[q];
      v[u] = vals[q];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (p + u * kBinThreads < it.p1) {
        unsigned long long xl, xh;
        to_fixed(v[u], xl, xh);
        const unsigned long long old = atomicAdd(&alo[rr[u]], xl);
        const unsigned long long up = xh + (old + xl < old ? 1ull : 0ull);
        if (up) atomicAdd(&ahi[rr[u]], up);
      }
    }
  }
  __syncthreads();
  const int32_t r0 = it.bin << kBinShiftBack;
  const int nr = min(n - r0, kRows);
  if (it.slot < 0) {
    for (int t = tid; t < nr; t += kBinThreads) epi.apply(r0 + t, from_fixed(alo[t], ahi[t]), epi.load(r0 + t));
  } else {
    unsigned long long* dst = partials + (size_t)it.slot * kRows * 2;
    for (int t = tid; t < nr; t += kBinThreads) {
      dst[2 * t] = alo[t];
      dst[2 * t + 1] = ahi[t];
    }
  }
}

template <class Epi>
__global__ void bin_combine_back_kernel(const BinSplit* __restrict__ splits, int32_t n, Epi epi,
                                        const unsigned long long* __restrict__ partials) {
  constexpr int kRows = 1 << kBinShiftBack;
  constexpr int kPer = kRows / 256;
  const BinSplit sp = splits[blockIdx.x / kPer];
  const int t = (blockIdx.x % kPer) * 256 + threadIdx.x;
  const int32_t r = (sp.bin << kBinShiftBack) + t;
  if (r >= n) return;
  unsigned long long lo = 0ull, hi = 0ull;
  for (int q = 0; q < sp.nslot; ++q) {
    const unsigned long long* p = partials + ((size_t)(sp.slot0 + q) * kRows + t) * 2;
    const unsigned long long pl = p[0];
    lo += pl;
    hi += p[1] + (lo < pl ? 1ull : 0ull);
  }
  epi.apply(r, from_fixed(lo, hi), epi.load(r));
}

template <class Epi>
void binned_forward_level(es_ctx* ctx, const es_graph* g, const int64_t* q, const Epi& ep) {
  const BinnedPlan& b = g->bfwd;
  int64_t* vals = (int64_t*)g->bin_vals;
  if (b.nranges > 0)
    bin_scatter_kernel<int64_t><<<b.nranges, kBinThreads, 0, ctx->stream>>>(b.ranges, b.src_local, b.pos, q, vals);
  bin_acc_fwd_kernel<Epi><<<b.nitems, kBinThreads, 0, ctx->stream>>>(b.items, b.row_local, vals, g->n, ep,
                                                                     (int64_t*)b.partials);
  if (b.nsplits > 0)
    bin_combine_fwd_kernel<Epi><<<b.nsplits * ((1 << kBinShiftFwd) / 256), 256, 0, ctx->stream>>>(
        b.splits, g->n, ep, (const int64_t*)b.partials);
}

template <class Epi>
void binned_backward_level(es_ctx* ctx, const es_graph* g, const double* s, const Epi& ep) {
  const BinnedPlan& b = g->bback;
  double* vals = (double*)g->bin_vals;
  if (b.nranges > 0)
    bin_scatter_kernel<double><<<b.nranges, kBinThreads, 0, ctx->stream>>>(b.ranges, b.src_local, b.pos, s, vals);
  bin_acc_back_kernel<Epi><<<b.nitems, kBinThreads, 0, ctx->stream>>>(b.items, b.row_local, vals, g->n, ep,
                                                                      (unsigned long long*)b.partials);
  if (b.nsplits > 0)
    bin_combine_back_kernel<Epi><<<b.nsplits * ((1 << kBinShiftBack) / 256), 256, 0, ctx->stream>>>(
        b.splits, g->n, ep, (const unsigned long long*)b.partials);
}

// pi^0 = (1 - sqrt c) e_u, q^0 = round(pi^0 / d_in * 2^62)
__global__ void forward_init_kernel(int32_t n, int32_t u, double pi0, const double* __restrict__ inv_din,
                                    double* __restrict__ lvl0, int64_t* __restrict__ q0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == u) {
    lvl0[i] = pi0;
    q0[i] = (int64_t)rint((pi0 * inv_din[i]) * kFix);
  } else {
    lvl0[i] = 0.0;
    q0[i] = 0;
  }
}

// pi(k) = sum_{l=0}^{L} pi^l(k), added in order of l
__global__ void sum_levels_kernel(int32_t n, int32_t L, const double* __restrict__ levels, double* __restrict__ pi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = levels[i];
  for (int l = 1; l <= L; ++l) acc = acc + levels[(int64_t)l * n + i];
  pi[i] = acc;
}

// s^0 = D pi^L / (1 - sqrt c)
__global__ void backward_init_kernel(int32_t n, double a, const double* __restrict__ D,
                                     const double* __restrict__ piL, double* __restrict__ s0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  s0[i] = a * (D[i] * piL[i]);
}

// ---- sparse linearization (Section 3.2, Lemma 2) ---------------------------
//
// After level l is computed densely, level_keep_kernel adds it to pi and
// appends its entries > theta to one list shared by all levels: a block takes
// kKeepPer x kKeepThreads consecutive rows, counts its kept entries with wave
// ballots and reserves their slots with one atomic on the running total, so
// level l's entries follow those of levels < l (their order within a level is
// unspecified; each node appears at most once per level).

constexpr int kKeepThreads = 256;
constexpr int kKeepPer = 16;
constexpr int kKeepRows = kKeepThreads * kKeepPer;

__global__ __launch_bounds__(kKeepThreads) void level_keep_kernel(int64_t n, const double* __restrict__ lvl,
                                                                  double theta, int first, double* __restrict__ pi,
                                                                  int32_t* __restrict__ sp_idx,
                                                                  double* __restrict__ sp_val, uint64_t cap,
                                                                  unsigned long long* __restrict__ cnt_level,
                                                                  unsigned long long* __restrict__ cnt_total) {
  __shared__ uint32_t wave_cnt[kKeepThreads / 64];
  __shared__ unsigned long long block_base;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kKeepRows + threadIdx.x;
  double v[kKeepPer];
  unsigned long long bal[kKeepPer];
  uint32_t kept = 0;
#pragma unroll
  for (int t = 0; t < kKeepPer; ++t) {
    const int64_t i = r0 + (int64_t)t * kKeepThreads;
    double x = 0.0;
    if (i < n) {
      x = lvl[i];
      pi[i] = first ? x : pi[i] + x;
    }
    v[t] = x;
    bal[t] = __ballot(x > theta);
    kept += (uint32_t)__popcll(bal[t]);
  }
  if (lane == 0) wave_cnt[wave] = kept;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kKeepThreads / 64; ++w) tot += wave_cnt[w];
    unsigned long long base = 0;
    if (tot) {
      base = atomicAdd(cnt_total, (unsigned long long)tot);
      atomicAdd(cnt_level, (unsigned long long)tot);
    }
    block_base = base;
  }
  __syncthreads();
  unsigned long long pos = block_base;
  for (int w = 0; w < wave; ++w) pos += wave_cnt[w];
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int t = 0; t < kKeepPer; ++t) {
    if ((bal[t] >> lane) & 1ull) {
      const unsigned long long p = pos + (unsigned long long)__popcll(bal[t] & below);
      if (p < cap) {
        sp_idx[p] = (int32_t)(r0 + (int64_t)t * kKeepThreads);
        sp_val[p] = v[t];
      }
    }
    pos += (unsigned long long)__popcll(bal[t]);
  }
}

// [first, end) of level l in the list, clamped to the capacity
__device__ __forceinline__ void level_range(int32_t l, const unsigned long long* cnt, uint64_t cap,
                                            unsigned long long* first, unsigned long long* end) {
  unsigned long long b = 0;
  for (int32_t k = 0; k < l; ++k) b += cnt[k];
  const unsigned long long e = b + cnt[l];
  *first = b < cap ? b : cap;
  *end = e < cap ? e : cap;
}

// s(j) += a D(j) pi^l(j) over the stored entries of level l
__global__ void level_scatter_kernel(int32_t l, const unsigned long long* __restrict__ cnt, uint64_t cap,
                                     const int32_t* __restrict__ sp_idx, const double* __restrict__ sp_val,
                                     const double* __restrict__ D, double a, double* __restrict__ s) {
  __shared__ unsigned long long range[2];
  if (threadIdx.x == 0) level_range(l, cnt, cap, &range[0], &range[1]);
  __syncthreads();
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long p = range[0] + (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; p < range[1];
       p += stride) {
    const int32_t j = sp_idx[p];
    s[j] = s[j] + a * (D[j] * sp_val[p]);
  }
}

// ids of the whole list, internal -> external
__global__ void sparse_ids_kernel(int32_t L, const unsigned long long* __restrict__ cnt, uint64_t cap,
                                  const int32_t* __restrict__ ext_of, int32_t* __restrict__ sp_idx) {
  __shared__ unsigned long long end;
  if (threadIdx.x == 0) {
    unsigned long long first;
    level_range(L, cnt, cap, &first, &end);
  }
  __syncthreads();
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long p = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; p < end; p += stride)
    sp_idx[p] = ext_of[sp_idx[p]];
}

__global__ void fill_u64_kernel(int64_t count, unsigned long long* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

__global__ void fill_f64_kernel(int64_t count, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// blocks for a grid-stride pass over at most `count` list entries
int scatter_blocks(uint64_t count) {
  const uint64_t b = (count + 255) / 256;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(b, 1024));
}

}  // namespace

es_status launch_level_keep(es_ctx* ctx, int64_t n, const double* lvl, bool first, double* pi, const SparseLevels& sp,
                            int32_t level, int32_t L) {
  level_keep_kernel<<<ceil_div(n, kKeepRows), kKeepThreads, 0, ctx->stream>>>(
      n, lvl, sp.theta, first ? 1 : 0, pi, sp.idx, sp.val, sp.cap, sp.cnt + level, sp.cnt + L + 1);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

es_status launch_level_scatter(es_ctx* ctx, int64_t n, const SparseLevels& sp, int32_t level, const double* D,
                               double a, double* s) {
  level_scatter_kernel<<<scatter_blocks(std::min<uint64_t>(sp.cap, (uint64_t)n)), 256, 0, ctx->stream>>>(
      level, sp.cnt, sp.cap, sp.idx, sp.val, D, a, s);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

es_status launch_fill(es_ctx* ctx, int64_t count, unsigned long long* p) {
  if (count > 0) fill_u64_kernel<<<ceil_div(count, 256), 256, 0, ctx->stream>>>(count, p);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

es_status launch_fill(es_ctx* ctx, int64_t count, double* p) {
  if (count > 0) fill_f64_kernel<<<ceil_div(count, 256), 256, 0, ctx->stream>>>(count, p);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

uint64_t sparse_capacity(int32_t n, int64_t m, int32_t L, double theta) {
  const double dense = (double)(L + 1) * (double)n;
  // kept entries exceed theta and the levels' mass is at most 1 plus the
  // fixed-point rounding of the forward pass (below 2^-62 per edge and level)
  const double slack = (double)(L + 1) * ((double)m + (double)n) * 0x1p-62;
  const double bound = std::floor((1.0 + slack) / theta) + 1.0;
  return (uint64_t)(bound < dense ? bound : dense);
}

es_status launch_sparse_ids(es_ctx* ctx, const es_graph* g, int32_t L, const SparseLevels& sp) {
  sparse_ids_kernel<<<scatter_blocks(sp.cap), 256, 0, ctx->stream>>>(L, sp.cnt, sp.cap, g->ext_of, sp.idx);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

es_status launch_forward(es_ctx* ctx, const es_graph* g, int32_t u, double c, int32_t L, double* levels, double* pi,
                         int64_t* q0, int64_t* q1, const SparseLevels* sp) {
  const int32_t n = g->n;
  const double sc = std::sqrt(c);
  const int tb = 256;
  const int nb = ceil_div(n, tb);
  // dense: level l in slot l; sparse: levels below nkeep in their slots, the rest share slot nkeep
  auto slot = [&](int32_t l) -> double* {
    const int32_t k = (sp && l >= sp->nkeep) ? sp->nkeep : l;
    return levels + (int64_t)k * n;
  };
  const int kb = ceil_div(n, kKeepRows);
  if (sp) fill_u64_kernel<<<ceil_div(L + 2, tb), tb, 0, ctx->stream>>>(L + 2, sp->cnt);
  forward_init_kernel<<<nb, tb, 0, ctx->stream>>>(n, u, 1.0 - sc, g->inv_din, slot(0), q0);
  if (sp)
    level_keep_kernel<<<kb, kKeepThreads, 0, ctx->stream>>>(n, slot(0), sp->theta, 1, pi, sp->idx, sp->val,
                                                            sp->cap, sp->cnt, sp->cnt + L + 1);
  int64_t* qp = q0;
  int64_t* qn = q1;
  for (int32_t l = 1; l <= L; ++l) {
    FwdGather ga{qp};
    FwdEpi ep{sc, g->inv_din, slot(l), qn};
    if (g->binned)
      binned_forward_level(ctx, g, qp, ep);
    else if (g->fwd.nblocks > 0)
      spmv_pull_kernel<int64_t, FwdGather, FwdEpi><<<g->fwd.nblocks, kSpmvThreads, 0, ctx->stream>>>(
          g->fwd.blocks, g->out_off, g->out_idx, ga, ep, (int64_t*)g->fwd.partials, g->fwd.long_p0, g->fwd.long_nch,
          g->fwd.counters);
    if (sp)
      level_keep_kernel<<<kb, kKeepThreads, 0, ctx->stream>>>(n, slot(l), sp->theta, 0, pi, sp->idx, sp->val,
                                                              sp->cap, sp->cnt + l, sp->cnt + L + 1);
    std::swap(qp, qn);
  }
  if (!sp) sum_levels_kernel<<<nb, tb, 0, ctx->stream>>>(n, L, levels, pi);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

es_status launch_backward(es_ctx* ctx, const es_graph* g, const double* levels, int32_t L, const double* D, double c,
                          double* s, double* s_tmp, const SparseLevels* sp) {
  const int32_t n = g->n;
  const double sc = std::sqrt(c);
  const double a = 1.0 / (1.0 - sc);
  const int tb = 256;
  const int nb = ceil_div(n, tb);
  // ping-pong so that level L lands in s
  double* cur = (L % 2 == 0) ? s : s_tmp;
  double* nxt = (L % 2 == 0) ? s_tmp : s;
  if (sp) {
    const int sb = scatter_blocks(std::min<uint64_t>(sp->cap, (uint64_t)n));
    fill_f64_kernel<<<nb, tb, 0, ctx->stream>>>(n, cur);
    level_scatter_kernel<<<sb, 256, 0, ctx->stream>>>(L, sp->cnt, sp->cap, sp->idx, sp->val, D, a, cur);
    for (int32_t l = 1; l <= L; ++l) {
      BackGather ga{cur};
      BackEpiSparse ep{sc, g->inv_din, nxt};
      if (g->binned)
        binned_backward_level(ctx, g, cur, ep);
      else if (g->back.nblocks > 0)
        spmv_pull_kernel<double, BackGather, BackEpiSparse><<<g->back.nblocks, kSpmvThreads, 0, ctx->stream>>>(
            g->back.blocks, g->in_off, g->in_idx, ga, ep, (double*)g->back.partials, g->back.long_p0,
            g->back.long_nch, g->back.counters);
      level_scatter_kernel<<<sb, 256, 0, ctx->stream>>>(L - l, sp->cnt, sp->cap, sp->idx, sp->val, D, a, nxt);
      std::swap(cur, nxt);
    }
    ES_CHECK_HIP(ctx, hipGetLastError());
    return ES_OK;
  }
  backward_init_kernel<<<nb, tb, 0, ctx->stream>>>(n, a, D, levels + (int64_t)L * n, cur);
  for (int32_t l = 1; l <= L; ++l) {
    BackGather ga{cur};
    BackEpi ep{sc, a, g->inv_din, D, levels + (int64_t)(L - l) * n, nxt};
    if (g->binned)
      binned_backward_level(ctx, g, cur, ep);
    else if (g->back.nblocks > 0)
      spmv_pull_kernel<double, BackGather, BackEpi><<<g->back.nblocks, kSpmvThreads, 0, ctx->stream>>>(
          g->back.blocks, g->in_off, g->in_idx, ga, ep, (double*)g->back.partials, g->back.long_p0,
          g->back.long_nch, g->back.counters);
    std::swap(cur, nxt);
  }
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

}  // namespace es
