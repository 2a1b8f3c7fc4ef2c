// Context, graph construction and host-side constants of libexactsim.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>

#include "es_internal.h"

namespace es {

namespace {

__global__ void walk_adj_kernel(int64_t m, const int32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx,
                                WalkEntry* __restrict__ adj) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = in_idx[e];
    const int32_t o = in_off[v];
    const int32_t d = in_off[v + 1] - o;
    adj[e] = WalkEntry{d > 0 ? o : -1 - v, d, 0, 0};
  }
}

}  // namespace

es_status fail(es_ctx* ctx, es_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return st;
}

es_status hip_fail(es_ctx* ctx, hipError_t e, const char* what) {
  // a failed runtime call also leaves its code as the thread's last error;
  // consume it, or the next launch check would report it as its own
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory) return fail(ctx, ES_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(ctx, ES_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

uint64_t workspace_total(const es_ctx* ctx) {
  uint64_t t = 0;
  for (size_t b : ctx->ws_bytes) t += b;
  return t;
}

void* workspace(es_ctx* ctx, int slot, size_t bytes, es_status* st) {
  *st = ES_OK;
  if ((int)ctx->ws.size() <= slot) {
    ctx->ws.resize(slot + 1, nullptr);
    ctx->ws_bytes.resize(slot + 1, 0);
  }
  if (bytes == 0) bytes = 8;
  if (ctx->ws_bytes[slot] < bytes) {
    if (ctx->ws[slot]) {
      // the stream may still use the old buffer
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(ctx->ws[slot]);
      ctx->ws[slot] = nullptr;
      ctx->ws_bytes[slot] = 0;
    }
    size_t want = bytes + bytes / 8;
    hipError_t e = hipMalloc(&ctx->ws[slot], want);
    if (e != hipSuccess) {
      *st = hip_fail(ctx, e, "hipMalloc(workspace)");
      return nullptr;
    }
    ctx->ws_bytes[slot] = want;
  }
  return ctx->ws[slot];
}

int32_t num_levels(double c, double eps) {
  // smallest L >= 0 with c^L <= eps/2
  int32_t L = 0;
  double p = 1.0;
  const double half = eps / 2.0;
  while (p > half) {
    p = p * c;
    ++L;
  }
  return L;
}

double total_samples(int32_t n, double c, double eps, double r_scale) {
  const double sc = std::sqrt(c);
  const double om = 1.0 - sc;
  const double om2 = om * om;
  const double om4 = om2 * om2;
  return 6.0 * std::log((double)n) / (om4 * (eps * eps)) * r_scale;
}

es_status lifetime_table(es_ctx* ctx, double c) {
  if (ctx->thr && ctx->thr_c == c) return ES_OK;
  constexpr int kCap = 4096;
  std::vector<uint64_t> thr(kCap + 1, 0);
  double p = 1.0;
  int t = 1;
  for (; t <= kCap; ++t) {
    p = p * c;
    const double v = p * 18446744073709551616.0;  // 2^64
    const uint64_t u = (v >= 18446744073709551616.0) ? ~0ull : (uint64_t)v;
    if (u == 0) break;
    thr[t] = u;
  }
  const int tmax = t - 1;
  if (!ctx->thr) ES_CHECK_HIP(ctx, hipMalloc(&ctx->thr, sizeof(uint64_t) * (kCap + 1)));
  // the whole table, zeros past tmax: the walk kernels read a fixed number of
  // leading thresholds whatever c is
  ES_CHECK_HIP(ctx, hipMemcpyAsync(ctx->thr, thr.data(), sizeof(uint64_t) * (kCap + 1), hipMemcpyHostToDevice,
                                   ctx->stream));
  ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->tmax = tmax;
  ctx->thr_c = c;
  return ES_OK;
}

es_status build_plan(es_ctx* ctx, const int32_t* off, int32_t n, SpmvPlan* plan) {
  std::vector<BlockDesc> longs, shorts;
  std::vector<int32_t> long_p0, long_nch;
  int32_t nslots = 0;
  int32_t maxnnz = 0;
  int32_t r = 0;
  while (r < n) {
    const int32_t deg = off[r + 1] - off[r];
    maxnnz = std::max(maxnnz, deg);
    if (deg > kSpmvNnz) {
      const int32_t lid = (int32_t)long_p0.size();
      const int32_t nch = ceil_div(deg, kLongChunk);
      long_p0.push_back(nslots);
      long_nch.push_back(nch);
      nslots += nch;
      for (int32_t c = 0; c < nch; ++c) {
        const int32_t e0 = off[r] + c * kLongChunk;
        const int32_t e1 = std::min<int32_t>(e0 + kLongChunk, off[r + 1]);
        longs.push_back(BlockDesc{r, -(lid + 1), e0, e1});
      }
      ++r;
      continue;
    }
    const int32_t r0 = r, e0 = off[r];
    while (r < n && r - r0 < kSpmvRows && off[r + 1] - e0 <= kSpmvNnz) {
      maxnnz = std::max(maxnnz, off[r + 1] - off[r]);
      ++r;
    }
    shorts.push_back(BlockDesc{r0, r, e0, off[r]});
  }
  std::vector<BlockDesc> all;
  all.reserve(longs.size() + shorts.size());
  all.insert(all.end(), longs.begin(), longs.end());
  all.insert(all.end(), shorts.begin(), shorts.end());
  plan->nblocks = (int32_t)all.size();
  plan->nlong = (int32_t)long_p0.size();
  plan->nslots = nslots;
  plan->max_row_nnz = maxnnz;
  ES_CHECK_HIP(ctx, hipMalloc(&plan->blocks, sizeof(BlockDesc) * std::max<size_t>(1, all.size())));
  ES_CHECK_HIP(ctx, hipMemcpy(plan->blocks, all.data(), sizeof(BlockDesc) * all.size(), hipMemcpyHostToDevice));
  const size_t nl = std::max<size_t>(1, long_p0.size());
  ES_CHECK_HIP(ctx, hipMalloc(&plan->long_p0, sizeof(int32_t) * nl));
  ES_CHECK_HIP(ctx, hipMalloc(&plan->long_nch, sizeof(int32_t) * nl));
  ES_CHECK_HIP(ctx, hipMalloc(&plan->counters, sizeof(uint32_t) * nl));
  ES_CHECK_HIP(ctx, hipMalloc(&plan->partials, 8 * std::max<size_t>(1, nslots)));
  ES_CHECK_HIP(ctx, hipMemset(plan->counters, 0, sizeof(uint32_t) * nl));
  if (!long_p0.empty()) {
    ES_CHECK_HIP(ctx, hipMemcpy(plan->long_p0, long_p0.data(), sizeof(int32_t) * long_p0.size(),
                                hipMemcpyHostToDevice));
    ES_CHECK_HIP(ctx, hipMemcpy(plan->long_nch, long_nch.data(), sizeof(int32_t) * long_nch.size(),
                                hipMemcpyHostToDevice));
  }
  return ES_OK;
}

void free_plan(SpmvPlan* plan) {
  (void)hipFree(plan->blocks);
  (void)hipFree(plan->long_p0);
  (void)hipFree(plan->long_nch);
  (void)hipFree(plan->counters);
  (void)hipFree(plan->partials);
  *plan = SpmvPlan{};
}

// ---------------------------------------------------------------------------
// Host-side parallel helpers for graph construction (std::thread; the worker
// count is OMP_NUM_THREADS when set, else the hardware count capped at 16).

int host_threads() {
  static const int t = [] {
    if (const char* e = std::getenv("OMP_NUM_THREADS")) {
      const int v = std::atoi(e);
      if (v >= 1) return std::min(v, 256);
    }
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(hc, 16u));
  }();
  return t;
}

// f(lo, hi) over [0, n) in dynamically dispatched blocks of at least `grain`.
template <class F>
void par_for(int64_t n, int64_t grain, F f) {
  if (n <= 0) return;
  const int T = host_threads();
  const int64_t nblk_target = (int64_t)T * 16;
  const int64_t blk = std::max<int64_t>(grain, (n + nblk_target - 1) / nblk_target);
  const int64_t nblk = (n + blk - 1) / blk;
  if (T == 1 || nblk == 1) {
    f((int64_t)0, n);
    return;
  }
  std::atomic<int64_t> next{0};
  auto work = [&] {
    for (;;) {
      const int64_t b = next.fetch_add(1, std::memory_order_relaxed);
      if (b >= nblk) return;
      f(b * blk, std::min(n, (b + 1) * blk));
    }
  };
  std::vector<std::thread> pool;
  const int nt = (int)std::min<int64_t>(T, nblk);
  try {
    pool.reserve(nt - 1);
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  } catch (...) {
    // fewer workers: the calling thread still drains every block
  }
  work();
  for (auto& th : pool) th.join();
}

// Ascending sort of a uint64 array: sorted chunks, then pairwise merges.
void par_sort(std::vector<uint64_t>& a) {
  const int64_t n = (int64_t)a.size();
  const int T = host_threads();
  if (T == 1 || n < (1 << 20)) {
    std::sort(a.begin(), a.end());
    return;
  }
  int64_t nch = 1;
  while (nch < T) nch *= 2;
  std::vector<int64_t> cut(nch + 1);
  for (int64_t i = 0; i <= nch; ++i) cut[i] = n * i / nch;
  par_for(nch, 1, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) std::sort(a.begin() + cut[i], a.begin() + cut[i + 1]);
  });
  std::vector<uint64_t> buf(n);
  uint64_t* from = a.data();
  uint64_t* to = buf.data();
  for (int64_t w = 1; w < nch; w *= 2) {
    par_for(nch / (2 * w), 1, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        const int64_t l = cut[2 * w * i], mid = cut[2 * w * i + w], r = cut[2 * w * i + 2 * w];
        std::merge(from + l, from + mid, from + mid, from + r, to + l);
      }
    });
    std::swap(from, to);
  }
  if (from != a.data()) std::memcpy(a.data(), from, (size_t)n * sizeof(uint64_t));
}

// Degree-ordered relabelling and the two CSR copies under internal ids.
// keys: edges (src << 32 | dst) in external ids, sorted ascending, distinct
// or not (every key is one edge).
struct HostLayout {
  std::vector<int32_t> din_ext, dout_ext, ext_of, int_of;
  std::vector<int32_t> out_off, out_idx, in_off, in_idx, din_int;
  std::vector<double> inv_din;
};

// Offsets [0, n] of the keys of each external source (keys sorted by source).
static std::vector<int64_t> source_starts(const std::vector<uint64_t>& keys, int32_t n) {
  std::vector<int64_t> st((size_t)n + 1);
  const int64_t m = (int64_t)keys.size();
  // st[v] = first key index with source >= v, by binary search per block of ids
  par_for(n + 1, 1 << 14, [&](int64_t lo, int64_t hi) {
    int64_t e = std::lower_bound(keys.begin(), keys.end(), (uint64_t)lo << 32) - keys.begin();
    for (int64_t v = lo; v < hi; ++v) {
      while (e < m && (int64_t)(keys[e] >> 32) < v) ++e;
      st[v] = e;
    }
  });
  return st;
}

static void build_layout(const std::vector<uint64_t>& keys, int32_t n, HostLayout& h) {
  const int64_t m = (int64_t)keys.size();
  const std::vector<int64_t> sst = source_starts(keys, n);
  h.din_ext.assign(n, 0);
  h.dout_ext.resize(n);
  par_for(n, 1 << 14, [&](int64_t lo, int64_t hi) {
    for (int64_t v = lo; v < hi; ++v) h.dout_ext[v] = (int32_t)(sst[v + 1] - sst[v]);
  });
  int32_t* din = h.din_ext.data();
  par_for(m, 1 << 16, [&](int64_t lo, int64_t hi) {
    for (int64_t e = lo; e < hi; ++e) __atomic_fetch_add(&din[keys[e] & 0xffffffffu], 1, __ATOMIC_RELAXED);
  });
  // internal id = rank by total degree, descending, ties by external id:
  // ascending order of ((2^32 - 1 - degree) << 32 | id)
  {
    std::vector<uint64_t> rk(n);
    par_for(n, 1 << 14, [&](int64_t lo, int64_t hi) {
      for (int64_t v = lo; v < hi; ++v) {
        const uint64_t deg = (uint64_t)h.din_ext[v] + (uint64_t)h.dout_ext[v];
        rk[v] = ((0xffffffffull - deg) << 32) | (uint64_t)v;
      }
    });
    par_sort(rk);
    h.ext_of.resize(n);
    h.int_of.resize(n);
    par_for(n, 1 << 14, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        const int32_t v = (int32_t)(rk[i] & 0xffffffffu);
        h.ext_of[i] = v;
        h.int_of[v] = (int32_t)i;
      }
    });
  }
  // row offsets of both CSRs (internal rows)
  h.out_off.assign((size_t)n + 1, 0);
  h.in_off.assign((size_t)n + 1, 0);
  h.din_int.resize(n);
  h.inv_din.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = h.ext_of[i];
    const int32_t d = h.din_ext[v];
    h.din_int[i] = d;
    h.inv_din[i] = d > 0 ? 1.0 / (double)d : 0.0;
    h.out_off[i + 1] = h.out_off[i] + h.dout_ext[v];
    h.in_off[i + 1] = h.in_off[i] + d;
  }
  // out-CSR: the keys of external source v fill internal row int_of[v];
  // columns internal, ascending
  h.out_idx.resize(m);
  par_for(n, 1 << 12, [&](int64_t lo, int64_t hi) {
    for (int64_t v = lo; v < hi; ++v) {
      int32_t* row = h.out_idx.data() + h.out_off[h.int_of[v]];
      const int64_t b = sst[v], e = sst[v + 1];
      for (int64_t k = b; k < e; ++k) row[k - b] = h.int_of[keys[k] & 0xffffffffu];
      std::sort(row, row + (e - b));
    }
  });
  // in-CSR: rows in ascending external source order (the walk's order).
  // Stable partition of the keys (already in source order) into P row
  // ranges of about equal edge counts, then an in-order scatter per range:
  // every row receives its sources in key order, i.e. ascending.
  h.in_idx.resize(m);
  {
    const int T = host_threads();
    const int64_t P = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>((int64_t)T * 64, 65535), n));
    std::vector<int64_t> rstart(P + 1);
    for (int64_t b = 0; b <= P; ++b)
      rstart[b] = b == 0 ? 0 : b == P ? n : std::lower_bound(h.in_off.begin(), h.in_off.end() - 1, (int32_t)(m * b / P)) - h.in_off.begin();
    // range of the row of every external node
    std::vector<uint16_t> part(n);
    par_for(P, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo; b < hi; ++b)
        for (int64_t r = rstart[b]; r < rstart[b + 1]; ++r) part[h.ext_of[r]] = (uint16_t)b;
    });
    // counts per (key chunk, range); chunks are contiguous and in order
    const int64_t C = std::max<int64_t>(1, std::min<int64_t>((int64_t)T * 4, (m + (1 << 16) - 1) >> 16));
    std::vector<int64_t> cnt((size_t)(C * P), 0);
    par_for(C, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t c = lo; c < hi; ++c) {
        int64_t* q = cnt.data() + c * P;
        for (int64_t e = m * c / C; e < m * (c + 1) / C; ++e) q[part[keys[e] & 0xffffffffu]]++;
      }
    });
    // range-major, chunk-minor offsets
    std::vector<int64_t> pstart(P + 1, 0);
    int64_t acc = 0;
    for (int64_t b = 0; b < P; ++b) {
      pstart[b] = acc;
      for (int64_t c = 0; c < C; ++c) {
        const int64_t k = cnt[c * P + b];
        cnt[c * P + b] = acc;
        acc += k;
      }
    }
    pstart[P] = acc;
    // (internal row << 32 | internal source) in stable order per range
    std::vector<uint64_t> tmp(m);
    par_for(C, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t c = lo; c < hi; ++c) {
        int64_t* q = cnt.data() + c * P;
        for (int64_t e = m * c / C; e < m * (c + 1) / C; ++e) {
          const uint64_t k = keys[e];
          const uint32_t d = (uint32_t)(k & 0xffffffffu);
          tmp[q[part[d]]++] = ((uint64_t)(uint32_t)h.int_of[d] << 32) | (uint32_t)h.int_of[k >> 32];
        }
      }
    });
    // next free slot of every row; each range touches only its own rows
    std::vector<int32_t> pos(h.in_off.begin(), h.in_off.end() - 1);
    par_for(P, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo; b < hi; ++b)
        for (int64_t i = pstart[b]; i < pstart[b + 1]; ++i) {
          const uint64_t t = tmp[i];
          h.in_idx[pos[t >> 32]++] = (int32_t)(t & 0xffffffffu);
        }
    });
  }
}

}  // namespace es

using namespace es;

extern "C" {

const char* es_status_str(es_status s) {
  switch (s) {
    case ES_OK: return "ES_OK";
    case ES_EINVAL: return "ES_EINVAL: invalid argument";
    case ES_ERANGE: return "ES_ERANGE: size outside the int32 index range";
    case ES_ENOMEM: return "ES_ENOMEM: out of memory";
    case ES_EDEVICE: return "ES_EDEVICE: HIP runtime error";
    case ES_EOVERFLOW: return "ES_EOVERFLOW: sample count reaches 2^63";
    case ES_EUNSUPPORTED: return "ES_EUNSUPPORTED: not supported";
  }
  return "unknown es_status";
}

const char* es_last_error(const es_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

es_status es_ctx_create(int device, void* hip_stream, es_ctx** out) {
  if (!out) return ES_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return ES_EDEVICE;
  if (device < 0 || device >= ndev) return ES_EINVAL;
  es_ctx* ctx = new (std::nothrow) es_ctx();
  if (!ctx) return ES_ENOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return ES_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete ctx;
    return ES_EDEVICE;
  }
  ctx->num_cus = prop.multiProcessorCount;
  for (auto& e : ctx->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      delete ctx;
      return ES_EDEVICE;
    }
  }
  if (es::topk_scratch_init(ctx) != ES_OK) {
    es_ctx_destroy(ctx);
    return ES_EDEVICE;
  }
  *out = ctx;
  return ES_OK;
}

es_status es_ctx_destroy(es_ctx* ctx) {
  if (!ctx) return ES_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  es::free_batch_plans(ctx);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  for (void* p : ctx->ws) (void)hipFree(p);
  (void)hipFree(ctx->thr);
  (void)hipFree(ctx->mlp_w);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
  return ES_OK;
}

es_status es_ctx_sync(es_ctx* ctx) {
  if (!ctx) return ES_EINVAL;
  ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return ES_OK;
}

es_status es_num_levels(double c, double eps, int32_t* L) {
  if (!L || !(c > 0.0 && c < 1.0) || !(eps > 0.0 && eps < 1.0)) return ES_EINVAL;
  *L = num_levels(c, eps);
  return ES_OK;
}

es_status es_total_samples(int32_t n, double c, double eps, double r_scale, double* R) {
  if (!R || n < 1 || !(c > 0.0 && c < 1.0) || !(eps > 0.0 && eps < 1.0) || !(r_scale > 0.0)) return ES_EINVAL;
  *R = total_samples(n, c, eps, r_scale);
  return ES_OK;
}

es_status es_graph_from_edges(es_ctx* ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                              uint32_t flags, es_graph** out) {
  if (!ctx || !out) return ES_EINVAL;
  *out = nullptr;
  if (n < 1 || m < 0 || m >= (int64_t)INT32_MAX) return fail(ctx, ES_ERANGE, "n=%d m=%lld", n, (long long)m);
  if (m > 0 && (!src || !dst)) return fail(ctx, ES_EINVAL, "null edge array");
  std::vector<uint64_t> keys;
  try {
    keys.resize((size_t)m);
  } catch (...) {
    return fail(ctx, ES_ENOMEM, "host edge buffer");
  }
  // pack, validate and (optionally) drop self-loops, in parallel blocks;
  // per-block counts give each block its place in the compacted array
  {
    const int64_t kBlk = 1 << 20;
    const int64_t nblk = (m + kBlk - 1) / kBlk;
    std::vector<int64_t> kept((size_t)nblk + 1, 0), bad((size_t)nblk, -1);
    std::vector<uint8_t> blk_sorted((size_t)nblk, 1);
    const bool drop = (flags & ES_DROP_SELF_LOOPS) != 0;
    par_for(nblk, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo; b < hi; ++b) {
        int64_t k = 0;
        for (int64_t e = b * kBlk; e < std::min(m, (b + 1) * kBlk); ++e) {
          const int32_t s = src[e], d = dst[e];
          if (s < 0 || s >= n || d < 0 || d >= n) {
            bad[b] = e;
            break;
          }
          if (!(drop && s == d)) ++k;
        }
        kept[b + 1] = k;
      }
    });
    for (int64_t b = 0; b < nblk; ++b)
      if (bad[b] >= 0) {
        const int64_t e = bad[b];
        return fail(ctx, ES_EINVAL, "edge %lld (%d -> %d) outside [0, %d)", (long long)e, src[e], dst[e], n);
      }
    for (int64_t b = 0; b < nblk; ++b) kept[b + 1] += kept[b];
    par_for(nblk, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo; b < hi; ++b) {
        int64_t w = kept[b];
        uint64_t prev = 0;
        bool first = true;
        for (int64_t e = b * kBlk; e < std::min(m, (b + 1) * kBlk); ++e) {
          const int32_t s = src[e], d = dst[e];
          if (drop && s == d) continue;
          const uint64_t key = ((uint64_t)(uint32_t)s << 32) | (uint32_t)d;
          if (!first && key <= prev) blk_sorted[b] = 0;
          prev = key;
          first = false;
          keys[w++] = key;
        }
      }
    });
    keys.resize((size_t)kept[nblk]);
    bool sorted = true;
    for (int64_t b = 0; b < nblk; ++b) sorted = sorted && blk_sorted[b];
    for (int64_t b = 1; sorted && b < nblk; ++b)
      if (kept[b] > 0 && kept[b] < (int64_t)keys.size() && keys[kept[b]] <= keys[kept[b] - 1]) sorted = false;
    if (!sorted) par_sort(keys);
  }
  if (flags & ES_DEDUP) keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  es_graph* g = new (std::nothrow) es_graph();
  if (!g) return fail(ctx, ES_ENOMEM, "graph handle");
  static std::atomic<uint64_t> next_uid{0};
  g->uid = ++next_uid;
  g->device = ctx->device;
  g->n = n;
  g->m = (int64_t)keys.size();
  HostLayout h;
  try {
    build_layout(keys, n, h);
  } catch (...) {
    delete g;
    return fail(ctx, ES_ENOMEM, "host graph layout");
  }
  std::vector<uint64_t>().swap(keys);
  auto up = [&](void** dptr, const void* host, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dptr, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) return e;
    if (bytes) e = hipMemcpy(*dptr, host, bytes, hipMemcpyHostToDevice);
    return e;
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up((void**)&g->out_off, h.out_off.data(), 4 * h.out_off.size());
  if (e == hipSuccess) e = up((void**)&g->out_idx, h.out_idx.data(), 4 * h.out_idx.size());
  if (e == hipSuccess) e = up((void**)&g->in_off, h.in_off.data(), 4 * h.in_off.size());
  if (e == hipSuccess) e = up((void**)&g->in_idx, h.in_idx.data(), 4 * h.in_idx.size());
  if (e == hipSuccess) e = up((void**)&g->inv_din, h.inv_din.data(), 8 * h.inv_din.size());
  if (e == hipSuccess) e = up((void**)&g->din_int, h.din_int.data(), 4 * h.din_int.size());
  if (e == hipSuccess) e = up((void**)&g->din_ext, h.din_ext.data(), 4 * h.din_ext.size());
  if (e == hipSuccess) e = up((void**)&g->dout_ext, h.dout_ext.data(), 4 * h.dout_ext.size());
  if (e == hipSuccess) e = up((void**)&g->ext_of, h.ext_of.data(), 4 * h.ext_of.size());
  if (e == hipSuccess) e = up((void**)&g->int_of, h.int_of.data(), 4 * h.int_of.size());
  if (e == hipSuccess) e = hipMalloc((void**)&g->walk_adj, sizeof(WalkEntry) * std::max<size_t>(1, h.in_idx.size()));
  if (e == hipSuccess && !h.in_idx.empty()) {
    const int64_t mm = (int64_t)h.in_idx.size();
    const int blocks = (int)std::min<int64_t>((mm + 255) / 256, (int64_t)ctx->num_cus * 64);
    walk_adj_kernel<<<blocks, 256>>>(mm, g->in_off, g->in_idx, g->walk_adj);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    es_graph_destroy(g);
    return hip_fail(ctx, e, "graph upload");
  }
  g->h_int_of = std::move(h.int_of);
  g->h_out_off = h.out_off;
  g->h_in_off = h.in_off;
  es_status st = build_plan(ctx, h.out_off.data(), n, &g->fwd);
  if (st == ES_OK) st = build_plan(ctx, h.in_off.data(), n, &g->back);
  if (st != ES_OK) {
    es_graph_destroy(g);
    return st;
  }
  *out = g;
  return ES_OK;
}

es_status es_graph_destroy(es_graph* g) {
  if (!g) return ES_EINVAL;
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(g->out_off);
  (void)hipFree(g->out_idx);
  (void)hipFree(g->in_off);
  (void)hipFree(g->in_idx);
  (void)hipFree(g->walk_adj);
  (void)hipFree(g->inv_din);
  (void)hipFree(g->din_int);
  (void)hipFree(g->din_ext);
  (void)hipFree(g->dout_ext);
  (void)hipFree(g->ext_of);
  (void)hipFree(g->int_of);
  (void)hipFree(g->vhat);
  (void)hipFree(g->lde_n1);
  (void)hipFree(g->lde_g);
  free_plan(&g->fwd);
  free_plan(&g->back);
  delete g;
  return ES_OK;
}

es_status es_graph_info(const es_graph* g, int32_t* n, int64_t* m) {
  if (!g) return ES_EINVAL;
  if (n) *n = g->n;
  if (m) *m = g->m;
  return ES_OK;
}

}  // extern "C"
