// Context, graph construction and host-side constants of libexactsim.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>

#include "es_internal.h"

namespace es {

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
  if (e == hipErrorOutOfMemory) return fail(ctx, ES_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(ctx, ES_EDEVICE, "%s: %s", what, hipGetErrorString(e));
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
      hipStreamSynchronize(ctx->stream);
      hipFree(ctx->ws[slot]);
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
  ES_CHECK_HIP(ctx, hipMemcpyAsync(ctx->thr, thr.data(), sizeof(uint64_t) * (tmax + 1), hipMemcpyHostToDevice,
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
  hipFree(plan->blocks);
  hipFree(plan->long_p0);
  hipFree(plan->long_nch);
  hipFree(plan->counters);
  hipFree(plan->partials);
  *plan = SpmvPlan{};
}

// Build CSR (offsets, column ids ascending within each row) of the edge keys
// (row << 32 | col) that are already sorted: the out-CSR directly.
static void csr_from_sorted(const std::vector<uint64_t>& keys, int32_t n, std::vector<int32_t>& off,
                            std::vector<int32_t>& idx) {
  off.assign((size_t)n + 1, 0);
  idx.resize(keys.size());
  for (size_t e = 0; e < keys.size(); ++e) {
    off[(keys[e] >> 32) + 1]++;
    idx[e] = (int32_t)(keys[e] & 0xffffffffu);
  }
  for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
}

// Transpose with a stable counting sort: rows of the result list their
// columns in ascending order because the input is sorted by (row, col).
static void csr_transpose(const std::vector<uint64_t>& keys, int32_t n, std::vector<int32_t>& off,
                          std::vector<int32_t>& idx) {
  off.assign((size_t)n + 1, 0);
  idx.resize(keys.size());
  for (size_t e = 0; e < keys.size(); ++e) off[(keys[e] & 0xffffffffu) + 1]++;
  for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  std::vector<int32_t> pos(off.begin(), off.end() - 1);
  for (size_t e = 0; e < keys.size(); ++e) {
    const uint32_t col = (uint32_t)(keys[e] & 0xffffffffu);
    idx[pos[col]++] = (int32_t)(keys[e] >> 32);
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
  *out = ctx;
  return ES_OK;
}

es_status es_ctx_destroy(es_ctx* ctx) {
  if (!ctx) return ES_EINVAL;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (void* p : ctx->ws) hipFree(p);
  hipFree(ctx->thr);
  hipFree(ctx->mlp_w);
  for (auto& e : ctx->ev)
    if (e) hipEventDestroy(e);
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
    keys.reserve((size_t)m);
  } catch (...) {
    return fail(ctx, ES_ENOMEM, "host edge buffer");
  }
  bool sorted = true;
  for (int64_t e = 0; e < m; ++e) {
    const int32_t s = src[e], d = dst[e];
    if (s < 0 || s >= n || d < 0 || d >= n)
      return fail(ctx, ES_EINVAL, "edge %lld (%d -> %d) outside [0, %d)", (long long)e, s, d, n);
    if ((flags & ES_DROP_SELF_LOOPS) && s == d) continue;
    const uint64_t key = ((uint64_t)(uint32_t)s << 32) | (uint32_t)d;
    if (!keys.empty() && key <= keys.back()) sorted = false;
    keys.push_back(key);
  }
  if (!sorted) std::sort(keys.begin(), keys.end());
  if (flags & ES_DEDUP) keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  std::vector<int32_t> out_off, out_idx, in_off, in_idx;
  csr_from_sorted(keys, n, out_off, out_idx);
  csr_transpose(keys, n, in_off, in_idx);
  std::vector<double> inv((size_t)n);
  for (int32_t v = 0; v < n; ++v) {
    const int32_t d = in_off[v + 1] - in_off[v];
    inv[v] = d > 0 ? 1.0 / (double)d : 0.0;
  }
  es_graph* g = new (std::nothrow) es_graph();
  if (!g) return fail(ctx, ES_ENOMEM, "graph handle");
  g->device = ctx->device;
  g->n = n;
  g->m = (int64_t)keys.size();
  std::vector<uint64_t>().swap(keys);
  auto up = [&](void** dptr, const void* host, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dptr, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) return e;
    if (bytes) e = hipMemcpy(*dptr, host, bytes, hipMemcpyHostToDevice);
    return e;
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up((void**)&g->out_off, out_off.data(), 4 * out_off.size());
  if (e == hipSuccess) e = up((void**)&g->out_idx, out_idx.data(), 4 * out_idx.size());
  if (e == hipSuccess) e = up((void**)&g->in_off, in_off.data(), 4 * in_off.size());
  if (e == hipSuccess) e = up((void**)&g->in_idx, in_idx.data(), 4 * in_idx.size());
  if (e == hipSuccess) e = up((void**)&g->inv_din, inv.data(), 8 * inv.size());
  if (e != hipSuccess) {
    es_graph_destroy(g);
    return hip_fail(ctx, e, "graph upload");
  }
  es_status st = build_plan(ctx, out_off.data(), n, &g->fwd);
  if (st == ES_OK) st = build_plan(ctx, in_off.data(), n, &g->back);
  if (st != ES_OK) {
    es_graph_destroy(g);
    return st;
  }
  *out = g;
  return ES_OK;
}

es_status es_graph_destroy(es_graph* g) {
  if (!g) return ES_EINVAL;
  hipSetDevice(g->device);
  hipDeviceSynchronize();
  hipFree(g->out_off);
  hipFree(g->out_idx);
  hipFree(g->in_off);
  hipFree(g->in_idx);
  hipFree(g->inv_din);
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
