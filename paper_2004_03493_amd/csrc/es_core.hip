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
  (void)hipFree(plan->blocks);
  (void)hipFree(plan->long_p0);
  (void)hipFree(plan->long_nch);
  (void)hipFree(plan->counters);
  (void)hipFree(plan->partials);
  *plan = SpmvPlan{};
}

// Degree-ordered relabelling and the two CSR copies under internal ids.
// keys: edges (src << 32 | dst) in external ids, sorted ascending.
struct HostLayout {
  std::vector<int32_t> din_ext, dout_ext, ext_of, int_of;
  std::vector<int32_t> out_off, out_idx, in_off, in_idx, din_int;
  std::vector<double> inv_din;
};

static void build_layout(const std::vector<uint64_t>& keys, int32_t n, HostLayout& h) {
  const size_t m = keys.size();
  h.din_ext.assign(n, 0);
  h.dout_ext.assign(n, 0);
  for (uint64_t k : keys) {
    h.dout_ext[k >> 32]++;
    h.din_ext[k & 0xffffffffu]++;
  }
  // internal id = rank by total degree, descending, ties by external id
  h.ext_of.resize(n);
  for (int32_t v = 0; v < n; ++v) h.ext_of[v] = v;
  std::stable_sort(h.ext_of.begin(), h.ext_of.end(), [&](int32_t a, int32_t b) {
    return (int64_t)h.din_ext[a] + h.dout_ext[a] > (int64_t)h.din_ext[b] + h.dout_ext[b];
  });
  h.int_of.resize(n);
  for (int32_t i = 0; i < n; ++i) h.int_of[h.ext_of[i]] = i;
  // out-CSR: internal rows, internal columns ascending
  h.out_off.assign((size_t)n + 1, 0);
  for (int32_t i = 0; i < n; ++i) h.out_off[i + 1] = h.out_off[i] + h.dout_ext[h.ext_of[i]];
  h.out_idx.resize(m);
  {
    std::vector<int32_t> pos(h.out_off.begin(), h.out_off.end() - 1);
    for (uint64_t k : keys) {
      const int32_t r = h.int_of[k >> 32];
      h.out_idx[pos[r]++] = h.int_of[k & 0xffffffffu];
    }
    for (int32_t i = 0; i < n; ++i) std::sort(h.out_idx.begin() + h.out_off[i], h.out_idx.begin() + h.out_off[i + 1]);
  }
  // in-CSR: internal rows; a stable pass over keys sorted by external source
  // keeps every row in ascending external source order (the walk's order)
  h.in_off.assign((size_t)n + 1, 0);
  h.din_int.resize(n);
  h.inv_din.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t d = h.din_ext[h.ext_of[i]];
    h.din_int[i] = d;
    h.inv_din[i] = d > 0 ? 1.0 / (double)d : 0.0;
    h.in_off[i + 1] = h.in_off[i] + d;
  }
  h.in_idx.resize(m);
  {
    std::vector<int32_t> pos(h.in_off.begin(), h.in_off.end() - 1);
    for (uint64_t k : keys) {
      const int32_t r = h.int_of[k & 0xffffffffu];
      h.in_idx[pos[r]++] = h.int_of[k >> 32];
    }
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
  es_graph* g = new (std::nothrow) es_graph();
  if (!g) return fail(ctx, ES_ENOMEM, "graph handle");
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
  (void)hipFree(g->inv_din);
  (void)hipFree(g->din_int);
  (void)hipFree(g->din_ext);
  (void)hipFree(g->dout_ext);
  (void)hipFree(g->ext_of);
  (void)hipFree(g->int_of);
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
