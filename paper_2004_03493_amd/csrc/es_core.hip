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
    WalkEntry w{};
    w.key = d > 0 ? o : -1 - v;
    w.deg = d;
    adj[e] = w;
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
  for (int q = 0; q < 16; ++q) ctx->thr_head[q] = thr[q + 1];
  ctx->tmax = tmax;
  ctx->thr_c = c;
  return ES_OK;
}

es_status build_plan(es_ctx* ctx, const int32_t* off, int32_t n, SpmvPlan* plan) {
  SpmvPartition part;
  try {
    spmv_partition(off, n, part);
  } catch (...) {
    return fail(ctx, ES_ENOMEM, "SpMV partition");
  }
  const std::vector<BlockDesc>& all = part.blocks;
  const std::vector<int32_t>& long_p0 = part.long_p0;
  const std::vector<int32_t>& long_nch = part.long_nch;
  const int32_t nslots = part.nslots;
  const int32_t maxnnz = part.max_row_nnz;
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

es_status build_binned_plan(es_ctx* ctx, const int32_t* off, const int32_t* idx, int32_t n, int32_t shift,
                            size_t row_bytes, BinnedPlan* plan) {
  BinnedLayout b;
  try {
    build_binned(off, idx, n, shift, b);
  } catch (...) {
    return fail(ctx, ES_ENOMEM, "binned level layout");
  }
  *plan = BinnedPlan{};
  plan->shift = shift;
  plan->nbins = b.nbins;
  plan->nranges = (int32_t)b.ranges.size();
  plan->nitems = (int32_t)b.items.size();
  plan->nsplits = (int32_t)b.splits.size();
  plan->nslots = b.nslots;
  auto up = [&](void** dptr, const void* host, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dptr, std::max<size_t>(bytes, 8));
    if (e != hipSuccess) return e;
    if (bytes) e = hipMemcpy(*dptr, host, bytes, hipMemcpyHostToDevice);
    return e;
  };
  hipError_t e = up((void**)&plan->ranges, b.ranges.data(), sizeof(BinRange) * b.ranges.size());
  if (e == hipSuccess) e = up((void**)&plan->src_local, b.src_local.data(), 2 * b.src_local.size());
  if (e == hipSuccess) e = up((void**)&plan->pos, b.pos.data(), 4 * b.pos.size());
  if (e == hipSuccess) e = up((void**)&plan->row_local, b.row_local.data(), 2 * b.row_local.size());
  if (e == hipSuccess) e = up((void**)&plan->items, b.items.data(), sizeof(BinItem) * b.items.size());
  if (e == hipSuccess) e = up((void**)&plan->splits, b.splits.data(), sizeof(BinSplit) * b.splits.size());
  if (e == hipSuccess)
    e = hipMalloc(&plan->partials, std::max<size_t>(8, (size_t)b.nslots * ((size_t)1 << shift) * row_bytes));
  if (e != hipSuccess) {
    free_binned_plan(plan);
    return hip_fail(ctx, e, "binned level layout upload");
  }
  return ES_OK;
}

void free_binned_plan(BinnedPlan* plan) {
  (void)hipFree(plan->ranges);
  (void)hipFree(plan->src_local);
  (void)hipFree(plan->pos);
  (void)hipFree(plan->row_local);
  (void)hipFree(plan->items);
  (void)hipFree(plan->splits);
  (void)hipFree(plan->partials);
  *plan = BinnedPlan{};
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
  if ((flags & ES_LEVELS_PULL) && (flags & ES_LEVELS_BINNED))
    return fail(ctx, ES_EINVAL, "ES_LEVELS_PULL and ES_LEVELS_BINNED together");
  if (flags & ~(uint32_t)(ES_DEDUP | ES_DROP_SELF_LOOPS | ES_LEVELS_PULL | ES_LEVELS_BINNED))
    return fail(ctx, ES_EINVAL, "unknown flags 0x%x", flags);
  if (m > 0 && (!src || !dst)) return fail(ctx, ES_EINVAL, "null edge array");
  std::vector<uint64_t> keys;
  int64_t bad = -1;
  try {
    if (!pack_edges(n, m, src, dst, (flags & ES_DROP_SELF_LOOPS) != 0, (flags & ES_DEDUP) != 0, keys, &bad))
      return fail(ctx, ES_EINVAL, "edge %lld (%d -> %d) outside [0, %d)", (long long)bad, src[bad], dst[bad], n);
  } catch (...) {
    return fail(ctx, ES_ENOMEM, "host edge buffer");
  }
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
  g->binned = (flags & ES_LEVELS_BINNED) || (!(flags & ES_LEVELS_PULL) && n >= kBinnedAutoNodes);
  if (st == ES_OK && g->binned) {
    st = build_binned_plan(ctx, h.in_off.data(), h.in_idx.data(), n, kBinShiftFwd, 8, &g->bfwd);
    if (st == ES_OK) st = build_binned_plan(ctx, h.out_off.data(), h.out_idx.data(), n, kBinShiftBack, 16, &g->bback);
    if (st == ES_OK) {
      const hipError_t he = hipMalloc(&g->bin_vals, 8 * std::max<size_t>(1, (size_t)g->m));
      if (he != hipSuccess) st = hip_fail(ctx, he, "binned level values");
    }
  }
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
  free_binned_plan(&g->bfwd);
  free_binned_plan(&g->bback);
  (void)hipFree(g->bin_vals);
  delete g;
  return ES_OK;
}

es_status es_graph_level_pass(const es_graph* g, int32_t* binned) {
  if (!g || !binned) return ES_EINVAL;
  *binned = g->binned ? 1 : 0;
  return ES_OK;
}

es_status es_graph_info(const es_graph* g, int32_t* n, int64_t* m) {
  if (!g) return ES_EINVAL;
  if (n) *n = g->n;
  if (m) *m = g->m;
  return ES_OK;
}

}  // extern "C"
