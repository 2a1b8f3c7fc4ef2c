// Public entry points for the steps of a query and the whole query.
#include <algorithm>
#include <cmath>
#include <vector>

#include "es_internal.h"

namespace es {
namespace {

__global__ void permute_rows_kernel(int32_t n, const double* __restrict__ src, const int32_t* __restrict__ map,
                                    double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t row = (int64_t)blockIdx.y * n;
  dst[row + i] = src[row + map[i]];
}

bool valid_c(double c) { return c > 0.0 && c <= 0.99; }

}  // namespace

es_status launch_permute_f64(es_ctx* ctx, int32_t n, int32_t rows, const double* src, const int32_t* map,
                             double* dst) {
  if (n <= 0 || rows <= 0) return ES_OK;
  for (int32_t r0 = 0; r0 < rows; r0 += 65535) {
    const int32_t nr = std::min<int32_t>(65535, rows - r0);
    dim3 grid(ceil_div(n, 256), nr);
    permute_rows_kernel<<<grid, 256, 0, ctx->stream>>>(n, src + (int64_t)r0 * n, map, dst + (int64_t)r0 * n);
  }
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

}  // namespace es

using namespace es;

extern "C" {

es_status es_graph_degrees(es_ctx* ctx, const es_graph* g, int32_t* din, int32_t* dout) {
  if (!ctx || !g) return ES_EINVAL;
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  if (din) ES_CHECK_HIP(ctx, hipMemcpyAsync(din, g->din_ext, 4 * (size_t)g->n, hipMemcpyDeviceToDevice, ctx->stream));
  if (dout)
    ES_CHECK_HIP(ctx, hipMemcpyAsync(dout, g->dout_ext, 4 * (size_t)g->n, hipMemcpyDeviceToDevice, ctx->stream));
  return ES_OK;
}

es_status es_forward(es_ctx* ctx, const es_graph* g, int32_t u, double c, int32_t L, double* levels, double* pi) {
  if (!ctx || !g) return ES_EINVAL;
  if (u < 0 || u >= g->n) return fail(ctx, ES_EINVAL, "source %d outside [0, %d)", u, g->n);
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  if (L < 0 || !levels || !pi) return fail(ctx, ES_EINVAL, "bad L or null output");
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  es_status st;
  const int32_t n = g->n;
  auto* q0 = (int64_t*)workspace(ctx, kWsQ0, sizeof(int64_t) * (size_t)n, &st);
  if (!q0) return st;
  auto* q1 = (int64_t*)workspace(ctx, kWsQ1, sizeof(int64_t) * (size_t)n, &st);
  if (!q1) return st;
  auto* lv = (double*)workspace(ctx, kWsLevels, sizeof(double) * (size_t)(L + 1) * n, &st);
  if (!lv) return st;
  auto* pii = (double*)workspace(ctx, kWsPi, sizeof(double) * (size_t)n, &st);
  if (!pii) return st;
  ES_TRY(launch_forward(ctx, g, g->h_int_of[u], c, L, lv, pii, q0, q1));
  ES_TRY(launch_permute_f64(ctx, n, L + 1, lv, g->int_of, levels));
  return launch_permute_f64(ctx, n, 1, pii, g->int_of, pi);
}

es_status es_sparse_capacity(int32_t n, int64_t m, int32_t L, double c, double sparse_eps, int64_t* cap) {
  if (!cap || n < 0 || m < 0 || L < 0) return ES_EINVAL;
  if (!valid_c(c) || !(sparse_eps > 0.0 && sparse_eps < 1.0)) return ES_EINVAL;
  const double sc = std::sqrt(c);
  *cap = (int64_t)sparse_capacity(n, m, L, (1.0 - sc) * (1.0 - sc) * sparse_eps);
  return ES_OK;
}

es_status es_forward_sparse(es_ctx* ctx, const es_graph* g, int32_t u, double c, int32_t L, double sparse_eps,
                            int64_t cap, int32_t* idx, double* val, uint64_t* counts, double* pi) {
  if (!ctx || !g) return ES_EINVAL;
  if (u < 0 || u >= g->n) return fail(ctx, ES_EINVAL, "source %d outside [0, %d)", u, g->n);
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  if (L < 0 || !counts) return fail(ctx, ES_EINVAL, "bad L or null counts");
  if (!(sparse_eps > 0.0 && sparse_eps < 1.0)) return fail(ctx, ES_EINVAL, "sparse_eps=%g outside (0, 1)", sparse_eps);
  if (cap < 0 || (cap > 0 && (!idx || !val))) return fail(ctx, ES_EINVAL, "bad capacity or null list");
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  es_status st;
  const int32_t n = g->n;
  auto* q0 = (int64_t*)workspace(ctx, kWsQ0, sizeof(int64_t) * (size_t)n, &st);
  if (!q0) return st;
  auto* q1 = (int64_t*)workspace(ctx, kWsQ1, sizeof(int64_t) * (size_t)n, &st);
  if (!q1) return st;
  auto* lv = (double*)workspace(ctx, kWsLevels, sizeof(double) * (size_t)n, &st);
  if (!lv) return st;
  auto* pii = (double*)workspace(ctx, kWsPi, sizeof(double) * (size_t)n, &st);
  if (!pii) return st;
  auto* cnt = (unsigned long long*)workspace(ctx, kWsSpCnt, sizeof(uint64_t) * (size_t)(L + 2), &st);
  if (!cnt) return st;
  const double sc = std::sqrt(c);
  SparseLevels sp{(1.0 - sc) * (1.0 - sc) * sparse_eps, 0, idx, val, cnt, (uint64_t)cap};
  ES_TRY(launch_forward(ctx, g, g->h_int_of[u], c, L, lv, pii, q0, q1, &sp));
  ES_TRY(launch_sparse_ids(ctx, g, L, sp));
  if (pi) ES_TRY(launch_permute_f64(ctx, n, 1, pii, g->int_of, pi));
  std::vector<uint64_t> h((size_t)L + 2);
  ES_CHECK_HIP(ctx, hipMemcpyAsync(h.data(), cnt, 8 * h.size(), hipMemcpyDeviceToHost, ctx->stream));
  ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int32_t l = 0; l <= L; ++l) counts[l] = h[l];
  if (h[L + 1] > (uint64_t)cap)
    return fail(ctx, ES_EOVERFLOW, "%llu entries above the threshold, capacity %lld", (unsigned long long)h[L + 1],
                (long long)cap);
  return ES_OK;
}

es_status es_budget(es_ctx* ctx, const es_graph* g, const double* pi, double R, int32_t alloc,
                    int32_t exact_small_din, uint64_t* Rk, uint64_t* total) {
  if (!ctx || !g || !pi || !Rk) return ES_EINVAL;
  if (!(R > 0.0)) return fail(ctx, ES_EINVAL, "R=%g must be positive", R);
  if (alloc != ES_ALLOC_PI2 && alloc != ES_ALLOC_PI && alloc != ES_ALLOC_LEARNED)
    return fail(ctx, ES_EINVAL, "unknown allocation %d", alloc);
  if (alloc == ES_ALLOC_LEARNED)
    return fail(ctx, ES_EINVAL, "learned allocation runs inside es_single_source after es_mlp_load");
  // sum_k ceil(R pi(k)^2) <= R sum pi^2 + n <= R + n, since sum_k pi(k) <= 1
  if (R + (double)g->n >= 9.2e18) return fail(ctx, ES_EOVERFLOW, "R=%g: sample count may reach 2^63", R);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  ES_TRY(launch_budget(ctx, g, pi, g->din_ext, R, alloc, exact_small_din, nullptr, 0.0, Rk));
  if (total) {
    std::vector<uint64_t> h((size_t)g->n);
    ES_CHECK_HIP(ctx, hipMemcpyAsync(h.data(), Rk, 8 * h.size(), hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    uint64_t s = 0;
    for (uint64_t v : h) s += v;
    *total = s;
  }
  return ES_OK;
}

es_status es_walk_pairs(es_ctx* ctx, const es_graph* g, const uint64_t* r_begin, const uint64_t* r_end,
                        uint64_t seed, double c, uint64_t* M) {
  if (!ctx || !g || !r_end || !M) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  WalkTotals* tot = nullptr;
  ES_TRY(launch_walks(ctx, g, r_begin, r_end, seed, c, M, true, &tot));
  WalkTotals h;
  ES_CHECK_HIP(ctx, hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h.overflow) return fail(ctx, ES_EOVERFLOW, "sample count reaches 2^63");
  return ES_OK;
}

es_status es_walk_pairs_lde(es_ctx* ctx, const es_graph* g, const uint64_t* r_begin, const uint64_t* r_end,
                            const int32_t* ell, uint64_t seed, double c, uint64_t* M) {
  if (!ctx || !g || !r_end || !ell || !M) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  WalkTotals* tot = nullptr;
  ES_TRY(launch_walks(ctx, g, r_begin, r_end, seed, c, M, true, &tot, ell));
  WalkTotals h;
  ES_CHECK_HIP(ctx, hipMemcpyAsync(&h, tot, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h.overflow) return fail(ctx, ES_EOVERFLOW, "sample count reaches 2^63");
  return ES_OK;
}

es_status es_diag(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, const uint64_t* M, double c,
                  int32_t exact_small_din, double* D) {
  if (!ctx || !g || !Rk || !M || !D) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  return launch_diag(ctx, g, Rk, M, g->din_ext, c, exact_small_din, D);
}

es_status es_backward(es_ctx* ctx, const es_graph* g, const double* levels, int32_t L, const double* D, double c,
                      double* s) {
  if (!ctx || !g || !levels || !D || !s) return ES_EINVAL;
  if (L < 0) return fail(ctx, ES_EINVAL, "L=%d", L);
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  es_status st;
  const int32_t n = g->n;
  auto* lv = (double*)workspace(ctx, kWsLevels, sizeof(double) * (size_t)(L + 1) * n, &st);
  if (!lv) return st;
  auto* Di = (double*)workspace(ctx, kWsD, sizeof(double) * (size_t)n, &st);
  if (!Di) return st;
  auto* s0 = (double*)workspace(ctx, kWsS0, sizeof(double) * (size_t)n, &st);
  if (!s0) return st;
  auto* tmp = (double*)workspace(ctx, kWsS1, sizeof(double) * (size_t)n, &st);
  if (!tmp) return st;
  ES_TRY(launch_permute_f64(ctx, n, L + 1, levels, g->ext_of, lv));
  ES_TRY(launch_permute_f64(ctx, n, 1, D, g->ext_of, Di));
  ES_TRY(launch_backward(ctx, g, lv, L, Di, c, s0, tmp));
  return launch_permute_f64(ctx, n, 1, s0, g->int_of, s);
}

es_status es_single_source(es_ctx* ctx, const es_graph* g, int32_t u, const es_query_opts* o, double* s_out,
                           es_stats* stats) {
  if (!ctx || !g || !o || !s_out) return ES_EINVAL;
  if (u < 0 || u >= g->n) return fail(ctx, ES_EINVAL, "source %d outside [0, %d)", u, g->n);
  if (!valid_c(o->c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", o->c);
  if (!(o->eps > 0.0 && o->eps < 1.0)) return fail(ctx, ES_EINVAL, "eps=%g outside (0, 1)", o->eps);
  if (!(o->r_scale > 0.0)) return fail(ctx, ES_EINVAL, "r_scale=%g must be positive", o->r_scale);
  if (o->alloc != ES_ALLOC_PI2 && o->alloc != ES_ALLOC_PI && o->alloc != ES_ALLOC_LEARNED)
    return fail(ctx, ES_EINVAL, "unknown allocation %d", o->alloc);
  if (o->alloc == ES_ALLOC_LEARNED && !ctx->mlp_w)
    return fail(ctx, ES_EINVAL, "learned allocation requested but no network loaded");
  if (o->alloc == ES_ALLOC_LEARNED && !(o->v_floor_ratio >= 0.0 && o->v_floor_ratio <= 1.0))
    return fail(ctx, ES_EINVAL, "v_floor_ratio=%g outside [0, 1]", o->v_floor_ratio);
  if (o->lde < 0 || o->lde > 2) return fail(ctx, ES_EINVAL, "lde=%d outside 0..2", o->lde);
  if (!(o->sparse_eps >= 0.0 && o->sparse_eps < 1.0))
    return fail(ctx, ES_EINVAL, "sparse_eps=%g outside [0, 1)", o->sparse_eps);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  const int32_t n = g->n;
  const int32_t L = num_levels(o->c, o->eps);
  const double R = total_samples(n, o->c, o->eps, o->r_scale);
  if (!o->d_override && R + (double)n >= 9.2e18)
    return fail(ctx, ES_EOVERFLOW, "R=%g: sample count may reach 2^63", R);
  es_status st;
  const bool sparse = o->sparse_eps > 0.0;
  SparseLevels sp{};
  int32_t dense_slots = L + 1;
  if (sparse) {
    const double sc = std::sqrt(o->c);
    sp.theta = (1.0 - sc) * (1.0 - sc) * o->sparse_eps;
    sp.nkeep = 0;
    sp.cap = sparse_capacity(n, g->m, L, sp.theta);
    dense_slots = std::min(L + 1, sp.nkeep + 1);
    sp.idx = (int32_t*)workspace(ctx, kWsSpIdx, sizeof(int32_t) * (size_t)sp.cap, &st);
    if (!sp.idx) return st;
    sp.val = (double*)workspace(ctx, kWsSpVal, sizeof(double) * (size_t)sp.cap, &st);
    if (!sp.val) return st;
    sp.cnt = (unsigned long long*)workspace(ctx, kWsSpCnt, sizeof(uint64_t) * (size_t)(L + 2), &st);
    if (!sp.cnt) return st;
  }
  const SparseLevels* spp = sparse ? &sp : nullptr;
  auto* levels = (double*)workspace(ctx, kWsLevels, sizeof(double) * (size_t)dense_slots * n, &st);
  if (!levels) return st;
  auto* pi = (double*)workspace(ctx, kWsPi, sizeof(double) * (size_t)n, &st);
  if (!pi) return st;
  auto* q0 = (int64_t*)workspace(ctx, kWsQ0, sizeof(int64_t) * (size_t)n, &st);
  if (!q0) return st;
  auto* q1 = (int64_t*)workspace(ctx, kWsQ1, sizeof(int64_t) * (size_t)n, &st);
  if (!q1) return st;
  auto* stmp = (double*)workspace(ctx, kWsS1, sizeof(double) * (size_t)n, &st);
  if (!stmp) return st;
  auto* sint = (double*)workspace(ctx, kWsS0, sizeof(double) * (size_t)n, &st);
  if (!sint) return st;
  auto* Dh = (double*)workspace(ctx, kWsD, sizeof(double) * (size_t)n, &st);
  if (!Dh) return st;
  hipEvent_t* ev = ctx->ev;
  ES_CHECK_HIP(ctx, hipEventRecord(ev[0], ctx->stream));
  ES_TRY(launch_forward(ctx, g, g->h_int_of[u], o->c, L, levels, pi, q0, q1, spp));
  ES_CHECK_HIP(ctx, hipEventRecord(ev[1], ctx->stream));
  WalkTotals* tot = nullptr;
  int32_t lde_level = 0;
  double lde_zsum = 0.0;
  if (!o->d_override) {
    auto* Rk = (uint64_t*)workspace(ctx, kWsRk, sizeof(uint64_t) * (size_t)n, &st);
    if (!Rk) return st;
    auto* M = (uint64_t*)workspace(ctx, kWsM, sizeof(uint64_t) * (size_t)n, &st);
    if (!M) return st;
    if (o->alloc == ES_ALLOC_LEARNED)
      ES_TRY(launch_learned_budget(ctx, g, pi, R, o->c, o->exact_small_din, o->v_floor_ratio, Rk));
    else
      ES_TRY(launch_budget(ctx, g, pi, g->din_int, R, o->alloc, o->exact_small_din, nullptr, 0.0, Rk));
    const uint64_t* Rwalk = Rk;
    LdeOut lo{nullptr, nullptr, nullptr};
    if (o->lde) {
      // Algorithm 3: exact first levels, then non-stop pairs on R'(k)
      lo.ell = (int32_t*)workspace(ctx, kWsLdeEll, sizeof(int32_t) * (size_t)n, &st);
      if (!lo.ell) return st;
      lo.zsum = (double*)workspace(ctx, kWsLdeZ, sizeof(double) * (size_t)n, &st);
      if (!lo.zsum) return st;
      lo.Rk2 = (uint64_t*)workspace(ctx, kWsLdeR, sizeof(uint64_t) * (size_t)n, &st);
      if (!lo.Rk2) return st;
      ES_TRY(launch_lde(ctx, g, Rk, o->c, o->lde, o->lde_max_level, lo));
      if (stats) {
        ES_CHECK_HIP(ctx, hipMemcpy(&lde_level, lo.ell + g->h_int_of[u], 4, hipMemcpyDeviceToHost));
        ES_CHECK_HIP(ctx, hipMemcpy(&lde_zsum, lo.zsum + g->h_int_of[u], 8, hipMemcpyDeviceToHost));
      }
      Rwalk = lo.Rk2;
    }
    ctx->ev_walk_begin = ev[2];  // recorded between the sample-space scan and the walk kernel
    const es_status ws = launch_walks(ctx, g, nullptr, Rwalk, o->seed, o->c, M, false, &tot, lo.ell);
    ctx->ev_walk_begin = nullptr;
    ES_TRY(ws);
    ES_CHECK_HIP(ctx, hipEventRecord(ev[3], ctx->stream));
    if (o->lde)
      ES_TRY(launch_diag_lde(ctx, n, Rwalk, M, lo.ell, lo.zsum, g->din_int, o->c, o->exact_small_din, Dh));
    else
      ES_TRY(launch_diag(ctx, g, Rk, M, g->din_int, o->c, o->exact_small_din, Dh));
    ES_CHECK_HIP(ctx, hipEventRecord(ev[4], ctx->stream));
  } else {
    ES_CHECK_HIP(ctx, hipEventRecord(ev[2], ctx->stream));
    ES_CHECK_HIP(ctx, hipEventRecord(ev[3], ctx->stream));
    ES_TRY(launch_permute_f64(ctx, n, 1, o->d_override, g->ext_of, Dh));
    ES_CHECK_HIP(ctx, hipEventRecord(ev[4], ctx->stream));
  }
  ES_TRY(launch_backward(ctx, g, levels, L, Dh, o->c, sint, stmp, spp));
  ES_TRY(launch_permute_f64(ctx, n, 1, sint, g->int_of, s_out));
  ES_CHECK_HIP(ctx, hipEventRecord(ev[5], ctx->stream));
  if (stats) {
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    es_stats s{};
    s.L = L;
    s.R = R;
    if (tot) {
      WalkTotals h;
      ES_CHECK_HIP(ctx, hipMemcpy(&h, tot, sizeof(h), hipMemcpyDeviceToHost));
      s.pairs = h.total;
      s.pairs_requested = h.total;
      s.active_nodes = h.n_active;
      s.meets = h.meets;
      s.philox_blocks = h.blocks;
      s.walk_steps = h.steps;
    }
    ES_CHECK_HIP(ctx, hipEventElapsedTime(&s.ms_forward, ev[0], ev[1]));
    ES_CHECK_HIP(ctx, hipEventElapsedTime(&s.ms_budget, ev[1], ev[2]));
    ES_CHECK_HIP(ctx, hipEventElapsedTime(&s.ms_walk, ev[2], ev[3]));
    ES_CHECK_HIP(ctx, hipEventElapsedTime(&s.ms_diag, ev[3], ev[4]));
    ES_CHECK_HIP(ctx, hipEventElapsedTime(&s.ms_backward, ev[4], ev[5]));
    s.lde_source_level = lde_level;
    s.lde_source_zsum = lde_zsum;
    if (sparse) {
      unsigned long long kept = 0;
      ES_CHECK_HIP(ctx, hipMemcpy(&kept, sp.cnt + L + 1, sizeof(kept), hipMemcpyDeviceToHost));
      if (kept > sp.cap)
        return fail(ctx, ES_EOVERFLOW, "%llu entries above the threshold, capacity %llu", kept,
                    (unsigned long long)sp.cap);
      s.level_entries = kept;
      s.level_bytes = 12ull * kept + 8ull * (uint64_t)dense_slots * (uint64_t)n;
    } else {
      s.level_entries = (uint64_t)(L + 1) * (uint64_t)n;
      s.level_bytes = 8ull * s.level_entries;
    }
    s.workspace_bytes = workspace_total(ctx);
    *stats = s;
  }
  return ES_OK;
}

}  // extern "C"
