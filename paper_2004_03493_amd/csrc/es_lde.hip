// Local deterministic exploitation for D(k,k) (Section 3.3, Algorithm 3,
// Lemma 4).
//
// Z_l(k) is the probability that two sqrt(c)-walks from v_k first meet at
// their l-th step; D(k,k) = 1 - sum_l Z_l(k).  Algorithm 3 computes the first
// l(k) terms exactly and estimates the rest with pairs that do not stop
// during their first l(k) steps:
//   D^(k,k) = (1 - sum_{l <= l(k)} Z_l(k)) - c^l(k) M(k) / R'(k).
//
// Summing Lemma 4 over the meeting node gives Z_l in terms of collision
// numbers C_m(x) = sum_q (P^T)^m(x, q)^2 (the probability that two walks
// from x that never stop share a node at step m; C_1(x) = 1/d_in(x)):
//   Z_1(k) = c C_1(k),
//   Z_2(k) = c^2 (C_2(k) - d_in(k)^-2 sum_{a in I(k)} C_1(a)),
//   Z_3(k) = c^3 (C_3(k) - sum_q (P^T)^2(k, q)^2 C_1(q)
//                 + d_in(k)^-2 sum_{a in I(k)} d_in(a)^-2 sum_{q in I(a)} C_1(q)
//                 - d_in(k)^-2 sum_{a in I(k)} C_2(a)).
// For the query source u the forward levels already hold the walk
// distributions: (P^T)^m(u, .) = pi^m / ((1 - sqrt c) sqrt(c)^m), so C_m(u)
// and the second term of Z_3 are reductions over pi^1..pi^3.  C_2(a) for the
// in-neighbours a of u comes from the two-step distribution of each a,
// accumulated in 2^-62 fixed point (exact integer sums) and squared in fixed
// point.  The source takes l(u) <= 3 levels, every other node l(k) <= 1
// (Z_1 is a closed form), each as far as the edge budget of Algorithm 3
// allows: the deterministic work (in-walks of length <= l from v_k, those of
// length 3 charged at their GPU cost) must stay within 2 R(k) / sqrt(c).
//
// Reductions run over fixed grids in a fixed order, so every result is
// reproducible bit for bit.
#include <cmath>
#include <vector>

#include "es_internal.h"

namespace es {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 512;   // fixed grid of the level reductions
constexpr int kMaxSourceLevel = 3;
// Work charged per three-step in-walk of the source's third level, in walk
// steps: each one is two atomic updates of a node-sized array, measured on
// MI355X at about 2 steps while that array (8n bytes) stays within 128 MiB
// of the Infinity Cache and about 24 once its updates go to HBM.
double level3_path_cost(int32_t n) { return 8.0 * (double)n <= 134217728.0 ? 2.0 : 24.0; }

// Small per-query record on the device (host reads the first part).
struct LdeSource {
  uint64_t Ru;       // R(u)
  int64_t E[3];      // edges traversed up to levels 1, 2, 3
  double A1;         // sum_{a in I(u)} C_1(a)
  double A2;         // sum_{a in I(u)} d_in(a)^-2 sum_{q in I(a)} C_1(q)
  double zsum;       // sum_{l <= l(u)} Z_l(u)
  double Z[4];       // Z_1..Z_3 (index 0 unused)
};

template <int N>
__device__ void block_sum(double (&v)[N], double (*sh)[N]) {
  for (int m = 32; m > 0; m >>= 1)
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], m, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) sh[w][i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double t = 0.0;
      for (int j = 0; j < kRedThreads / 64; ++j) t += sh[j][i];
      v[i] = t;
    }
}

// One block per in-neighbour a = I(u)[blockIdx.x]: sum_{b in I(a)} d_in(b)
// (int64) and sum_{b in I(a)} C_1(b).
__global__ __launch_bounds__(kRedThreads) void source_nb_kernel(int32_t u, const int32_t* __restrict__ in_off,
                                                                const int32_t* __restrict__ in_idx,
                                                                const int32_t* __restrict__ din,
                                                                const double* __restrict__ inv_din,
                                                                long long* __restrict__ deg2,
                                                                double* __restrict__ inv2) {
  __shared__ double sh[kRedThreads / 64][1];
  __shared__ long long shi[kRedThreads / 64];
  const int32_t a = in_idx[in_off[u] + blockIdx.x];
  long long s = 0;
  double r[1] = {0.0};
  for (int32_t e = in_off[a] + (int32_t)threadIdx.x; e < in_off[a + 1]; e += kRedThreads) {
    const int32_t b = in_idx[e];
    s += din[b];
    r[0] += inv_din[b];
  }
  for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
  if ((threadIdx.x & 63) == 0) shi[threadIdx.x >> 6] = s;
  block_sum<1>(r, sh);
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int j = 0; j < kRedThreads / 64; ++j) t += shi[j];
    deg2[blockIdx.x] = t;
    inv2[blockIdx.x] = r[0];
  }
}

// Sequential over the in-neighbours of u, in CSR order.
__global__ void source_costs_kernel(int32_t u, const int32_t* __restrict__ in_off, const int32_t* __restrict__ in_idx,
                                    const int32_t* __restrict__ din, const double* __restrict__ inv_din,
                                    const long long* __restrict__ deg2, const double* __restrict__ inv2,
                                    const uint64_t* __restrict__ Rk, LdeSource* __restrict__ src) {
  const int32_t b = in_off[u], e = in_off[u + 1];
  long long e2 = 0, e3 = 0;
  double a1 = 0.0, a2 = 0.0;
  for (int32_t i = b; i < e; ++i) {
    const int32_t a = in_idx[i];
    const double ia = inv_din[a];
    e2 += din[a];
    e3 += deg2[i - b];
    a1 += ia;
    a2 += (ia * ia) * inv2[i - b];
  }
  src->Ru = Rk[u];
  src->E[0] = e - b;
  src->E[1] = (long long)(e - b) + e2;
  src->E[2] = (long long)(e - b) + e2 + e3;
  src->A1 = a1;
  src->A2 = a2;
}

// Per-block partial sums over n (fixed grid): sum pi^1^2, sum pi^2^2,
// sum pi^3^2, sum pi^2^2 C_1.
__global__ __launch_bounds__(kRedThreads) void level_dots_kernel(int32_t n, const double* __restrict__ lv1,
                                                                 const double* __restrict__ lv2,
                                                                 const double* __restrict__ lv3,
                                                                 const double* __restrict__ inv_din,
                                                                 double* __restrict__ part) {
  __shared__ double sh[kRedThreads / 64][4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t q = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; q < n; q += (int64_t)kRedBlocks * kRedThreads) {
    const double p1 = lv1[q], p2 = lv2[q], p3 = lv3 ? lv3[q] : 0.0;
    v[0] += p1 * p1;
    v[1] += p2 * p2;
    v[2] += p3 * p3;
    v[3] += (p2 * p2) * inv_din[q];
  }
  block_sum<4>(v, sh);
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) part[blockIdx.x * 4 + i] = v[i];
}

// Two-step distribution of the origin a = I(u)[o]: W[q] += Q(C_1(a) C_1(b))
// for every in-walk a -> b -> q.  Rows b with many in-neighbours are swept by
// the whole grid, the others by one wave each.
constexpr int32_t kWideRow = 1024;

template <class F>
__device__ __forceinline__ void for_two_step(int32_t u, int32_t o, const int32_t* __restrict__ in_off,
                                             const int32_t* __restrict__ in_idx, F f) {
  const int32_t a = in_idx[in_off[u] + o];
  const int32_t b0 = in_off[a], b1 = in_off[a + 1];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  // wide rows: every thread of the grid strides the row
  for (int32_t e = b0; e < b1; ++e) {
    const int32_t b = in_idx[e];
    const int32_t c0 = in_off[b], c1 = in_off[b + 1];
    if (c1 - c0 < kWideRow) continue;
    for (int64_t x = c0 + tid; x < c1; x += nthreads) f(a, b, in_idx[x]);
  }
  // narrow rows: one wave per row
  const int lane = threadIdx.x & 63;
  for (int64_t e = b0 + (tid >> 6); e < b1; e += nthreads >> 6) {
    const int32_t b = in_idx[e];
    const int32_t c0 = in_off[b], c1 = in_off[b + 1];
    if (c1 - c0 >= kWideRow) continue;
    for (int32_t x = c0 + lane; x < c1; x += 64) f(a, b, in_idx[x]);
  }
}

__global__ __launch_bounds__(256) void c2_scatter_kernel(int32_t u, int32_t o, const int32_t* __restrict__ in_off,
                                                         const int32_t* __restrict__ in_idx,
                                                         const double* __restrict__ inv_din,
                                                         unsigned long long* __restrict__ W) {
  for_two_step(u, o, in_off, in_idx, [&](int32_t a, int32_t b, int32_t q) {
    const unsigned long long w = (unsigned long long)(int64_t)rint((inv_din[a] * inv_din[b]) * 0x1p62);
    atomicAdd(&W[q], w);
  });
}

// sum over the distinct q of Q((W[q] 2^-62)^2): each q's value is taken out
// (and W[q] cleared) by the first visit; acc[o] receives the integer sum.
__global__ __launch_bounds__(256) void c2_exchange_kernel(int32_t u, int32_t o, const int32_t* __restrict__ in_off,
                                                          const int32_t* __restrict__ in_idx,
                                                          unsigned long long* __restrict__ W,
                                                          unsigned long long* __restrict__ acc) {
  unsigned long long s = 0;
  for_two_step(u, o, in_off, in_idx, [&](int32_t, int32_t, int32_t q) {
    const unsigned long long v = atomicExch(&W[q], 0ull);
    if (v) {
      const double x = (double)v * 0x1p-62;
      s += (unsigned long long)(int64_t)rint((x * x) * 0x1p62);
    }
  });
  for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(&acc[o], s);
}

__global__ void zero_u64(int64_t n, unsigned long long* __restrict__ p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Z_1..Z_lu of the source and their sum.
__global__ void source_z_kernel(int32_t lu, int32_t du, double c, double sc, const double* __restrict__ part,
                                const unsigned long long* __restrict__ c2acc, const double* __restrict__ inv_din,
                                int32_t u, LdeSource* __restrict__ src) {
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  if (lu >= 2)
    for (int b = 0; b < kRedBlocks; ++b)
      for (int i = 0; i < 4; ++i) S[i] += part[b * 4 + i];
  double A3 = 0.0;
  if (lu >= 3)
    for (int o = 0; o < du; ++o) A3 += (double)c2acc[o] * 0x1p-62;
  // (P^T)^m(u, q) = pi^m(q) / f_m, f_m = (1 - sqrt c) sqrt(c)^m
  const double f0 = 1.0 - sc;
  const double f2 = (f0 * sc) * sc, f3 = f2 * sc;
  const double C2 = S[1] / (f2 * f2);
  const double C3 = S[2] / (f3 * f3);
  const double T2 = S[3] / (f2 * f2);
  const double iu = inv_din[u];
  const double iu2 = iu * iu;
  const double c2 = c * c, c3 = c2 * c;
  double Z[4] = {0.0, c * iu, 0.0, 0.0};
  if (lu >= 2) Z[2] = c2 * (C2 - iu2 * src->A1);
  if (lu >= 3) Z[3] = c3 * (((C3 - T2) + iu2 * src->A2) - iu2 * A3);
  double z = 0.0;
  for (int l = 1; l <= lu; ++l) z += Z[l];
  for (int l = 0; l < 4; ++l) src->Z[l] = Z[l];
  src->zsum = lu > 0 ? z : 0.0;
}

// l(k), sum Z and R'(k) of every node (any id order: din and Rk alike).
__global__ void lde_plan_kernel(int32_t n, const uint64_t* __restrict__ Rk, const int32_t* __restrict__ din,
                                int32_t u, int32_t lu, const LdeSource* __restrict__ src, double c, double sc,
                                int32_t mode, double cl1, double cl2, double cl3, int32_t* __restrict__ ell,
                                double* __restrict__ zsum, uint64_t* __restrict__ Rk2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint64_t r = Rk[k];
  const int32_t d = din[k];
  int32_t l = 0;
  double z = 0.0;
  if (mode == 0) {
    l = 0;
  } else if (k == u) {
    l = lu;
    z = src->zsum;
  } else if (r > 0 && (double)d <= (2.0 * (double)r) / sc) {
    l = 1;
    z = d > 0 ? c / (double)d : 0.0;
  }
  uint64_t r2 = r;
  if (mode == 2 && r > 0 && l > 0) {
    const double cl = l == 1 ? cl1 : (l == 2 ? cl2 : cl3);
    r2 = (uint64_t)ceil((double)r * cl);
  }
  ell[k] = l;
  zsum[k] = z;
  Rk2[k] = r2;
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

}  // namespace

es_status launch_lde(es_ctx* ctx, const es_graph* g, int32_t u, const double* lv, int32_t L, const uint64_t* Rk,
                     double c, int32_t mode, LdeOut out, int32_t* level_u, double* zsum_u) {
  const int32_t n = g->n;
  const double sc = std::sqrt(c);
  const int32_t du = g->h_in_off[u + 1] - g->h_in_off[u];
  es_status st;
  // misc: LdeSource, per-in-neighbour sums, level partials, C_2 accumulators
  const size_t off_nb = 256;
  const size_t off_part = off_nb + 16 * (size_t)std::max(du, 1);
  const size_t off_acc = off_part + sizeof(double) * 4 * kRedBlocks;
  const size_t misc_bytes = off_acc + 8 * (size_t)std::max(du, 1);
  auto* misc = (char*)workspace(ctx, kWsLdeMisc, misc_bytes, &st);
  if (!misc) return st;
  auto* src = (LdeSource*)misc;
  auto* deg2 = (long long*)(misc + off_nb);
  auto* inv2 = (double*)(misc + off_nb + 8 * (size_t)std::max(du, 1));
  auto* part = (double*)(misc + off_part);
  auto* c2acc = (unsigned long long*)(misc + off_acc);
  const int tb = 256;
  int32_t lu = 0;
  if (mode != 0) {
    if (du > 0)
      source_nb_kernel<<<du, kRedThreads, 0, ctx->stream>>>(u, g->in_off, g->in_idx, g->din_int, g->inv_din, deg2,
                                                            inv2);
    source_costs_kernel<<<1, 1, 0, ctx->stream>>>(u, g->in_off, g->in_idx, g->din_int, g->inv_din, deg2, inv2, Rk,
                                                  src);
    ES_CHECK_HIP(ctx, hipGetLastError());
    LdeSource h;
    ES_CHECK_HIP(ctx, hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    // the largest l <= min(3, L) whose work E_l(u) fits 2 R(u) / sqrt(c)
    if (h.Ru > 0) {
      const double budget = (2.0 * (double)h.Ru) / sc;
      const double work[3] = {(double)h.E[0], (double)h.E[1],
                              (double)h.E[1] + level3_path_cost(n) * (double)(h.E[2] - h.E[1])};
      for (int l = 1; l <= std::min(kMaxSourceLevel, (int)L); ++l)
        if (work[l - 1] <= budget) lu = l;
    }
    if (lu >= 2) {
      const double* lv3 = lu >= 3 ? lv + 3 * (size_t)n : nullptr;
      level_dots_kernel<<<kRedBlocks, kRedThreads, 0, ctx->stream>>>(n, lv + (size_t)n, lv + 2 * (size_t)n, lv3,
                                                                    g->inv_din, part);
    }
    if (lu >= 3) {
      auto* W = (unsigned long long*)workspace(ctx, kWsLdeW, sizeof(uint64_t) * (size_t)n, &st);
      if (!W) return st;
      const int zb = std::max(1, std::min(ceil_div(n, tb), ctx->num_cus * 8));
      zero_u64<<<zb, tb, 0, ctx->stream>>>(n, W);
      zero_u64<<<1, tb, 0, ctx->stream>>>(du, c2acc);
      const int grid = ctx->num_cus * 8;
      for (int32_t o = 0; o < du; ++o) {
        c2_scatter_kernel<<<grid, 256, 0, ctx->stream>>>(u, o, g->in_off, g->in_idx, g->inv_din, W);
        c2_exchange_kernel<<<grid, 256, 0, ctx->stream>>>(u, o, g->in_off, g->in_idx, W, c2acc);
      }
    }
    source_z_kernel<<<1, 1, 0, ctx->stream>>>(lu, du, c, sc, part, c2acc, g->inv_din, u, src);
    ES_CHECK_HIP(ctx, hipGetLastError());
  }
  if (mode == 0) {
    // no exploitation: l = 0, R' = R (the plan kernel with an impossible source)
    lde_plan_kernel<<<ceil_div(n, tb), tb, 0, ctx->stream>>>(n, Rk, g->din_int, -1, 0, src, c, sc, 0, 1.0, 1.0, 1.0,
                                                             out.ell, out.zsum, out.Rk2);
  } else {
    lde_plan_kernel<<<ceil_div(n, tb), tb, 0, ctx->stream>>>(n, Rk, g->din_int, u, lu, src, c, sc, mode,
                                                             c_power(c, 1), c_power(c, 2), c_power(c, 3), out.ell,
                                                             out.zsum, out.Rk2);
  }
  ES_CHECK_HIP(ctx, hipGetLastError());
  if (level_u) *level_u = lu;
  if (zsum_u) {
    double z = 0.0;
    if (mode != 0) {
      ES_CHECK_HIP(ctx, hipMemcpyAsync(&z, &src->zsum, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    *zsum_u = z;
  }
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

es_status es_lde_plan(es_ctx* ctx, const es_graph* g, int32_t u, const double* levels, int32_t L, const uint64_t* Rk,
                      double c, int32_t mode, int32_t* ell, double* zsum, uint64_t* Rk_out) {
  if (!ctx || !g || !levels || !Rk || !ell || !zsum || !Rk_out) return ES_EINVAL;
  if (u < 0 || u >= g->n) return fail(ctx, ES_EINVAL, "source %d outside [0, %d)", u, g->n);
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  if (L < 1) return fail(ctx, ES_EINVAL, "L=%d must be at least 1", L);
  if (mode < 0 || mode > 2) return fail(ctx, ES_EINVAL, "exploitation mode %d outside 0..2", mode);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  const int32_t n = g->n;
  const int32_t nl = std::min(L, kMaxSourceLevel) + 1;
  es_status st;
  auto* lv = (double*)workspace(ctx, kWsLdeLv, sizeof(double) * (size_t)nl * n, &st);
  if (!lv) return st;
  auto* rin = (uint64_t*)workspace(ctx, kWsLdeRin, sizeof(uint64_t) * (size_t)n, &st);
  if (!rin) return st;
  auto* e_int = (int32_t*)workspace(ctx, kWsLdeEll, sizeof(int32_t) * (size_t)n, &st);
  if (!e_int) return st;
  auto* z_int = (double*)workspace(ctx, kWsLdeZ, sizeof(double) * (size_t)n, &st);
  if (!z_int) return st;
  auto* r_int = (uint64_t*)workspace(ctx, kWsLdeR, sizeof(uint64_t) * (size_t)n, &st);
  if (!r_int) return st;
  // caller order -> internal order (levels 0..min(3, L), sample counts bit for bit)
  ES_TRY(launch_permute_f64(ctx, n, nl, levels, g->ext_of, lv));
  ES_TRY(launch_permute_f64(ctx, n, 1, (const double*)Rk, g->ext_of, (double*)rin));
  ES_TRY(launch_lde(ctx, g, g->h_int_of[u], lv, L, rin, c, mode, LdeOut{e_int, z_int, r_int}, nullptr, nullptr));
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
