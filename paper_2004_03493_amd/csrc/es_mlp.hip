// Learned walk budget: features, the 6-64-64-1 network (inference, gradient,
// Adam), and the variance-weighted sample allocation.
//
// The variance bound of Lemma 1 (Section 3.1) keeps the Bernoulli variance
// D(k,k)(1 - D(k,k)) of each pair before the paper bounds it by 1; under a fixed
// total, the worst case over targets is smallest when R(k) is proportional to
// pi(k)^2 D(1-D).  The network predicts the meeting probability p(k) = 1 - D(k,k)
// from local degree features, v(k) = max(p(1-p), 1e-6), and
//   R(k) = ceil((R * pi(k)^2) * (v(k) * S2 / S1)),
//   S1 = sum Q(pi^2 v), S2 = sum Q(pi^2), Q(x) = round(x 2^62), exact int64 sums,
// so the total matches the pi^2 rule and every node with pi(k) > 0 keeps at least
// one pair: the estimator stays unbiased whatever the network predicts.
//
// All network arithmetic is float32 on the vector ALUs: at width 64 each
// sample is a few thousand multiply-adds against weights held in LDS.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <vector>

#include "es_internal.h"

namespace es {
namespace {

constexpr int NF = 6, H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = H * NF, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1;
constexpr float V_FLOOR = 1e-6f;
constexpr int kInferThreads = 256;
constexpr int kGradRows = 256;                 // rows per gradient block
constexpr int kGradThreads = 2 * kGradRows;    // two threads per row
constexpr int kPartStride = (NPARAM + 3) & ~3;  // floats per block partial gradient
constexpr int kSumGroup = 64;                  // partials added per first-level sum
constexpr uint64_t kWeightCap = 65536;  // a node's weight in the loss: min(R(k), cap)

// ---- features ----------------------------------------------------------------

// feats[v] for v in [0, n): k = to_int ? to_int[v] : v (internal id).  One
// wave per node (grid-stride): the lanes stride k's in-neighbour list for the
// integer sum and max of their in-degrees and the float64 sum of their
// reciprocal in-degrees, reduced by a fixed butterfly, so a node's features
// depend only on its row (identical under either id order).
__global__ __launch_bounds__(256) void features_kernel(int32_t n, const int32_t* __restrict__ to_int,
                                                       const int32_t* __restrict__ in_off,
                                                       const int32_t* __restrict__ in_idx,
                                                       const int32_t* __restrict__ din,
                                                       const int32_t* __restrict__ out_off, float c,
                                                       float* __restrict__ F) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < n; v += nwaves) {
    const int32_t k = to_int ? to_int[v] : (int32_t)v;
    const int32_t b = in_off[k], e = in_off[k + 1];
    int64_t s = 0;
    int32_t mx = 0;
    double rs = 0.0;
    for (int32_t i = b + lane; i < e; i += 64) {
      const int32_t dd = din[in_idx[i]];
      s += dd;
      mx = dd > mx ? dd : mx;
      rs += dd > 0 ? 1.0 / (double)dd : 0.0;
    }
    for (int m = 32; m > 0; m >>= 1) {
      s += __shfl_xor(s, m, 64);
      const int32_t o = __shfl_xor(mx, m, 64);
      mx = o > mx ? o : mx;
      rs += __shfl_xor(rs, m, 64);
    }
    if (lane == 0) {
      const int32_t d = e - b;
      const int32_t dout = out_off[k + 1] - out_off[k];
      float* f = F + v * NF;
      f[0] = log1pf((float)d);
      f[1] = log1pf((float)dout);
      f[2] = d > 0 ? log1pf((float)((double)s / (double)d)) : 0.0f;
      f[3] = log1pf((float)mx);
      f[4] = d > 0 ? (float)(rs / (double)d) : 0.0f;
      f[5] = d > 0 ? c / (float)d : 0.0f;
    }
  }
}

unsigned feature_blocks(const es_ctx* ctx, int32_t n) {
  const int64_t want = ((int64_t)n + 3) / 4;  // four waves per block
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->num_cus * 64));
}

// S[0] += Q(pi^2 w), S[1] += Q(pi^2) over nodes that take samples, with
// w = max(v, *thr) (thr may be NULL: w = v; v may be NULL: S[1] only).
// Grid-stride blocks of 256 reduce in registers, then across their four
// waves in LDS, and add once per block: integer sums, so any split gives
// the same totals.
__global__ __launch_bounds__(256) void weighted_sums_kernel(int32_t n, const double* __restrict__ pi,
                                                            const float* __restrict__ v,
                                                            const int32_t* __restrict__ din, int32_t exact_small_din,
                                                            const double* __restrict__ thr,
                                                            unsigned long long* __restrict__ S) {
  __shared__ unsigned long long part[2][4];
  unsigned long long a = 0, b = 0;
  const double t = thr ? *thr : 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const double p = pi[k];
    const bool take = p > 0.0 && (!exact_small_din || din[k] >= 2);
    if (take) {
      const double p2 = p * p;
      if (v) {
        double w = (double)v[k];
        if (thr && t > w) w = t;
        a += (unsigned long long)(int64_t)rint((p2 * w) * 0x1p62);
      }
      b += (unsigned long long)(int64_t)rint(p2 * 0x1p62);
    }
  }
  for (int m = 32; m > 0; m >>= 1) {
    a += __shfl_xor(a, m, 64);
    b += __shfl_xor(b, m, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][wave] = a;
    part[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long sa = part[0][0] + part[0][1] + part[0][2] + part[0][3];
    const unsigned long long sb = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    if (sa | sb) {
      atomicAdd(&S[0], sa);
      atomicAdd(&S[1], sb);
    }
  }
}

// thr = floor_ratio * vbar, vbar = S[0] / S[1] (0 when no node takes samples)
__global__ void floor_kernel(const unsigned long long* __restrict__ S, double floor_ratio, double* __restrict__ thr) {
  const int64_t s1 = (int64_t)S[0], s2 = (int64_t)S[1];
  *thr = s1 > 0 ? floor_ratio * ((double)s1 / (double)s2) : 0.0;
}

__global__ void vbar_kernel(const unsigned long long* __restrict__ S, double* __restrict__ vbar_inv) {
  const int64_t s1 = (int64_t)S[0], s2 = (int64_t)S[1];
  *vbar_inv = s1 > 0 ? (double)s2 / (double)s1 : -1.0;
}

// R(k) = ceil((R * (pi*pi)) * (max(v, thr) * vbar_inv)); plain pi^2 rule if vbar_inv < 0
__global__ void budget_weighted_kernel(int32_t n, const double* __restrict__ pi, const float* __restrict__ v,
                                       const int32_t* __restrict__ din, double R, int32_t exact_small_din,
                                       const double* __restrict__ thr_p, const double* __restrict__ vbar_inv_p,
                                       uint64_t* __restrict__ Rk) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double p = pi[k];
  const double vi = *vbar_inv_p;
  double want = R * (p * p);
  if (vi >= 0.0) {
    double w = (double)v[k];
    if (*thr_p > w) w = *thr_p;
    want = want * (w * vi);
  }
  uint64_t r = (uint64_t)ceil(want);
  if (!(p > 0.0)) r = 0;
  if (exact_small_din && din[k] <= 1) r = 0;
  Rk[k] = r;
}

__global__ void zero_sums(unsigned long long* S, int n) {
  if ((int)threadIdx.x < n) S[threadIdx.x] = 0ull;
}

// ---- network ------------------------------------------------------------------

__device__ __forceinline__ void load_weights(const float* __restrict__ w, float* sw) {
  for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) sw[i] = w[i];
}

// p_out (nullable): c * sigmoid(z); v_out (nullable): max(p(1-p), V_FLOOR)
__global__ __launch_bounds__(kInferThreads) void infer_kernel(int64_t N, const float* __restrict__ F,
                                                              const float* __restrict__ w, float c,
                                                              float* __restrict__ p_out, float* __restrict__ v_out) {
  __shared__ float sw[NPARAM];
  load_weights(w, sw);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float x[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) x[j] = F[i * NF + j];
  float h1[H];
#pragma unroll
  for (int a = 0; a < H; ++a) {
    float s = sw[OFF_B1 + a];
#pragma unroll
    for (int j = 0; j < NF; ++j) s += sw[OFF_W1 + a * NF + j] * x[j];
    h1[a] = s > 0.0f ? s : 0.0f;
  }
  float z = sw[OFF_B3];
  for (int a = 0; a < H; ++a) {
    float s = sw[OFF_B2 + a];
#pragma unroll
    for (int j = 0; j < H; ++j) s += sw[OFF_W2 + a * H + j] * h1[j];
    z += sw[OFF_W3 + a] * (s > 0.0f ? s : 0.0f);
  }
  const float p = c / (1.0f + expf(-z));
  if (p_out) p_out[i] = p;
  if (v_out) {
    const float vv = p * (1.0f - p);
    v_out[i] = vv > V_FLOOR ? vv : V_FLOOR;
  }
}

// LDS index of element c of row q in a [rows][H] array whose 16-byte groups
// are permuted per row (group g of row q sits at g ^ (q mod 16)): 64 lanes
// writing their own rows at one column spread over 16 bank groups, and row
// reads (one row for the whole wave) and column reads stay conflict-free.
__device__ __forceinline__ int swz(int q, int c) { return q * H + ((((c >> 2) ^ (q & 15)) << 2) | (c & 3)); }

// Unnormalised gradient of sum_i w_i BCE(y_i, p_i) over the block's rows and
// the loss sum: part[b][NPARAM] and pacc[b][2] (loss, sum of weights) for
// block b, each entry written by one thread (the blocks' partials are added
// in block order afterwards, so the gradient does not depend on timing).
// Labels: y = M(k)/R(k), the observed meeting fraction of R(k) pairs, weight
// min(R(k), cap) (rows with R(k) = 0 carry no weight).  Two threads per row,
// each for half of the hidden units (the halves are whole waves): the
// forward pass and dh1 run in registers against the weights in LDS (16-byte
// broadcast reads); the block's sums over its rows (dW2 as 2 x 4 register
// tiles per thread, the rest as column sums) read the rows back from LDS.
__global__ __launch_bounds__(kGradThreads) void grad_kernel(int64_t N, const float* __restrict__ F,
                                                            const uint64_t* __restrict__ Rn,
                                                            const uint64_t* __restrict__ Mn,
                                                            const float* __restrict__ w, float c,
                                                            float* __restrict__ part, double* __restrict__ pacc) {
  __shared__ __align__(16) float sw[NPARAM];
  __shared__ __align__(16) float HS[kGradRows * H];  // h1 rows, later dh1 rows
  __shared__ __align__(16) float DS[kGradRows * H];  // h2 rows, later dz2 rows
  __shared__ float XS[kGradRows * NF];
  __shared__ float GZ[kGradRows];
  __shared__ float ZP[2][kGradRows];  // each half's share of z
  __shared__ double red[2][kGradRows / 64];
  load_weights(w, sw);
  const int t = threadIdx.x;
  const int q0 = t & (kGradRows - 1);  // this thread's row
  const int hf = t / kGradRows;        // its half of the hidden units
  const int64_t i = (int64_t)blockIdx.x * kGradRows + q0;
  const bool live = i < N;
  float* __restrict__ grad = part + (int64_t)blockIdx.x * kPartStride;
  float x[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) x[j] = live ? F[i * NF + j] : 0.0f;
  if (hf == 0) {
#pragma unroll
    for (int j = 0; j < NF; ++j) XS[q0 * NF + j] = x[j];
  }
  __syncthreads();
  // layer 1, all units in both halves: h1 in registers, its ReLU pattern in m1
  float h[H];
  uint64_t m1 = 0;
#pragma unroll
  for (int a = 0; a < H; ++a) {
    float s = sw[OFF_B1 + a];
#pragma unroll
    for (int j = 0; j < NF; ++j) s = fmaf(sw[OFF_W1 + a * NF + j], x[j], s);
    h[a] = s > 0.0f ? s : 0.0f;
    m1 |= (uint64_t)(s > 0.0f ? 1u : 0u) << a;
  }
  // this half's 16-byte groups of the h1 row
  if (hf == 0) {
#pragma unroll
    for (int g = 0; g < H / 8; ++g)
      *(float4*)&HS[q0 * H + ((g ^ (q0 & 15)) << 2)] = make_float4(h[4 * g], h[4 * g + 1], h[4 * g + 2], h[4 * g + 3]);
  } else {
#pragma unroll
    for (int g = H / 8; g < H / 4; ++g)
      *(float4*)&HS[q0 * H + ((g ^ (q0 & 15)) << 2)] = make_float4(h[4 * g], h[4 * g + 1], h[4 * g + 2], h[4 * g + 3]);
  }
  // layer 2 for this half's units, four rows of W2 at a time: h2 to LDS,
  // the ReLU pattern in m2 (this half's bits), the share of z in ZP
  uint64_t m2 = 0;
  float zp = 0.0f;
  for (int a = hf * (H / 2); a < (hf + 1) * (H / 2); a += 4) {
    float s[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = sw[OFF_B2 + a + k];
#pragma unroll
    for (int g = 0; g < H / 4; ++g) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 v = *(const float4*)&sw[OFF_W2 + (a + k) * H + 4 * g];
        s[k] = fmaf(v.x, h[4 * g], s[k]);
        s[k] = fmaf(v.y, h[4 * g + 1], s[k]);
        s[k] = fmaf(v.z, h[4 * g + 2], s[k]);
        s[k] = fmaf(v.w, h[4 * g + 3], s[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float r = s[k] > 0.0f ? s[k] : 0.0f;
      DS[swz(q0, a + k)] = r;
      m2 |= (uint64_t)(s[k] > 0.0f ? 1u : 0u) << (a + k);
      zp = fmaf(sw[OFF_W3 + a + k], r, zp);
    }
  }
  ZP[hf][q0] = zp;
  __syncthreads();
  const float z = (sw[OFF_B3] + ZP[0][q0]) + ZP[1][q0];
  const float sig = 1.0f / (1.0f + expf(-z));
  const float p = c * sig;
  float gz = 0.0f;
  double lsum = 0.0, wsum = 0.0;
  if (live && Rn[i] > 0) {
    const uint64_t rr = Rn[i];
    const float yy = (float)((double)Mn[i] / (double)rr);
    const float ww = (float)(rr < kWeightCap ? rr : kWeightCap);
    // d/dz of w * BCE(y, c sigmoid(z)) = w (1 - p/c) (-y + (1 - y) p/(1 - p))
    gz = ww * (1.0f - p / c) * (-yy + (1.0f - yy) * p / (1.0f - p));
    if (hf == 0) {
      lsum = -(double)ww * ((double)yy * log((double)p) + (1.0 - (double)yy) * log1p(-(double)p));
      wsum = ww;
    }
  }
  if (hf == 0) {
    GZ[q0] = gz;
    for (int m = 32; m > 0; m >>= 1) {
      lsum += __shfl_xor(lsum, m, 64);
      wsum += __shfl_xor(wsum, m, 64);
    }
    if ((t & 63) == 0) {
      red[0][t >> 6] = lsum;
      red[1][t >> 6] = wsum;
    }
  }
  __syncthreads();
  if (t == 0) {
    double l = 0.0, ws = 0.0;
    for (int q = 0; q < kGradRows / 64; ++q) {
      l += red[0][q];
      ws += red[1][q];
    }
    pacc[2 * (int64_t)blockIdx.x] = l;
    pacc[2 * (int64_t)blockIdx.x + 1] = ws;
  }
  // dW3[a] = sum_q gz_q h2_{q,a}, db3 = sum_q gz_q
  if (t < H) {
    float s = 0.0f;
    for (int q = 0; q < kGradRows; ++q) s = fmaf(GZ[q], DS[swz(q, t)], s);
    grad[OFF_W3 + t] = s;
  } else if (t == H) {
    float s = 0.0f;
    for (int q = 0; q < kGradRows; ++q) s += GZ[q];
    grad[OFF_B3] = s;
  }
  __syncthreads();
  // dz2 (pre-activation gradient of layer 2), this half's groups, over the h2 rows
#pragma unroll
  for (int g = 0; g < H / 8; ++g) {
    const int gg = hf * (H / 8) + g;
    float d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = 4 * gg + k;
      d[k] = ((m2 >> a) & 1ull) ? gz * sw[OFF_W3 + a] : 0.0f;
    }
    *(float4*)&DS[q0 * H + ((gg ^ (q0 & 15)) << 2)] = make_float4(d[0], d[1], d[2], d[3]);
  }
  __syncthreads();
  // dW2[a][j] = sum_q dz2_{q,a} h1_{q,j}: thread t sums the 2 x 4 tile at
  // a = 2 (t / 16), j = 4 (t mod 16)
  {
    const int a0 = 2 * (t >> 4), gj = t & 15;
    float s[2][4] = {};
    for (int q = 0; q < kGradRows; ++q) {
      const float2 dv = *(const float2*)&DS[q * H + ((((a0 >> 2) ^ (q & 15)) << 2) | (a0 & 3))];
      const float4 hv = *(const float4*)&HS[q * H + ((gj ^ (q & 15)) << 2)];
      const float dd[2] = {dv.x, dv.y}, hh[4] = {hv.x, hv.y, hv.z, hv.w};
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) s[r][k] = fmaf(dd[r], hh[k], s[r][k]);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) grad[OFF_W2 + (a0 + r) * H + 4 * gj + k] = s[r][k];
  }
  // db2[a] = sum_q dz2_{q,a}
  if (t < H) {
    float s = 0.0f;
    for (int q = 0; q < kGradRows; ++q) s += DS[swz(q, t)];
    grad[OFF_B2 + t] = s;
  }
  __syncthreads();
  // dh1[j] = [h1_j > 0] sum_a W2[a][j] dz2_a for this half's j, over the h1 rows
  {
    float dh[H / 2];
#pragma unroll
    for (int j = 0; j < H / 2; ++j) dh[j] = 0.0f;
    for (int a = 0; a < H; ++a) {
      const float d = DS[swz(q0, a)];
      const float4* wr = (const float4*)&sw[OFF_W2 + a * H + hf * (H / 2)];
#pragma unroll
      for (int g = 0; g < H / 8; ++g) {
        const float4 v = wr[g];
        dh[4 * g] = fmaf(d, v.x, dh[4 * g]);
        dh[4 * g + 1] = fmaf(d, v.y, dh[4 * g + 1]);
        dh[4 * g + 2] = fmaf(d, v.z, dh[4 * g + 2]);
        dh[4 * g + 3] = fmaf(d, v.w, dh[4 * g + 3]);
      }
    }
#pragma unroll
    for (int g = 0; g < H / 8; ++g) {
      const int gg = hf * (H / 8) + g;
      float e[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) e[k] = ((m1 >> (4 * gg + k)) & 1ull) ? dh[4 * g + k] : 0.0f;
      *(float4*)&HS[q0 * H + ((gg ^ (q0 & 15)) << 2)] = make_float4(e[0], e[1], e[2], e[3]);
    }
  }
  __syncthreads();
  // dW1[a][j] = sum_q dh1_{q,a} x_{q,j} (thread a NF + j), db1[a] = sum_q dh1_{q,a}
  if (t < H * NF) {
    const int a = t / NF, j = t - a * NF;
    float s = 0.0f;
    for (int q = 0; q < kGradRows; ++q) s = fmaf(HS[swz(q, a)], XS[q * NF + j], s);
    grad[OFF_W1 + t] = s;
  } else if (t < H * NF + H) {
    const int a = t - H * NF;
    float s = 0.0f;
    for (int q = 0; q < kGradRows; ++q) s += HS[swz(q, a)];
    grad[OFF_B1 + a] = s;
  }
}

// out[g][j] = sum of in[r][j] over rows r in [g G, min((g + 1) G, nrows)),
// added in row order (rows of `stride` elements, ncols used).
template <typename T>
__global__ void sum_rows_kernel(int64_t nrows, int32_t G, int32_t ncols, int32_t stride, const T* __restrict__ in,
                                T* __restrict__ out) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncols) return;
  const int64_t r0 = (int64_t)blockIdx.y * G;
  const int64_t r1 = min(nrows, r0 + G);
  T s = 0;
  for (int64_t r = r0; r < r1; ++r) s += in[r * stride + j];
  out[(int64_t)blockIdx.y * stride + j] = s;
}

__global__ void zero_f32(int n, float* p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// grad /= sum of weights
__global__ void normalise_kernel(float* __restrict__ grad, const double* __restrict__ acc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NPARAM && acc[1] > 0.0) grad[i] = (float)((double)grad[i] / acc[1]);
}

// Adam (Kingma and Ba, 2015) on the normalised gradient
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ grad, float* __restrict__ m,
                            float* __restrict__ v, const double* __restrict__ acc, float lr, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float g = acc[1] > 0.0 ? (float)((double)grad[i] / acc[1]) : 0.0f;
  const float mi = 0.9f * m[i] + 0.1f * g;
  const float vi = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

__global__ void record_loss(const double* __restrict__ acc, float* __restrict__ out) {
  *out = acc[1] > 0.0 ? (float)(acc[0] / acc[1]) : 0.0f;
}

bool valid_c(double c) { return c > 0.0 && c <= 0.99; }

// Scratch of one gradient evaluation over N rows: the blocks' partials and the
// first-level sums, after `lead` floats the caller keeps for itself (Adam's
// state in training).
struct GradScratch {
  float* lead;    // lead floats
  float* part;    // [nb][kPartStride], then [ng][kPartStride]
  double* acc;    // acc[0] loss, acc[1] sum of weights
  double* pacc;   // [nb][2], then [ng][2]
  int64_t nb, ng;
  int32_t G;      // blocks per first-level sum
};

es_status grad_scratch(es_ctx* ctx, int64_t N, size_t lead, GradScratch* gs) {
  es_status st;
  gs->nb = (N + kGradRows - 1) / kGradRows;
  gs->G = (int32_t)std::max<int64_t>(kSumGroup, (gs->nb + 32767) / 32768);  // at most 32768 first-level sums
  gs->ng = (gs->nb + gs->G - 1) / gs->G;
  const size_t lead4 = (lead + 3) & ~(size_t)3;
  auto* f = (float*)workspace(ctx, kWsMlpGrad, sizeof(float) * (lead4 + (size_t)(gs->nb + gs->ng) * kPartStride), &st);
  if (!f) return st;
  auto* d = (double*)workspace(ctx, kWsMlpAcc, sizeof(double) * (2 + 2 * (size_t)(gs->nb + gs->ng)), &st);
  if (!d) return st;
  gs->lead = f;
  gs->part = f + lead4;
  gs->acc = d;
  gs->pacc = d + 2;
  return ES_OK;
}

// grad_out[NPARAM] and gs.acc[0..1]: the block partials of the rows added in
// block order (two levels), so the result is the same on every run.
void launch_grad(es_ctx* ctx, const GradScratch& gs, int64_t N, const float* feats, const uint64_t* R,
                 const uint64_t* M, const float* weights, double c, float* grad_out) {
  float* part2 = gs.part + gs.nb * kPartStride;
  double* pacc2 = gs.pacc + 2 * gs.nb;
  grad_kernel<<<(unsigned)gs.nb, kGradThreads, 0, ctx->stream>>>(N, feats, R, M, weights, (float)c, gs.part,
                                                                  gs.pacc);
  const unsigned cols = (unsigned)ceil_div(NPARAM, 256);
  sum_rows_kernel<float><<<dim3(cols, (unsigned)gs.ng), 256, 0, ctx->stream>>>(gs.nb, gs.G, NPARAM, kPartStride,
                                                                              gs.part, part2);
  sum_rows_kernel<float><<<dim3(cols, 1), 256, 0, ctx->stream>>>(gs.ng, (int32_t)gs.ng, NPARAM, kPartStride, part2,
                                                                grad_out);
  sum_rows_kernel<double><<<dim3(1, (unsigned)gs.ng), 64, 0, ctx->stream>>>(gs.nb, gs.G, 2, 2, gs.pacc, pacc2);
  sum_rows_kernel<double><<<dim3(1, 1), 64, 0, ctx->stream>>>(gs.ng, (int32_t)gs.ng, 2, 2, pacc2, gs.acc);
}

}  // namespace

// The weighted allocation of R over n nodes (din indexed like pi and v).
static es_status launch_weighted(es_ctx* ctx, int32_t n, const double* pi, const float* v, const int32_t* din, double R,
                          int32_t exact_small_din, double floor_ratio, uint64_t* Rk) {
  es_status st;
  auto* S = (unsigned long long*)workspace(ctx, kWsMlpSums, 64, &st);
  if (!S) return st;
  double* thr = (double*)(S + 4);
  double* vbar_inv = (double*)(S + 5);
  const int tb = 256;
  const unsigned nb = ceil_div(n, tb);
  const unsigned nsum = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nb, (int64_t)ctx->num_cus * 8));
  zero_sums<<<1, 64, 0, ctx->stream>>>(S, 4);
  // S[0] = sum Q(pi^2 v), S[1] = sum Q(pi^2); thr = floor_ratio * S[0] / S[1]
  weighted_sums_kernel<<<nsum, tb, 0, ctx->stream>>>(n, pi, v, din, exact_small_din, nullptr, S);
  floor_kernel<<<1, 1, 0, ctx->stream>>>(S, floor_ratio, thr);
  // S[2] = sum Q(pi^2 max(v, thr)), S[3] = sum Q(pi^2); vbar_inv = S[3] / S[2]
  weighted_sums_kernel<<<nsum, tb, 0, ctx->stream>>>(n, pi, v, din, exact_small_din, thr, S + 2);
  vbar_kernel<<<1, 1, 0, ctx->stream>>>(S + 2, vbar_inv);
  budget_weighted_kernel<<<nb, tb, 0, ctx->stream>>>(n, pi, v, din, R, exact_small_din, thr, vbar_inv, Rk);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

// Learned budget inside a query (internal node order): predicted variances
// (cached in the graph per network and decay), then the weighted allocation.
es_status ensure_vhat(es_ctx* ctx, const es_graph* g, double c) {
  const int32_t n = g->n;
  es_status st;
  if (!g->vhat || g->vhat_net != ctx->mlp_id || g->vhat_c != c) {
    // predictions for this network and decay: features, then inference, once
    if (!g->vhat) ES_CHECK_HIP(ctx, hipMalloc((void**)&g->vhat, sizeof(float) * std::max<int32_t>(n, 1)));
    auto* F = (float*)workspace(ctx, kWsFeat, sizeof(float) * NF * (size_t)n, &st);
    if (!F) return st;
    features_kernel<<<feature_blocks(ctx, n), 256, 0, ctx->stream>>>(n, nullptr, g->in_off, g->in_idx, g->din_int,
                                                                     g->out_off, (float)c, F);
    infer_kernel<<<ceil_div(n, kInferThreads), kInferThreads, 0, ctx->stream>>>(n, F, ctx->mlp_w, (float)c, nullptr,
                                                                                g->vhat);
    ES_CHECK_HIP(ctx, hipGetLastError());
    g->vhat_net = ctx->mlp_id;
    g->vhat_c = c;
  }
  return ES_OK;
}

es_status launch_learned_budget(es_ctx* ctx, const es_graph* g, const double* pi, double R, double c,
                                int32_t exact_small_din, double floor_ratio, uint64_t* Rk) {
  ES_TRY(ensure_vhat(ctx, g, c));
  return launch_weighted(ctx, g->n, pi, g->vhat, g->din_int, R, exact_small_din, floor_ratio, Rk);
}

}  // namespace es

using namespace es;

extern "C" {

es_status es_mlp_features(es_ctx* ctx, const es_graph* g, double c, float* feats) {
  if (!ctx || !g || !feats) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  features_kernel<<<feature_blocks(ctx, g->n), 256, 0, ctx->stream>>>(g->n, g->int_of, g->in_off, g->in_idx,
                                                                      g->din_int, g->out_off, (float)c, feats);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

es_status es_mlp_infer(es_ctx* ctx, const float* weights, const float* feats, int64_t N, double c, float* p_out,
                       float* v_out) {
  if (!ctx || !weights || (!feats && N > 0) || N < 0 || (!p_out && !v_out)) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  if (N == 0) return ES_OK;
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  infer_kernel<<<(unsigned)((N + kInferThreads - 1) / kInferThreads), kInferThreads, 0, ctx->stream>>>(
      N, feats, weights, (float)c, p_out, v_out);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

es_status es_mlp_grad(es_ctx* ctx, const float* weights, const float* feats, const uint64_t* R, const uint64_t* M,
                      int64_t N, double c, float* grad, double* loss) {
  if (!ctx || !weights || !feats || !R || !M || N < 1 || !grad) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  GradScratch gs;
  ES_TRY(grad_scratch(ctx, N, 0, &gs));
  double* acc = gs.acc;
  launch_grad(ctx, gs, N, feats, R, M, weights, c, grad);
  normalise_kernel<<<ceil_div(NPARAM, 256), 256, 0, ctx->stream>>>(grad, acc);
  ES_CHECK_HIP(ctx, hipGetLastError());
  if (loss) {
    double h[2];
    ES_CHECK_HIP(ctx, hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *loss = h[1] > 0 ? h[0] / h[1] : 0.0;
  }
  return ES_OK;
}

es_status es_mlp_train(es_ctx* ctx, const float* feats, const uint64_t* R, const uint64_t* M, int64_t N, double c,
                       int32_t epochs, float lr, float* weights, float* losses) {
  if (!ctx || !feats || !R || !M || N < 1 || epochs < 1 || !(lr > 0.0f) || !weights) return ES_EINVAL;
  if (!valid_c(c)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", c);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  es_status st;
  GradScratch gs;
  ES_TRY(grad_scratch(ctx, N, 3 * (size_t)NPARAM, &gs));
  float* grad = gs.lead;
  float* m = grad + NPARAM;
  float* v = grad + 2 * NPARAM;
  double* acc = gs.acc;
  auto* dl = (float*)workspace(ctx, kWsMlpLoss, sizeof(float) * (size_t)epochs, &st);
  if (!dl) return st;
  zero_f32<<<ceil_div(3 * NPARAM, 256), 256, 0, ctx->stream>>>(3 * NPARAM, grad);
  double b1t = 1.0, b2t = 1.0;
  for (int32_t ep = 0; ep < epochs; ++ep) {
    b1t *= 0.9;
    b2t *= 0.999;
    launch_grad(ctx, gs, N, feats, R, M, weights, c, grad);
    record_loss<<<1, 1, 0, ctx->stream>>>(acc, dl + ep);
    adam_kernel<<<ceil_div(NPARAM, 256), 256, 0, ctx->stream>>>(weights, grad, m, v, acc, lr, (float)(1.0 - b1t),
                                                                 (float)(1.0 - b2t));
  }
  ES_CHECK_HIP(ctx, hipGetLastError());
  if (losses) {
    ES_CHECK_HIP(ctx, hipMemcpyAsync(losses, dl, sizeof(float) * epochs, hipMemcpyDeviceToHost, ctx->stream));
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return ES_OK;
}

es_status es_mlp_load(es_ctx* ctx, const float* weights) {
  if (!ctx) return ES_EINVAL;
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  if (!weights) {
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ES_CHECK_HIP(ctx, hipFree(ctx->mlp_w));
    ctx->mlp_w = nullptr;
    ctx->mlp_id = 0;
    return ES_OK;
  }
  if (!ctx->mlp_w) ES_CHECK_HIP(ctx, hipMalloc(&ctx->mlp_w, sizeof(float) * NPARAM));
  ES_CHECK_HIP(ctx, hipMemcpyAsync(ctx->mlp_w, weights, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, ctx->stream));
  // a new identity: predictions cached in graphs for other weights go stale
  static std::atomic<uint64_t> next_id{0};
  ctx->mlp_id = ++next_id;
  return ES_OK;
}

es_status es_budget_weighted(es_ctx* ctx, const es_graph* g, const double* pi, const float* v, double R,
                             int32_t exact_small_din, double floor_ratio, uint64_t* Rk) {
  if (!ctx || !g || !pi || !v || !Rk) return ES_EINVAL;
  if (!(R > 0.0)) return fail(ctx, ES_EINVAL, "R=%g must be positive", R);
  if (!(floor_ratio >= 0.0 && floor_ratio <= 1.0)) return fail(ctx, ES_EINVAL, "floor ratio %g outside [0, 1]", floor_ratio);
  if (R + (double)g->n >= 9.2e18) return fail(ctx, ES_EOVERFLOW, "R=%g: sample count may reach 2^63", R);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  return launch_weighted(ctx, g->n, pi, v, g->din_ext, R, exact_small_din, floor_ratio, Rk);
}

int32_t es_mlp_num_params(void) { return NPARAM; }

}  // extern "C"
