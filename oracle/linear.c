/*
 * ExactSim oracle: the two linear passes of Algorithm 1 on plain CSR arrays,
 * for graphs whose sparse-matrix form would not fit the Python oracle
 * (a billion edges and more).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library.
 *
 * Graph: n nodes, m directed edges src[e] -> dst[e], distinct, no
 * self-loops, sorted ascending by (src, dst).  Then
 *   - the out-neighbour lists O(i) are the dst entries of i's run of edges,
 *     in ascending order;
 *   - the in-neighbour lists I(j) (ascending source id, the walk sampler's
 *     order) follow by one stable counting pass over the edges by dst.
 *
 * Forward (Algorithm 1, l-hop PPR), in the fixed-point rounding that makes
 * the sample counts reproducible:
 *   pi^0 = (1 - sqrt c) e_u;
 *   q(j) = round_to_nearest_even(pi^(l-1)(j) * (1/d_in(j)) * 2^62)  (int64)
 *   pi^l(i) = sqrt c * ((double)(sum_{j in O(i)} q(j)) * 2^-62)
 *   pi = pi^0 + pi^1 + ... + pi^L, added in that order.
 * Each integer sum is exact, so the result does not depend on its order.
 *
 * Back-accumulation (Algorithm 1), with a = 1/(1 - sqrt c):
 *   s^0(j) = a * (D(j) * pi^L(j));
 *   s^l(j) = sqrt c * ((1/d_in(j)) * sum_{i in I(j)} s^(l-1)(i))
 *            + a * (D(j) * pi^(L-l)(j)),   l = 1..L;
 *   returns s^L.
 *
 * Compile with -ffp-contract=off (no fused multiply-add anywhere).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* d_in, 1/d_in and the in-CSR (in_off int64[n+1], in_idx int32[m]).
 * Returns 0, or -1 if an edge is out of range, a self-loop, or out of
 * (src, dst) order. */
int oracle_in_csr(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int64_t* din,
                  double* inv_din, int64_t* in_off, int32_t* in_idx) {
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n || src[e] == dst[e]) return -1;
    if (e > 0 && (src[e] < src[e - 1] || (src[e] == src[e - 1] && dst[e] <= dst[e - 1]))) return -1;
  }
  memset(din, 0, (size_t)n * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) din[dst[e]]++;
  in_off[0] = 0;
  for (int64_t j = 0; j < n; ++j) {
    in_off[j + 1] = in_off[j] + din[j];
    inv_din[j] = din[j] > 0 ? 1.0 / (double)din[j] : 0.0;
  }
  int64_t* next = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!next) return -2;
  memcpy(next, in_off, (size_t)n * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) in_idx[next[dst[e]]++] = src[e];
  free(next);
  return 0;
}

/* out_off int64[n+1] from the sorted edge list (out_idx is dst itself). */
void oracle_out_off(int64_t n, int64_t m, const int32_t* src, int64_t* out_off) {
  memset(out_off, 0, (size_t)(n + 1) * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) out_off[src[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) out_off[i + 1] += out_off[i];
}

/* levels: (L+1) * n doubles, level l at levels + l*n; pi: n doubles. */
int oracle_forward(int64_t n, const int64_t* out_off, const int32_t* out_idx, const double* inv_din,
                   int64_t u, double c, int L, double* levels, double* pi) {
  if (u < 0 || u >= n || L < 0 || !(c > 0.0 && c < 1.0)) return -1;
  const double sc = sqrt(c);
  int64_t* q = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!q) return -2;
  memset(levels, 0, (size_t)n * sizeof(double));
  levels[u] = 1.0 - sc;
  memcpy(pi, levels, (size_t)n * sizeof(double));
  for (int l = 1; l <= L; ++l) {
    const double* prev = levels + (size_t)(l - 1) * (size_t)n;
    double* cur = levels + (size_t)l * (size_t)n;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
      const double term = prev[j] * inv_din[j];
      q[j] = (int64_t)llrint(term * 0x1p62);
    }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
      int64_t acc = 0;
      for (int64_t e = out_off[i]; e < out_off[i + 1]; ++e) acc += q[out_idx[e]];
      cur[i] = sc * ((double)acc * 0x1p-62);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) pi[i] = pi[i] + cur[i];
  }
  free(q);
  return 0;
}

int oracle_backward(int64_t n, const int64_t* in_off, const int32_t* in_idx, const double* inv_din,
                    const double* levels, int L, const double* D, double c, double* s) {
  if (L < 0 || !(c > 0.0 && c < 1.0)) return -1;
  const double sc = sqrt(c);
  const double a = 1.0 / (1.0 - sc);
  double* prev = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!prev) return -2;
  const double* top = levels + (size_t)L * (size_t)n;
  for (int64_t j = 0; j < n; ++j) s[j] = a * (D[j] * top[j]);
  for (int l = 1; l <= L; ++l) {
    memcpy(prev, s, (size_t)n * sizeof(double));
    const double* lv = levels + (size_t)(L - l) * (size_t)n;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t j = 0; j < n; ++j) {
      double sum = 0.0;
      for (int64_t e = in_off[j]; e < in_off[j + 1]; ++e) sum += prev[in_idx[e]];
      s[j] = sc * (inv_din[j] * sum) + a * (D[j] * lv[j]);
    }
  }
  free(prev);
  return 0;
}
