/*
 * ExactSim oracle: plain C Monte Carlo estimation of the diagonal
 * correction by the basic estimator of Algorithm 2: for node k, simulate
 * R(k) pairs of sqrt(c)-walks from v_k and count the pairs that meet.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library; both implement the same published random number
 * generator and the same sampling rule, written separately.
 *
 * Sampling rule for pair r of node k (all integers unsigned 64-bit), with
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011; 10 rounds) under key (seed, 0):
 *
 *   Two independent sqrt(c)-walks can meet at step t only if both are still
 *   walking at step t; that happens with probability sqrt(c)^t * sqrt(c)^t =
 *   c^t.  The pair's joint lifetime T is drawn by inverse transform from the
 *   word u = Philox(counter (k, floor(r/4), 0, 1))[r mod 4] (one block serves
 *   four consecutive pairs): T = #{ t >= 1 : u < thr[t] }, thr[t] =
 *   floor(c^t * 2^64) with c^t formed by repeated double multiplication, so
 *   Pr[T >= t] = c^t to within double rounding.
 *
 *   The words that move the walks at step t come from the block
 *   b_j = Philox(counter (k, r, j, 0)) with j = floor((t-1)/2):
 *   (wx, wy) = (b_j[0], b_j[1]) for odd t, (b_j[2], b_j[3]) for even t.
 *
 *   Both walks start at v_k.  For t = 1..T: if either walk sits on a node
 *   with no in-neighbour it cannot move and the pair ends without meeting;
 *   otherwise walk x moves to in-neighbour number mulhi64(wx, d_in(x)) of x
 *   (in-neighbours listed in ascending id order) and walk y to number
 *   mulhi64(wy, d_in(y)) of y.  The pair meets if x == y after the move
 *   (meeting at step 0, where both sit at v_k, does not count).
 *
 * M(k) = number of meeting pairs among r = 0 .. R(k)-1.
 *
 * Non-stop variant (Algorithm 3, the sampling part of the local
 * deterministic exploitation): with nonstop(k) = l > 0 both walks of every
 * pair of node k take their first l steps without stopping (the joint
 * lifetime becomes l + T); a meeting at a step t <= l ends the pair without
 * counting (those meetings are accounted for exactly), meetings at t > l
 * count as before.  l = 0 is the rule above.
 *
 * Compile with -ffp-contract=off (no fused multiply-add anywhere).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_TMAX 4096

static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

/* Philox4x64 with 10 rounds; counter ctr, key key, output out. */
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ x1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ x3 ^ k1;
    uint64_t n3 = lo0;
    x0 = n0; x1 = n1; x2 = n2; x3 = n3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* floor(w * d / 2^64): a uniform index in [0, d) from a uniform 64-bit word. */
uint64_t oracle_mulhi64(uint64_t w, uint64_t d) {
  return (uint64_t)(((unsigned __int128)w * d) >> 64);
}

/* Joint-lifetime thresholds: thr[t] = floor(c^t * 2^64) for t = 1..; returns
 * the number of positive entries written (at most cap).  thr[0] is unused. */
int oracle_lifetime_table(double c, uint64_t* thr, int cap) {
  double p = 1.0;
  int t;
  thr[0] = 0;
  for (t = 1; t < cap; ++t) {
    p = p * c;
    double v = p * 18446744073709551616.0; /* 2^64 */
    uint64_t u = (v >= 18446744073709551616.0) ? ~0ull : (uint64_t)v;
    if (u == 0) break;
    thr[t] = u;
  }
  return t - 1;
}

/* One walk pair: returns 1 if the two walks meet (after step `nonstop`), 0 otherwise. */
int oracle_walk_pair(const int64_t* in_off, const int32_t* in_idx, uint64_t seed, const uint64_t* thr,
                     int tmax, uint64_t k, uint64_t r, int nonstop) {
  const uint64_t key[2] = {seed, 0};
  uint64_t life[4];
  const uint64_t life_ctr[4] = {k, r / 4, 0, 1};
  oracle_philox4x64_10(life_ctr, key, life);
  const uint64_t u = life[r % 4];
  int T = 0;
  while (T < tmax && u < thr[T + 1]) ++T;
  T += nonstop;
  uint64_t x = k, y = k;
  uint64_t b[4];
  for (int t = 1; t <= T; ++t) {
    if (t % 2 == 1) {
      const uint64_t ctr[4] = {k, r, (uint64_t)((t - 1) / 2), 0};
      oracle_philox4x64_10(ctr, key, b);
    }
    const uint64_t wx = (t % 2 == 1) ? b[0] : b[2];
    const uint64_t wy = (t % 2 == 1) ? b[1] : b[3];
    uint64_t dx = (uint64_t)(in_off[x + 1] - in_off[x]);
    uint64_t dy = (uint64_t)(in_off[y + 1] - in_off[y]);
    if (dx == 0 || dy == 0) return 0;
    x = (uint64_t)in_idx[in_off[x] + (int64_t)oracle_mulhi64(wx, dx)];
    y = (uint64_t)in_idx[in_off[y] + (int64_t)oracle_mulhi64(wy, dy)];
    if (x == y) return t > nonstop ? 1 : 0;
  }
  return 0;
}

/* M[k] = number of meeting pairs among pairs r in [r_begin[k], r_end[k]) of
 * node k, for k = 0..n-1 (r_begin may be NULL, meaning 0; nonstop may be
 * NULL, meaning 0 for every node).  Returns 0, or -1 if c is outside (0, 1). */
int oracle_walk_counts(int64_t n, const int64_t* in_off, const int32_t* in_idx, const uint64_t* r_begin,
                       const uint64_t* r_end, const int32_t* nonstop, uint64_t seed, double c, uint64_t* M,
                       int threads) {
  if (!(c > 0.0 && c < 1.0)) return -1;
  uint64_t* thr = (uint64_t*)malloc(sizeof(uint64_t) * (ORACLE_TMAX + 1));
  int tmax = oracle_lifetime_table(c, thr, ORACLE_TMAX + 1);
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  const uint64_t big = 1u << 14;
  /* nodes with few pairs: one thread per node */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < n; ++k) {
    uint64_t b = r_begin ? r_begin[k] : 0, e = r_end[k];
    if (e <= b || e - b >= big) continue;
    uint64_t cnt = 0;
    const int l = nonstop ? nonstop[k] : 0;
    for (uint64_t r = b; r < e; ++r)
      cnt += (uint64_t)oracle_walk_pair(in_off, in_idx, seed, thr, tmax, (uint64_t)k, r, l);
    M[k] = cnt;
  }
  /* nodes with many pairs: split the pairs over threads */
  for (int64_t k = 0; k < n; ++k) {
    uint64_t b = r_begin ? r_begin[k] : 0, e = r_end[k];
    if (e <= b) {
      M[k] = 0;
      continue;
    }
    if (e - b < big) continue;
    uint64_t cnt = 0;
    const int l = nonstop ? nonstop[k] : 0;
#pragma omp parallel for schedule(static) reduction(+ : cnt)
    for (int64_t r = (int64_t)b; r < (int64_t)e; ++r)
      cnt += (uint64_t)oracle_walk_pair(in_off, in_idx, seed, thr, tmax, (uint64_t)k, (uint64_t)r, l);
    M[k] = cnt;
  }
  free(thr);
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
