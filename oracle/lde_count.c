/*
 * Algorithm 3's stopping rule for the local deterministic exploitation
 * (Section 3.2, "Local deterministic exploitation for D", Algorithm 3):
 * test infrastructure, part of the CPU oracle.
 *
 * Algorithm 3 walks the transition tables of v_k level by level.  In round
 * l (l = 0, 1, 2, ...) it first evaluates Z_l(k, .) and then, for every
 * l' = 0..l and every node q' that a walk from v_k reaches in exactly l - l'
 * steps, extends the table of q' by one step: for every node x that a walk
 * from q' reaches in exactly l' steps and every in-neighbour q of x it adds
 * one term and counts one traversed edge in E_k.  As soon as E_k reaches
 * 2 R(k) / sqrt(c) the exploitation stops and l(k) = l.
 *
 * The sets involved are supports: "reached in exactly j steps" means
 * (P^T)^j(q', x) > 0, each node once however many walks reach it.  Round l
 * therefore traverses
 *     sum_{l'=0..l} sum_{q' in S_{l-l'}(k)} sum_{x in S_{l'}(q')} d_in(x)
 * edges, S_j(v) being the exact-j-step support of v.  The printed loop is
 * open-ended; two readings close it:
 *   - when round l traverses no edge at all, no walk from v_k survives l + 1
 *     steps, every first meeting lies within l steps and l(k) = l (the
 *     exploitation is then exact);
 *   - the caller passes a cap: l(k) = min(l_printed(k), cap), so rounds
 *     0..cap-1 are the only ones ever counted.
 * The threshold test is the float64 comparison (double)E >= T with
 * T = (2 R(k)) / sqrt(c) computed by the caller.
 *
 * The loops below follow that description directly: each support is
 * rebuilt by a breadth-first sweep whenever the printed loop needs it
 * (nothing is cached between origins), with a per-thread stamp array to
 * keep every node once per level.  Nodes are independent (OpenMP).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t* mark;   /* stamp per node */
  uint32_t stamp;
  int32_t* buf[2]; /* level lists of the inner sweep */
  int64_t cap_buf[2];
  int32_t** lev;   /* outer levels S_0(k) .. S_{cap-1}(k) */
  int64_t* lev_n;
  int64_t* lev_cap;
} Scratch;

static void* grow(void* p, int64_t* cap, int64_t need, size_t elem) {
  if (need <= *cap) return p;
  int64_t c = *cap ? *cap : 1024;
  while (c < need) c *= 2;
  p = realloc(p, (size_t)c * elem);
  if (!p) abort();
  *cap = c;
  return p;
}

static uint32_t next_stamp(Scratch* s, int32_t n) {
  if (++s->stamp == 0x7fffffffu) {
    memset(s->mark, 0, sizeof(int32_t) * (size_t)n);
    s->stamp = 1;
  }
  return s->stamp;
}

/* out <- distinct in-neighbours of the nodes in `in` (one step of the
 * support: S_{j+1} = union over x in S_j of I(x)); returns its size. */
static int64_t step_support(Scratch* s, int32_t n, const int64_t* in_off, const int32_t* in_idx, const int32_t* in,
                            int64_t nin, int32_t** out, int64_t* out_cap) {
  const int32_t st = (int32_t)next_stamp(s, n);
  int64_t cnt = 0;
  for (int64_t i = 0; i < nin; ++i) {
    const int32_t x = in[i];
    for (int64_t e = in_off[x]; e < in_off[x + 1]; ++e) {
      const int32_t q = in_idx[e];
      if (s->mark[q] != st) {
        s->mark[q] = st;
        *out = (int32_t*)grow(*out, out_cap, cnt + 1, sizeof(int32_t));
        (*out)[cnt++] = q;
      }
    }
  }
  return cnt;
}

/* sum of d_in(x) over x in S_j(origin): the edges the printed loop traverses
 * when it extends the origin's table from step j to step j + 1. */
static int64_t edges_from_level(Scratch* s, int32_t n, const int64_t* in_off, const int32_t* in_idx, int32_t origin,
                                int32_t j) {
  s->buf[0] = (int32_t*)grow(s->buf[0], &s->cap_buf[0], 1, sizeof(int32_t));
  s->buf[0][0] = origin;
  int64_t cnt = 1;
  int cur = 0;
  for (int32_t t = 0; t < j && cnt > 0; ++t) {
    cnt = step_support(s, n, in_off, in_idx, s->buf[cur], cnt, &s->buf[1 - cur], &s->cap_buf[1 - cur]);
    cur = 1 - cur;
  }
  int64_t e = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    const int32_t x = s->buf[cur][i];
    e += in_off[x + 1] - in_off[x];
  }
  return e;
}

/* min(l_printed(k), cap) for one node; costs[l] (if non-NULL) receives the
 * edges traversed in round l for the rounds that ran (-1 for the others;
 * a round cut short by the threshold records the edges up to the cut). */
static int32_t node_level(Scratch* s, int32_t n, const int64_t* in_off, const int32_t* in_idx, int32_t k, double T,
                          int32_t cap, int64_t* costs) {
  if (costs)
    for (int32_t l = 0; l < cap; ++l) costs[l] = -1;
  /* outer supports S_0(k) = {k}, S_1(k), ... as the rounds need them */
  s->lev[0] = (int32_t*)grow(s->lev[0], &s->lev_cap[0], 1, sizeof(int32_t));
  s->lev[0][0] = k;
  s->lev_n[0] = 1;
  int64_t E = 0;
  for (int32_t l = 0; l < cap; ++l) {
    if (l > 0)
      s->lev_n[l] = step_support(s, n, in_off, in_idx, s->lev[l - 1], s->lev_n[l - 1], &s->lev[l], &s->lev_cap[l]);
    int64_t cost = 0;
    for (int32_t lp = 0; lp <= l; ++lp) {
      const int32_t d = l - lp;
      for (int64_t i = 0; i < s->lev_n[d]; ++i) {
        cost += edges_from_level(s, n, in_off, in_idx, s->lev[d][i], lp);
        if ((double)(E + cost) >= T) {
          if (costs) costs[l] = cost;
          return l;
        }
      }
    }
    if (costs) costs[l] = cost;
    if (cost == 0) return l; /* no walk from v_k survives l + 1 steps */
    E += cost;
  }
  return cap;
}

/* ell[i] = min(l_printed(nodes[i]), cap) with threshold T[i]; costs
 * (nullable) [nnodes][cap] as in node_level.  in_off int64 [n+1], in_idx
 * int32 [m]: in-neighbour lists.  Returns 0, or -1 for a bad argument. */
int lde_levels(int32_t n, const int64_t* in_off, const int32_t* in_idx, int64_t nnodes, const int32_t* nodes,
               const double* T, int32_t cap, int32_t* ell, int64_t* costs) {
  if (n < 1 || cap < 0 || nnodes < 0) return -1;
  int bad = 0;
#pragma omp parallel reduction(| : bad)
  {
    Scratch s;
    memset(&s, 0, sizeof(s));
    s.mark = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    const int32_t nl = cap > 0 ? cap : 1;
    s.lev = (int32_t**)calloc((size_t)nl, sizeof(int32_t*));
    s.lev_n = (int64_t*)calloc((size_t)nl, sizeof(int64_t));
    s.lev_cap = (int64_t*)calloc((size_t)nl, sizeof(int64_t));
    if (!s.mark || !s.lev || !s.lev_n || !s.lev_cap) abort();
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < nnodes; ++i) {
      const int32_t k = nodes[i];
      if (k < 0 || k >= n) {
        bad = 1;
        continue;
      }
      ell[i] = node_level(&s, n, in_off, in_idx, k, T[i], cap, costs ? costs + i * (int64_t)cap : NULL);
    }
    for (int32_t l = 0; l < nl; ++l) free(s.lev[l]);
    free(s.lev);
    free(s.lev_n);
    free(s.lev_cap);
    free(s.buf[0]);
    free(s.buf[1]);
    free(s.mark);
  }
  return bad ? -1 : 0;
}
