/*
 * exactsim.h -- C ABI of the MI355X ExactSim library (libexactsim.so).
 *
 * ExactSim (Wang, Wei, Yuan, Du, Wen: "Exact Single-Source SimRank
 * Computation on Large Graphs", SIGMOD 2020) answers a single-source SimRank
 * query: given a directed graph G, a source node u, the decay factor c and an
 * additive error eps, return s(u, .), an estimate of column u of the SimRank
 * matrix S of Eq. 1 (Section 1) with error at most eps for every node with
 * probability at least 1 - 1/n (Theorem 1, Section 3.1), and optionally its
 * top-k entries (Section 1, single-source and top-k queries).
 *
 * A query runs the steps of Algorithm 1 (basic ExactSim) with the sample
 * allocation of Section 3.2:
 *   es_forward      l-hop Personalized PageRank vectors pi^l and pi
 *                   (Algorithm 1)
 *   es_budget       per-node walk-pair counts R(k) (Algorithm 1;
 *                   Section 3.2, sampling in proportion to pi(k)^2)
 *   es_walk_pairs   meeting counts M(k) of R(k) pairs of sqrt(c)-walks from
 *                   each node (Algorithm 2)
 *   es_diag         D^(k,k) = (R(k) - M(k)) / R(k) (Algorithm 2; the exact
 *                   cases that open Algorithm 3)
 *   es_backward     s^L = 1/(1-sqrt c) sum_l (sqrt c P^T)^l D^ pi^l by the
 *                   nested recursion of Algorithm 1's back-accumulation
 *   es_topk         k largest entries of s (Section 1, top-k query)
 * es_single_source runs all of them; es_batch runs many sources and many
 * graphs at once with shared walk samples.
 *
 * Conventions for every call:
 *  - Nothing is thrown across this boundary.  Every call returns an
 *    es_status; es_last_error(ctx) holds a message for the last failure on
 *    that context.
 *  - "device" pointers are HIP device memory owned by the caller (for
 *    example PyTorch tensors); "host" pointers are ordinary host memory.
 *    Handles (es_ctx, es_graph) are owned by the library and released with
 *    their *_destroy call.
 *  - Work is enqueued asynchronously on the context's HIP stream.  Calls that
 *    return values through host pointers synchronize that stream first.
 *  - One context per host thread; calls on one context must not overlap.
 *    A graph handle holds the level passes' scratch (partial sums, the
 *    binned values), so calls on one graph must not overlap either, even
 *    from different contexts.
 *  - Node ids are int32 in [0, n); edge and sample counts are 64-bit.
 *  - Results are a pure function of the graph, the source, the options of
 *    es_query_opts and the network weights: they do not depend on launch
 *    shapes, batch composition or stream.  pi^l, R(k) and M(k) are bit-exact; s is float64
 *    with summation order left to the kernels.
 */
#ifndef EXACTSIM_H
#define EXACTSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct es_ctx es_ctx;
typedef struct es_graph es_graph;

typedef enum {
  ES_OK = 0,
  ES_EINVAL = -1,        /* an argument is out of its documented range */
  ES_ERANGE = -2,        /* n or m exceeds the int32 index range */
  ES_ENOMEM = -3,        /* device or host allocation failed */
  ES_EDEVICE = -4,       /* a HIP runtime call failed */
  ES_EOVERFLOW = -5,     /* the total sample count would reach 2^63 */
  ES_EUNSUPPORTED = -6   /* valid request the library does not implement */
} es_status;

typedef enum {
  ES_ALLOC_PI2 = 0,      /* R(k) = ceil(R pi(k)^2)          (Section 3.2)      */
  ES_ALLOC_PI = 1,       /* R(k) = ceil(R pi(k))            (Algorithm 1)     */
  ES_ALLOC_LEARNED = 2   /* R(k) = ceil(R pi(k)^2 v(k)/vbar), v from the budget
                            network; see es_mlp_load                          */
} es_alloc;

/* es_graph_from_edges flags */
#define ES_DEDUP 1u            /* merge repeated (src, dst) pairs: Eq. 1 uses neighbour sets */
#define ES_DROP_SELF_LOOPS 2u  /* drop (v, v) edges */
/* Level pass of es_forward / es_backward (and of a whole query); with neither
 * flag, graphs of at least 2^24 nodes take the binned pass, smaller ones the
 * pull pass.  Both give the same pi^l bit for bit. */
#define ES_LEVELS_PULL 4u      /* each row gathers its terms (two int32 CSRs only)          */
#define ES_LEVELS_BINNED 8u    /* push form in bins of destination rows: the sources are
                                  streamed, one 8-byte value per edge is written to its
                                  bin and summed there in LDS; costs 24 bytes per edge of
                                  device memory more (per direction a 2-byte source slot,
                                  a 4-byte position and a 2-byte row slot; the values)
                                  and is the faster pass once the level vectors no
                                  longer fit in the caches                               */

typedef struct {
  double c;                  /* decay factor, 0 < c <= 0.99 (the paper uses 0.6)            */
  double eps;                /* additive error, 0 < eps < 1                                 */
  uint64_t seed;             /* word 0 of the Philox key of the walk stream                 */
  double r_scale;            /* multiplies R = 6 ln n / ((1-sqrt c)^4 eps^2); 1 = the paper */
  int32_t alloc;             /* es_alloc                                                    */
  int32_t exact_small_din;   /* nonzero: nodes with d_in 0 / 1 take D = 1 / 1-c, no samples  */
  const double* d_override;  /* device [n] or NULL: use this diagonal instead of sampling   */
  double v_floor_ratio;      /* ES_ALLOC_LEARNED: floor f in [0, 1] on v(k) / vbar (below;
                                ES_LEARNED_FLOOR = 1/2 recommended, 0 = none)              */
  int32_t lde;               /* local deterministic exploitation (Algorithm 3; below):
                                ES_LDE_OFF, ES_LDE_AS_PRINTED or ES_LDE_REDUCED            */
  double sparse_eps;         /* sparse linearization (Section 3.2, Lemma 2): 0 keeps the
                                levels dense; in (0, 1) the back-accumulation reads only
                                the entries pi^l(k) > (1-sqrt c)^2 sparse_eps, which
                                lowers s(u, j) by at most sparse_eps (es_forward_sparse) */
  int32_t lde_max_level;     /* Algorithm 3: cap on l(k), 1..ES_LDE_MAX_LEVEL; any other
                                value runs the printed rule uncapped (es_lde_plan)         */
} es_query_opts;

typedef enum {
  ES_LDE_OFF = 0,         /* Algorithm 2 for every node                                   */
  ES_LDE_AS_PRINTED = 1,  /* Algorithm 3 with R(k) non-stop pairs                         */
  ES_LDE_REDUCED = 2      /* Algorithm 3 with ceil(R(k) c^l(k)) non-stop pairs            */
} es_lde_mode;

#define ES_LEARNED_FLOOR 0.5
#define ES_LDE_MAX_LEVEL 3     /* exact levels this library evaluates (Z_1..Z_3)          */

typedef struct {
  int32_t L;                 /* number of levels                                    */
  int32_t active_nodes;      /* nodes with R(k) > 0                                 */
  double R;                  /* total sample parameter (already times r_scale)     */
  uint64_t pairs;            /* walk pairs simulated (sum_k R(k); a batch shares them) */
  uint64_t pairs_requested;  /* sum over queries of sum_k R(k)                       */
  uint64_t meets;            /* sum_k M(k)                                          */
  uint64_t philox_blocks;    /* Philox4x64-10 blocks drawn by the walk kernel        */
  uint64_t walk_steps;       /* joint steps taken by the walk pairs                  */
  float ms_forward;          /* HIP-event times on the context stream: forward levels */
  float ms_budget;           /*   budget and sample-space scan                       */
  float ms_walk;             /*   the walk-pair kernel alone                         */
  float ms_diag;             /*   diagonal estimate                                  */
  float ms_backward;         /*   back-accumulation                                  */
  int32_t lde_source_level;  /* l(u) of the source under Algorithm 3 (0 when off)    */
  double lde_source_zsum;    /* sum_{l <= l(u)} Z_l(u), the source's exact part      */
  uint64_t level_entries;    /* pi^l entries stored for the back-accumulation:      */
                             /*   (L+1) n dense, the kept ones with sparse_eps > 0  */
  uint64_t level_bytes;      /* device bytes holding the levels: 8 (L+1) n dense;   */
                             /*   12 per kept entry plus the dense working slots    */
  uint64_t workspace_bytes;  /* device bytes the context's workspaces hold after the */
                             /*   call (they grow on demand and are kept)           */
} es_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the handle. */
es_status es_ctx_create(int device, void* hip_stream, es_ctx** out);
es_status es_ctx_destroy(es_ctx* ctx);
/* Block until all work enqueued on the context's stream has finished. */
es_status es_ctx_sync(es_ctx* ctx);
const char* es_status_str(es_status s);
/* Message for the last failing call on ctx (never NULL; "" if none). */
const char* es_last_error(const es_ctx* ctx);

/* ---- graph -------------------------------------------------------------- */

/* Build the device graph from m host edges src[e] -> dst[e].
 * The library keeps two int32 CSR copies in device memory: rows of the
 * out-CSR list O(v) (used by the forward pass P pi, pull form), rows of the
 * in-CSR list I(v) in ascending id order (walks and the backward pass
 * P^T s), plus 1/d_in(v) as float64 (Section 2: P(i,j) = 1/d_in(v_j) for
 * v_i in I(v_j)).  flags: ES_DEDUP, ES_DROP_SELF_LOOPS, and at most one of
 * ES_LEVELS_PULL / ES_LEVELS_BINNED.  Errors: ES_EINVAL (id outside [0,n),
 * NULL pointer, unknown or conflicting flags), ES_ERANGE (n < 1, n or
 * m >= 2^31), ES_ENOMEM. */
es_status es_graph_from_edges(es_ctx* ctx, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                              uint32_t flags, es_graph** out);
es_status es_graph_destroy(es_graph* g);
/* Node count and edge count after flags were applied (host outputs). */
es_status es_graph_info(const es_graph* g, int32_t* n, int64_t* m);
/* *binned (host) = 1 if the graph's level passes run binned, 0 if pull. */
es_status es_graph_level_pass(const es_graph* g, int32_t* binned);
/* Copy the in-degrees (device int32 [n]) and out-degrees (device int32 [n]);
 * either pointer may be NULL. */
es_status es_graph_degrees(es_ctx* ctx, const es_graph* g, int32_t* din, int32_t* dout);

/* ---- host constants ---------------------------------------------------- */

/* L = ceil(log_{1/c}(2/eps)), Algorithm 1's level count, computed as the smallest
 * L >= 0 with c^L <= eps/2 (c^L by repeated float64 multiplication). */
es_status es_num_levels(double c, double eps, int32_t* L);
/* R = 6 ln(n) / ((1-sqrt c)^4 eps^2) * r_scale (Algorithm 1), float64,
 * evaluated as ((6*log(n)) / (om4*(eps*eps))) * r_scale with om = 1-sqrt(c),
 * om4 = (om*om)*(om*om). */
es_status es_total_samples(int32_t n, double c, double eps, double r_scale, double* R);

/* ---- the steps of one query ------------------------------------------- */

/* Algorithm 1, l-hop PPR.  levels: device float64 [(L+1) * n], row l holds
 * pi^l = (1-sqrt c)(sqrt c P)^l e_u; pi: device float64 [n] = sum_l pi^l
 * summed in order of l.  Each pi^l(i) = sqrt(c) * (A * 2^-62) where A is the
 * exact int64 sum over j in O(v_i) of round(pi^(l-1)(j)/d_in(j) * 2^62)
 * (ties to even).  Errors: ES_EINVAL (u outside [0,n), L < 0, c outside
 * (0, 0.99]). */
es_status es_forward(es_ctx* ctx, const es_graph* g, int32_t u, double c, int32_t L, double* levels,
                     double* pi);

/* Sparse linearization (Section 3.2, Lemma 2).  Runs Algorithm 1's l-hop PPR
 * exactly as es_forward (same pi^l, same pi) but stores only the entries
 * pi^l(k) > theta = ((1-sqrt c)*(1-sqrt c))*sparse_eps (float64, in that
 * order): idx (device int32 [cap], node ids) and val (device float64 [cap],
 * pi^l(k)) receive the kept entries of level 0, then of level 1, ..., then of
 * level L, in no particular order within a level (each node at most once per
 * level); counts (host uint64 [L+1]) receives the number per level and pi
 * (device float64 [n], nullable) the full pi.  The levels' mass is at most 1,
 * so at most 1/theta entries are kept; es_sparse_capacity gives a cap that
 * always suffices.  Synchronizes the stream.  Errors: ES_EINVAL (as
 * es_forward; sparse_eps outside (0, 1); cap < 0; a NULL list with cap > 0),
 * ES_EOVERFLOW (more than cap entries: the lists hold the first cap). */
es_status es_forward_sparse(es_ctx* ctx, const es_graph* g, int32_t u, double c, int32_t L, double sparse_eps,
                            int64_t cap, int32_t* idx, double* val, uint64_t* counts, double* pi);
/* *cap = min((L+1) n, floor((1 + (L+1)(m+n) 2^-62)/theta) + 1): the kept entries
 * exceed theta and sum to at most the levels' mass, 1 plus the forward pass's
 * rounding.  Errors: ES_EINVAL (negative sizes, c or sparse_eps out of range). */
es_status es_sparse_capacity(int32_t n, int64_t m, int32_t L, double c, double sparse_eps, int64_t* cap);

/* Algorithm 1's sample budget and Section 3.2.  Rk: device uint64 [n] receives
 * R(k) = ceil(R * (pi(k)*pi(k))) (ES_ALLOC_PI2) or ceil(R * pi(k))
 * (ES_ALLOC_PI); 0 where pi(k) = 0 and, with exact_small_din, where
 * d_in(k) <= 1.  ES_ALLOC_LEARNED needs weights loaded by es_mlp_load.
 * If total is non-NULL (host), the stream is synchronized and sum_k R(k)
 * written there.  Errors: ES_EINVAL, ES_EOVERFLOW (R + n >= 2^63). */
es_status es_budget(es_ctx* ctx, const es_graph* g, const double* pi, double R, int32_t alloc,
                    int32_t exact_small_din, uint64_t* Rk, uint64_t* total);

/* Algorithm 2.  M: device uint64 [n] receives, for every node k, the number
 * of meeting pairs among pairs r in [r_begin(k), r_end(k)) of sqrt(c)-walk
 * pairs from v_k (r_begin: device uint64 [n] or NULL for 0; r_end: device
 * uint64 [n], usually R(k)).  Pair r of node k draws its randomness from
 * Philox4x64-10 under key (seed, 0): its joint lifetime T (Pr[T >= t] = c^t,
 * inverse transform against floor(c^t 2^64)) from word r mod 4 of the block
 * with counter (k, floor(r/4), 0, 1), and the words that move both walks at
 * step t from the block with counter (k, r, floor((t-1)/2), 0), words 0-1 at
 * odd t and 2-3 at even t.  A walk moves to in-neighbour floor(w * d_in / 2^64)
 * of its node in ascending id order, a walk on a node without in-neighbours
 * ends the pair, and the pair meets when both walks stand on the same node
 * after the same step t >= 1.  Because each pair is a pure function of
 * (seed, k, r), any split of the sample ranges gives the same counts.
 * Errors: ES_EINVAL (c outside (0, 0.99]), ES_EOVERFLOW (total >= 2^63). */
es_status es_walk_pairs(es_ctx* ctx, const es_graph* g, const uint64_t* r_begin, const uint64_t* r_end,
                        uint64_t seed, double c, uint64_t* M);

/* Algorithm 2 (estimate) and the exact cases that open Algorithm 3.  D: device float64 [n]:
 * (R(k) - M(k)) / R(k) where R(k) > 0; with exact_small_din, 1 where
 * d_in(k) = 0 and 1 - c where d_in(k) = 1; 1 elsewhere (pi(k) = 0, unused). */
es_status es_diag(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, const uint64_t* M, double c,
                  int32_t exact_small_din, double* D);

/* Algorithm 1, back-accumulation.  levels as written by es_forward (L+1 rows),
 * D: device float64 [n]; s: device float64 [n] receives
 * s^L with s^0 = D pi^L/(1-sqrt c) and
 * s^l(j) = sqrt(c) * (1/d_in(j)) * sum_{i in I(v_j)} s^(l-1)(i) + D(j) pi^(L-l)(j)/(1-sqrt c).
 * The sum over I(v_j) is float64 added in list order on a pull-pass graph;
 * on a binned graph every term is rounded to a multiple of 2^-72 (ties away
 * from zero), summed exactly in 128-bit integers and converted to float64
 * (terms of magnitude 2^24 or more are outside its range; with D in [0, 1]
 * and c <= 0.99 every term is below 1/(1-sqrt c)^2 < 2^16, since P^T
 * averages).  Both orders are fixed, so a graph's results repeat bit for
 * bit. */
es_status es_backward(es_ctx* ctx, const es_graph* g, const double* levels, int32_t L, const double* D,
                      double c, double* s);

/* Whole query: every step above with library-owned workspaces.
 * s_out: device float64 [n].  stats (host, nullable) is filled after a
 * stream synchronization.  With opts->sparse_eps > 0 the forward pass keeps
 * the levels as es_forward_sparse does, the sample budget uses the full pi, and
 * s^l(j) = sqrt(c) (1/d_in(j)) sum_{i in I(v_j)} s^(l-1)(i), plus
 * D(j) pi^(L-l)(j)/(1-sqrt c) where pi^(L-l)(j) is kept.  Errors: as the
 * steps, plus ES_EINVAL for r_scale <= 0, eps outside (0, 1) or sparse_eps
 * outside [0, 1), and ES_EUNSUPPORTED when an uncapped Algorithm 3 needs
 * more than ES_LDE_MAX_LEVEL exact levels (es_lde_plan). */
es_status es_single_source(es_ctx* ctx, const es_graph* g, int32_t u, const es_query_opts* opts,
                           double* s_out, es_stats* stats);

/* Top-k query (Section 1): the k largest s(j) over j != exclude (exclude < 0:
 * none), in descending order, ties broken towards the smaller id.
 * s: device float64 [n]; idx_out: device int32 [k]; val_out: device float64
 * [k] or NULL.  Errors: ES_EINVAL (k < 1, k > n - (exclude >= 0)). */
es_status es_topk(es_ctx* ctx, const double* s, int32_t n, int32_t exclude, int32_t k, int32_t* idx_out,
                  double* val_out);

/* es_topk for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * selection and the same results, with its scratch (the selection state and
 * 4096 candidate keys and ids) in a fixed 64 KiB array that each device holds
 * for the life of the process, so the call allocates nothing.  Every call on
 * one device shares that array (each call re-initialises it): calls that
 * overlap in time on one device race, also across contexts.  Errors: as
 * es_topk, and ES_EINVAL for k > 4096 (the array's capacity). */
es_status es_topk_noalloc(es_ctx* ctx, const double* s, int32_t n, int32_t exclude, int32_t k, int32_t* idx_out,
                          double* val_out);

/* ---- local deterministic exploitation (Section 3.2, Algorithm 3) ----------
 * Z_l(k) is the probability that two sqrt(c)-walks from v_k first meet at
 * step l (Lemma 4 gives it from the transition probabilities), and
 * D(k,k) = 1 - sum_l Z_l(k).  Algorithm 3 computes Z_1..Z_l(k) exactly and
 * estimates the rest with R'(k) pairs of walks that do not stop during their
 * first l(k) steps (sqrt(c)-walks afterwards); M(k) counts those meeting
 * after step l(k) without meeting before:
 *   D^(k,k) = (1 - sum_{l <= l(k)} Z_l(k)) - c^l(k) M(k) / R'(k).
 * The level l(k) follows Algorithm 3's edge counter, for every node with
 * R(k) > 0: round l (l = 0, 1, ...) extends, for l' = 0..l and every node q'
 * that a walk from v_k reaches in exactly l - l' steps, the transition table
 * of q' from step l' to l' + 1 and counts one edge per in-neighbour of each
 * node in that table's support (each node once); l(k) is the round in which
 * the count reaches 2 R(k) / sqrt(c) (float64: E >= (2 R(k)) / sqrt(c)), or
 * the first round that counts no edge (then no walk survives another step
 * and the exact part is all of 1 - D(k,k)).  R'(k) = R(k)
 * (ES_LDE_AS_PRINTED) or ceil(R(k) c^l(k)) (ES_LDE_REDUCED: every pair weighs
 * at most 1/R(k) and has Bernoulli variance at most 1/4, so the Bernstein
 * bound of Theorem 1 holds as for R(k) plain pairs). */

/* Rk: device uint64 [n] (es_budget).  Writes, by external id: ell (device
 * int32 [n]) = l(k) = min(l_printed(k), max_level) for max_level in
 * 1..ES_LDE_MAX_LEVEL; for any other max_level the printed rule itself.
 * zsum (device float64 [n]) = sum_{l <= l(k)} Z_l(k), Rk_out (device uint64
 * [n]) = R'(k).  mode: es_lde_mode (ES_LDE_OFF gives l = 0 and R' = R).
 * Synchronizes the stream.  Errors: ES_EINVAL (c outside (0, 0.99], mode
 * outside 0..2), ES_EUNSUPPORTED (uncapped, and some node's rule asks for
 * more than ES_LDE_MAX_LEVEL levels; the outputs are then undefined). */
es_status es_lde_plan(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, double c, int32_t mode,
                      int32_t max_level, int32_t* ell, double* zsum, uint64_t* Rk_out);
/* Algorithm 3's sampling: es_walk_pairs with the pairs of node k taking
 * ell[k] (device int32 [n], 0..L) non-stop steps first; a meeting at a step
 * t <= ell[k] ends the pair uncounted, the joint lifetime is ell[k] + T. */
es_status es_walk_pairs_lde(es_ctx* ctx, const es_graph* g, const uint64_t* r_begin, const uint64_t* r_end,
                            const int32_t* ell, uint64_t seed, double c, uint64_t* M);
/* D^ above where ell[k] > 0, (R - M)/R where ell[k] = 0, the exact values of
 * es_diag for d_in <= 1 with exact_small_din. */
es_status es_diag_lde(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, const uint64_t* M, const int32_t* ell,
                      const double* zsum, double c, int32_t exact_small_din, double* D);

/* ---- learned walk budget --------------------------------------------------
 * Lemma 1 (Section 3.1) bounds the variance of s^L(j) by a sum over nodes k of
 * pi_i(k)^2 pi_j(k)^2 D(k,k)(1 - D(k,k)) / rho(k); the paper then bounds the
 * Bernoulli variance D(1-D) by 1 and allocates rho(k) ~ pi(k)^2 (Section 3.2).
 * The learned allocation keeps that factor: a network (6 -> 64 -> 64 -> 1,
 * ReLU, float32) predicts the meeting probability p(k) = 1 - D(k,k) in
 * (0, c) from local features, v(k) = max(p(1-p), 1e-6), and
 *   vbar = S1/S2, w(k) = max(v(k), f vbar),
 *   R(k) = ceil((R * (pi(k)*pi(k))) * (w(k) * S2/S3)),
 *   S1 = sum Q(pi^2 v), S2 = sum Q(pi^2), S3 = sum Q(pi^2 w),
 *   Q(x) = round(x * 2^62) (exact int64 sums over the nodes that take samples),
 * which keeps the pi^2 rule's total and gives every node with pi(k) > 0 at
 * least one pair, so D^ stays unbiased.  The floor f keeps every node at no
 * less than about f times its pi^2 share: the bound behind Theorem 1
 * (Bernstein's inequality) has a range term besides the variance, and a node
 * left with a handful of pairs has a heavy-tailed error however small its
 * variance.  Weights: float32 [es_mlp_num_params()]
 * = W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3.
 * Features per node: log1p d_in, log1p d_out, log1p of the mean and of the
 * max in-degree of its in-neighbours, the mean of 1/d_in over its
 * in-neighbours (0 for those without in-neighbours), c/d_in.  D(k,k) does
 * not depend on the query source, and neither does any feature: a learned
 * query computes the predictions for its graph once per loaded network and
 * decay c, caches them in the graph (float32 [n] of device memory, freed by
 * es_graph_destroy) and reuses them for later queries.  Learned queries on
 * one graph from several contexts must therefore not overlap in time. */

int32_t es_mlp_num_params(void);
/* feats: device float32 [n][6] by external id. */
es_status es_mlp_features(es_ctx* ctx, const es_graph* g, double c, float* feats);
/* p_out, v_out: device float32 [N] (either may be NULL): p and v of each row of feats. */
es_status es_mlp_infer(es_ctx* ctx, const float* weights, const float* feats, int64_t N, double c, float* p_out,
                       float* v_out);
/* Training rows: feats [N][6], R, M device uint64 [N]: R(k) pairs of Algorithm 2
 * of which M(k) met.  Loss: sum_k w_k BCE(y_k, p_k) / sum_k w_k with the
 * observed meeting fraction y_k = M/R and weight w_k = min(R, 65536) (rows
 * with R = 0 carry no weight).  grad: device float32 [num_params]; loss
 * (host, nullable) receives the loss (synchronizes).  The sums over rows are
 * formed per block of 256 rows and added in block order, so the gradient
 * and a training run are the same bit for bit on every call; the context
 * keeps about 19 KB of device scratch per 256 rows for them. */
es_status es_mlp_grad(es_ctx* ctx, const float* weights, const float* feats, const uint64_t* R, const uint64_t* M,
                      int64_t N, double c, float* grad, double* loss);
/* `epochs` full-batch Adam steps (lr, betas 0.9 / 0.999, eps 1e-8) on that
 * loss, updating weights (device) in place; losses (host float [epochs],
 * nullable) gets the loss before each step (synchronizes). */
es_status es_mlp_train(es_ctx* ctx, const float* feats, const uint64_t* R, const uint64_t* M, int64_t N, double c,
                       int32_t epochs, float lr, float* weights, float* losses);
/* Copy the weights into the context for ES_ALLOC_LEARNED (NULL: unload).
 * Every call gives the context's network a new identity, so predictions
 * cached in graphs for earlier weights are recomputed on next use. */
es_status es_mlp_load(es_ctx* ctx, const float* weights);
/* The weighted allocation above with a given v (device float32 [n], external
 * order) and floor ratio f in [0, 1]: Rk device uint64 [n]. */
es_status es_budget_weighted(es_ctx* ctx, const es_graph* g, const double* pi, const float* v, double R,
                             int32_t exact_small_din, double floor_ratio, uint64_t* Rk);

/* ---- batches ------------------------------------------------------------ */

typedef struct {
  int32_t use_hip_graph;  /* nonzero: capture the batch in a hipGraph and replay it when the same
                             plan (graphs, block widths, options, workspace) comes again          */
  int32_t autotune;       /* nonzero: on first use of a (graph, block width) time the candidate
                             tilings of the level SpMM and keep the fastest                        */
  int32_t force_width;    /* 0, or lanes per row of the level SpMM (8, 16, 32 or 64, >= block width) */
  int32_t force_rows;     /* 0, or entries per lane per tile (rows per wave pass)                   */
  int32_t block_width;    /* 0: sources per block chosen by the autotuner when it is on (the width
                             of 64, 32, 16 or 8 whose level SpMM costs least per source), else 64;
                             1..64: that many sources per block                                    */
} es_batch_opts;

/* Many single-source queries at once (same c, eps, seed, r_scale, alloc):
 * query q asks for s(sources[q], .) on graphs[graph_of_query[q]].  Queries of
 * one graph are grouped in source blocks of at most 64 (es_batch_opts
 * block_width); each block runs the
 * level SpMV as one SpMM over its sources (Algorithm 1's l-hop PPR and
 * back-accumulation for every source at once) in a single fused launch per level across all blocks
 * and graphs, and the blocks draw shared walk samples: node k of a block
 * simulates max_b R_b(k) pairs once and source b uses pairs r < R_b(k)
 * (Algorithm 2), so every source's counts, and therefore its D^ and s, are the
 * ones its own single-source query gives.
 * graphs: host array [ngraphs]; graph_of_query, sources: host int32 [nq];
 * s_out: host array [nq] of device float64 [n of that graph] outputs.
 * bopts may be NULL (defaults: no hipGraph, autotune on).
 * With opts->sparse_eps > 0 every source keeps only its level entries above
 * (1-sqrt c)^2 sparse_eps, as its single-source query does, in one list for
 * the whole batch (the dense level of the moment stays in one slot).
 * With opts->alloc = ES_ALLOC_LEARNED every source takes its own weighted
 * allocation (the floor and the normalisation from that source's pi, as in
 * es_budget_weighted) over the graph's cached predictions.
 * stats (nullable): pairs = pairs simulated, pairs_requested = sum over queries,
 * meets = sum over queries of sum_k M(k), level_entries / level_bytes over the
 * batch; times are 0 except ms_walk (all walks).
 * Errors: as es_single_source; ES_EINVAL for a bad graph index, source,
 * width or block width, the learned allocation without a loaded network;
 * ES_EUNSUPPORTED for d_override, Algorithm 3 (lde != 0), or sparse levels
 * when a batch holds 2^31 or more (node, source) entries. */
es_status es_batch(es_ctx* ctx, const es_graph* const* graphs, int32_t ngraphs, const int32_t* graph_of_query,
                   const int32_t* sources, int32_t nq, const es_query_opts* opts, const es_batch_opts* bopts,
                   double* const* s_out, es_stats* stats);

/* The tiling the autotuner chose for graph g and source-block width B
 * (host outputs; 0 if not tuned yet). */
es_status es_batch_tuning(const es_graph* g, int32_t B, int32_t* width, int32_t* rows);
/* The source-block width the autotuner chose for a batch of S queries on g
 * (host output; 0 if not tuned yet). */
es_status es_batch_block_width(const es_graph* g, int32_t S, int32_t* width);

#ifdef __cplusplus
}
#endif

#endif /* EXACTSIM_H */
