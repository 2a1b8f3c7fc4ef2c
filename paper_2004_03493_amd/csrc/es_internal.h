// Internal declarations shared by the HIP translation units of libexactsim.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "es_host.h"
#include "exactsim.h"

namespace es {

// ---------------------------------------------------------------------------
// Sparse row partition used by both SpMV directions (pull form).
//
// The rows of a CSR matrix are cut into work blocks, one workgroup each:
//  * a multi-row block holds consecutive rows whose entries together fit the
//    workgroup's LDS staging buffer (kSpmvNnz values, at most kSpmvRows rows);
//  * a row with more than kSpmvNnz entries is a long row; it is cut into
//    chunks of kLongChunk entries, one workgroup per chunk, whose partial
//    sums are combined in chunk order by the last chunk to finish.
// ---------------------------------------------------------------------------
constexpr int kSpmvThreads = 512;
// kSpmvNnz, kSpmvRows, kLongChunk and BlockDesc: es_host.h

struct SpmvPlan {
  BlockDesc* blocks = nullptr;  // device
  int32_t nblocks = 0;
  int32_t nlong = 0;
  int32_t* long_p0 = nullptr;   // device [nlong]: first partial slot of each long row
  int32_t* long_nch = nullptr;  // device [nlong]: chunk count of each long row
  uint32_t* counters = nullptr; // device [nlong]: chunks finished (reset by the last one)
  void* partials = nullptr;     // device [nslots] x 8 bytes
  int32_t nslots = 0;
  int32_t max_row_nnz = 0;
};

// Binned level pass of one direction (push form; the layout is built on the
// host by build_binned): device copies plus the partial sums of split bins.
struct BinnedPlan {
  int32_t shift = 0, nbins = 0, nranges = 0, nitems = 0, nsplits = 0, nslots = 0;
  BinRange* ranges = nullptr;
  uint16_t* src_local = nullptr;
  uint32_t* pos = nullptr;
  uint16_t* row_local = nullptr;
  BinItem* items = nullptr;
  BinSplit* splits = nullptr;
  void* partials = nullptr;  // [nslots x 2^shift] row sums (8 or 16 bytes each)
};

struct BatchPlan;

// Source-independent sums of a node's transition tables (Algorithm 3's level
// rule and Lemma 4), cached per graph once computed: with S_j(v) the support
// of (P^T)^j(v, .), N_j = sum of d_in over S_j, SN1_2 = sum over S_2 of
// sum_{a in I(q)} d_in(a), C_j = sum_q (P^T)^j(v, q)^2, Cw_2 = sum_q
// (P^T)^2(v, q)^2 / d_in(q).  Computed in exact integer arithmetic, so a
// cached value equals a fresh one bit for bit.
struct LdeNodeStats {
  bool has2 = false, has3 = false;
  uint64_t N2 = 0, SN1_2 = 0, N3 = 0;
  double C2 = 0.0, Cw2 = 0.0, C3 = 0.0;
};

}  // namespace es

// One in-CSR entry for the walks: the in-neighbour's own row, so a walk step
// is one dependent load.  key names the node: its row offset when it has
// in-neighbours (such nodes have distinct offsets), -1 - id when it has none
// (never an offset, and never dereferenced); deg is its in-degree.  Eight
// bytes: half the footprint of a 16-byte record, 7% fewer fills from the
// memory side and 5% more pairs per second on R-MAT 2^20.
struct alignas(8) WalkEntry {
  int32_t key;
  int32_t deg;
};

// Device graph.  Nodes are stored under internal ids: the rank of the node by
// total degree (descending, ties by id), so that the hub entries every SpMV
// level gathers share few cache lines.  Callers only ever see external ids.
struct es_graph {
  int device = 0;
  uint64_t uid = 0;            // unique per handle in the process, never reused (keys cached batch plans)
  int32_t n = 0;
  int64_t m = 0;
  int32_t* out_off = nullptr;  // [n+1]  internal rows list O(v) (internal ids, ascending)
  int32_t* out_idx = nullptr;  // [m]
  int32_t* in_off = nullptr;   // [n+1]  internal rows list I(v): internal ids in ascending EXTERNAL id order
  int32_t* in_idx = nullptr;   // [m]
  WalkEntry* walk_adj = nullptr;  // [m]  in_idx[e] as its row: (key, d_in)
  double* inv_din = nullptr;   // [n]    1/d_in(v) by internal id, 0 where d_in = 0
  int32_t* din_int = nullptr;  // [n]    d_in by internal id
  int32_t* din_ext = nullptr;  // [n]    d_in by external id
  int32_t* dout_ext = nullptr; // [n]    d_out by external id
  int32_t* ext_of = nullptr;   // [n]    internal id -> external id
  int32_t* int_of = nullptr;   // [n]    external id -> internal id
  std::vector<int32_t> h_int_of;
  std::vector<int32_t> h_out_off, h_in_off;  // host copies of the offsets (batch tiling)
  // autotuned batch tiling per source-block width B: lanes per row W, entries
  // per lane G and the forward SpMM's time for three levels (ms)
  struct Tuned {
    int32_t B, W, G;
    float ms;
  };
  std::vector<Tuned> tuned;
  // block width the tuner chose for a graph's batch of S queries, by S
  std::vector<std::pair<int32_t, int32_t>> tuned_block;
  es::SpmvPlan fwd;            // over the out-CSR
  es::SpmvPlan back;           // over the in-CSR
  // binned level pass (graphs too large for the caches, or on request):
  // forward pushes along the in-lists, backward along the out-lists; one
  // 8-byte value per edge in between
  bool binned = false;
  es::BinnedPlan bfwd, bback;
  void* bin_vals = nullptr;    // [m] x 8 bytes
  // learned allocation: predicted variances v(k) by internal id for the
  // network identified by vhat_net at decay vhat_c (features and network
  // are source-independent, so one prediction serves every query)
  mutable float* vhat = nullptr;
  mutable uint64_t vhat_net = 0;
  mutable double vhat_c = 0.0;
  // Algorithm 3's level rule, by internal id (computed on first use):
  // sum of d_in over I(v), and sum of 1/d_in over I(v)
  mutable long long* lde_n1 = nullptr;
  mutable double* lde_g = nullptr;
  mutable std::unordered_map<int32_t, es::LdeNodeStats> lde_cache;
  mutable std::mutex lde_mu;
};

struct es_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 0;
  std::string last_error;
  // growable device workspaces, by slot
  std::vector<void*> ws;
  std::vector<size_t> ws_bytes;
  // walk lifetime thresholds for the cached decay factor
  uint64_t* thr = nullptr;
  uint64_t thr_head[16] = {};  // host copy of thresholds 1..16 (zeros past tmax)
  int32_t tmax = 0;
  double thr_c = -1.0;
  hipEvent_t ev[8] = {};
  hipEvent_t ev_walk_begin = nullptr;  // set while a query records stage times
  // learned-budget network weights (device), nullptr until loaded; mlp_id
  // is unique per es_mlp_load call across all contexts (0: none loaded)
  float* mlp_w = nullptr;
  uint64_t mlp_id = 0;
  // batch plans (tiles, descriptors, captured graph), by plan key
  es::BatchPlan* plans = nullptr;
  hipStream_t capture_stream = nullptr;
};

namespace es {

// workspace slots
enum Slot : int {
  kWsLevels = 0,
  kWsPi,
  kWsQ0,
  kWsQ1,
  kWsRk,
  kWsM,
  kWsD,
  kWsS0,
  kWsS1,
  kWsActive,
  kWsPrefix,
  kWsScanCnt,
  kWsScanSum,
  kWsTotals,
  kWsTopk,
  kWsMisc,
  kWsBatchT,
  kWsBatchMisc,
  kWsFeat,
  kWsVhat,
  kWsMlpSums,
  kWsMlpAcc,
  kWsMlpGrad,
  kWsMlpLoss,
  kWsLdeEll,
  kWsLdeZ,
  kWsLdeR,
  kWsLdeW,
  kWsLdeMisc,
  kWsLdeRin,
  kWsLdeCand,
  kWsLdeStats,
  kWsLdeEnt0,
  kWsLdeEnt1,
  kWsLdeCnt,
  kWsLdePre,
  kWsLdeTsum,
  kWsLdeKeys,
  kWsLdeVals,
  kWsLdeReg,
  kWsLdeSums,
  kWsLdeRows,
  kWsSpIdx,
  kWsSpVal,
  kWsSpCnt,
  kWsCount
};

// device-side totals of a sample-space scan
struct WalkTotals {
  unsigned long long total;     // sum of sample counts
  unsigned long long cursor;    // work-queue cursor of the walk kernel
  unsigned long long meets;     // sum of meeting counts
  unsigned long long blocks;    // Philox4x64-10 blocks drawn
  unsigned long long steps;     // joint walk steps taken
  int32_t n_active;             // nodes with a non-empty sample range
  int32_t overflow;             // nonzero if the sum reached 2^63
};

es_status fail(es_ctx* ctx, es_status st, const char* fmt, ...);
es_status hip_fail(es_ctx* ctx, hipError_t e, const char* what);
void* workspace(es_ctx* ctx, int slot, size_t bytes, es_status* st);
// device bytes held by the context's workspaces
uint64_t workspace_total(const es_ctx* ctx);

// lifetime threshold table for decay c, cached on the context
es_status lifetime_table(es_ctx* ctx, double c);

// Sparse linearization (Section 3.2, Lemma 2): the stored levels keep only the
// entries pi^l(k) > theta, in one list of (internal id, value) for all levels;
// level l's entries follow those of levels < l, in no particular order within
// the level.  cnt[l] counts level l's entries and cnt[L + 1] all of them; the
// list holds at most cap entries (more cannot occur: see sparse_capacity).
struct SparseLevels {
  double theta;
  int32_t nkeep;             // levels 0..nkeep-1 also stay dense in their slots
  int32_t* idx;              // device [cap]
  double* val;               // device [cap]
  unsigned long long* cnt;   // device [L + 2]
  uint64_t cap;
};
// An upper bound on the entries above theta over levels 0..L: their mass is at most 1.
uint64_t sparse_capacity(int32_t n, int64_t m, int32_t L, double theta);
// internal -> external ids over the whole list
es_status launch_sparse_ids(es_ctx* ctx, const es_graph* g, int32_t L, const SparseLevels& sp);
// Over a flat array of n elements (level l of any layout, ids < 2^31): add the
// level to pi (pi = level when first) and append its entries above theta.
es_status launch_level_keep(es_ctx* ctx, int64_t n, const double* lvl, bool first, double* pi, const SparseLevels& sp,
                            int32_t level, int32_t L);
// s[j] += a D[j] pi^level(j) over the stored entries of one level.
es_status launch_level_scatter(es_ctx* ctx, int64_t n, const SparseLevels& sp, int32_t level, const double* D,
                               double a, double* s);
es_status launch_fill(es_ctx* ctx, int64_t count, unsigned long long* p);
es_status launch_fill(es_ctx* ctx, int64_t count, double* p);

// launchers (enqueue on ctx->stream)
// Forward levels.  sp == NULL: levels holds L + 1 dense slots (pi^l in slot l).
// sp != NULL: levels holds sp->nkeep + 1 dense slots (pi^l in slot min(l, nkeep))
// and the kept entries go to sp.
es_status launch_forward(es_ctx* ctx, const es_graph* g, int32_t u, double c, int32_t L, double* levels,
                         double* pi, int64_t* q0, int64_t* q1, const SparseLevels* sp = nullptr);
es_status launch_budget(es_ctx* ctx, const es_graph* g, const double* pi, const int32_t* din, double R,
                        int32_t alloc, int32_t exact_small_din, const float* vhat, double vbar_inv, uint64_t* Rk);
// Walk pairs over sample counts indexed by internal ids (external_counts = false)
// or by external ids (external_counts = true); M is indexed like the counts.
// nonstop (indexed like the counts, or NULL): the non-stop pairs of Algorithm 3.
es_status launch_walks(es_ctx* ctx, const es_graph* g, const uint64_t* r_begin, const uint64_t* r_end,
                       uint64_t seed, double c, uint64_t* M, bool external_counts, WalkTotals** totals_out,
                       const int32_t* nonstop = nullptr);
// Shared samples of a block of B sources: Rmax[k] pairs per internal node k,
// meetings bucketed by T (ascending thresholds per node, stride B) into H[k * B + j].
es_status launch_walks_buckets(es_ctx* ctx, const es_graph* g, const uint64_t* Rmax, const uint64_t* T, int32_t B,
                               uint64_t seed, double c, uint64_t* H, WalkTotals** totals_out);
// Learned allocation (internal order): features, network, weighted budget.
// ensure_vhat computes the graph's predicted variances for the loaded
// network and decay c unless they are cached (stream-ordered; not capturable).
es_status ensure_vhat(es_ctx* ctx, const es_graph* g, double c);
es_status launch_learned_budget(es_ctx* ctx, const es_graph* g, const double* pi, double R, double c,
                                int32_t exact_small_din, double floor_ratio, uint64_t* Rk);
es_status launch_diag(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, const uint64_t* M, const int32_t* din,
                      double c, int32_t exact_small_din, double* D);

// Local deterministic exploitation (Algorithm 3), internal order.  Rk: budget.
// Writes l(k) = min(l_printed(k), max_level) (max_level outside 1..3: the
// printed rule uncapped, ES_EUNSUPPORTED where it needs more than 3 levels),
// the exact part sum_{l <= l(k)} Z_l(k) and the pair counts R'(k).
// Synchronizes the stream.
struct LdeOut {
  int32_t* ell;
  double* zsum;
  uint64_t* Rk2;
};
es_status launch_lde(es_ctx* ctx, const es_graph* g, const uint64_t* Rk, double c, int32_t mode, int32_t max_level,
                     LdeOut out);
es_status launch_diag_lde(es_ctx* ctx, int32_t n, const uint64_t* Rk, const uint64_t* M, const int32_t* ell,
                          const double* zsum, const int32_t* din, double c, int32_t exact_small_din, double* D);
// dst[row * n + i] = src[row * n + map[i]] for rows = 0..rows-1
es_status launch_permute_f64(es_ctx* ctx, int32_t n, int32_t rows, const double* src, const int32_t* map, double* dst);
// Back-accumulation from the dense levels (sp == NULL, levels [L + 1][n]) or
// from the stored entries of sparse linearization (levels unused).
es_status launch_backward(es_ctx* ctx, const es_graph* g, const double* levels, int32_t L, const double* D,
                          double c, double* s, double* s_tmp, const SparseLevels* sp = nullptr);
es_status launch_topk(es_ctx* ctx, const double* s, int32_t n, int32_t exclude, int32_t k, int32_t* idx_out,
                      double* val_out);
// Finds this context's device copy of the fixed top-k scratch (context creation).
es_status topk_scratch_init(es_ctx* ctx);
es_status build_plan(es_ctx* ctx, const int32_t* off_host, int32_t n, SpmvPlan* plan);
void free_batch_plans(es_ctx* ctx);
void free_plan(SpmvPlan* plan);
// Binned layout of the push lists (off, idx) uploaded with partial-sum room
// of row_bytes per row of every split bin.
es_status build_binned_plan(es_ctx* ctx, const int32_t* off, const int32_t* idx, int32_t n, int32_t shift,
                            size_t row_bytes, BinnedPlan* plan);
void free_binned_plan(BinnedPlan* plan);
// rows per bin of the two directions: 2^14 int64 sums (forward, 128 KiB of
// LDS), 2^12 128-bit sums (backward, 64 KiB)
constexpr int32_t kBinShiftFwd = 14;
constexpr int32_t kBinShiftBack = 12;
// graphs with at least this many nodes take the binned pass unless the
// caller asks for the pull pass
constexpr int32_t kBinnedAutoNodes = 1 << 24;

// host constants
int32_t num_levels(double c, double eps);
double total_samples(int32_t n, double c, double eps, double r_scale);

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace es

#define ES_CHECK_HIP(ctx, call)                          \
  do {                                                   \
    hipError_t es_e_ = (call);                           \
    if (es_e_ != hipSuccess) return es::hip_fail((ctx), es_e_, #call); \
  } while (0)

#define ES_TRY(expr)                 \
  do {                               \
    es_status es_s_ = (expr);        \
    if (es_s_ != ES_OK) return es_s_; \
  } while (0)
