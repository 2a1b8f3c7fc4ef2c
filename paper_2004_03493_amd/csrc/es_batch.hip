// Batched queries: blocks of up to 64 sources on one or more graphs.
//
// Per (node, source) arrays of every block live in flat buffers, node-major
// within a block (element base + r * B + b), so that one SpMM edge gathers the
// B contiguous values of a row.  The level SpMM (Algorithm 1's l-hop PPR and
// back-accumulation for all sources at once) runs as one launch per level over a tile list
// that covers every block of every graph: a tile is a run of rows of one block
// handled by one wave, whose 64 lanes form 64/W groups of W lanes; lane b of a
// group owns source column b.  Rows longer than kLongRow are cut into chunks
// that whole waves sum into one partial slot per chunk; a small launch after
// the level adds each row's partials in chunk order, so the sums do not
// depend on which wave finishes first.  The walk phase shares samples inside a
// block: node k simulates max_b R_b(k) pairs and the meetings are bucketed by
// the block's sorted per-source counts, so source b sees exactly the meetings of
// its own pairs r < R_b(k).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "es_internal.h"

namespace es {

namespace {

constexpr int kBatchMaxB = 64;
constexpr int kSpmmThreads = 256;  // four independent waves
constexpr double kFix = 0x1p62;
constexpr double kFixInv = 0x1p-62;

struct BEntry {
  const int32_t* out_off;
  const int32_t* out_idx;
  const int32_t* in_off;
  const int32_t* in_idx;
  const double* inv_din;
  const int32_t* din;
  const int32_t* int_of;
  const float* vhat;  // learned allocation: predicted variances by internal id (else unused)
  int32_t n;
  int32_t B;
  int32_t W;
  int32_t nlong_fwd;
  int32_t nlong_back;
  int32_t pad;
  double R;           // total sample parameter of the block's graph
  int64_t base;       // first flat element of the block
  int64_t node_base;  // first flat node of the block (arrays of length n)
  int64_t long_base;  // first long-row slot (x B) of the block
  int64_t src_base;   // first source / output index of the block
};

// ---- level operators ------------------------------------------------------

struct FwdOp {
  using V = int64_t;
  static constexpr bool kForward = true;
  const int64_t* __restrict__ qprev;
  int64_t* __restrict__ qnext;
  double* __restrict__ lvl;
  long long* __restrict__ acc;  // long-row chunk partials
  double sc;
  __device__ __forceinline__ V gather(const BEntry& E, int32_t col, int sub) const {
    return qprev[E.base + (int64_t)col * E.B + sub];
  }
  __device__ __forceinline__ void epi(const BEntry& E, int32_t r, int sub, V a) const {
    const int64_t i = E.base + (int64_t)r * E.B + sub;
    const double p = sc * ((double)a * kFixInv);
    lvl[i] = p;
    qnext[i] = (int64_t)rint((p * E.inv_din[r]) * kFix);
  }
  __device__ __forceinline__ void long_put(const BEntry& E, int32_t slot, int sub, V a) const {
    acc[(E.long_base + slot) * kBatchMaxB + sub] = a;
  }
  __device__ __forceinline__ V long_get(const BEntry& E, int32_t slot, int sub) const {
    return acc[(E.long_base + slot) * kBatchMaxB + sub];
  }
};

struct BackOp {
  using V = double;
  static constexpr bool kForward = false;
  const double* __restrict__ sprev;
  double* __restrict__ snext;
  const double* __restrict__ D;
  const double* __restrict__ lvl;  // level L - l; NULL: sparse levels, added afterwards by a scatter
  double* __restrict__ acc;
  double sc, a;
  __device__ __forceinline__ V gather(const BEntry& E, int32_t col, int sub) const {
    return sprev[E.base + (int64_t)col * E.B + sub];
  }
  __device__ __forceinline__ void epi(const BEntry& E, int32_t r, int sub, V v) const {
    const int64_t i = E.base + (int64_t)r * E.B + sub;
    if (lvl) snext[i] = sc * (E.inv_din[r] * v) + a * (D[i] * lvl[i]);
    else snext[i] = sc * (E.inv_din[r] * v);
  }
  __device__ __forceinline__ void long_put(const BEntry& E, int32_t slot, int sub, V v) const {
    acc[(E.long_base + slot) * kBatchMaxB + sub] = v;
  }
  __device__ __forceinline__ V long_get(const BEntry& E, int32_t slot, int sub) const {
    return acc[(E.long_base + slot) * kBatchMaxB + sub];
  }
};

// Column ids come in one coalesced load per group (W of them; 64 per wave on a
// long-row chunk) and are broadcast by lane shuffles, so a row's gathers are
// issued eight at a time instead of behind their own index loads.  Each group
// adds its entries in increasing entry order, as a plain loop would.
template <class Op>
__global__ __launch_bounds__(kSpmmThreads) void spmm_kernel(const MTile* __restrict__ tiles, int32_t ntiles,
                                                            const BEntry* __restrict__ ents, Op op) {
  using V = typename Op::V;
  const int wave = blockIdx.x * (kSpmmThreads / 64) + (threadIdx.x >> 6);
  if (wave >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const MTile t = tiles[wave];
  const BEntry E = ents[t.entry];
  const int W = E.W;
  const int P = 64 / W;
  const int grp = lane / W, sub = lane - grp * W;
  const int gl = grp * W;  // the group's first lane
  const bool vb = sub < E.B;
  const int32_t* __restrict__ off = Op::kForward ? E.out_off : E.in_off;
  const int32_t* __restrict__ idx = Op::kForward ? E.out_idx : E.in_idx;
  if (t.row1 >= 0) {
    // the shuffles read lanes of the reader's own group, which runs the same row
    for (int32_t r = t.row0 + grp; r < t.row1; r += P) {
      const int32_t e0 = off[r], e1 = off[r + 1];
      V acc = 0;
      for (int32_t eb = e0; eb < e1; eb += W) {
        const int32_t nc = min(W, e1 - eb);
        const int32_t col = sub < nc ? idx[eb + sub] : 0;
        int32_t j = 0;
        for (; j + 8 <= nc; j += 8) {
          int32_t c[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) c[u] = __shfl(col, gl + j + u, 64);
          if (vb) {
            V v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = op.gather(E, c[u], sub);
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
          }
        }
        for (; j < nc; ++j) {
          const int32_t c0 = __shfl(col, gl + j, 64);
          if (vb) acc += op.gather(E, c0, sub);
        }
      }
      if (vb) op.epi(E, r, sub, acc);
    }
  } else {
    // one chunk of a long row: group grp takes the entries grp, grp + P, ...
    // (wave-uniform trip counts, so every shuffle has all lanes active)
    V acc = 0;
    for (int32_t eb = t.e0; eb < t.e1; eb += 64) {
      const int32_t nb = min(64, t.e1 - eb);
      const int32_t col = lane < nb ? idx[eb + lane] : 0;
      for (int32_t j0 = 0; j0 < nb; j0 += 8 * P) {
        int32_t c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int32_t j = j0 + grp + u * P;
          c[u] = __shfl(col, j < 64 ? j : 63, 64);
        }
        if (vb) {
          V v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = (j0 + grp + u * P < nb) ? op.gather(E, c[u], sub) : (V)0;
#pragma unroll
          for (int u = 0; u < 8; ++u) acc += v[u];
        }
      }
    }
    for (int m = W; m < 64; m <<= 1) acc += __shfl_xor(acc, m, 64);
    if (grp == 0 && vb) op.long_put(E, -t.row1 - 1, sub, acc);
  }
}

template <class Op>
__global__ void long_finish_kernel(const LongRow* __restrict__ rows, int32_t nrows, const BEntry* __restrict__ ents,
                                   Op op) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t lr = i / kBatchMaxB;
  const int sub = (int)(i % kBatchMaxB);
  if (lr >= nrows) return;
  const LongRow L = rows[lr];
  const BEntry E = ents[L.entry];
  if (sub >= E.B) return;
  typename Op::V v = 0;
  for (int32_t c = 0; c < L.nch; ++c) v += op.long_get(E, L.slot + c, sub);
  op.epi(E, L.row, sub, v);
}

// ---- per-block elementwise kernels (grid.y = block) -------------------------

__global__ void bat_forward_init(const BEntry* __restrict__ ents, const int32_t* __restrict__ src_int, double pi0,
                                 double* __restrict__ lvl0, int64_t* __restrict__ q0) {
  const BEntry E = ents[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (int64_t)E.n * E.B;
  if (i >= nb) return;
  const int32_t r = (int32_t)(i / E.B);
  const int32_t b = (int32_t)(i - (int64_t)r * E.B);
  const bool hit = src_int[E.src_base + b] == r;
  lvl0[E.base + i] = hit ? pi0 : 0.0;
  q0[E.base + i] = hit ? (int64_t)rint((pi0 * E.inv_din[r]) * kFix) : 0;
}

__global__ void bat_sum_levels(int64_t NB, int32_t L, const double* __restrict__ levels, double* __restrict__ pi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NB) return;
  double acc = levels[i];
  for (int l = 1; l <= L; ++l) acc = acc + levels[(int64_t)l * NB + i];
  pi[i] = acc;
}

__global__ void bat_budget(const BEntry* __restrict__ ents, const double* __restrict__ pi, int32_t alloc,
                           int32_t exact_small_din, uint64_t* __restrict__ Rk) {
  const BEntry E = ents[blockIdx.y];
  const double R = E.R;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (int64_t)E.n * E.B;
  if (i >= nb) return;
  const int32_t r = (int32_t)(i / E.B);
  const double p = pi[E.base + i];
  const double want = alloc == ES_ALLOC_PI ? R * p : R * (p * p);
  uint64_t c = (uint64_t)ceil(want);
  if (p == 0.0) c = 0;
  if (exact_small_din && E.din[r] <= 1) c = 0;
  Rk[E.base + i] = c;
}

// Learned allocation per source of a block, the single-source rule in the
// block layout: pass 0 adds Q(pi^2 v) and Q(pi^2) over the source's nodes,
// pass 1 Q(pi^2 max(v, thr)) and Q(pi^2) (Q(x) = round(x 2^62), exact
// integer sums); each thread keeps one source's sums, then LDS, then one
// global add per workgroup and source.
__global__ __launch_bounds__(256) void bat_learned_sums(const BEntry* __restrict__ ents, const double* __restrict__ pi,
                                                        const double* __restrict__ thr, int32_t exact_small_din,
                                                        int32_t pass, unsigned long long* __restrict__ S) {
  __shared__ unsigned long long sa[kBatchMaxB], sb[kBatchMaxB];
  const BEntry E = ents[blockIdx.y];
  const int tid = threadIdx.x;
  if (tid < kBatchMaxB) {
    sa[tid] = 0ull;
    sb[tid] = 0ull;
  }
  __syncthreads();
  const int rows = blockDim.x / E.B;  // nodes per workgroup step
  const int b = tid % E.B;
  const int rl = tid / E.B;
  unsigned long long a = 0, c = 0;
  if (rl < rows) {
    const double t = pass ? thr[E.src_base + b] : 0.0;
    for (int64_t r = (int64_t)blockIdx.x * rows + rl; r < E.n; r += (int64_t)gridDim.x * rows) {
      const double p = pi[E.base + r * E.B + b];
      if (p > 0.0 && (!exact_small_din || E.din[r] >= 2)) {
        const double p2 = p * p;
        double w = (double)E.vhat[r];
        if (pass && t > w) w = t;
        a += (unsigned long long)(int64_t)rint((p2 * w) * 0x1p62);
        c += (unsigned long long)(int64_t)rint(p2 * 0x1p62);
      }
    }
    atomicAdd(&sa[b], a);
    atomicAdd(&sb[b], c);
  }
  __syncthreads();
  if (tid < E.B) {
    unsigned long long* d = S + (E.src_base + tid) * 4 + 2 * pass;
    if (sa[tid]) atomicAdd(&d[0], sa[tid]);
    if (sb[tid]) atomicAdd(&d[1], sb[tid]);
  }
}

// Per source: the floor thr = f * vbar after pass 0, vbar_inv = S3 / S2 after
// pass 1 (-1: no weighted mass, the plain pi^2 rule).
__global__ void bat_learned_scalars(int32_t nq, const unsigned long long* __restrict__ S, double floor_ratio,
                                    int32_t pass, double* __restrict__ thr, double* __restrict__ vbar_inv) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const unsigned long long* s = S + (int64_t)q * 4;
  if (pass == 0) {
    const int64_t s1 = (int64_t)s[0], s2 = (int64_t)s[1];
    thr[q] = s1 > 0 ? floor_ratio * ((double)s1 / (double)s2) : 0.0;
  } else {
    const int64_t s1 = (int64_t)s[2], s2 = (int64_t)s[3];
    vbar_inv[q] = s1 > 0 ? (double)s2 / (double)s1 : -1.0;
  }
}

__global__ void bat_budget_learned(const BEntry* __restrict__ ents, const double* __restrict__ pi,
                                   int32_t exact_small_din, const double* __restrict__ thr,
                                   const double* __restrict__ vbar_inv, uint64_t* __restrict__ Rk) {
  const BEntry E = ents[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (int64_t)E.n * E.B;
  if (i >= nb) return;
  const int32_t r = (int32_t)(i / E.B);
  const int32_t b = (int32_t)(i - (int64_t)r * E.B);
  const double p = pi[E.base + i];
  const double vi = vbar_inv[E.src_base + b];
  double want = E.R * (p * p);
  if (vi >= 0.0) {
    double w = (double)E.vhat[r];
    const double t = thr[E.src_base + b];
    if (t > w) w = t;
    want = want * (w * vi);
  }
  uint64_t c = (uint64_t)ceil(want);
  if (!(p > 0.0)) c = 0;
  if (exact_small_din && E.din[r] <= 1) c = 0;
  Rk[E.base + i] = c;
}

// One wave per node: sort the block's B counts ascending into T, Rmax = largest.
__global__ void bat_sort_counts(const BEntry* __restrict__ ents, const uint64_t* __restrict__ Rk,
                                uint64_t* __restrict__ T, uint64_t* __restrict__ Rmax) {
  const BEntry E = ents[blockIdx.y];
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= E.n) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = E.base + r * E.B;
  // lanes past B hold 0 and sort first; the B real counts end up in lanes 64-B..63
  uint64_t v = lane < E.B ? Rk[row + lane] : 0ull;
  for (int size = 2; size <= 64; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint64_t o = __shfl_xor(v, stride, 64);
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      // ascending runs where up, descending otherwise
      const bool take_min = (lower == up);
      v = take_min ? (o < v ? o : v) : (o > v ? o : v);
    }
  }
  const int j = lane - (64 - E.B);
  if (j >= 0) T[row + j] = v;
  if (lane == 63) Rmax[E.node_base + r] = v;
}

// M_b(k) = sum_{j <= #{b' : R_b'(k) < R_b(k)}} H[k][j];  D^ as in the single-source path.
// One group of B consecutive lanes per node (64 / B nodes per wave, the wave's
// spare lanes idle): the group scans the node's bucket counts, each source finds
// its bucket by a fixed-step search over the node's thresholds held one per
// lane, and reads the inclusive prefix there.  Grid-stride over a grid sized to
// the resident waves, so the two totals take few atomics.
__global__ void bat_finish_diag(const BEntry* __restrict__ ents, const uint64_t* __restrict__ Rk,
                                const uint64_t* __restrict__ T, const uint64_t* __restrict__ H, double c,
                                int32_t exact_small_din, double* __restrict__ D, unsigned long long* __restrict__ sums) {
  const BEntry E = ents[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int B = E.B;
  const int gpw = 64 / B;  // nodes per wave
  const int grp = lane / B;
  const int b = lane - grp * B;
  const bool used = grp < gpw;
  const int64_t nw = ((int64_t)E.n + gpw - 1) / gpw;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
  unsigned long long req = 0, met = 0;
  for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < nw; w += stride) {
    const int64_t r = w * gpw + grp;
    const bool live = used && r < E.n;
    const int64_t row = E.base + r * B;
    uint64_t h = live ? H[row + b] : 0ull;
    const uint64_t R = live ? Rk[row + b] : 0ull;
    const uint64_t Tb = live ? T[row + b] : ~0ull;
    for (int o = 1; o < B; o <<= 1) {  // inclusive scan within the group
      const uint64_t t = __shfl_up(h, o, 64);
      if (b >= o) h += t;
    }
    // lo = #{j : T[j] < R}, the thresholds ascending (R itself is one of them)
    int32_t lo = 0;
    for (int st = 64; st > 0; st >>= 1) {
      const int32_t j = lo + st - 1;
      const uint64_t t = __shfl(Tb, grp * B + (j < B ? j : B - 1), 64);
      if (j < B && t < R) lo += st;
    }
    if (lo > B - 1) lo = B - 1;
    const uint64_t M = __shfl(h, grp * B + lo, 64);
    if (live) {
      double d = 1.0;
      if (R > 0) {
        d = (double)(R - M) / (double)R;
        req += R;
        met += M;
      }
      if (exact_small_din) {
        const int32_t din = E.din[r];
        if (din == 0) d = 1.0;
        else if (din == 1) d = 1.0 - c;
      }
      D[row + b] = d;
    }
  }
  for (int m = 32; m > 0; m >>= 1) {
    req += __shfl_xor(req, m, 64);
    met += __shfl_xor(met, m, 64);
  }
  if (lane == 0 && (req | met)) {
    atomicAdd(&sums[0], req);
    atomicAdd(&sums[1], met);
  }
}

__global__ void bat_back_init(int64_t NB, double a, const double* __restrict__ D, const double* __restrict__ lvlL,
                              double* __restrict__ s0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NB) return;
  s0[i] = a * (D[i] * lvlL[i]);
}

// s_out[q][v] = S[int_of[v]][b] for external node v
// Source index fastest: a node's B results are one contiguous read, and the
// writes of neighbouring nodes to each output meet in the same cache lines.
__global__ void bat_output(const BEntry* __restrict__ ents, const double* __restrict__ S, double* const* __restrict__ outs) {
  const BEntry E = ents[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (int64_t)E.n * E.B;
  if (i >= nb) return;
  const int32_t v = (int32_t)(i / E.B);
  const int32_t b = (int32_t)(i - (int64_t)v * E.B);
  outs[E.src_base + b][v] = S[E.base + (int64_t)E.int_of[v] * E.B + b];
}

__global__ void bat_accumulate_walk(const WalkTotals* __restrict__ tot, unsigned long long* __restrict__ sums) {
  sums[2] += tot->total;
  sums[3] += tot->meets;
}

__global__ void zero_u64(int64_t n, unsigned long long* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

// ---- plans -------------------------------------------------------------------

struct BatchBlock {
  const es_graph* g;
  int32_t B;
  int32_t W, G;
  std::vector<int32_t> queries;  // query indices
};

struct BatchPlan {
  BatchPlan* next = nullptr;
  // key: graphs by handle identity (a destroyed graph's address can come
  // back for a new graph; its uid cannot)
  std::vector<const es_graph*> kg;
  std::vector<uint64_t> kid;
  std::vector<int32_t> kB, kW, kG;
  int32_t L = 0;
  double c = 0, eps = 0, r_scale = 0;
  uint64_t seed = 0;
  int32_t alloc = 0, small = 0;
  int32_t nq = 0;
  double sparse_eps = 0;
  double v_floor = 0;   // learned allocation: floor ratio and the network's load id
  uint64_t mlp_id = 0;
  // device data
  BEntry* ents = nullptr;
  int32_t nent = 0;
  MTile* tiles_fwd = nullptr;
  MTile* tiles_back = nullptr;
  int32_t ntf = 0, ntb = 0;
  LongRow* long_fwd = nullptr;
  LongRow* long_back = nullptr;
  int32_t nlf = 0, nlb = 0;
  int32_t* src_int = nullptr;    // [nq] internal source ids, block order
  double** outs = nullptr;       // [nq] device pointer array, block order
  unsigned long long* lsums = nullptr;  // learned allocation: [nq][4] sums, thresholds, vbar_inv
  double* lthr = nullptr;
  double* lvbi = nullptr;
  int64_t NB = 0, NN = 0, NLONG = 0;
  int32_t max_nb_blocks = 0;     // grid.x for per-block elementwise kernels
  int32_t max_n = 0;
  std::vector<int64_t> node_base, base;
  std::vector<int32_t> order;    // block-order position -> query index
  // workspace pointers the plan was built with (a change forces a rebuild)
  std::vector<void*> ws;
  hipGraphExec_t exec = nullptr;
};

void free_batch_plans(es_ctx* ctx) {
  BatchPlan* p = ctx->plans;
  while (p) {
    BatchPlan* nx = p->next;
    (void)hipFree(p->ents);
    (void)hipFree(p->tiles_fwd);
    (void)hipFree(p->tiles_back);
    (void)hipFree(p->long_fwd);
    (void)hipFree(p->long_back);
    (void)hipFree(p->src_int);
    (void)hipFree(p->outs);
    (void)hipFree(p->lsums);
    (void)hipFree(p->lthr);
    (void)hipFree(p->lvbi);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    delete p;
    p = nx;
  }
  ctx->plans = nullptr;
}

namespace {

int32_t pow2_at_least(int32_t x) {
  int32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

bool find_tuned(const es_graph* g, int32_t B, int32_t* W, int32_t* G, float* ms = nullptr) {
  for (auto& t : g->tuned)
    if (t.B == B) {
      *W = t.W;
      *G = t.G;
      if (ms) *ms = t.ms;
      return true;
    }
  return false;
}

template <class T>
es_status upload(es_ctx* ctx, T** dptr, const std::vector<T>& h) {
  ES_CHECK_HIP(ctx, hipMalloc((void**)dptr, sizeof(T) * std::max<size_t>(1, h.size())));
  if (!h.empty()) ES_CHECK_HIP(ctx, hipMemcpy(*dptr, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return ES_OK;
}

struct BatchBuffers {
  double* levels;
  int64_t* q[2];
  double* pi;
  uint64_t* Rk;
  uint64_t* T;
  uint64_t* H;
  double* D;
  double* s[2];
  uint64_t* Rmax;
  long long* acc;
  unsigned long long* sums;  // [0] pairs requested, [1] meets, [2] pairs simulated, [3] raw meets
  SparseLevels sp;           // sparse linearization: the kept level entries (sp.idx NULL when dense)
};

// Capacity of the kept entries of a batch: each source keeps at most its own bound.
uint64_t batch_sparse_capacity(const BatchPlan& p, const std::vector<const es_graph*>& block_graphs, double theta) {
  uint64_t cap = 0;
  for (int32_t e = 0; e < p.nent; ++e)
    cap += (uint64_t)p.kB[e] * sparse_capacity(block_graphs[e]->n, block_graphs[e]->m, p.L, theta);
  return std::min<uint64_t>(cap, (uint64_t)(p.L + 1) * (uint64_t)p.NB);
}

es_status batch_buffers(es_ctx* ctx, const BatchPlan& p, BatchBuffers* b, double sparse_eps = 0.0,
                        const std::vector<const es_graph*>* block_graphs = nullptr) {
  es_status st;
  const size_t NB = (size_t)p.NB;
  const size_t L1 = (size_t)p.L + 1;
  b->sp = SparseLevels{};
  if (sparse_eps > 0.0) {
    // the level of the moment stays dense; the kept entries of all levels go to one list
    const double sc = std::sqrt(p.c);
    b->sp.theta = (1.0 - sc) * (1.0 - sc) * sparse_eps;
    b->sp.cap = batch_sparse_capacity(p, *block_graphs, b->sp.theta);
    b->sp.idx = (int32_t*)workspace(ctx, kWsSpIdx, sizeof(int32_t) * (size_t)b->sp.cap, &st);
    if (!b->sp.idx) return st;
    b->sp.val = (double*)workspace(ctx, kWsSpVal, sizeof(double) * (size_t)b->sp.cap, &st);
    if (!b->sp.val) return st;
    b->sp.cnt = (unsigned long long*)workspace(ctx, kWsSpCnt, sizeof(uint64_t) * (L1 + 1), &st);
    if (!b->sp.cnt) return st;
  }
  b->levels = (double*)workspace(ctx, kWsLevels, 8 * NB * (sparse_eps > 0.0 ? 1 : L1), &st);
  if (!b->levels) return st;
  b->q[0] = (int64_t*)workspace(ctx, kWsQ0, 8 * NB, &st);
  if (!b->q[0]) return st;
  b->q[1] = (int64_t*)workspace(ctx, kWsQ1, 8 * NB, &st);
  if (!b->q[1]) return st;
  b->pi = (double*)workspace(ctx, kWsPi, 8 * NB, &st);
  if (!b->pi) return st;
  b->Rk = (uint64_t*)workspace(ctx, kWsRk, 8 * NB, &st);
  if (!b->Rk) return st;
  b->H = (uint64_t*)workspace(ctx, kWsM, 8 * NB, &st);
  if (!b->H) return st;
  b->D = (double*)workspace(ctx, kWsD, 8 * NB, &st);
  if (!b->D) return st;
  b->s[0] = (double*)workspace(ctx, kWsS0, 8 * NB, &st);
  if (!b->s[0]) return st;
  b->s[1] = (double*)workspace(ctx, kWsS1, 8 * NB, &st);
  if (!b->s[1]) return st;
  b->T = (uint64_t*)workspace(ctx, kWsBatchT, 8 * NB, &st);
  if (!b->T) return st;
  char* misc = (char*)workspace(ctx, kWsBatchMisc,
                                8 * (size_t)p.NN + 8 * (size_t)std::max<int64_t>(1, p.NLONG) * kBatchMaxB + 64, &st);
  if (!misc) return st;
  b->Rmax = (uint64_t*)misc;
  b->acc = (long long*)(misc + 8 * (size_t)p.NN);
  b->sums = (unsigned long long*)(misc + 8 * (size_t)p.NN + 8 * (size_t)std::max<int64_t>(1, p.NLONG) * kBatchMaxB);
  return ES_OK;
}

// Enqueue the whole batch on ctx->stream (also used under stream capture).
es_status enqueue_batch(es_ctx* ctx, const BatchPlan& p, const BatchBuffers& b,
                        const std::vector<const es_graph*>& block_graphs, uint64_t seed) {
  hipStream_t stream = ctx->stream;
  const double sc = std::sqrt(p.c);
  const double a = 1.0 / (1.0 - sc);
  const int tb = 256;
  const int64_t NB = p.NB;
  const int64_t nacc = std::max<int64_t>(1, p.NLONG) * kBatchMaxB;
  dim3 egrid(p.max_nb_blocks, p.nent);
  zero_u64<<<1, 64, 0, stream>>>(4, b.sums);
  zero_u64<<<ceil_div(nacc, tb), tb, 0, stream>>>(nacc, (unsigned long long*)b.acc);
  const bool sparse = b.sp.idx != nullptr;
  // dense: level l in slot l; sparse: every level in slot 0, its kept entries appended to b.sp
  auto slot = [&](int32_t l) { return b.levels + (sparse ? 0 : (int64_t)l * NB); };
  if (sparse) ES_TRY(launch_fill(ctx, p.L + 2, b.sp.cnt));
  bat_forward_init<<<egrid, tb, 0, stream>>>(p.ents, p.src_int, 1.0 - sc, slot(0), b.q[0]);
  if (sparse) ES_TRY(launch_level_keep(ctx, NB, slot(0), true, b.pi, b.sp, 0, p.L));
  const int spmm_f = ceil_div(p.ntf, kSpmmThreads / 64);
  const int spmm_b = ceil_div(p.ntb, kSpmmThreads / 64);
  for (int32_t l = 1; l <= p.L; ++l) {
    FwdOp op{b.q[(l - 1) & 1], b.q[l & 1], slot(l), b.acc, sc};
    if (p.ntf) spmm_kernel<FwdOp><<<spmm_f, kSpmmThreads, 0, stream>>>(p.tiles_fwd, p.ntf, p.ents, op);
    if (p.nlf)
      long_finish_kernel<FwdOp><<<ceil_div((int64_t)p.nlf * kBatchMaxB, tb), tb, 0, stream>>>(p.long_fwd, p.nlf,
                                                                                               p.ents, op);
    if (sparse) ES_TRY(launch_level_keep(ctx, NB, slot(l), false, b.pi, b.sp, l, p.L));
  }
  if (!sparse) bat_sum_levels<<<ceil_div(NB, tb), tb, 0, stream>>>(NB, p.L, b.levels, b.pi);
  if (p.alloc == ES_ALLOC_LEARNED) {
    const int lgrid = std::min(p.max_nb_blocks, std::max(1, ctx->num_cus) * 4);
    dim3 lg(lgrid, p.nent);
    zero_u64<<<ceil_div((int64_t)p.nq * 4, tb), tb, 0, stream>>>((int64_t)p.nq * 4, p.lsums);
    bat_learned_sums<<<lg, tb, 0, stream>>>(p.ents, b.pi, p.lthr, p.small, 0, p.lsums);
    bat_learned_scalars<<<ceil_div(p.nq, tb), tb, 0, stream>>>(p.nq, p.lsums, p.v_floor, 0, p.lthr, p.lvbi);
    bat_learned_sums<<<lg, tb, 0, stream>>>(p.ents, b.pi, p.lthr, p.small, 1, p.lsums);
    bat_learned_scalars<<<ceil_div(p.nq, tb), tb, 0, stream>>>(p.nq, p.lsums, p.v_floor, 1, p.lthr, p.lvbi);
    bat_budget_learned<<<egrid, tb, 0, stream>>>(p.ents, b.pi, p.small, p.lthr, p.lvbi, b.Rk);
  } else {
    bat_budget<<<egrid, tb, 0, stream>>>(p.ents, b.pi, p.alloc, p.small, b.Rk);
  }
  dim3 sgrid(ceil_div(p.max_n, tb / 64), p.nent);
  bat_sort_counts<<<sgrid, tb, 0, stream>>>(p.ents, b.Rk, b.T, b.Rmax);
  for (int32_t e = 0; e < p.nent; ++e) {
    const es_graph* g = block_graphs[e];
    const int32_t B = p.kB[e];
    WalkTotals* tot = nullptr;
    ES_TRY(launch_walks_buckets(ctx, g, b.Rmax + p.node_base[e], b.T + p.base[e], B, seed, p.c, b.H + p.base[e],
                                &tot));
    bat_accumulate_walk<<<1, 1, 0, stream>>>(tot, b.sums);
  }
  dim3 dgrid(std::min(p.max_nb_blocks, std::max(1, ctx->num_cus) * 8), p.nent);
  bat_finish_diag<<<dgrid, tb, 0, stream>>>(p.ents, b.Rk, b.T, b.H, p.c, p.small, b.D, b.sums);
  // back-accumulation; level L lands in s[L & 1]
  if (sparse) {
    ES_TRY(launch_fill(ctx, NB, b.s[0]));
    ES_TRY(launch_level_scatter(ctx, NB, b.sp, p.L, b.D, a, b.s[0]));
  } else {
    bat_back_init<<<ceil_div(NB, tb), tb, 0, stream>>>(NB, a, b.D, b.levels + (int64_t)p.L * NB, b.s[0]);
  }
  for (int32_t l = 1; l <= p.L; ++l) {
    BackOp op{b.s[(l - 1) & 1], b.s[l & 1], b.D, sparse ? nullptr : b.levels + (int64_t)(p.L - l) * NB,
              (double*)b.acc, sc, a};
    if (p.ntb) spmm_kernel<BackOp><<<spmm_b, kSpmmThreads, 0, stream>>>(p.tiles_back, p.ntb, p.ents, op);
    if (p.nlb)
      long_finish_kernel<BackOp><<<ceil_div((int64_t)p.nlb * kBatchMaxB, tb), tb, 0, stream>>>(p.long_back, p.nlb,
                                                                                                p.ents, op);
    if (sparse) ES_TRY(launch_level_scatter(ctx, NB, b.sp, p.L - l, b.D, a, b.s[l & 1]));
  }
  bat_output<<<egrid, tb, 0, stream>>>(p.ents, b.s[p.L & 1], p.outs);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

bool same_key(const BatchPlan& p, const BatchPlan& q) {
  return p.kid == q.kid && p.kg == q.kg && p.kB == q.kB && p.kW == q.kW && p.kG == q.kG && p.L == q.L && p.c == q.c &&
         p.eps == q.eps && p.r_scale == q.r_scale && p.seed == q.seed && p.alloc == q.alloc && p.small == q.small &&
         p.nq == q.nq && p.sparse_eps == q.sparse_eps && p.v_floor == q.v_floor && p.mlp_id == q.mlp_id;
}

// Build tiles and descriptors of a plan whose key fields are set.
es_status build_batch_plan(es_ctx* ctx, BatchPlan& p, const std::vector<BatchBlock>& blocks) {
  std::vector<BEntry> ents;
  std::vector<MTile> tf, tbk;
  std::vector<LongRow> lf, lbk;
  int64_t base = 0, node_base = 0, long_base = 0, src_base = 0;
  p.max_n = 1;
  int64_t max_nb = 1;
  p.node_base.clear();
  p.base.clear();
  for (size_t e = 0; e < blocks.size(); ++e) {
    const BatchBlock& bl = blocks[e];
    const es_graph* g = bl.g;
    BEntry E{};
    E.out_off = g->out_off;
    E.out_idx = g->out_idx;
    E.in_off = g->in_off;
    E.in_idx = g->in_idx;
    E.inv_din = g->inv_din;
    E.din = g->din_int;
    E.int_of = g->int_of;
    E.vhat = g->vhat;
    E.n = g->n;
    E.B = bl.B;
    E.W = bl.W;
    E.R = total_samples(g->n, p.c, p.eps, p.r_scale);
    E.base = base;
    E.node_base = node_base;
    E.long_base = long_base;
    E.src_base = src_base;
    int32_t nlf = 0, nlb = 0;
    make_tiles(g->h_out_off, g->n, (int32_t)e, bl.W, bl.G, tf, lf, nlf);
    // backward chunks use slots after the forward ones of the same block
    std::vector<MTile> tb_e;
    std::vector<LongRow> lb_e;
    make_tiles(g->h_in_off, g->n, (int32_t)e, bl.W, bl.G, tb_e, lb_e, nlb);
    for (auto& t : tb_e) {
      if (t.row1 < 0) t.row1 = -((-t.row1 - 1) + nlf + 1);
      tbk.push_back(t);
    }
    for (auto& r : lb_e) {
      r.slot += nlf;
      lbk.push_back(r);
    }
    E.nlong_fwd = nlf;
    E.nlong_back = nlb;
    ents.push_back(E);
    p.base.push_back(base);
    p.node_base.push_back(node_base);
    base += (int64_t)g->n * bl.B;
    node_base += g->n;
    long_base += nlf + nlb;
    src_base += bl.B;
    p.max_n = std::max(p.max_n, g->n);
    max_nb = std::max<int64_t>(max_nb, (int64_t)g->n * bl.B);
  }
  p.NB = base;
  p.NN = node_base;
  p.NLONG = long_base;
  p.nent = (int32_t)ents.size();
  p.ntf = (int32_t)tf.size();
  p.ntb = (int32_t)tbk.size();
  p.nlf = (int32_t)lf.size();
  p.nlb = (int32_t)lbk.size();
  p.max_nb_blocks = ceil_div(max_nb, 256);
  ES_TRY(upload(ctx, &p.ents, ents));
  ES_TRY(upload(ctx, &p.tiles_fwd, tf));
  ES_TRY(upload(ctx, &p.tiles_back, tbk));
  ES_TRY(upload(ctx, &p.long_fwd, lf));
  ES_TRY(upload(ctx, &p.long_back, lbk));
  ES_CHECK_HIP(ctx, hipMalloc((void**)&p.src_int, sizeof(int32_t) * std::max(1, p.nq)));
  ES_CHECK_HIP(ctx, hipMalloc((void**)&p.outs, sizeof(double*) * std::max(1, p.nq)));
  if (p.alloc == ES_ALLOC_LEARNED) {
    ES_CHECK_HIP(ctx, hipMalloc((void**)&p.lsums, sizeof(unsigned long long) * 4 * std::max(1, p.nq)));
    ES_CHECK_HIP(ctx, hipMalloc((void**)&p.lthr, sizeof(double) * std::max(1, p.nq)));
    ES_CHECK_HIP(ctx, hipMalloc((void**)&p.lvbi, sizeof(double) * std::max(1, p.nq)));
  }
  return ES_OK;
}

// Time the forward SpMM of one block for each candidate tiling; keep the fastest.
es_status autotune(es_ctx* ctx, const es_graph* g, int32_t B, const es_query_opts* o, int32_t* bestW,
                   int32_t* bestG, float* best_ms) {
  std::vector<int32_t> widths;
  for (int32_t w = pow2_at_least(std::max(B, 1)); w <= 64; w <<= 1) widths.push_back(std::max(w, 8));
  widths.erase(std::unique(widths.begin(), widths.end()), widths.end());
  const int32_t rows_opts[] = {8, 32, 128};
  float best = 1e30f;
  *bestW = widths.front();
  *bestG = 32;
  hipEvent_t e0 = ctx->ev[6], e1 = ctx->ev[7];
  for (int32_t W : widths) {
    for (int32_t G : rows_opts) {
      BatchPlan p;
      p.c = o->c;
      p.eps = o->eps;
      p.r_scale = o->r_scale;
      p.L = 3;
      p.nq = B;
      std::vector<BatchBlock> blocks(1);
      blocks[0].g = g;
      blocks[0].B = B;
      blocks[0].W = W;
      blocks[0].G = G;
      es_status st = build_batch_plan(ctx, p, blocks);
      BatchBuffers bb{};
      if (st == ES_OK) st = batch_buffers(ctx, p, &bb);
      if (st == ES_OK) {
        // sources: the B highest-degree nodes (internal ids 0..B-1)
        std::vector<int32_t> src(B);
        for (int32_t b = 0; b < B; ++b) src[b] = std::min(b, g->n - 1);
        const hipError_t ec = hipMemcpy(p.src_int, src.data(), 4 * B, hipMemcpyHostToDevice);
        if (ec != hipSuccess) st = hip_fail(ctx, ec, "hipMemcpy(tuning sources)");
        const double sc = std::sqrt(o->c);
        dim3 egrid(p.max_nb_blocks, 1);
        bat_forward_init<<<egrid, 256, 0, ctx->stream>>>(p.ents, p.src_int, 1.0 - sc, bb.levels, bb.q[0]);
        const int spmm_f = ceil_div(p.ntf, kSpmmThreads / 64);
        float tot = 0;
        for (int rep = 0; rep < 2 && st == ES_OK; ++rep) {
          (void)hipEventRecord(e0, ctx->stream);
          for (int32_t l = 1; l <= p.L; ++l) {
            FwdOp op{bb.q[(l - 1) & 1], bb.q[l & 1], bb.levels + (int64_t)l * p.NB, bb.acc, sc};
            if (p.ntf) spmm_kernel<FwdOp><<<spmm_f, kSpmmThreads, 0, ctx->stream>>>(p.tiles_fwd, p.ntf, p.ents, op);
            if (p.nlf)
              long_finish_kernel<FwdOp><<<ceil_div((int64_t)p.nlf * kBatchMaxB, 256), 256, 0, ctx->stream>>>(
                  p.long_fwd, p.nlf, p.ents, op);
          }
          (void)hipEventRecord(e1, ctx->stream);
          const hipError_t es = hipEventSynchronize(e1);
          if (es != hipSuccess) st = hip_fail(ctx, es, "tuning launch");
          float ms = 0;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep == 1) tot = ms;
        }
        if (st == ES_OK && tot < best) {
          best = tot;
          *bestW = W;
          *bestG = G;
        }
      }
      (void)hipFree(p.ents);
      (void)hipFree(p.tiles_fwd);
      (void)hipFree(p.tiles_back);
      (void)hipFree(p.long_fwd);
      (void)hipFree(p.long_back);
      (void)hipFree(p.src_int);
      (void)hipFree(p.outs);
      ES_TRY(st);
    }
  }
  ES_CHECK_HIP(ctx, hipGetLastError());
  *best_ms = best;
  return ES_OK;
}

// The tiling of a block of width B on g: tuned once and kept in the graph.
es_status tiling_for(es_ctx* ctx, const es_graph* g, int32_t B, const es_query_opts* o, int32_t* W, int32_t* G,
                     float* ms) {
  if (find_tuned(g, B, W, G, ms)) return ES_OK;
  ES_TRY(autotune(ctx, g, B, o, W, G, ms));
  const_cast<es_graph*>(g)->tuned.push_back({B, *W, *G, *ms});
  return ES_OK;
}

// Source-block width for S queries on g: the width (64, 32, 16 or 8, not
// above what S fills) whose tuned level SpMM costs least per source.
es_status block_width_for(es_ctx* ctx, const es_graph* g, int32_t S, const es_query_opts* o, int32_t* width) {
  for (auto& t : g->tuned_block)
    if (t.first == S) {
      *width = t.second;
      return ES_OK;
    }
  int32_t best_w = std::min(S, kBatchMaxB);
  if (S > 8 && g->n >= kBatchMaxB) {
    float best = 1e30f;
    for (int32_t w = kBatchMaxB; w >= 8; w >>= 1) {
      if (w > pow2_at_least(S)) continue;
      const int32_t bw = std::min(w, S);
      int32_t W, G;
      float ms;
      ES_TRY(tiling_for(ctx, g, bw, o, &W, &G, &ms));
      const float per_source = ms / (float)bw;
      if (per_source < best) {
        best = per_source;
        best_w = bw;
      }
    }
  }
  const_cast<es_graph*>(g)->tuned_block.push_back({S, best_w});
  *width = best_w;
  return ES_OK;
}

}  // namespace
}  // namespace es

using namespace es;

extern "C" {

es_status es_batch_tuning(const es_graph* g, int32_t B, int32_t* width, int32_t* rows) {
  if (!g || !width || !rows) return ES_EINVAL;
  if (!find_tuned(g, B, width, rows)) {
    *width = 0;
    *rows = 0;
  }
  return ES_OK;
}

es_status es_batch_block_width(const es_graph* g, int32_t S, int32_t* width) {
  if (!g || !width) return ES_EINVAL;
  *width = 0;
  for (auto& t : g->tuned_block)
    if (t.first == S) *width = t.second;
  return ES_OK;
}

es_status es_batch(es_ctx* ctx, const es_graph* const* graphs, int32_t ngraphs, const int32_t* graph_of_query,
                   const int32_t* sources, int32_t nq, const es_query_opts* o, const es_batch_opts* bo,
                   double* const* s_out, es_stats* stats) {
  if (!ctx || !graphs || ngraphs < 1 || !graph_of_query || !sources || nq < 1 || !o || !s_out) return ES_EINVAL;
  if (!(o->c > 0.0 && o->c <= 0.99)) return fail(ctx, ES_EINVAL, "c=%g outside (0, 0.99]", o->c);
  if (!(o->eps > 0.0 && o->eps < 1.0)) return fail(ctx, ES_EINVAL, "eps=%g outside (0, 1)", o->eps);
  if (!(o->r_scale > 0.0)) return fail(ctx, ES_EINVAL, "r_scale=%g must be positive", o->r_scale);
  if (o->d_override) return fail(ctx, ES_EUNSUPPORTED, "d_override is single-source only");
  if (o->alloc != ES_ALLOC_PI2 && o->alloc != ES_ALLOC_PI && o->alloc != ES_ALLOC_LEARNED)
    return fail(ctx, ES_EINVAL, "allocation %d", o->alloc);
  if (o->alloc == ES_ALLOC_LEARNED) {
    if (!ctx->mlp_w) return fail(ctx, ES_EINVAL, "learned allocation without a loaded network (es_mlp_load)");
    if (!(o->v_floor_ratio >= 0.0 && o->v_floor_ratio <= 1.0))
      return fail(ctx, ES_EINVAL, "v_floor_ratio=%g outside [0, 1]", o->v_floor_ratio);
  }
  if (o->lde != 0) return fail(ctx, ES_EUNSUPPORTED, "batches run Algorithm 2 only (lde = 0)");
  if (!(o->sparse_eps >= 0.0 && o->sparse_eps < 1.0))
    return fail(ctx, ES_EINVAL, "sparse_eps=%g outside [0, 1)", o->sparse_eps);
  es_batch_opts defaults{0, 1, 0, 0, 0};
  const es_batch_opts& b = bo ? *bo : defaults;
  if (b.block_width < 0 || b.block_width > kBatchMaxB)
    return fail(ctx, ES_EINVAL, "block_width=%d outside 0..%d", b.block_width, kBatchMaxB);
  if (b.force_width && (b.force_width < 8 || b.force_width > 64 || (b.force_width & (b.force_width - 1))))
    return fail(ctx, ES_EINVAL, "force_width=%d", b.force_width);
  if (b.force_rows < 0) return fail(ctx, ES_EINVAL, "force_rows=%d", b.force_rows);
  for (int32_t gi = 0; gi < ngraphs; ++gi)
    if (!graphs[gi]) return fail(ctx, ES_EINVAL, "graph %d is NULL", gi);
  for (int32_t q = 0; q < nq; ++q) {
    const int32_t gi = graph_of_query[q];
    if (gi < 0 || gi >= ngraphs) return fail(ctx, ES_EINVAL, "query %d: graph index %d", q, gi);
    if (sources[q] < 0 || sources[q] >= graphs[gi]->n) return fail(ctx, ES_EINVAL, "query %d: source %d", q, sources[q]);
    if (!s_out[q]) return fail(ctx, ES_EINVAL, "query %d: null output", q);
  }
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  for (int32_t gi = 0; gi < ngraphs; ++gi) {
    const double R = total_samples(graphs[gi]->n, o->c, o->eps, o->r_scale);
    if (R + (double)graphs[gi]->n >= 9.2e18) return fail(ctx, ES_EOVERFLOW, "R=%g: sample count may reach 2^63", R);
  }
  // blocks per graph, in graph order: of the forced width, of the width the
  // tuner finds cheapest per source, or of 64
  std::vector<BatchBlock> blocks;
  for (int32_t gi = 0; gi < ngraphs; ++gi) {
    std::vector<int32_t> qs;
    for (int32_t q = 0; q < nq; ++q)
      if (graph_of_query[q] == gi) qs.push_back(q);
    if (qs.empty()) continue;
    int32_t bw = kBatchMaxB;
    if (b.block_width) bw = b.block_width;
    else if (b.autotune && !b.force_width && !b.force_rows)
      ES_TRY(block_width_for(ctx, graphs[gi], (int32_t)qs.size(), o, &bw));
    for (size_t s0 = 0; s0 < qs.size(); s0 += (size_t)bw) {
      BatchBlock bl;
      bl.g = graphs[gi];
      bl.queries.assign(qs.begin() + s0, qs.begin() + std::min(qs.size(), s0 + (size_t)bw));
      bl.B = (int32_t)bl.queries.size();
      blocks.push_back(bl);
    }
  }
  // tiling per block: forced, tuned or default
  for (auto& bl : blocks) {
    int32_t W = 0, G = 0;
    if (b.force_width || b.force_rows) {
      W = b.force_width ? b.force_width : std::max(8, pow2_at_least(bl.B));
      G = b.force_rows ? b.force_rows : 32;
      if (W < bl.B) return fail(ctx, ES_EINVAL, "force_width=%d below block width %d", W, bl.B);
    } else if (!find_tuned(bl.g, bl.B, &W, &G)) {
      if (b.autotune) {
        float ms;
        ES_TRY(tiling_for(ctx, bl.g, bl.B, o, &W, &G, &ms));
      } else {
        W = std::max(8, pow2_at_least(bl.B));
        G = 32;
      }
    }
    bl.W = W;
    bl.G = G;
  }
  // plan lookup
  BatchPlan key;
  for (auto& bl : blocks) {
    key.kg.push_back(bl.g);
    key.kid.push_back(bl.g->uid);
    key.kB.push_back(bl.B);
    key.kW.push_back(bl.W);
    key.kG.push_back(bl.G);
  }
  key.L = num_levels(o->c, o->eps);
  key.c = o->c;
  key.eps = o->eps;
  key.r_scale = o->r_scale;
  key.seed = o->seed;
  key.alloc = o->alloc;
  key.small = o->exact_small_din;
  key.nq = nq;
  key.sparse_eps = o->sparse_eps;
  if (o->alloc == ES_ALLOC_LEARNED) {
    // predictions first: the plan's descriptors point at them
    for (const auto& bl : blocks) ES_TRY(ensure_vhat(ctx, bl.g, o->c));
    key.v_floor = o->v_floor_ratio;
    key.mlp_id = ctx->mlp_id;
  }
  BatchPlan* plan = nullptr;
  for (BatchPlan* p = ctx->plans; p; p = p->next)
    if (same_key(*p, key)) plan = p;
  if (!plan) {
    plan = new BatchPlan(key);
    plan->next = nullptr;
    const es_status st = build_batch_plan(ctx, *plan, blocks);
    if (st != ES_OK) {
      BatchPlan* saved = ctx->plans;
      ctx->plans = plan;  // free_batch_plans releases exactly this one
      free_batch_plans(ctx);
      ctx->plans = saved;
      return st;
    }
    // keep at most eight plans: drop the oldest
    int count = 0;
    for (BatchPlan* q = ctx->plans; q; q = q->next)
      if (++count >= 8 && q->next) {
        (void)hipStreamSynchronize(ctx->stream);  // an evicted graph may still be running
        BatchPlan* rest = q->next;
        q->next = nullptr;
        BatchPlan* saved = ctx->plans;
        ctx->plans = rest;
        free_batch_plans(ctx);
        ctx->plans = saved;
        break;
      }
    plan->next = ctx->plans;
    ctx->plans = plan;
  }
  std::vector<const es_graph*> block_graphs;
  for (auto& bl : blocks) block_graphs.push_back(bl.g);
  // the kept entries are indexed by int32 flat positions
  if (o->sparse_eps > 0.0 && plan->NB >= (int64_t)INT32_MAX)
    return fail(ctx, ES_EUNSUPPORTED, "sparse levels need (nodes x sources) per batch below 2^31");
  // workspaces (allocated before any capture)
  BatchBuffers bb{};
  ES_TRY(batch_buffers(ctx, *plan, &bb, o->sparse_eps, &block_graphs));
  ES_TRY(lifetime_table(ctx, o->c));
  {
    es_status st;
    const int nbk = ceil_div(plan->max_n, 1024);
    if (!workspace(ctx, kWsTotals, sizeof(WalkTotals), &st)) return st;
    if (!workspace(ctx, kWsScanCnt, sizeof(uint32_t) * nbk, &st)) return st;
    if (!workspace(ctx, kWsScanSum, sizeof(uint64_t) * nbk, &st)) return st;
    if (!workspace(ctx, kWsActive, sizeof(int32_t) * (size_t)plan->max_n, &st)) return st;
    if (!workspace(ctx, kWsPrefix, sizeof(uint64_t) * ((size_t)plan->max_n + 1), &st)) return st;
  }
  std::vector<void*> ws_now(ctx->ws.begin(), ctx->ws.end());
  if (plan->exec && plan->ws != ws_now) {
    (void)hipGraphExecDestroy(plan->exec);
    plan->exec = nullptr;
  }
  // per-call inputs: sources (internal ids) and output pointers, in block order
  std::vector<int32_t> src_int;
  std::vector<double*> outs;
  for (auto& bl : blocks) {
    for (int32_t q : bl.queries) {
      src_int.push_back(bl.g->h_int_of[sources[q]]);
      outs.push_back(s_out[q]);
    }
  }
  ES_CHECK_HIP(ctx, hipMemcpyAsync(plan->src_int, src_int.data(), 4 * src_int.size(), hipMemcpyHostToDevice,
                                   ctx->stream));
  ES_CHECK_HIP(ctx, hipMemcpyAsync(plan->outs, outs.data(), sizeof(double*) * outs.size(), hipMemcpyHostToDevice,
                                   ctx->stream));
  ES_CHECK_HIP(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
  if (b.use_hip_graph) {
    if (!plan->exec) {
      if (!ctx->capture_stream) ES_CHECK_HIP(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
      // the inputs above must land before the captured work reads them
      ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
      hipStream_t user = ctx->stream;
      ctx->stream = ctx->capture_stream;
      ES_CHECK_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      es_status st = enqueue_batch(ctx, *plan, bb, block_graphs, o->seed);
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
      ctx->stream = user;
      ES_TRY(st);
      if (ec != hipSuccess) return hip_fail(ctx, ec, "hipStreamEndCapture");
      const hipError_t ei = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return hip_fail(ctx, ei, "hipGraphInstantiate");
      plan->ws = ws_now;
    }
    ES_CHECK_HIP(ctx, hipGraphLaunch(plan->exec, ctx->stream));
  } else {
    ES_TRY(enqueue_batch(ctx, *plan, bb, block_graphs, o->seed));
  }
  ES_CHECK_HIP(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
  if (stats) {
    ES_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    unsigned long long h[4];
    ES_CHECK_HIP(ctx, hipMemcpy(h, bb.sums, sizeof(h), hipMemcpyDeviceToHost));
    es_stats s{};
    s.L = plan->L;
    s.R = plan->nent ? total_samples(blocks[0].g->n, o->c, o->eps, o->r_scale) : 0.0;
    s.pairs_requested = h[0];
    s.meets = h[1];
    s.pairs = h[2];
    float ms = 0;
    ES_CHECK_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    s.ms_walk = ms;
    if (bb.sp.idx) {
      unsigned long long kept = 0;
      ES_CHECK_HIP(ctx, hipMemcpy(&kept, bb.sp.cnt + plan->L + 1, sizeof(kept), hipMemcpyDeviceToHost));
      if (kept > bb.sp.cap)
        return fail(ctx, ES_EOVERFLOW, "%llu entries above the threshold, capacity %llu", kept,
                    (unsigned long long)bb.sp.cap);
      s.level_entries = kept;
      s.level_bytes = 12ull * kept + 8ull * (uint64_t)plan->NB;
    } else {
      s.level_entries = (uint64_t)(plan->L + 1) * (uint64_t)plan->NB;
      s.level_bytes = 8ull * s.level_entries;
    }
    s.workspace_bytes = workspace_total(ctx);
    *stats = s;
  }
  return ES_OK;
}

}  // extern "C"
