// Top-k query (Section 1): the k largest s(j), j != exclude, ties to the smaller id.
//
// Radix select over order-preserving 64-bit keys of the float64 scores finds
// the k-th largest key tau in eight 8-bit passes; if more nodes tie at tau
// than are still needed, four more passes over the node ids pick the smallest
// ids among the ties.  The k survivors are then sorted by (score desc, id asc)
// with a bitonic sort in one workgroup's LDS.
#include <cstring>
#include <mutex>
#include <vector>

#include "es_internal.h"

namespace es {
namespace {

constexpr int kTopkMax = 4096;
constexpr int kHistThreads = 256;
// fixed scratch of the allocation-free entry point (state, candidate keys and ids)
constexpr size_t kTopkScratchBytes = 64 * 1024;

struct TopkState {
  unsigned long long prefix;  // key bits fixed so far
  unsigned long long mask;
  unsigned long long tau;
  uint32_t need;              // rank still to find among keys matching prefix
  uint32_t id_prefix;
  uint32_t id_mask;
  uint32_t id_need;           // how many ties at tau to take
  uint32_t id_active;         // 1 if the id passes are needed
  uint32_t id_limit;          // take ties with id <= id_limit
  uint32_t count;             // candidates written
  uint32_t hist[256];
};

__device__ __forceinline__ unsigned long long order_key(double s) {
  unsigned long long b = (unsigned long long)__double_as_longlong(s);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void topk_init_kernel(TopkState* st, uint32_t k) {
  const int t = threadIdx.x;
  if (t < 256) st->hist[t] = 0;
  if (t == 0) {
    st->prefix = 0;
    st->mask = 0;
    st->tau = 0;
    st->need = k;
    st->id_prefix = 0;
    st->id_mask = 0;
    st->id_need = 0;
    st->id_active = 0;
    st->id_limit = 0xffffffffu;
    st->count = 0;
  }
}

// histogram of one key digit (mode 0) or one id digit among ties (mode 1)
__global__ __launch_bounds__(kHistThreads) void topk_hist_kernel(int32_t n, const double* __restrict__ s,
                                                                 int32_t exclude, TopkState* st, int shift,
                                                                 int mode) {
  __shared__ uint32_t h[256];
  if (mode == 1 && !st->id_active) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const unsigned long long prefix = st->prefix, mask = st->mask, tau = st->tau;
  const uint32_t idp = st->id_prefix, idm = st->id_mask;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    if (j == exclude) continue;
    const unsigned long long key = order_key(s[j]);
    if (mode == 0) {
      if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
    } else {
      if (key == tau && (((uint32_t)j & idm) == idp)) atomicAdd(&h[((uint32_t)j >> shift) & 255u], 1u);
    }
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void topk_select_kernel(TopkState* st, int shift, int mode) {
  if (mode == 1 && !st->id_active) return;
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    // descending: find the digit holding the need-th largest
    uint32_t need = st->need;
    int d = 255;
    for (; d > 0; --d) {
      const uint32_t c = st->hist[d];
      if (c >= need) break;
      need -= c;
    }
    const uint32_t eq = st->hist[d];
    st->prefix |= (unsigned long long)d << shift;
    st->mask |= 255ull << shift;
    st->need = need;
    if (shift == 0) {
      st->tau = st->prefix;
      st->id_need = need;
      st->id_active = eq > need ? 1u : 0u;
    }
  } else {
    // ascending over ids among the ties: the id_need-th smallest
    uint32_t need = st->id_need;
    int d = 0;
    for (; d < 255; ++d) {
      const uint32_t c = st->hist[d];
      if (c >= need) break;
      need -= c;
    }
    st->id_prefix |= (uint32_t)d << shift;
    st->id_mask |= 255u << shift;
    st->id_need = need;
    if (shift == 0) st->id_limit = st->id_prefix;
  }
  for (int b = 0; b < 256; ++b) st->hist[b] = 0;
}

__global__ void topk_collect_kernel(int32_t n, const double* __restrict__ s, int32_t exclude, TopkState* st,
                                    unsigned long long* __restrict__ ckey, int32_t* __restrict__ cid) {
  const unsigned long long tau = st->tau;
  const uint32_t lim = st->id_limit;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    if (j == exclude) continue;
    const unsigned long long key = order_key(s[j]);
    if (key > tau || (key == tau && (uint32_t)j <= lim)) {
      const uint32_t pos = atomicAdd(&st->count, 1u);
      if (pos < kTopkMax) {
        ckey[pos] = key;
        cid[pos] = (int32_t)j;
      }
    }
  }
}

// (key desc, id asc) is "a before b"
__device__ __forceinline__ bool before(unsigned long long ka, int32_t ia, unsigned long long kb, int32_t ib) {
  return ka > kb || (ka == kb && ia < ib);
}

__global__ __launch_bounds__(1024) void topk_sort_kernel(int32_t k, const double* __restrict__ s,
                                                         const unsigned long long* __restrict__ ckey,
                                                         const int32_t* __restrict__ cid, int32_t* __restrict__ idx_out,
                                                         double* __restrict__ val_out) {
  __shared__ unsigned long long kk[kTopkMax];
  __shared__ int32_t ii[kTopkMax];
  int size = 1;
  while (size < k) size <<= 1;
  for (int t = threadIdx.x; t < size; t += blockDim.x) {
    if (t < k) {
      kk[t] = ckey[t];
      ii[t] = cid[t];
    } else {
      kk[t] = 0ull;  // below every real key
      ii[t] = 0x7fffffff;
    }
  }
  __syncthreads();
  for (int len = 2; len <= size; len <<= 1) {
    for (int stride = len >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < size; t += blockDim.x) {
        const int p = t ^ stride;
        if (p > t) {
          const bool up = (t & len) == 0;  // this run sorts in "before" order
          const bool ab = before(kk[t], ii[t], kk[p], ii[p]);
          if (up ? !ab : ab) {
            const unsigned long long tk = kk[t];
            kk[t] = kk[p];
            kk[p] = tk;
            const int32_t ti = ii[t];
            ii[t] = ii[p];
            ii[p] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    idx_out[t] = ii[t];
    if (val_out) val_out[t] = s[ii[t]];
  }
}

constexpr size_t kTopkBytes = ((sizeof(TopkState) + 15) & ~size_t(15)) +
                               kTopkMax * (sizeof(unsigned long long) + sizeof(int32_t));
static_assert(kTopkBytes <= kTopkScratchBytes, "top-k scratch too small");

// The whole selection in a caller-given device buffer of kTopkBytes.
es_status launch_topk_in(es_ctx* ctx, const double* s, int32_t n, int32_t exclude, int32_t k, int32_t* idx_out,
                         double* val_out, char* ws) {
  auto* st = (TopkState*)ws;
  auto* ckey = (unsigned long long*)(ws + ((sizeof(TopkState) + 15) & ~size_t(15)));
  auto* cid = (int32_t*)(ckey + kTopkMax);
  const int grid = std::max(1, std::min(ctx->num_cus * 4, ceil_div(n, kHistThreads)));
  topk_init_kernel<<<1, 256, 0, ctx->stream>>>(st, (uint32_t)k);
  for (int shift = 56; shift >= 0; shift -= 8) {
    topk_hist_kernel<<<grid, kHistThreads, 0, ctx->stream>>>(n, s, exclude, st, shift, 0);
    topk_select_kernel<<<1, 64, 0, ctx->stream>>>(st, shift, 0);
  }
  for (int shift = 24; shift >= 0; shift -= 8) {
    topk_hist_kernel<<<grid, kHistThreads, 0, ctx->stream>>>(n, s, exclude, st, shift, 1);
    topk_select_kernel<<<1, 64, 0, ctx->stream>>>(st, shift, 1);
  }
  topk_collect_kernel<<<grid, kHistThreads, 0, ctx->stream>>>(n, s, exclude, st, ckey, cid);
  topk_sort_kernel<<<1, 1024, 0, ctx->stream>>>(k, s, ckey, cid, idx_out, val_out);
  ES_CHECK_HIP(ctx, hipGetLastError());
  return ES_OK;
}

// Per device: the address of that device's copy of topk_scratch (found once,
// at context creation).
std::mutex scratch_mu;
std::vector<void*> scratch_ptr;

}  // namespace

es_status launch_topk(es_ctx* ctx, const double* s, int32_t n, int32_t exclude, int32_t k, int32_t* idx_out,
                      double* val_out) {
  es_status stt;
  char* ws = (char*)workspace(ctx, kWsTopk, kTopkBytes + 64, &stt);
  if (!ws) return stt;
  return launch_topk_in(ctx, s, n, exclude, k, idx_out, val_out, ws);
}

}  // namespace es

// Scratch of es_topk_noalloc: one copy per device for the life of the process.
static __device__ __align__(256) char topk_scratch[es::kTopkScratchBytes];

namespace es {

es_status topk_scratch_init(es_ctx* ctx) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  if ((int)scratch_ptr.size() <= ctx->device) scratch_ptr.resize(ctx->device + 1, nullptr);
  if (scratch_ptr[ctx->device]) return ES_OK;
  void* p = nullptr;
  // the device is current (es_ctx_create); the host name is not a device address
  ES_CHECK_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(topk_scratch)));
  scratch_ptr[ctx->device] = p;
  return ES_OK;
}

}  // namespace es

using namespace es;

extern "C" es_status es_topk(es_ctx* ctx, const double* s, int32_t n, int32_t exclude, int32_t k, int32_t* idx_out,
                             double* val_out) {
  if (!ctx || !s || !idx_out) return ES_EINVAL;
  const int32_t avail = n - ((exclude >= 0 && exclude < n) ? 1 : 0);
  if (n < 1 || k < 1 || k > avail) return fail(ctx, ES_EINVAL, "k=%d outside [1, %d]", k, avail);
  if (k > kTopkMax) return fail(ctx, ES_EUNSUPPORTED, "k=%d above %d", k, kTopkMax);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  return launch_topk(ctx, s, n, exclude, k, idx_out, val_out);
}

extern "C" es_status es_topk_noalloc(es_ctx* ctx, const double* s, int32_t n, int32_t exclude, int32_t k,
                                     int32_t* idx_out, double* val_out) {
  if (!ctx || !s || !idx_out) return ES_EINVAL;
  const int32_t avail = n - ((exclude >= 0 && exclude < n) ? 1 : 0);
  if (n < 1 || k < 1 || k > avail) return fail(ctx, ES_EINVAL, "k=%d outside [1, %d]", k, avail);
  if (k > kTopkMax) return fail(ctx, ES_EINVAL, "k=%d above the fixed scratch's %d", k, kTopkMax);
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (ctx->device < (int)scratch_ptr.size()) p = scratch_ptr[ctx->device];
  }
  if (!p) return fail(ctx, ES_EDEVICE, "top-k scratch of device %d not set up", ctx->device);
  ES_CHECK_HIP(ctx, hipSetDevice(ctx->device));
  return launch_topk_in(ctx, s, n, exclude, k, idx_out, val_out, (char*)p);
}
