// Host-side graph layout, edge packing and launch partitions (plain C++).
#include "es_host.h"

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <thread>

namespace es {

// ---------------------------------------------------------------------------
// Host-side parallel helpers for graph construction (std::thread; the worker
// count is OMP_NUM_THREADS when set, else the hardware count capped at 16).

int host_threads() {
  static const int t = [] {
    if (const char* e = std::getenv("OMP_NUM_THREADS")) {
      const int v = std::atoi(e);
      if (v >= 1) return std::min(v, 256);
    }
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(hc, 16u));
  }();
  return t;
}

// f(lo, hi) over [0, n) in dynamically dispatched blocks of at least `grain`.
template <class F>
void par_for(int64_t n, int64_t grain, F f) {
  if (n <= 0) return;
  const int T = host_threads();
  const int64_t nblk_target = (int64_t)T * 16;
  const int64_t blk = std::max<int64_t>(grain, (n + nblk_target - 1) / nblk_target);
  const int64_t nblk = (n + blk - 1) / blk;
  if (T == 1 || nblk == 1) {
    f((int64_t)0, n);
    return;
  }
  std::atomic<int64_t> next{0};
  auto work = [&] {
    for (;;) {
      const int64_t b = next.fetch_add(1, std::memory_order_relaxed);
      if (b >= nblk) return;
      f(b * blk, std::min(n, (b + 1) * blk));
    }
  };
  std::vector<std::thread> pool;
  const int nt = (int)std::min<int64_t>(T, nblk);
  try {
    pool.reserve(nt - 1);
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  } catch (...) {
    // fewer workers: the calling thread still drains every block
  }
  work();
  for (auto& th : pool) th.join();
}

void par_sort(std::vector<uint64_t>& a) {
  const int64_t n = (int64_t)a.size();
  const int T = host_threads();
  if (T == 1 || n < (1 << 20)) {
    std::sort(a.begin(), a.end());
    return;
  }
  int64_t nch = 1;
  while (nch < T) nch *= 2;
  std::vector<int64_t> cut(nch + 1);
  for (int64_t i = 0; i <= nch; ++i) cut[i] = n * i / nch;
  par_for(nch, 1, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) std::sort(a.begin() + cut[i], a.begin() + cut[i + 1]);
  });
  std::vector<uint64_t> buf(n);
  uint64_t* from = a.data();
  uint64_t* to = buf.data();
  for (int64_t w = 1; w < nch; w *= 2) {
    par_for(nch / (2 * w), 1, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        const int64_t l = cut[2 * w * i], mid = cut[2 * w * i + w], r = cut[2 * w * i + 2 * w];
        std::merge(from + l, from + mid, from + mid, from + r, to + l);
      }
    });
    std::swap(from, to);
  }
  if (from != a.data()) std::memcpy(a.data(), from, (size_t)n * sizeof(uint64_t));
}


// Offsets [0, n] of the keys of each external source (keys sorted by source).
std::vector<int64_t> source_starts(const std::vector<uint64_t>& keys, int32_t n) {
  std::vector<int64_t> st((size_t)n + 1);
  const int64_t m = (int64_t)keys.size();
  // st[v] = first key index with source >= v, by binary search per block of ids
  par_for(n + 1, 1 << 14, [&](int64_t lo, int64_t hi) {
    int64_t e = std::lower_bound(keys.begin(), keys.end(), (uint64_t)lo << 32) - keys.begin();
    for (int64_t v = lo; v < hi; ++v) {
      while (e < m && (int64_t)(keys[e] >> 32) < v) ++e;
      st[v] = e;
    }
  });
  return st;
}

void build_layout(const std::vector<uint64_t>& keys, int32_t n, HostLayout& h) {
  const int64_t m = (int64_t)keys.size();
  const std::vector<int64_t> sst = source_starts(keys, n);
  h.din_ext.assign(n, 0);
  h.dout_ext.resize(n);
  par_for(n, 1 << 14, [&](int64_t lo, int64_t hi) {
    for (int64_t v = lo; v < hi; ++v) h.dout_ext[v] = (int32_t)(sst[v + 1] - sst[v]);
  });
  int32_t* din = h.din_ext.data();
  par_for(m, 1 << 16, [&](int64_t lo, int64_t hi) {
    for (int64_t e = lo; e < hi; ++e) __atomic_fetch_add(&din[keys[e] & 0xffffffffu], 1, __ATOMIC_RELAXED);
  });
  // internal id = rank by total degree, descending, ties by external id:
  // ascending order of ((2^32 - 1 - degree) << 32 | id)
  {
    std::vector<uint64_t> rk(n);
    par_for(n, 1 << 14, [&](int64_t lo, int64_t hi) {
      for (int64_t v = lo; v < hi; ++v) {
        const uint64_t deg = (uint64_t)h.din_ext[v] + (uint64_t)h.dout_ext[v];
        rk[v] = ((0xffffffffull - deg) << 32) | (uint64_t)v;
      }
    });
    par_sort(rk);
    h.ext_of.resize(n);
    h.int_of.resize(n);
    par_for(n, 1 << 14, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        const int32_t v = (int32_t)(rk[i] & 0xffffffffu);
        h.ext_of[i] = v;
        h.int_of[v] = (int32_t)i;
      }
    });
  }
  // row offsets of both CSRs (internal rows)
  h.out_off.assign((size_t)n + 1, 0);
  h.in_off.assign((size_t)n + 1, 0);
  h.din_int.resize(n);
  h.inv_din.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = h.ext_of[i];
    const int32_t d = h.din_ext[v];
    h.din_int[i] = d;
    h.inv_din[i] = d > 0 ? 1.0 / (double)d : 0.0;
    h.out_off[i + 1] = h.out_off[i] + h.dout_ext[v];
    h.in_off[i + 1] = h.in_off[i] + d;
  }
  // out-CSR: the keys of external source v fill internal row int_of[v];
  // columns internal, ascending
  h.out_idx.resize(m);
  par_for(n, 1 << 12, [&](int64_t lo, int64_t hi) {
    for (int64_t v = lo; v < hi; ++v) {
      int32_t* row = h.out_idx.data() + h.out_off[h.int_of[v]];
      const int64_t b = sst[v], e = sst[v + 1];
      for (int64_t k = b; k < e; ++k) row[k - b] = h.int_of[keys[k] & 0xffffffffu];
      std::sort(row, row + (e - b));
    }
  });
  // in-CSR: rows in ascending external source order (the walk's order).
  // Stable partition of the keys (already in source order) into P row
  // ranges of about equal edge counts, then an in-order scatter per range:
  // every row receives its sources in key order, i.e. ascending.
  h.in_idx.resize(m);
  {
    const int T = host_threads();
    const int64_t P = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>((int64_t)T * 64, 65535), n));
    std::vector<int64_t> rstart(P + 1);
    for (int64_t b = 0; b <= P; ++b)
      rstart[b] = b == 0 ? 0 : b == P ? n : std::lower_bound(h.in_off.begin(), h.in_off.end() - 1, (int32_t)(m * b / P)) - h.in_off.begin();
    // range of the row of every external node
    std::vector<uint16_t> part(n);
    par_for(P, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo; b < hi; ++b)
        for (int64_t r = rstart[b]; r < rstart[b + 1]; ++r) part[h.ext_of[r]] = (uint16_t)b;
    });
    // counts per (key chunk, range); chunks are contiguous and in order
    const int64_t C = std::max<int64_t>(1, std::min<int64_t>((int64_t)T * 4, (m + (1 << 16) - 1) >> 16));
    std::vector<int64_t> cnt((size_t)(C * P), 0);
    par_for(C, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t c = lo; c < hi; ++c) {
        int64_t* q = cnt.data() + c * P;
        for (int64_t e = m * c / C; e < m * (c + 1) / C; ++e) q[part[keys[e] & 0xffffffffu]]++;
      }
    });
    // range-major, chunk-minor offsets
    std::vector<int64_t> pstart(P + 1, 0);
    int64_t acc = 0;
    for (int64_t b = 0; b < P; ++b) {
      pstart[b] = acc;
      for (int64_t c = 0; c < C; ++c) {
        const int64_t k = cnt[c * P + b];
        cnt[c * P + b] = acc;
        acc += k;
      }
    }
    pstart[P] = acc;
    // (internal row << 32 | internal source) in stable order per range
    std::vector<uint64_t> tmp(m);
    par_for(C, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t c = lo; c < hi; ++c) {
        int64_t* q = cnt.data() + c * P;
        for (int64_t e = m * c / C; e < m * (c + 1) / C; ++e) {
          const uint64_t k = keys[e];
          const uint32_t d = (uint32_t)(k & 0xffffffffu);
          tmp[q[part[d]]++] = ((uint64_t)(uint32_t)h.int_of[d] << 32) | (uint32_t)h.int_of[k >> 32];
        }
      }
    });
    // next free slot of every row; each range touches only its own rows
    std::vector<int32_t> pos(h.in_off.begin(), h.in_off.end() - 1);
    par_for(P, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo; b < hi; ++b)
        for (int64_t i = pstart[b]; i < pstart[b + 1]; ++i) {
          const uint64_t t = tmp[i];
          h.in_idx[pos[t >> 32]++] = (int32_t)(t & 0xffffffffu);
        }
    });
  }
}


bool pack_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, bool drop_self_loops, bool dedup,
                std::vector<uint64_t>& keys, int64_t* bad_edge) {
  keys.resize((size_t)m);
  // pack, validate and (optionally) drop self-loops, in parallel blocks;
  // per-block counts give each block its place in the compacted array
  {
    const int64_t kBlk = 1 << 20;
    const int64_t nblk = (m + kBlk - 1) / kBlk;
    std::vector<int64_t> kept((size_t)nblk + 1, 0), bad((size_t)nblk, -1);
    std::vector<uint8_t> blk_sorted((size_t)nblk, 1);
    const bool drop = drop_self_loops;
    par_for(nblk, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo; b < hi; ++b) {
        int64_t k = 0;
        for (int64_t e = b * kBlk; e < std::min(m, (b + 1) * kBlk); ++e) {
          const int32_t s = src[e], d = dst[e];
          if (s < 0 || s >= n || d < 0 || d >= n) {
            bad[b] = e;
            break;
          }
          if (!(drop && s == d)) ++k;
        }
        kept[b + 1] = k;
      }
    });
    for (int64_t b = 0; b < nblk; ++b)
      if (bad[b] >= 0) {
        *bad_edge = bad[b];
        return false;
      }
    for (int64_t b = 0; b < nblk; ++b) kept[b + 1] += kept[b];
    par_for(nblk, 1, [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo; b < hi; ++b) {
        int64_t w = kept[b];
        uint64_t prev = 0;
        bool first = true;
        for (int64_t e = b * kBlk; e < std::min(m, (b + 1) * kBlk); ++e) {
          const int32_t s = src[e], d = dst[e];
          if (drop && s == d) continue;
          const uint64_t key = ((uint64_t)(uint32_t)s << 32) | (uint32_t)d;
          if (!first && key <= prev) blk_sorted[b] = 0;
          prev = key;
          first = false;
          keys[w++] = key;
        }
      }
    });
    keys.resize((size_t)kept[nblk]);
    bool sorted = true;
    for (int64_t b = 0; b < nblk; ++b) sorted = sorted && blk_sorted[b];
    for (int64_t b = 1; sorted && b < nblk; ++b)
      if (kept[b] > 0 && kept[b] < (int64_t)keys.size() && keys[kept[b]] <= keys[kept[b] - 1]) sorted = false;
    if (!sorted) par_sort(keys);
  }
  if (dedup) keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  return true;
}

void spmv_partition(const int32_t* off, int32_t n, SpmvPartition& out) {
  std::vector<BlockDesc> longs, shorts;
  std::vector<int32_t> long_p0, long_nch;
  int32_t nslots = 0;
  int32_t maxnnz = 0;
  int32_t r = 0;
  while (r < n) {
    const int32_t deg = off[r + 1] - off[r];
    maxnnz = std::max(maxnnz, deg);
    if (deg > kSpmvNnz) {
      const int32_t lid = (int32_t)long_p0.size();
      const int32_t nch = (deg + kLongChunk - 1) / kLongChunk;
      long_p0.push_back(nslots);
      long_nch.push_back(nch);
      nslots += nch;
      for (int32_t c = 0; c < nch; ++c) {
        const int32_t e0 = off[r] + c * kLongChunk;
        const int32_t e1 = std::min<int32_t>(e0 + kLongChunk, off[r + 1]);
        longs.push_back(BlockDesc{r, -(lid + 1), e0, e1});
      }
      ++r;
      continue;
    }
    const int32_t r0 = r, e0 = off[r];
    while (r < n && r - r0 < kSpmvRows && off[r + 1] - e0 <= kSpmvNnz) {
      maxnnz = std::max(maxnnz, off[r + 1] - off[r]);
      ++r;
    }
    shorts.push_back(BlockDesc{r0, r, e0, off[r]});
  }
  std::vector<BlockDesc> all;
  all.reserve(longs.size() + shorts.size());
  all.insert(all.end(), longs.begin(), longs.end());
  all.insert(all.end(), shorts.begin(), shorts.end());
  out.blocks = std::move(all);
  out.long_p0 = std::move(long_p0);
  out.long_nch = std::move(long_nch);
  out.nslots = nslots;
  out.max_row_nnz = maxnnz;
}

// Tiles over the rows of one block for one CSR direction.
void make_tiles(const std::vector<int32_t>& off, int32_t n, int32_t entry, int32_t W, int32_t G,
                std::vector<MTile>& tiles, std::vector<LongRow>& longs, int32_t& nlong) {
  const int32_t P = 64 / W;
  const int64_t target = (int64_t)P * G;
  int32_t r = 0;
  while (r < n) {
    const int32_t deg = off[r + 1] - off[r];
    if (deg > kLongRow) {
      // one partial slot per chunk
      const int32_t first = nlong;
      for (int32_t e0 = off[r]; e0 < off[r + 1]; e0 += kLongRow)
        tiles.push_back(MTile{entry, r, -(nlong++ + 1), e0, std::min(e0 + kLongRow, off[r + 1]), r});
      longs.push_back(LongRow{entry, r, first, nlong - first});
      ++r;
      continue;
    }
    const int32_t r0 = r;
    int64_t acc = 0;
    while (r < n) {
      const int32_t d = off[r + 1] - off[r];
      if (d > kLongRow) break;
      const int64_t w = std::max<int32_t>(d, 1);
      if (r > r0 && acc + w > target) break;
      acc += w;
      ++r;
    }
    tiles.push_back(MTile{entry, r0, r, 0, 0, 0});
  }
}


// ---------------------------------------------------------------------------
// Binned level pass layout.

void build_binned(const int32_t* off, const int32_t* idx, int32_t n, int32_t shift, BinnedLayout& b,
                  int32_t max_src, int32_t max_ent, int32_t max_acc) {
  const int32_t m = off[n];
  const int32_t rows = 1 << shift;
  const uint32_t mask = (uint32_t)rows - 1u;
  b.shift = shift;
  b.nbins = (int32_t)(((int64_t)n + rows - 1) >> shift);
  b.ranges.clear();
  // 1. ranges of consecutive sources: at most max_src sources and max_ent
  // entries each; a source with more than max_ent entries is cut into ranges
  // of its own
  for (int32_t j = 0; j < n;) {
    const int32_t d = off[j + 1] - off[j];
    if (d > max_ent) {
      for (int32_t e = off[j]; e < off[j + 1]; e += max_ent)
        b.ranges.push_back(BinRange{j, j + 1, e, std::min(e + max_ent, off[j + 1]), 0, 0});
      ++j;
      continue;
    }
    const int32_t j0 = j;
    int32_t ents = 0;
    while (j < n && j - j0 < max_src) {
      const int32_t dj = off[j + 1] - off[j];
      if (dj > max_ent || ents + dj > max_ent) break;
      ents += dj;
      ++j;
    }
    b.ranges.push_back(BinRange{j0, j, off[j0], off[j], 0, 0});
  }
  const int64_t W = (int64_t)b.ranges.size();
  // 2. each range's entries in (bin, push-list) order: source slots, and the
  // destination rows in that order for step 4; its segments (bin, first entry)
  b.src_local.assign((size_t)m, 0);
  std::vector<uint16_t> tmp_row((size_t)m, 0);
  std::vector<std::vector<std::pair<int32_t, int32_t>>> rsegs((size_t)W);
  par_for(W, 1, [&](int64_t lo, int64_t hi) {
    std::vector<uint64_t> keys;
    std::vector<uint16_t> loc;
    for (int64_t w = lo; w < hi; ++w) {
      const BinRange& r = b.ranges[(size_t)w];
      const int32_t E = r.e1 - r.e0;
      keys.resize((size_t)E);
      loc.resize((size_t)E);
      for (int32_t j = r.j0; j < r.j1; ++j)
        for (int32_t e = std::max(off[j], r.e0); e < std::min(off[j + 1], r.e1); ++e)
          loc[(size_t)(e - r.e0)] = (uint16_t)(j - r.j0);
      for (int32_t t = 0; t < E; ++t)
        keys[(size_t)t] = ((uint64_t)((uint32_t)idx[r.e0 + t] >> shift) << 32) | (uint32_t)t;
      std::sort(keys.begin(), keys.end());
      auto& sg = rsegs[(size_t)w];
      int32_t last = -1;
      for (int32_t t = 0; t < E; ++t) {
        const int32_t bin = (int32_t)(keys[(size_t)t] >> 32);
        const uint32_t el = (uint32_t)keys[(size_t)t];
        b.src_local[(size_t)(r.e0 + t)] = loc[el];
        tmp_row[(size_t)(r.e0 + t)] = (uint16_t)((uint32_t)idx[r.e0 + (int32_t)el] & mask);
        if (bin != last) {
          sg.emplace_back(bin, t);
          last = bin;
        }
      }
    }
  });
  // 3. bin-major offsets, then each segment's output position: within a bin,
  // the ranges' segments in range order
  std::vector<int64_t> cnt((size_t)b.nbins, 0);
  int64_t nseg = 0;
  for (int64_t w = 0; w < W; ++w) {
    const BinRange& r = b.ranges[(size_t)w];
    const auto& sg = rsegs[(size_t)w];
    for (size_t i = 0; i < sg.size(); ++i) {
      const int32_t end = i + 1 < sg.size() ? sg[i + 1].second : r.e1 - r.e0;
      cnt[(size_t)sg[i].first] += end - sg[i].second;
    }
    nseg += (int64_t)sg.size();
  }
  b.bin_off.assign((size_t)b.nbins + 1, 0);
  for (int32_t k = 0; k < b.nbins; ++k) b.bin_off[(size_t)k + 1] = b.bin_off[(size_t)k] + (int32_t)cnt[(size_t)k];
  std::vector<int32_t> run(b.bin_off.begin(), b.bin_off.end() - 1);
  b.segs.clear();
  b.segs.reserve((size_t)nseg);
  for (int64_t w = 0; w < W; ++w) {
    BinRange& r = b.ranges[(size_t)w];
    const auto& sg = rsegs[(size_t)w];
    r.s0 = (int32_t)b.segs.size();
    for (size_t i = 0; i < sg.size(); ++i) {
      const int32_t end = i + 1 < sg.size() ? sg[i + 1].second : r.e1 - r.e0;
      b.segs.push_back(BinSeg{(uint32_t)(r.e0 + sg[i].second), (uint32_t)run[(size_t)sg[i].first]});
      run[(size_t)sg[i].first] += end - sg[i].second;
    }
    r.s1 = (int32_t)b.segs.size();
    std::vector<std::pair<int32_t, int32_t>>().swap(rsegs[(size_t)w]);
  }
  // 4. destination rows in bin-major order, each entry's value position
  b.row_local.assign((size_t)m, 0);
  b.pos.assign((size_t)m, 0);
  par_for(W, 1, [&](int64_t lo, int64_t hi) {
    for (int64_t w = lo; w < hi; ++w) {
      const BinRange& r = b.ranges[(size_t)w];
      for (int32_t s = r.s0; s < r.s1; ++s) {
        const uint32_t k = b.segs[(size_t)s].k, out = b.segs[(size_t)s].out;
        const uint32_t end = s + 1 < r.s1 ? b.segs[(size_t)s + 1].k : (uint32_t)r.e1;
        std::memcpy(&b.row_local[out], &tmp_row[k], sizeof(uint16_t) * (end - k));
        for (uint32_t t = k; t < end; ++t) b.pos[t] = out + (t - k);
      }
    }
  });
  // 5. accumulate items: one per bin, or one per max_acc entries with a
  // partial-sum slot each
  b.items.clear();
  b.splits.clear();
  b.nslots = 0;
  for (int32_t k = 0; k < b.nbins; ++k) {
    const int32_t p0 = b.bin_off[(size_t)k], p1 = b.bin_off[(size_t)k + 1];
    if (p1 - p0 <= max_acc) {
      b.items.push_back(BinItem{k, p0, p1, -1});
      continue;
    }
    const int32_t ns = (int32_t)(((int64_t)p1 - p0 + max_acc - 1) / max_acc);
    b.splits.push_back(BinSplit{k, b.nslots, ns});
    for (int32_t t = 0; t < ns; ++t)
      b.items.push_back(BinItem{k, p0 + t * max_acc, std::min(p1, p0 + (t + 1) * max_acc), b.nslots + t});
    b.nslots += ns;
  }
}

}  // namespace es
