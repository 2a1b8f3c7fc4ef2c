// Runs the library's host-side builders (es_host.cpp: edge packing, the
// degree-ordered CSR layout, the SpMV row partition, the batched SpMM tiles
// and the binned level pass layout) on edge cases, with invariant checks, so
// that a build with AddressSanitizer and UndefinedBehaviorSanitizer checks
// every access:
// one node, no edges, duplicate edges and self-loops, rows longer than the
// SpMV's 8192-entry and the SpMM's 1024-entry cuts, push lists and bins
// longer than the binned level pass's ranges and items, an id out of range.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "es_host.h"

using namespace es;

#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond);     \
      return 1;                                                      \
    }                                                                \
  } while (0)

// Every row covered once, entries in order, long rows cut into chunks.
static int check_partition(const std::vector<int32_t>& off, int32_t n) {
  SpmvPartition p;
  spmv_partition(off.data(), n, p);
  std::vector<int32_t> seen(n, 0);
  std::vector<int64_t> long_entries(p.long_p0.size(), 0);
  int32_t maxnnz = 0;
  for (int32_t r = 0; r < n; ++r) maxnnz = std::max(maxnnz, off[r + 1] - off[r]);
  CHECK(p.max_row_nnz == maxnnz);
  for (const BlockDesc& b : p.blocks) {
    if (b.row1 >= 0) {
      CHECK(b.row0 < b.row1 && b.row1 <= n && b.row1 - b.row0 <= kSpmvRows);
      CHECK(b.e0 == off[b.row0] && b.e1 == off[b.row1] && b.e1 - b.e0 <= kSpmvNnz);
      for (int32_t r = b.row0; r < b.row1; ++r) ++seen[r];
    } else {
      const int32_t lid = -b.row1 - 1;
      CHECK(lid >= 0 && lid < (int32_t)p.long_p0.size());
      CHECK(b.e0 >= off[b.row0] && b.e1 <= off[b.row0 + 1] && b.e1 - b.e0 <= kLongChunk && b.e0 < b.e1);
      long_entries[lid] += b.e1 - b.e0;
      if (b.e0 == off[b.row0]) ++seen[b.row0];
    }
  }
  for (int32_t r = 0; r < n; ++r) CHECK(seen[r] == 1);
  int32_t slots = 0;
  for (size_t i = 0; i < p.long_p0.size(); ++i) {
    CHECK(p.long_p0[i] == slots);
    slots += p.long_nch[i];
  }
  CHECK(slots == p.nslots);
  return 0;
}

// Tiles cover every row of the block once; long-row chunks cover their row.
static int check_tiles(const std::vector<int32_t>& off, int32_t n) {
  for (int32_t W : {8, 16, 64})
    for (int32_t G : {1, 8, 128}) {
      std::vector<MTile> tiles;
      std::vector<LongRow> longs;
      int32_t nlong = 5;  // slots already used by an earlier direction
      make_tiles(off, n, 3, W, G, tiles, longs, nlong);
      std::vector<int64_t> cover(n, 0);
      std::vector<int32_t> slot_used(nlong, 0);
      for (const MTile& t : tiles) {
        CHECK(t.entry == 3);
        if (t.row1 >= 0) {
          CHECK(t.row0 < t.row1 && t.row1 <= n);
          for (int32_t r = t.row0; r < t.row1; ++r) {
            CHECK(off[r + 1] - off[r] <= kLongRow);
            cover[r] += std::max(off[r + 1] - off[r], 1);
          }
        } else {
          const int32_t slot = -t.row1 - 1;
          CHECK(slot >= 5 && slot < nlong);
          ++slot_used[slot];
          CHECK(t.row == t.row0 && t.e0 >= off[t.row] && t.e1 <= off[t.row + 1] && t.e1 - t.e0 <= kLongRow);
          cover[t.row] += t.e1 - t.e0;
        }
      }
      for (int32_t r = 0; r < n; ++r) CHECK(cover[r] == std::max(off[r + 1] - off[r], 1));
      for (int32_t s = 5; s < nlong; ++s) CHECK(slot_used[s] == 1);
      int32_t nch = 0;
      for (const LongRow& l : longs) {
        CHECK(l.nch >= 2 && l.slot >= 5 && l.slot + l.nch <= nlong);
        CHECK(l.nch == (off[l.row + 1] - off[l.row] + kLongRow - 1) / kLongRow);
        nch += l.nch;
      }
      CHECK(nch == nlong - 5);
    }
  return 0;
}

// Binned layout: every edge appears once as (source, destination row), every
// value position once, ranges and items within their limits and in order.
static int check_binned(const std::vector<int32_t>& off, const std::vector<int32_t>& idx, int32_t n, int32_t shift,
                        int32_t max_src = kBinSrc, int32_t max_ent = kBinEnt, int32_t max_acc = kBinAccEnt) {
  BinnedLayout b;
  build_binned(off.data(), idx.data(), n, shift, b, max_src, max_ent, max_acc);
  const int32_t m = off[n];
  CHECK(b.nbins == (int32_t)(((int64_t)n + (1 << shift) - 1) >> shift));
  CHECK((int32_t)b.bin_off.size() == b.nbins + 1 && b.bin_off[0] == 0 && b.bin_off[b.nbins] == m);
  CHECK((int32_t)b.src_local.size() == m && (int32_t)b.row_local.size() == m && (int32_t)b.pos.size() == m);
  std::vector<uint64_t> want, got;
  for (int32_t j = 0; j < n; ++j)
    for (int32_t e = off[j]; e < off[j + 1]; ++e) want.push_back(((uint64_t)j << 32) | (uint32_t)idx[e]);
  std::vector<uint8_t> hit((size_t)m, 0);
  int32_t next_e = 0, next_j = 0;
  for (const BinRange& r : b.ranges) {
    CHECK(r.e0 == next_e && r.e0 <= r.e1 && r.e1 - r.e0 <= max_ent);
    CHECK(r.j0 < r.j1 && r.j1 - r.j0 <= max_src && r.j1 <= n);
    CHECK(r.j0 == next_j || (r.j0 == next_j - 1 && r.j1 == r.j0 + 1));  // cut lists repeat their source
    CHECK(r.e0 >= off[r.j0] && r.e1 <= off[r.j1]);
    next_e = r.e1;
    next_j = r.j1;
    CHECK(r.s0 <= r.s1 && r.s1 <= (int32_t)b.segs.size());
    CHECK((r.e1 > r.e0) == (r.s1 > r.s0));
    int32_t last_bin = -1;
    for (int32_t s = r.s0; s < r.s1; ++s) {
      const BinSeg& g = b.segs[(size_t)s];
      const uint32_t end = s + 1 < r.s1 ? b.segs[(size_t)s + 1].k : (uint32_t)r.e1;
      CHECK(g.k >= (uint32_t)r.e0 && g.k < end && end <= (uint32_t)r.e1);
      if (s == r.s0) CHECK(g.k == (uint32_t)r.e0);
      const int32_t bin = (int32_t)(std::upper_bound(b.bin_off.begin(), b.bin_off.end(), (int32_t)g.out) -
                                    b.bin_off.begin()) - 1;
      CHECK(bin > last_bin && bin < b.nbins);
      last_bin = bin;
      CHECK(g.out + (end - g.k) <= (uint32_t)b.bin_off[(size_t)bin + 1]);
      for (uint32_t k = g.k; k < end; ++k) {
        const uint32_t pos = g.out + (k - g.k);
        CHECK(b.pos[k] == pos);
        CHECK(hit[pos] == 0);
        hit[pos] = 1;
        const int32_t j = r.j0 + b.src_local[k];
        CHECK(j < r.j1);
        const int64_t row = ((int64_t)bin << shift) | b.row_local[pos];
        CHECK(row < n);
        got.push_back(((uint64_t)j << 32) | (uint32_t)row);
      }
    }
  }
  CHECK(next_e == m && (m == 0 || next_j == n || off[next_j] == m));
  std::sort(want.begin(), want.end());
  std::sort(got.begin(), got.end());
  CHECK(want == got);
  // items: each bin's entries exactly once, in order; split bins own their slots
  int32_t it = 0, slots = 0;
  size_t sp = 0;
  for (int32_t bin = 0; bin < b.nbins; ++bin) {
    int32_t p = b.bin_off[(size_t)bin];
    int32_t count = 0;
    while (it < (int32_t)b.items.size() && b.items[(size_t)it].bin == bin) {
      const BinItem& x = b.items[(size_t)it];
      CHECK(x.p0 == p && x.p0 <= x.p1 && x.p1 - x.p0 <= max_acc);
      p = x.p1;
      ++count;
      ++it;
      if (x.slot >= 0) CHECK(x.slot == slots++);
    }
    CHECK(count >= 1 && p == b.bin_off[(size_t)bin + 1]);
    if (count > 1) {
      CHECK(sp < b.splits.size() && b.splits[sp].bin == bin && b.splits[sp].nslot == count);
      CHECK(b.splits[sp].slot0 + count == slots);
      ++sp;
    }
  }
  CHECK(it == (int32_t)b.items.size() && sp == b.splits.size() && slots == b.nslots);
  return 0;
}

static int run(const char* name, int32_t n, const std::vector<int32_t>& src, const std::vector<int32_t>& dst,
               bool drop, bool dedup) {
  std::vector<uint64_t> keys;
  int64_t bad = -1;
  CHECK(pack_edges(n, (int64_t)src.size(), src.data(), dst.data(), drop, dedup, keys, &bad));
  CHECK(std::is_sorted(keys.begin(), keys.end()));
  if (dedup) CHECK(std::adjacent_find(keys.begin(), keys.end()) == keys.end());
  if (drop)
    for (uint64_t k : keys) CHECK((k >> 32) != (k & 0xffffffffu));
  HostLayout h;
  build_layout(keys, n, h);
  const int64_t m = (int64_t)keys.size();
  CHECK((int64_t)h.out_off.size() == n + 1 && (int64_t)h.in_off.size() == n + 1);
  CHECK(h.out_off[n] == m && h.in_off[n] == m);
  // the permutation, the degree order, both CSRs against the keys
  std::vector<int32_t> din(n, 0), dout(n, 0);
  for (uint64_t k : keys) {
    ++dout[k >> 32];
    ++din[k & 0xffffffffu];
  }
  for (int32_t v = 0; v < n; ++v) {
    CHECK(h.ext_of[h.int_of[v]] == v);
    CHECK(h.din_ext[v] == din[v] && h.dout_ext[v] == dout[v]);
  }
  for (int32_t i = 1; i < n; ++i) {
    const int32_t a = h.ext_of[i - 1], b = h.ext_of[i];
    CHECK(din[a] + dout[a] > din[b] + dout[b] || (din[a] + dout[a] == din[b] + dout[b] && a < b));
  }
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = h.ext_of[i];
    CHECK(h.din_int[i] == din[v] && h.in_off[i + 1] - h.in_off[i] == din[v]);
    CHECK(h.out_off[i + 1] - h.out_off[i] == dout[v]);
    CHECK(h.inv_din[i] == (din[v] ? 1.0 / din[v] : 0.0));
    for (int32_t e = h.out_off[i] + 1; e < h.out_off[i + 1]; ++e) CHECK(h.out_idx[e - 1] < h.out_idx[e] || !dedup);
    for (int32_t e = h.in_off[i] + 1; e < h.in_off[i + 1]; ++e)
      CHECK(h.ext_of[h.in_idx[e - 1]] <= h.ext_of[h.in_idx[e]]);
  }
  std::vector<uint64_t> rebuilt;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = h.in_off[i]; e < h.in_off[i + 1]; ++e)
      rebuilt.push_back(((uint64_t)(uint32_t)h.ext_of[h.in_idx[e]] << 32) | (uint32_t)h.ext_of[i]);
  std::sort(rebuilt.begin(), rebuilt.end());
  CHECK(rebuilt == keys);
  if (check_partition(h.out_off, n) || check_partition(h.in_off, n)) return 1;
  if (check_tiles(h.out_off, n) || check_tiles(h.in_off, n)) return 1;
  for (int32_t shift : {1, 4, 12, 14})
    if (check_binned(h.in_off, h.in_idx, n, shift) || check_binned(h.out_off, h.out_idx, n, shift)) return 1;
  // small limits: cut push lists, split bins, source-bound ranges
  if (check_binned(h.in_off, h.in_idx, n, 12, 100, 5000, 3000) ||
      check_binned(h.out_off, h.out_idx, n, 12, 100, 5000, 3000))
    return 1;
  std::printf("%s: n=%d m=%lld ok\n", name, n, (long long)m);
  return 0;
}

int main() {
  int rc = 0;
  rc |= run("one node", 1, {}, {}, true, true);
  rc |= run("one node, self-loop kept", 1, {0, 0}, {0, 0}, false, false);
  rc |= run("no edges", 7, {}, {}, true, true);
  rc |= run("duplicates and self-loops", 5, {0, 0, 1, 1, 2, 2, 3, 4, 4}, {1, 1, 1, 2, 2, 0, 3, 0, 0}, true, true);
  rc |= run("duplicates kept", 5, {0, 0, 1, 2}, {1, 1, 2, 0}, false, false);
  {
    // a hub with more in- and out-neighbours than either cut, plus random edges
    const int32_t n = 30000;
    std::mt19937_64 rng(7);
    std::vector<int32_t> s, d;
    for (int32_t v = 1; v < n; ++v) {
      s.push_back(v);
      d.push_back(0);
      if (v < 12000) {
        s.push_back(0);
        d.push_back(v);
      }
    }
    for (int32_t v = 1; v < 1500; ++v) {
      s.push_back(n - 1 - v);
      d.push_back(n - 1);
    }
    for (int i = 0; i < 60000; ++i) {
      s.push_back((int32_t)(rng() % n));
      d.push_back((int32_t)(rng() % n));
    }
    std::vector<size_t> ord(s.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
    std::shuffle(ord.begin(), ord.end(), rng);
    std::vector<int32_t> s2, d2;
    for (size_t i : ord) {
      s2.push_back(s[i]);
      d2.push_back(d[i]);
    }
    rc |= run("hub rows over both cuts, unsorted input", n, s2, d2, true, true);
  }
  {
    // several packing blocks of 2^20 edges, the parallel sort's merges and
    // the in-CSR's range partition
    const int32_t n = 200000;
    std::mt19937_64 rng(11);
    std::vector<int32_t> s(2500000), d(2500000);
    for (size_t i = 0; i < s.size(); ++i) {
      s[i] = (int32_t)(rng() % n);
      d[i] = (int32_t)((rng() % 7 == 0) ? s[i] : rng() % 64);  // self-loops, and 64 hubs of in-degree ~3e4
    }
    rc |= run("2.5e6 unsorted edges", n, s, d, true, true);
  }
  {
    // a node with more in- and out-neighbours than a scatter range and an
    // accumulate item take at the default limits: cut push lists, split bins
    const int32_t n = 1100001;
    std::vector<int32_t> s, d;
    for (int32_t v = 1; v < n; ++v) {
      s.push_back(v);
      d.push_back(0);
      s.push_back(0);
      d.push_back(v);
    }
    rc |= run("star of 1.1e6 leaves both ways", n, s, d, true, true);
  }
  {
    // an endpoint out of range is reported, not read past
    std::vector<uint64_t> keys;
    int64_t bad = -1;
    const std::vector<int32_t> s{0, 1, 2}, d{1, 5, 0};
    if (pack_edges(3, 3, s.data(), d.data(), true, true, keys, &bad) || bad != 1) {
      std::printf("FAIL bad edge not reported\n");
      rc = 1;
    }
  }
  if (rc == 0) std::printf("ok\n");
  return rc;
}
