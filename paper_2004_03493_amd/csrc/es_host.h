// Host-side graph layout, edge packing and launch partitions of libexactsim:
// plain C++ (no HIP), so the library links it and the tests can also build
// it alone with sanitizers.
#pragma once

#include <cstdint>
#include <vector>

namespace es {

// Sparse row partition used by both SpMV directions (pull form); see
// es_internal.h for how the blocks are processed.
constexpr int kSpmvNnz = 8192;
constexpr int kSpmvRows = 512;
constexpr int kLongChunk = 8192;

struct BlockDesc {
  int32_t row0;  // first row
  int32_t row1;  // one past the last row; < 0: long-row chunk of long row (-row1 - 1)
  int32_t e0;    // first entry
  int32_t e1;    // one past the last entry
};

struct SpmvPartition {
  std::vector<BlockDesc> blocks;  // long-row chunks first, then multi-row blocks
  std::vector<int32_t> long_p0;   // first partial slot of each long row
  std::vector<int32_t> long_nch;  // chunk count of each long row
  int32_t nslots = 0;
  int32_t max_row_nnz = 0;
};

// Rows 0..n-1 of a CSR with offsets off[0..n] cut into work blocks.
void spmv_partition(const int32_t* off, int32_t n, SpmvPartition& out);

// Batched SpMM tiles (es_batch): a tile is a run of rows of one block for one
// wave, or one chunk of a row longer than kLongRow.
constexpr int kLongRow = 1024;

struct MTile {
  int32_t entry;
  int32_t row0;
  int32_t row1;  // < 0: chunk of long row slot (-row1 - 1)
  int32_t e0;
  int32_t e1;
  int32_t row;   // long chunk: the row
};

struct LongRow {
  int32_t entry;
  int32_t row;
  int32_t slot;  // first partial slot; the row's chunks use slot .. slot + nch - 1
  int32_t nch;
};

// Tiles over the rows of one block (descriptor `entry`) for one CSR
// direction: rows grouped so that a wave of 64/W lane groups gets about
// (64/W)*G entries; long rows split into chunks with one partial slot each
// (nlong counts the slots and is advanced).
void make_tiles(const std::vector<int32_t>& off, int32_t n, int32_t entry, int32_t W, int32_t G,
                std::vector<MTile>& tiles, std::vector<LongRow>& longs, int32_t& nlong);

// Worker count of the host-side builders: OMP_NUM_THREADS when set, else the
// hardware count capped at 16.
int host_threads();

// Ascending sort of a uint64 array: sorted chunks, then pairwise merges.
void par_sort(std::vector<uint64_t>& a);

// Edge keys (src << 32 | dst) of m host edges: validated (*bad = the first
// edge with an endpoint outside [0, n), and the function returns false),
// self-loops dropped if drop_self_loops, sorted ascending, duplicates merged
// if dedup.
bool pack_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, bool drop_self_loops, bool dedup,
                std::vector<uint64_t>& keys, int64_t* bad);

// Binned (propagation-blocked) level pass: the level product is computed in
// push form.  A scatter pass streams the sources in order, each workgroup
// staging the values of one range of sources and writing one value per edge
// into the bin of the edge's destination row; an accumulate pass then sums
// each bin's values into its rows in LDS.  Every access to the level vectors
// is a sequential one; the per-edge traffic is a 2-byte source slot and a
// 4-byte position, the 8-byte value written and read back, and a 2-byte row
// slot.
constexpr int kBinSrc = 16384;       // sources staged per scatter workgroup (128 KiB of values)
constexpr int kBinEnt = 1 << 20;     // entries per scatter workgroup
constexpr int kBinAccEnt = 1 << 20;  // entries per accumulate workgroup (longer bins are split)

struct BinRange {
  int32_t j0, j1;  // sources [j0, j1) (one source when its list is cut into several ranges)
  int32_t e0, e1;  // its entries [e0, e1) in push-list order
  int32_t s0, s1;  // its segments (one per bin it writes), ascending bin
};

struct BinSeg {
  uint32_t k;    // first entry of the segment (absolute, within [e0, e1) of its range)
  uint32_t out;  // position of that entry's value in the bin-major value array
};

struct BinItem {
  int32_t bin;
  int32_t p0, p1;  // bin-major entries [p0, p1)
  int32_t slot;    // -1: the item completes the bin; else its partial-sum slot
};

struct BinSplit {
  int32_t bin;
  int32_t slot0, nslot;  // partial-sum slots of a bin split over several items
};

struct BinnedLayout {
  int32_t shift = 0;  // rows per bin = 2^shift
  int32_t nbins = 0;
  int32_t nslots = 0;
  std::vector<BinRange> ranges;
  std::vector<BinSeg> segs;
  std::vector<uint16_t> src_local;  // [m] source - j0 of each entry, each range's entries in bin order
  std::vector<uint32_t> pos;        // [m] each entry's position in the bin-major value array
  std::vector<uint16_t> row_local;  // [m] destination row - bin * 2^shift, bin-major
  std::vector<int32_t> bin_off;     // [nbins + 1] bin-major offsets
  std::vector<BinItem> items;       // every bin has at least one item (its rows are written even when empty)
  std::vector<BinSplit> splits;
};

// Push lists: source j sends to idx[off[j] .. off[j+1]) (destination rows in
// [0, n)); shift in [1, 16].  max_src / max_ent / max_acc (at most the
// defaults) bound the sources and entries of a scatter range and the entries
// of an accumulate item.
void build_binned(const int32_t* off, const int32_t* idx, int32_t n, int32_t shift, BinnedLayout& b,
                  int32_t max_src = kBinSrc, int32_t max_ent = kBinEnt, int32_t max_acc = kBinAccEnt);

// Degree-ordered relabelling and the two CSR copies under internal ids.
// keys: edges (src << 32 | dst) in external ids, sorted ascending, distinct
// or not (every key is one edge).
struct HostLayout {
  std::vector<int32_t> din_ext, dout_ext, ext_of, int_of;
  std::vector<int32_t> out_off, out_idx, in_off, in_idx, din_int;
  std::vector<double> inv_din;
};

void build_layout(const std::vector<uint64_t>& keys, int32_t n, HostLayout& h);

}  // namespace es
