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
