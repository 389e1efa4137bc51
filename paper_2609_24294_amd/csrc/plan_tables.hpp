// plan_tables.hpp -- host-side construction of a chunk plan's run tables
// (plain C++, no HIP: also built on its own for host sanitizer runs).
//
// A plan covers chunks laid out as in the paper's transpositions (Section
// II-B: every rank sends a sub-array to every other rank): chunk c has
// levels[c] levels at chunk_base[c] + z * level_stride[c], and rows
// row_start[c] .. row_start[c+1]-1, row r at further offset row_offset[r]
// with row_len[r] contiguous points.  Rows are taken in fours (row groups,
// as wide as their longest row) and each chunk is coded as its own array of
// 4x4x4 blocks, numbered by level block, then row group, then x block.
#pragma once

#include <stdint.h>

#include <vector>

namespace zfpx {

// One run of x-blocks: (chunk, level block, row group).  Each lane finds the
// run holding its block and gathers/scatters its 4x4x4 values through it.
struct SegDesc {
  int64_t rbase[4];  // element offset of row (4g+dy, clamped) at level 4*bz
  int64_t lstride;   // elements between levels
  int32_t block0;    // first global block id of the run
  int32_t nbx;       // x blocks in the run
  int32_t nlev;      // levels present in this level block (1..4)
  int32_t nrow;      // rows present in this row group (1..4)
  int32_t rlen[4];   // row lengths (missing rows repeat the last row)
};

// Largest number of blocks a plan may hold (block ids are int32).
constexpr int64_t kMaxPlanBlocks = 0x7fffffffLL;

struct PlanTables {
  std::vector<SegDesc> segs;          // runs in block order
  std::vector<int32_t> seg_block0;    // [nseg + 1]: first block of each run, then the total
  std::vector<int32_t> tile_seg;      // [max(ntiles, 1)]: run holding block 64 t
  std::vector<int64_t> chunk_blocks;  // [nchunks]
  std::vector<int64_t> chunk_first;   // [nchunks + 1]: first block of each chunk, then the total
  int64_t nblocks = 0;                // blocks in all chunks
  int64_t nvalues = 0;                // real (unpadded) values in all chunks
  int64_t min_elems = 0;              // smallest buffer (elements) every chunk fits in
  bool vec4 = true;                   // every chunk row starts 16-byte aligned in a 16-byte
                                      // aligned buffer
};

// Checks the chunk description and builds its tables.  Returns 0, or -1
// (invalid argument: negative counts, offsets or strides, rows of fewer than
// one point, row_start not starting at 0 or decreasing, more than
// kMaxPlanBlocks blocks).
int build_plan_tables(int32_t nchunks, const int64_t* chunk_base, const int64_t* level_stride,
                      const int32_t* levels, const int32_t* row_start, const int64_t* row_offset,
                      const int32_t* row_len, PlanTables* t);

}  // namespace zfpx
