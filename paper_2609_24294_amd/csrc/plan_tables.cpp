// plan_tables.cpp -- host-side construction of a chunk plan's run tables.
#include "plan_tables.hpp"

#include <algorithm>

namespace zfpx {

namespace {
int64_t ceil4(int64_t n) { return (n + 3) / 4; }
}  // namespace

int build_plan_tables(int32_t nchunks, const int64_t* chunk_base, const int64_t* level_stride,
                      const int32_t* levels, const int32_t* row_start, const int64_t* row_offset,
                      const int32_t* row_len, PlanTables* t) {
  constexpr int kInvalid = -1;
  if (!t || nchunks < 0) return kInvalid;
  if (nchunks > 0 && (!chunk_base || !level_stride || !levels || !row_start)) return kInvalid;
  if (nchunks > 0 && row_start[0] != 0) return kInvalid;
  for (int c = 0; c < nchunks; c++) {
    if (row_start[c + 1] < row_start[c] || levels[c] < 0 || level_stride[c] < 0 ||
        chunk_base[c] < 0)
      return kInvalid;
  }
  const int64_t nrows_total = nchunks > 0 ? row_start[nchunks] : 0;
  if (nrows_total > 0 && (!row_offset || !row_len)) return kInvalid;
  for (int64_t r = 0; r < nrows_total; r++)
    if (row_len[r] < 1 || row_offset[r] < 0) return kInvalid;

  *t = PlanTables{};
  t->chunk_blocks.assign(nchunks, 0);
  t->chunk_first.assign((size_t)nchunks + 1, 0);
  std::vector<SegDesc>& segs = t->segs;
  int64_t total = 0, values = 0, min_elems = 0;
  bool vec4 = true;
  for (int c = 0; c < nchunks; c++) {
    const int64_t r0 = row_start[c], nrows = row_start[c + 1] - r0, L = levels[c];
    const int64_t ngroups = ceil4(nrows);
    std::vector<int64_t> width(ngroups, 0);
    for (int64_t g = 0; g < ngroups; g++)
      for (int64_t r = 4 * g; r < std::min(4 * g + 4, nrows); r++)
        width[g] = std::max<int64_t>(width[g], row_len[r0 + r]);
    int64_t per_lb = 0;
    for (int64_t g = 0; g < ngroups; g++) per_lb += ceil4(width[g]);
    const int64_t cb = (L > 0 && nrows > 0) ? ceil4(L) * per_lb : 0;
    t->chunk_first[c] = total;
    t->chunk_blocks[c] = cb;
    if (total + cb > kMaxPlanBlocks) return kInvalid;
    if (cb > 0) {
      if ((level_stride[c] & 3) != 0 || (chunk_base[c] & 3) != 0) vec4 = false;
      for (int64_t r = r0; r < r0 + nrows; r++) {
        if ((row_offset[r] & 3) != 0) vec4 = false;
        values += L * row_len[r];
        min_elems = std::max(min_elems, chunk_base[c] + (L - 1) * level_stride[c] + row_offset[r] +
                                            row_len[r]);
      }
      int64_t run = total;  // block0 of each run: running sum in run order
      for (int64_t bz = 0; bz < ceil4(L); bz++) {
        for (int64_t g = 0; g < ngroups; g++) {
          SegDesc d{};
          for (int dy = 0; dy < 4; dy++) {
            const int64_t r = r0 + std::min<int64_t>(4 * g + dy, nrows - 1);
            d.rbase[dy] = chunk_base[c] + 4 * bz * level_stride[c] + row_offset[r];
            d.rlen[dy] = row_len[r];
          }
          d.lstride = level_stride[c];
          d.block0 = (int32_t)run;
          d.nbx = (int32_t)ceil4(width[g]);
          d.nlev = (int32_t)std::min<int64_t>(4, L - 4 * bz);
          d.nrow = (int32_t)std::min<int64_t>(4, nrows - 4 * g);
          segs.push_back(d);
          run += d.nbx;
        }
      }
    }
    total += cb;
  }
  t->chunk_first[nchunks] = total;
  t->nblocks = total;
  t->nvalues = values;
  t->min_elems = min_elems;
  t->vec4 = vec4;

  // run starts and the tile -> run table
  t->seg_block0.resize(segs.size() + 1);
  for (size_t i = 0; i < segs.size(); i++) t->seg_block0[i] = segs[i].block0;
  t->seg_block0[segs.size()] = (int32_t)total;
  const int64_t ntiles = (total + 63) / 64;
  t->tile_seg.assign((size_t)std::max<int64_t>(ntiles, 1), 0);
  size_t s = 0;
  for (int64_t tl = 0; tl < ntiles; tl++) {
    const int64_t b = 64 * tl;
    while (s + 1 < segs.size() && t->seg_block0[s + 1] <= b) s++;
    t->tile_seg[tl] = (int32_t)s;
  }
  return 0;
}

}  // namespace zfpx
