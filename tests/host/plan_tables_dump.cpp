// Host-only driver for the plan-table builder (for sanitizer runs): reads a
// chunk description as whitespace-separated integers on stdin
//   nchunks, chunk_base[nchunks], level_stride[nchunks], levels[nchunks],
//   row_start[nchunks + 1], row_offset[nrows], row_len[nrows]
// and prints the tables: a status line, then one line per run
// (block0 nbx nlev nrow lstride rbase0..3 rlen0..3), then the tile -> run
// table and the plan totals.
#include <stdio.h>

#include <vector>

#include "../../paper_2609_24294_amd/csrc/plan_tables.hpp"

template <class T>
static bool read_vec(std::vector<T>& v, size_t n) {
  v.resize(n);
  for (size_t i = 0; i < n; i++) {
    long long x;
    if (scanf("%lld", &x) != 1) return false;
    v[i] = (T)x;
  }
  return true;
}

int main() {
  int nchunks = 0;
  if (scanf("%d", &nchunks) != 1 || nchunks < 0) return 2;
  std::vector<int64_t> base, lstride, roff;
  std::vector<int32_t> levels, rstart, rlen;
  if (!read_vec(base, nchunks) || !read_vec(lstride, nchunks) || !read_vec(levels, nchunks) ||
      !read_vec(rstart, nchunks + 1))
    return 2;
  const size_t nrows = nchunks > 0 ? (size_t)rstart[nchunks] : 0;
  if (!read_vec(roff, nrows) || !read_vec(rlen, nrows)) return 2;
  zfpx::PlanTables t;
  const int st = zfpx::build_plan_tables(nchunks, base.data(), lstride.data(), levels.data(),
                                         rstart.data(), roff.data(), rlen.data(), &t);
  printf("status %d\n", st);
  if (st != 0) return 0;
  printf("runs %zu\n", t.segs.size());
  for (const zfpx::SegDesc& d : t.segs)
    printf("%d %d %d %d %lld %lld %lld %lld %lld %d %d %d %d\n", d.block0, d.nbx, d.nlev, d.nrow,
           (long long)d.lstride, (long long)d.rbase[0], (long long)d.rbase[1],
           (long long)d.rbase[2], (long long)d.rbase[3], d.rlen[0], d.rlen[1], d.rlen[2],
           d.rlen[3]);
  printf("seg_block0");
  for (int32_t b : t.seg_block0) printf(" %d", b);
  printf("\ntile_seg");
  for (int32_t s : t.tile_seg) printf(" %d", s);
  printf("\ntotals %lld %lld %lld %d\n", (long long)t.nblocks, (long long)t.nvalues,
         (long long)t.min_elems, t.vec4 ? 1 : 0);
  return 0;
}
