// internal.hpp -- plan tables and kernel launchers shared by the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
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

// Device-side view of a plan.
struct PlanDev {
  const SegDesc* segs;
  const int32_t* seg_block0;  // [nseg + 1], last entry = total blocks
  const int32_t* tile_seg;    // [ntiles]: run holding block 64 * t
};

// Regular strided array as a geometry.
struct RegularDev {
  int64_t nx, ny, nz;
  int64_t sx, sy, sz;
  int32_t nbx, nby;
};

// Launch configuration: threads per workgroup and persistent grid (0 = one
// 64-block tile per wavefront).
struct LaunchCfg {
  int wg = 256;
  int grid = 0;
};

constexpr int kOpEncode = 0;
constexpr int kOpDecode = 1;

// Launchers (kernels.hip).  Blocks [b_begin, b_end) of the geometry.
hipError_t launch_plan_encode(const PlanDev& p, bool vec4, const float* src, uint64_t* out,
                              int rate, int32_t b_begin, int32_t b_end, LaunchCfg cfg,
                              hipStream_t s);
hipError_t launch_plan_decode(const PlanDev& p, bool vec4, const uint64_t* in, float* dst,
                              int rate, int32_t b_begin, int32_t b_end, LaunchCfg cfg,
                              hipStream_t s);
hipError_t launch_regular_encode(const RegularDev& g, bool vec4, const float* src,
                                 uint64_t* out, int rate, int32_t nblocks, LaunchCfg cfg,
                                 hipStream_t s);
hipError_t launch_regular_decode(const RegularDev& g, bool vec4, const uint64_t* in, float* dst,
                                 int rate, int32_t nblocks, LaunchCfg cfg, hipStream_t s);
hipError_t launch_f16_truncate(const float* in, size_t n, uint16_t* out, hipStream_t s);
hipError_t launch_f16_restore(const uint16_t* in, size_t n, float* out, hipStream_t s);

// LDS bytes a workgroup of `wg` threads needs at `rate`.
size_t lds_bytes(int wg, int rate);
// Largest LDS per workgroup of the current device (cached).
size_t device_max_lds();
int device_cu_count();

}  // namespace zfpx
