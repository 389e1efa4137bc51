// internal.hpp -- plan tables and kernel launchers shared by the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "plan_tables.hpp"

namespace zfpx {

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

// 64-block tiles covering n blocks (n up to 2^31 - 1, counted without
// overflowing 32 bits).
__host__ __device__ inline int32_t tiles_of(int32_t n) {
  return (int32_t)(((int64_t)n + 63) >> 6);
}

// Launch configuration: threads per workgroup and persistent grid (0 = one
// 64-block tile per wavefront).
struct LaunchCfg {
  int wg = 128;
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
// Variable-size modes over a whole plan: the encoder's scratch is a staging
// area of var_stage_words 32-bit words plus one count per tile.
size_t var_stage_words(int64_t nblocks, int cap);
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_plan_encode_var(const PlanDev& p, bool vec4, const float* src, uint32_t* out,
                                  uint64_t out_words, uint8_t* nd, int64_t* tile_off,
                                  uint32_t* stage, uint32_t* tile_count, int cap,
                                  int32_t nblocks, int maxprec, int minexp, hipStream_t s);
hipError_t launch_plan_decode_var(const PlanDev& p, bool vec4, const uint32_t* in,
                                  uint64_t in_words, const uint8_t* nd, const int64_t* tile_off,
                                  float* dst, int cap, int32_t nblocks, int maxprec, int minexp,
                                  hipStream_t s);
// Scratch of the allocation-free variable-size encoder: a file-scope device
// array of kNoAllocScratchBytes (kernels.hip), one copy per GPU.  Returns its
// address on the current device (looked up once per device).
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
hipError_t noalloc_scratch(void** ptr);
hipError_t launch_var_chunk_offsets(const int64_t* chunk_first, int32_t nchunks,
                                    const uint8_t* nd, const int64_t* tile_off,
                                    int64_t* chunk_off, hipStream_t s);
hipError_t launch_f16_truncate(const float* in, size_t n, uint16_t* out, hipStream_t s);
hipError_t launch_f16_restore(const uint16_t* in, size_t n, float* out, hipStream_t s);

// ---------------------------------------------------------------------------
// Serving: a request ring shared by the host (writer) and a persistent
// device loop (reader).
// ---------------------------------------------------------------------------
struct ServeDesc {   // one admitted request; host-coherent memory, slot = seq % cap
  uint64_t seq;      // request number
  int32_t op;        // 0 = encode (float32 -> words), 1 = decode
  int32_t rate;
  int32_t nblocks, ntiles;
  uint32_t vspan;     // float32 array span in bytes when it is 16-byte accessible
                      // within 4 GiB (unit x stride, aligned rows), else 0
  int32_t per_claim;  // tiles per wavefront of a workgroup's claim (1..8)
  RegularDev geo;
  uint64_t in, out;  // device addresses
};

struct ServeCtl {        // host-coherent control block
  uint64_t published;    // requests 0 .. published-1 are in the ring
  uint64_t oldest;       // no request older than this has work left (a hint)
  uint32_t stop;         // set by the host to end the device loop
  uint32_t pad;
};

struct ServeDevCtl {     // device-memory mirror written by the dispatcher
  uint64_t published;    // requests copied into ring_dev
  uint64_t stop;         // set once the host asked the loop to stop
  uint64_t oldest;       // a copy of the host's hint; it may lag, never lead
};

struct ServeDev {        // arguments of the device loop
  ServeCtl* ctl;         // device view of the host control block
  const ServeDesc* ring; // device view of the host ring (cap entries)
  uint64_t* done_flag;   // host-coherent, per slot: seq + 1 once complete
  ServeDevCtl* dctl;     // device memory
  ServeDesc* ring_dev;   // device memory copy of the ring
  uint64_t* claim;       // device memory, per slot: (seq << 32) | tiles claimed
  uint64_t* done;        // device memory, per slot: (seq << 32) | tiles done
  int32_t cap;
  int32_t pad;
  uint64_t idle_ticks;   // leave after this long without work (real-time ticks)
  uint64_t max_ticks;    // and in any case after this long
};

hipError_t launch_serve(const ServeDev& d, int workgroups, hipStream_t s);
constexpr int kServeWaves = 8;  // wavefronts per workgroup of the device loop

// LDS bytes a workgroup of `wg` threads needs at `rate`.
size_t lds_bytes(int wg, int rate);
// Largest LDS per workgroup of the current device (cached).
size_t device_max_lds();
int device_cu_count();

}  // namespace zfpx
