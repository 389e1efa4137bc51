// kernels.hip -- HIP kernels for gfx950: fused gather + encode, decode +
// scatter, and the float16 comparator.
//
// Mapping.  One 4x4x4 block per lane; one wavefront handles a tile of 64
// consecutive blocks (consecutive x blocks of a row group, so the 16 row
// segments a lane reads are contiguous 16-byte pieces and a wavefront's loads
// of one row are one contiguous 1 KiB stretch).  The coded words of a tile are
// contiguous in the output, so each lane codes into its own slice of LDS
// (stride rate|1 words to spread the banks) and the wavefront then copies the
// tile out (or in, for decoding) with coalesced 8-byte accesses.  Workgroups
// loop over tiles with a grid stride, so the same kernel serves as a
// one-tile-per-wave launch and as a persistent launch.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>

#include "block_codec.hpp"
#include "internal.hpp"

namespace zfpx {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Block location
// ---------------------------------------------------------------------------

struct BlockView {
  int64_t rbase[4];
  int64_t lstride;
  int64_t sx;
  int32_t nlev, nrow;
  int32_t rlen[4];
  int32_t x0;  // first x of the block
};

// Loads through the constant address space: with a wave-uniform address they
// become scalar loads (no per-lane round trip).
template <class T>
__device__ __forceinline__ T uniform_load(const T* p, int64_t i) {
  return ((const __attribute__((address_space(4))) T*)p)[i];
}

// A tile whose 64 blocks all lie in one run: everything but the x offset is
// wave-uniform (scalar registers), so whole blocks load through a scalar row
// base plus a per-lane offset.
struct RunView {
  int64_t rbase[4];
  int64_t lstride;
  int32_t nlev, nrow, block0;
  int32_t minlen;  // shortest row of the group
  int32_t rlen[4];
};

struct PlanGeo {
  PlanDev p;
  // True (the same on every lane) when blocks b0 .. b0 + nact - 1 lie in one
  // run; r then describes it.
  __device__ __forceinline__ bool one_run(int32_t b0, int nact, RunView& r) const {
    int32_t s = uniform_load(p.tile_seg, b0 >> 6);
    while (uniform_load(p.seg_block0, s + 1) <= b0) s++;
    if (uniform_load(p.seg_block0, s + 1) <= b0 + nact - 1) return false;
    const SegDesc* d = p.segs + s;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      r.rbase[i] = uniform_load(&d->rbase[i], 0);
      r.rlen[i] = uniform_load(&d->rlen[i], 0);
    }
    r.lstride = uniform_load(&d->lstride, 0);
    r.nlev = uniform_load(&d->nlev, 0);
    r.nrow = uniform_load(&d->nrow, 0);
    r.block0 = uniform_load(&d->block0, 0);
    r.minlen = min(min(r.rlen[0], r.rlen[1]), min(r.rlen[2], r.rlen[3]));
    return true;
  }
  // Any block: find its run from the run table.
  __device__ __forceinline__ void locate(int32_t b, BlockView& v) const {
    int32_t s = p.tile_seg[b >> 6];
    while (p.seg_block0[s + 1] <= b) s++;
    const SegDesc& d = p.segs[s];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      v.rbase[i] = d.rbase[i];
      v.rlen[i] = d.rlen[i];
    }
    v.lstride = d.lstride;
    v.sx = 1;
    v.nlev = d.nlev;
    v.nrow = d.nrow;
    v.x0 = 4 * (b - d.block0);
  }
  // Block b0 + lane of a tile whose first block b0 is the same on every lane
  // and whose last active block is b0 + nact - 1.  A tile that meets at most
  // two runs reads both descriptors with scalar loads and each lane picks
  // its own; other tiles look every block up.
  __device__ __forceinline__ void locate_tile(int32_t b0, int lane, int nact,
                                              BlockView& v) const {
    int32_t s = uniform_load(p.tile_seg, b0 >> 6);
    while (uniform_load(p.seg_block0, s + 1) <= b0) s++;
    const int32_t last = b0 + nact - 1;
    const int32_t e1 = uniform_load(p.seg_block0, s + 1);
    // e1 <= last < total blocks, so run s + 1 exists and so does entry s + 2
    if (e1 <= last && uniform_load(p.seg_block0, s + 2) <= last) {
      locate(b0 + lane, v);
      return;
    }
    const int32_t b = b0 + lane;
    const int32_t s1 = e1 <= last ? s + 1 : s;
    const bool second = b >= e1;
    const SegDesc* d0 = p.segs + s;
    const SegDesc* d1 = p.segs + s1;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int64_t r0 = uniform_load(&d0->rbase[i], 0), r1 = uniform_load(&d1->rbase[i], 0);
      const int32_t l0 = uniform_load(&d0->rlen[i], 0), l1 = uniform_load(&d1->rlen[i], 0);
      v.rbase[i] = second ? r1 : r0;
      v.rlen[i] = second ? l1 : l0;
    }
    const int64_t ls0 = uniform_load(&d0->lstride, 0), ls1 = uniform_load(&d1->lstride, 0);
    const int32_t nl0 = uniform_load(&d0->nlev, 0), nl1 = uniform_load(&d1->nlev, 0);
    const int32_t nr0 = uniform_load(&d0->nrow, 0), nr1 = uniform_load(&d1->nrow, 0);
    const int32_t bb0 = uniform_load(&d0->block0, 0), bb1 = uniform_load(&d1->block0, 0);
    v.lstride = second ? ls1 : ls0;
    v.sx = 1;
    v.nlev = second ? nl1 : nl0;
    v.nrow = second ? nr1 : nr0;
    v.x0 = 4 * (b - (second ? bb1 : bb0));
  }
};

struct RegularGeo {
  RegularDev g;
  __device__ __forceinline__ void locate(int32_t b, BlockView& v) const {
    uint32_t ub = (uint32_t)b;
    uint32_t t = ub / (uint32_t)g.nbx;
    uint32_t bx = ub - t * (uint32_t)g.nbx;
    uint32_t bz = t / (uint32_t)g.nby;
    uint32_t by = t - bz * (uint32_t)g.nby;
    int64_t y0 = 4 * (int64_t)by, z0 = 4 * (int64_t)bz;
    int64_t zoff = z0 * g.sz;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      int64_t y = y0 + i < g.ny ? y0 + i : g.ny - 1;
      v.rbase[i] = zoff + y * g.sy;
      v.rlen[i] = (int32_t)g.nx;
    }
    v.lstride = g.sz;
    v.sx = g.sx;
    v.nlev = (int32_t)(g.nz - z0 < 4 ? g.nz - z0 : 4);
    v.nrow = (int32_t)(g.ny - y0 < 4 ? g.ny - y0 : 4);
    v.x0 = (int32_t)(4 * bx);
  }
  __device__ __forceinline__ void locate_tile(int32_t b0, int lane, int, BlockView& v) const {
    locate(b0 + lane, v);
  }
  __device__ __forceinline__ bool one_run(int32_t, int, RunView&) const { return false; }
};

// COH: system-coherent element accesses that bypass the (per-XCD) L2, used by
// the serving loop so that no cache write-back is needed between requests.
__device__ __forceinline__ float coh_load(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void coh_store(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// System-coherent 16-byte accesses for the serving loop, through a buffer
// resource over the request's array (base and size wave-uniform): loads miss
// the per-XCD L2 and stores write through to memory (scope bits sc0 sc1), so
// no cache invalidation or write-back is needed between requests.  Offsets
// past the resource read zero and drop stores.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kSystemScope = 1 | 16;  // sc0 | sc1
__device__ __forceinline__ __amdgpu_buffer_rsrc_t coh_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}

// A whole block: 4 levels and 4 rows present, its 4 points inside every row,
// unit x stride.
__device__ __forceinline__ bool whole_block(const BlockView& v) {
  int len = min(min(v.rlen[0], v.rlen[1]), min(v.rlen[2], v.rlen[3]));
  return v.nlev == 4 && v.nrow == 4 && v.sx == 1 && v.x0 + 3 < len;
}

// Gather the 64 values of a block.  A whole block takes sixteen 16-byte
// loads with no branch between them, so that all of them are in flight at
// once; any other block loads every element from its clamped position
// (repeating the last level, row or point), also without branches.
template <bool VEC4, bool COH = false>
__device__ __forceinline__ void gather(const float* __restrict__ src, const BlockView& v,
                                       float* val, uint32_t vspan = 0) {
  if (COH && vspan != 0 && whole_block(v)) {
    const __amdgpu_buffer_rsrc_t rs = coh_rsrc(src, vspan);
#pragma unroll
    for (int dz = 0; dz < 4; dz++) {
#pragma unroll
      for (int dy = 0; dy < 4; dy++) {
        const uint32_t off = (uint32_t)(4 * (v.rbase[dy] + dz * v.lstride + v.x0));
        f32x4 f = __builtin_bit_cast(
            f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kSystemScope));
        float* o = val + 16 * dz + 4 * dy;
        o[0] = f.x;
        o[1] = f.y;
        o[2] = f.z;
        o[3] = f.w;
      }
    }
    return;
  }
  if (VEC4 && !COH && whole_block(v)) {
#pragma unroll
    for (int dz = 0; dz < 4; dz++) {
#pragma unroll
      for (int dy = 0; dy < 4; dy++) {
        f32x4 f = *reinterpret_cast<const f32x4*>(src + v.rbase[dy] + dz * v.lstride + v.x0);
        float* o = val + 16 * dz + 4 * dy;
        o[0] = f.x;
        o[1] = f.y;
        o[2] = f.z;
        o[3] = f.w;
      }
    }
    return;
  }
#pragma unroll
  for (int dz = 0; dz < 4; dz++) {
    int64_t zoff = (int64_t)(dz < v.nlev ? dz : v.nlev - 1) * v.lstride;
#pragma unroll
    for (int dy = 0; dy < 4; dy++) {
      int64_t base = v.rbase[dy] + zoff;
      int len = v.rlen[dy];
      float* o = val + 16 * dz + 4 * dy;
#pragma unroll
      for (int dx = 0; dx < 4; dx++) {
        int x = v.x0 + dx < len ? v.x0 + dx : len - 1;
        o[dx] = COH ? coh_load(src + base + (int64_t)x * v.sx) : src[base + (int64_t)x * v.sx];
      }
    }
  }
}

// NT: whole blocks are stored with the non-temporal hint.
template <bool VEC4, bool COH = false, bool NT = false>
__device__ __forceinline__ void scatter(float* __restrict__ dst, const BlockView& v,
                                        const float* val, uint32_t vspan = 0) {
  if (COH && vspan != 0 && whole_block(v)) {
    const __amdgpu_buffer_rsrc_t rs = coh_rsrc(dst, vspan);
#pragma unroll
    for (int dz = 0; dz < 4; dz++) {
#pragma unroll
      for (int dy = 0; dy < 4; dy++) {
        const float* o = val + 16 * dz + 4 * dy;
        f32x4 f = {o[0], o[1], o[2], o[3]};
        const uint32_t off = (uint32_t)(4 * (v.rbase[dy] + dz * v.lstride + v.x0));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, f), rs, (int)off, 0,
                                               kSystemScope);
      }
    }
    return;
  }
  if (VEC4 && !COH && whole_block(v)) {
#pragma unroll
    for (int dz = 0; dz < 4; dz++) {
#pragma unroll
      for (int dy = 0; dy < 4; dy++) {
        const float* o = val + 16 * dz + 4 * dy;
        f32x4 f = {o[0], o[1], o[2], o[3]};
        f32x4* q = reinterpret_cast<f32x4*>(dst + v.rbase[dy] + dz * v.lstride + v.x0);
        if (NT)
          __builtin_nontemporal_store(f, q);
        else
          *q = f;
      }
    }
    return;
  }
#pragma unroll
  for (int dz = 0; dz < 4; dz++) {
    if (dz < v.nlev) {
      int64_t zoff = (int64_t)dz * v.lstride;
#pragma unroll
      for (int dy = 0; dy < 4; dy++) {
        if (dy < v.nrow) {
          int64_t base = v.rbase[dy] + zoff;
          int len = v.rlen[dy];
          const float* o = val + 16 * dz + 4 * dy;
          if (VEC4 && !COH && v.x0 + 3 < len) {
            f32x4 f = {o[0], o[1], o[2], o[3]};
            *reinterpret_cast<f32x4*>(dst + base + v.x0) = f;
          } else {
#pragma unroll
            for (int dx = 0; dx < 4; dx++)
              if (v.x0 + dx < len) {
                if (COH)
                  coh_store(dst + base + (int64_t)(v.x0 + dx) * v.sx, o[dx]);
                else
                  dst[base + (int64_t)(v.x0 + dx) * v.sx] = o[dx];
              }
          }
        }
      }
    }
  }
}

// Block b of a one-run tile: whole blocks load sixteen 16-byte pieces at a
// scalar row address plus the lane's x offset; others take the clamped
// element path of gather().
template <bool VEC4>
__device__ __forceinline__ void gather_run(const float* __restrict__ src, const RunView& r,
                                           int32_t b, float* val) {
  const int32_t x0 = 4 * (b - r.block0);
  if (VEC4 && r.nlev == 4 && r.nrow == 4 && x0 + 3 < r.minlen) {
#pragma unroll
    for (int dz = 0; dz < 4; dz++) {
#pragma unroll
      for (int dy = 0; dy < 4; dy++) {
        const float* row = src + (r.rbase[dy] + dz * r.lstride);
        // read once: a streaming (non-temporal) load
        f32x4 f = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(row + (uint32_t)x0));
        float* o = val + 16 * dz + 4 * dy;
        o[0] = f.x;
        o[1] = f.y;
        o[2] = f.z;
        o[3] = f.w;
      }
    }
    return;
  }
  BlockView v;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    v.rbase[i] = r.rbase[i];
    v.rlen[i] = r.rlen[i];
  }
  v.lstride = r.lstride;
  v.sx = 1;
  v.nlev = r.nlev;
  v.nrow = r.nrow;
  v.x0 = x0;
  gather<false>(src, v, val);
}

template <bool VEC4>
__device__ __forceinline__ void scatter_run(float* __restrict__ dst, const RunView& r, int32_t b,
                                            const float* val) {
  const int32_t x0 = 4 * (b - r.block0);
  if (VEC4 && r.nlev == 4 && r.nrow == 4 && x0 + 3 < r.minlen) {
#pragma unroll
    for (int dz = 0; dz < 4; dz++) {
#pragma unroll
      for (int dy = 0; dy < 4; dy++) {
        float* row = dst + (r.rbase[dy] + dz * r.lstride);
        const float* o = val + 16 * dz + 4 * dy;
        f32x4 f = {o[0], o[1], o[2], o[3]};
        *reinterpret_cast<f32x4*>(row + (uint32_t)x0) = f;
      }
    }
    return;
  }
  BlockView v;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    v.rbase[i] = r.rbase[i];
    v.rlen[i] = r.rlen[i];
  }
  v.lstride = r.lstride;
  v.sx = 1;
  v.nlev = r.nlev;
  v.nrow = r.nrow;
  v.x0 = x0;
  scatter<VEC4>(dst, v, val);
}

// Make loaded values available at this point (an empty asm that reads and
// writes them): the loads are then all issued before the first wait, instead
// of one round trip each behind the guards of their uses.
__device__ __forceinline__ void pin_words64(uint64_t (&v)[4]) {
  asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
}
__device__ __forceinline__ void pin_words32(uint32_t (&v)[4]) {
  asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
}
__device__ __forceinline__ void pin_words32(uint32_t (&v)[8]) {
  asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),
               "+v"(v[6]), "+v"(v[7]));
}

// Copy a tile's coded words between LDS slices (stride words per block) and
// global memory (rate words per block, contiguous).  For rates dividing 64,
// lane l always handles word l % rate of every (64/rate)-th block, so the
// addresses are a per-lane base plus compile-time offsets.
template <bool COH>
__device__ __forceinline__ void gstore64(uint64_t* p, uint64_t v) {
  if (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  else
    __builtin_nontemporal_store(v, p);  // written once: streaming
}
template <bool COH>
__device__ __forceinline__ uint64_t gload64(const uint64_t* p) {
  if (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  return *p;
}

template <int RATE, bool TO_GLOBAL, bool COH = false>
__device__ __forceinline__ void copy_tile(uint64_t* __restrict__ g, uint64_t* lds, int lane,
                                          int nact, int rate_rt) {
  if constexpr (RATE > 0 && 64 % RATE == 0) {
    constexpr int stride = (RATE + kSlackWords) | 1;
    constexpr int step = 64 / RATE;  // blocks per row of 64 words
    const int b = lane / RATE, idx = lane % RATE;
    uint64_t* l = lds + b * stride + idx;
    if (nact == 64) {
      // A whole tile (nact is wave-uniform): every read is issued before any
      // is waited for, one round trip in all (behind per-word guards the
      // compiler waits for each word before the next).
      uint64_t v[RATE];
      if (TO_GLOBAL) {
#pragma unroll
        for (int j = 0; j < RATE; j++) v[j] = l[j * step * stride];
#pragma unroll
        for (int j = 0; j < RATE; j++) gstore64<COH>(g + lane + 64 * j, v[j]);
      } else {
#pragma unroll
        for (int j = 0; j < RATE; j++) v[j] = gload64<COH>(g + lane + 64 * j);
#pragma unroll
        for (int j = 0; j < RATE; j++) l[j * step * stride] = v[j];
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < RATE; j++) {
      if (b + j * step < nact) {
        if (TO_GLOBAL)
          gstore64<COH>(g + lane + 64 * j, l[j * step * stride]);
        else
          l[j * step * stride] = gload64<COH>(g + lane + 64 * j);
      }
    }
  } else {
    const int rate = RATE > 0 ? RATE : rate_rt;
    const int stride = (rate + kSlackWords) | 1;
    const int nw = nact * rate;
    // four words per lane per round, all read before any is waited for
    // (reads past the end repeat word 0 and are not stored)
    for (int w0 = lane; w0 < nw; w0 += 256) {
      uint64_t v[4];
      int at[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int w = w0 + 64 * j < nw ? w0 + 64 * j : 0;
        const int blk = w / rate;
        at[j] = blk * stride + (w - blk * rate);
        v[j] = TO_GLOBAL ? lds[at[j]] : gload64<COH>(g + w);
      }
      pin_words64(v);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int w = w0 + 64 * j;
        if (w < nw) {
          if (TO_GLOBAL)
            gstore64<COH>(g + w, v[j]);
          else
            lds[at[j]] = v[j];
        }
      }
    }
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Words per lane slice: the stream plus zero slack, odd to spread LDS banks.
__host__ __device__ constexpr int lds_stride(int rate) { return (rate + kSlackWords) | 1; }

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Returns x unchanged but hides its value from the optimiser, so that work
// derived from it is not hoisted out of the tile loop (which would hold that
// work in registers for the whole kernel and cut occupancy).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// One 64-block tile: gather + encode into the lane slices, then copy the
// tile's words out (encode), or copy in + decode + scatter (decode).
template <int RATE, bool VEC4, bool COH = false, class Geo>
__device__ __forceinline__ void encode_tile(const Geo& geo, const float* __restrict__ src,
                                            uint64_t* __restrict__ out, int rate, int lane,
                                            uint64_t* wlds, int32_t b0, int nact,
                                            uint32_t vspan = 0) {
  const int stride = lds_stride(RATE > 0 ? RATE : rate);
  uint64_t* slice = wlds + lane * stride;
  for (int i = 0; i < stride; i++) slice[i] = 0;
  RunView run;
  const bool uniform = !COH && geo.one_run(b0, nact, run);
  if (lane < nact) {
    float val[64];
    if (uniform) {
      gather_run<VEC4>(src, run, b0 + lane, val);
    } else {
      BlockView v;
      geo.locate_tile(b0, lane, nact, v);
      gather<VEC4, COH>(src, v, val, vspan);
    }
    encode_block<RATE>(val, slice, rate);
  }
  wave_sync_lds();
  copy_tile<RATE, true, COH>(out + (int64_t)b0 * rate, wlds, opaque(lane), nact, rate);
}

template <int RATE, bool VEC4, bool COH = false, class Geo>
__device__ __forceinline__ void decode_tile(const Geo& geo, const uint64_t* __restrict__ in,
                                            float* __restrict__ dst, int rate, int lane,
                                            uint64_t* wlds, int32_t b0, int nact,
                                            uint32_t vspan = 0) {
  const int stride = lds_stride(RATE > 0 ? RATE : rate);
  for (int i = (RATE > 0 ? RATE : rate); i < stride; i++) wlds[lane * stride + i] = 0;
  copy_tile<RATE, false, COH>(const_cast<uint64_t*>(in) + (int64_t)b0 * rate, wlds, lane, nact,
                              rate);
  wave_sync_lds();
  if (lane < nact) {
    float val[64];
    decode_block<RATE>(wlds + opaque(lane) * stride, val, rate);
    RunView run;
    if (!COH && geo.one_run(b0, nact, run)) {
      scatter_run<VEC4>(dst, run, b0 + lane, val);
    } else {
      BlockView v;
      geo.locate_tile(b0, lane, nact, v);
      scatter<VEC4, COH>(dst, v, val, vspan);
    }
  }
}

// Workgroups cover the tiles of blocks [b_begin, b_end): one tile per
// wavefront, or (PERSIST) a grid-stride loop over tiles.
template <int RATE, bool VEC4, bool PERSIST, class Geo>
__global__ __launch_bounds__(256) void k_encode(Geo geo, const float* __restrict__ src,
                                                uint64_t* __restrict__ out, int rate_rt,
                                                int32_t b_begin, int32_t b_end) {
  extern __shared__ uint64_t lds[];
  const int rate = RATE > 0 ? RATE : rate_rt;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int waves = blockDim.x >> 6;
  uint64_t* wlds = lds + (size_t)wave * 64 * lds_stride(rate);
  const int32_t ntiles = tiles_of(b_end - b_begin);
  int32_t t = blockIdx.x * waves + wave;
  if (t >= ntiles) return;
  for (;;) {
    const int32_t b0 = b_begin + (t << 6);
    const int nact = b_end - b0 < 64 ? b_end - b0 : 64;
    encode_tile<RATE, VEC4>(geo, src, out, rate, opaque(lane), wlds, b0, nact);
    if (!PERSIST) break;
    t += gridDim.x * waves;
    if (t >= ntiles) break;
    wave_sync_lds();
  }
}

// Workgroup i runs on XCD i % 8 (dispatch is round-robin over the XCDs).
// Renumbered in groups of 64, each XCD takes 8 consecutive workgroups of a
// group: neighbouring tiles, which share the cache lines at their ends, then
// mostly meet in one L2 (merged there instead of written back in parts from
// two), while all XCDs stay in one region of the buffer.  A partial last
// group keeps its order.  A bijection on [0, n).
__device__ __forceinline__ int32_t xcd_grouped(uint32_t i, uint32_t n) {
  constexpr uint32_t kXcds = 8, kRun = 8, kGroup = kXcds * kRun;
  if (i >= n / kGroup * kGroup) return (int32_t)i;
  const uint32_t x = i % kXcds, k = i / kXcds;
  return (int32_t)((k / kRun) * kGroup + x * kRun + k % kRun);
}

// The decoder's time is that of its writes (16 rows of 1 KB per tile): a
// fourth wavefront per SIMD pays for the few registers it spills (three per
// SIMD are slower), and its tiles are taken in XCD-grouped order, so that the
// cache lines shared by neighbouring tiles are merged in one L2 rather than
// written back in parts from two (the encoder, bound by instruction issue,
// gains nothing from the order).
template <int RATE, bool VEC4, bool PERSIST, class Geo>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_decode(Geo geo, const uint64_t* __restrict__ in,
                                                float* __restrict__ dst, int rate_rt,
                                                int32_t b_begin, int32_t b_end) {
  extern __shared__ uint64_t lds[];
  const int rate = RATE > 0 ? RATE : rate_rt;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int waves = blockDim.x >> 6;
  uint64_t* wlds = lds + (size_t)wave * 64 * lds_stride(rate);
  const int32_t ntiles = tiles_of(b_end - b_begin);
  int32_t t = (PERSIST ? (int32_t)blockIdx.x : xcd_grouped(blockIdx.x, gridDim.x)) * waves + wave;
  if (t >= ntiles) return;
  for (;;) {
    const int32_t b0 = b_begin + (t << 6);
    const int nact = b_end - b0 < 64 ? b_end - b0 : 64;
    decode_tile<RATE, VEC4>(geo, in, dst, rate, opaque(lane), wlds, b0, nact);
    if (!PERSIST) break;
    t += gridDim.x * waves;
    if (t >= ntiles) break;
    wave_sync_lds();
  }
}


// ---------------------------------------------------------------------------
// Variable-size modes (fixed precision, fixed accuracy)
// ---------------------------------------------------------------------------
// Block b takes nd[b] = ceil(bits / 32) 32-bit words at word offset
// nd[0] + ... + nd[b-1].  A tile's offset depends on every earlier tile's
// size, so encoding runs in stages that never wait on each other's progress:
// (1) each wavefront codes its 64-block tile as in fixed rate and writes the
// tile's words, compacted, to its own staging slot of 64 * 2 * cap words,
// plus the per-block counts and the tile's count; (2) a chunked scan (three
// short launches) turns the tile counts into tile offsets; (3) each wavefront
// copies its tile's words from the staging slot to the tile's offset.  The words, which
// are the bulk of the traffic, are stored as contiguous 256-byte stretches
// per wavefront instruction in both (1) and (3).

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

template <int CAP, bool VEC4, class Geo>
__global__ __launch_bounds__(256) void k_encode_var(Geo geo, const float* __restrict__ src,
                                                    uint32_t* __restrict__ stage,
                                                    uint32_t* __restrict__ tile_count,
                                                    uint8_t* __restrict__ nd_out, int cap_rt,
                                                    int32_t nblocks, int maxprec, int minexp) {
  extern __shared__ uint64_t lds[];
  const int cap = CAP > 0 ? CAP : cap_rt;
  const int stride = lds_stride(cap);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int waves = blockDim.x >> 6;
  uint64_t* wlds = lds + (size_t)wave * 64 * stride;
  uint64_t* slice = wlds + lane * stride;
  const int32_t ntiles = tiles_of(nblocks);
  const int32_t t = blockIdx.x * waves + wave;
  if (t >= ntiles) return;
  const int32_t b0 = t << 6;
  const int nact = nblocks - b0 < 64 ? nblocks - b0 : 64;
  for (int i = 0; i < stride; i++) slice[i] = 0;
  uint32_t bits = 0;
  if (lane < nact) {
    BlockView v;
    geo.locate_tile(b0, lane, nact, v);
    float val[64];
    gather<VEC4>(src, v, val);
    bits = encode_block<CAP>(val, slice, cap, maxprec, minexp);
  }
  const uint32_t nd = (bits + 31) >> 5;
  if (lane < nact) nd_out[b0 + lane] = (uint8_t)nd;
  const uint32_t excl = wave_incl_scan(nd, lane) - nd;
  const uint32_t count = __builtin_amdgcn_readlane(excl + nd, 63);
  if (lane == 0) tile_count[t] = count;
  wave_sync_lds();
  // word q of the tile belongs to the last block whose first word is <= q
  // (blocks have at least one word; lanes past the tile start at `count`)
  const uint32_t* w32 = reinterpret_cast<const uint32_t*>(wlds);
  uint32_t* out = stage + (size_t)t * 64 * 2 * cap;
  for (uint32_t q0 = 0; q0 < count; q0 += 64) {
    const uint32_t q = q0 + lane;
    int lo = 0;
    uint32_t elo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      const uint32_t e = __shfl(excl, lo + step, 64);
      if (e <= q) {
        lo += step;
        elo = e;
      }
    }
    if (q < count) out[q] = w32[(uint32_t)lo * 2 * stride + (q - elo)];
  }
}

// Tile offsets = exclusive prefix sum of the tile counts, in three launches
// over chunks of kScanChunk counts (8 per thread of a 1024-thread group):
// (1) each chunk's sum, parked in tile_off at the chunk's first position;
// (2) one group scans the chunk sums in place into chunk bases and writes the
// total at tile_off[ntiles]; (3) each chunk reads its base, then scans its
// counts into tile_off.  Each launch reads and writes only positions the
// previous one left ready, so no launch waits on another's progress.
constexpr int kScanPer = 8, kScanChunk = 1024 * kScanPer;

// Load chunk c's counts (zero past ntiles) and return this thread's eight
// consecutive counts and their sum, with the group's exclusive prefix of sums
// before this thread in *before and the chunk total in *total.
__device__ __forceinline__ void scan_chunk_counts(const uint32_t* __restrict__ tile_count,
                                                  int32_t ntiles, int64_t base, uint32_t* buf,
                                                  uint32_t* wtot, uint32_t v[kScanPer],
                                                  uint32_t* before, uint32_t* total) {
  const int i = threadIdx.x, lane = i & 63, w = i >> 6;
#pragma unroll
  for (int j = 0; j < kScanPer; j++) {
    const int64_t k = base + j * 1024 + i;
    buf[j * 1024 + i] = k < ntiles ? tile_count[k] : 0u;
  }
  __syncthreads();
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; j++) {
    v[j] = buf[i * kScanPer + j];
    sum += v[j];
  }
  const uint32_t incl = wave_incl_scan(sum, lane);
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  uint32_t b = 0, t = 0;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    const uint32_t x = wtot[k];
    b += k < w ? x : 0u;
    t += x;
  }
  *before = b + (incl - sum);
  *total = t;
}

__global__ __launch_bounds__(1024) void k_var_scan_sums(const uint32_t* __restrict__ tile_count,
                                                        int32_t ntiles,
                                                        int64_t* __restrict__ tile_off) {
  __shared__ uint32_t buf[kScanChunk];
  __shared__ uint32_t wtot[16];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t v[kScanPer], before, total;
  scan_chunk_counts(tile_count, ntiles, base, buf, wtot, v, &before, &total);
  if (threadIdx.x == 0) tile_off[base] = total;
}

__global__ __launch_bounds__(1024) void k_var_scan_bases(int32_t nchunks, int32_t ntiles,
                                                         int64_t* __restrict__ tile_off) {
  __shared__ int64_t wtot[16];
  const int i = threadIdx.x, lane = i & 63, w = i >> 6;
  int64_t carry = 0;
  for (int32_t c0 = 0; c0 < nchunks; c0 += 1024) {
    const int32_t c = c0 + i;
    const int64_t x = c < nchunks ? tile_off[(int64_t)c * kScanChunk] : 0;
    int64_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int64_t before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
      const int64_t t = wtot[k];
      before += k < w ? t : 0;
      total += t;
    }
    if (c < nchunks) tile_off[(int64_t)c * kScanChunk] = carry + before + (incl - x);
    carry += total;
    __syncthreads();  // wtot is rewritten by the next round
  }
  if (i == 0) tile_off[ntiles] = carry;
}

__global__ __launch_bounds__(1024) void k_var_scan_chunks(const uint32_t* __restrict__ tile_count,
                                                          int32_t ntiles,
                                                          int64_t* __restrict__ tile_off) {
  __shared__ uint32_t buf[kScanChunk];
  __shared__ uint32_t wtot[16];
  __shared__ int64_t chunk_base;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  if (threadIdx.x == 0) chunk_base = tile_off[base];
  uint32_t v[kScanPer], before, total;
  scan_chunk_counts(tile_count, ntiles, base, buf, wtot, v, &before, &total);
  // chunk_base was read before the first barrier inside scan_chunk_counts
  int64_t run = chunk_base + before;
#pragma unroll
  for (int j = 0; j < kScanPer; j++) {
    const int64_t k = base + threadIdx.x * kScanPer + j;
    if (k < ntiles) tile_off[k] = run;
    run += v[j];
  }
}

// Copy each tile's words from its staging slot to its offset; words at or
// past out_words are not written.
__global__ __launch_bounds__(256) void k_var_place(const uint32_t* __restrict__ stage,
                                                   const uint32_t* __restrict__ tile_count,
                                                   const int64_t* __restrict__ tile_off,
                                                   int32_t ntiles, int cap,
                                                   uint32_t* __restrict__ out,
                                                   uint64_t out_words) {
  const int lane = threadIdx.x & 63;
  const int waves = blockDim.x >> 6;
  const int32_t t = blockIdx.x * waves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (t >= ntiles) return;
  const uint32_t count = uniform_load(tile_count, t);
  const uint64_t o = (uint64_t)uniform_load(tile_off, t);
  const uint32_t* in = stage + (size_t)t * 64 * 2 * cap;
  for (uint32_t q0 = lane; q0 < count; q0 += 256) {
    // four words per lane read at once (past the count: word 0, not stored)
    uint32_t r[4];
#pragma unroll
    for (int j = 0; j < 4; j++) r[j] = in[q0 + 64 * j < count ? q0 + 64 * j : 0];
    pin_words32(r);
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const uint32_t q = q0 + 64 * j;
      if (q < count && o + q < out_words) out[o + q] = r[j];
    }
  }
}

// Any content of the stream, counts and offsets decodes without a fault:
// counts are clamped to the cap and words outside the stream read as zero.
template <int CAP, bool VEC4, class Geo>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_decode_var(
    Geo geo, const uint32_t* __restrict__ in, uint64_t in_words, const uint8_t* __restrict__ nd_in,
    const int64_t* __restrict__ tile_off, float* __restrict__ dst, int cap_rt, int32_t nblocks,
    int maxprec, int minexp) {
  extern __shared__ uint64_t lds[];
  const int cap = CAP > 0 ? CAP : cap_rt;
  const int stride = lds_stride(cap);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int waves = blockDim.x >> 6;
  uint64_t* slice = lds + (size_t)(wave * 64 + lane) * stride;
  const int32_t ntiles = tiles_of(nblocks);
  const int32_t t = xcd_grouped(blockIdx.x, gridDim.x) * waves + wave;
  if (t >= ntiles) return;
  const int32_t b0 = t << 6;
  const int nact = nblocks - b0 < 64 ? nblocks - b0 : 64;
  uint32_t nd = lane < nact ? nd_in[b0 + lane] : 0;
  nd = nd < 2u * cap ? nd : 2u * cap;
  const uint32_t incl = wave_incl_scan(nd, lane);
  const uint64_t o = (uint64_t)uniform_load(tile_off, t) + (incl - nd);
  for (int i = 0; i < stride; i++) slice[i] = 0;
  uint32_t* s32 = reinterpret_cast<uint32_t*>(slice);
  if (in_words == 0) nd = 0;  // nothing to read: every block decodes from zeros
  for (uint32_t i0 = 0; i0 < nd; i0 += 8) {
    // eight words read at once (words outside the stream are read at 0 and
    // replaced by zero), then written to the slice
    uint32_t r[8];
    bool ok[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const uint64_t w = o + i0 + j;
      ok[j] = i0 + j < nd && w < in_words && w >= o;
      r[j] = in[ok[j] ? w : 0];
    }
    pin_words32(r);
#pragma unroll
    for (int j = 0; j < 8; j++)
      if (i0 + j < nd) s32[i0 + j] = ok[j] ? r[j] : 0u;
  }
  wave_sync_lds();
  if (lane < nact) {
    float val[64];
    decode_block<CAP, true>(slice, val, cap, maxprec, minexp);
    BlockView v;
    geo.locate_tile(b0, lane, nact, v);
    // streaming stores: 9% faster here on a 9.47 GB output; the fixed-rate
    // decoders gain nothing from them
    scatter<VEC4, false, true>(dst, v, val);
  }
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Word offset of each chunk's first block (and the total at index nchunks).
__global__ void k_var_chunk_offsets(const int64_t* __restrict__ chunk_first, int32_t nchunks,
                                    const uint8_t* __restrict__ nd,
                                    const int64_t* __restrict__ tile_off,
                                    int64_t* __restrict__ chunk_off) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > nchunks) return;
  const int64_t b = chunk_first[c];
  int64_t o = tile_off[b >> 6];
  for (int64_t i = b & ~(int64_t)63; i < b; i++) o += nd[i];
  chunk_off[c] = o;
}

// ---------------------------------------------------------------------------
// Serving loop
// ---------------------------------------------------------------------------
// Wavefront 0 of workgroup 0 is the dispatcher: it alone polls the host's
// control block (over PCIe, with a pause between polls) and copies newly
// published descriptors into a ring in device memory, then publishes them to
// the workers through a device-memory counter.  Every other workgroup is an
// independent worker: its first wavefront walks the device ring in order
// (cursor = request number) and claims runs of 64-block tiles of the request
// at its cursor with a fetch-add on a per-slot counter tagged with the
// request number (so a slot reused for a later request is never confused
// with the earlier one); the workgroup's wavefronts code the run's tiles, and
// the run is counted done; the workgroup that completes a request's last
// tile raises the request's completion flag in host memory.  Requests
// overlap on the device as soon as they are published.  Every workgroup
// leaves when the host asks to stop, after `idle_ticks` without work, or after
// `max_ticks` in total, so the grid always drains.

// All control accesses of the loop are relaxed atomics: on this part an
// acquire or release at agent or system scope means a whole-L2 invalidate or
// write-back, far too costly per tile.  Ordering comes from the hardware
// instead: coherent (cache-bypassing) atomic accesses, program order of
// dependent loads, and explicit waits for outstanding memory operations
// (s_waitcnt) before a store or atomic that publishes earlier writes.
__device__ __forceinline__ uint64_t sys_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t sys_load32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t dev_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Every memory access before this point has completed before any access
// after it is issued; the compiler fences keep the accesses on their sides.
__device__ __forceinline__ void wait_memory() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ int32_t dev_load32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t dev_load64i(const int64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every lane loaded the same descriptor word: make that explicit (scalar).
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void serve_tile(const ServeDesc& q, int lane, uint64_t* wlds,
                                           int32_t tile) {
  RegularGeo geo{q.geo};
  const int32_t b0 = tile << 6;
  const int nact = q.nblocks - b0 < 64 ? q.nblocks - b0 : 64;
  const uint32_t vspan = __builtin_amdgcn_readfirstlane(q.vspan);
  if (q.op == 0) {
    const float* src = reinterpret_cast<const float*>(uniform64(q.in));
    uint64_t* out = reinterpret_cast<uint64_t*>(q.out);
    if (q.rate == 8)
      encode_tile<8, false, true>(geo, src, out, 8, lane, wlds, b0, nact, vspan);
    else if (q.rate == 16)
      encode_tile<16, false, true>(geo, src, out, 16, lane, wlds, b0, nact, vspan);
    else if (q.rate == 32)
      encode_tile<32, false, true>(geo, src, out, 32, lane, wlds, b0, nact, vspan);
    else
      encode_tile<0, false, true>(geo, src, out, q.rate, lane, wlds, b0, nact, vspan);
  } else {
    const uint64_t* in = reinterpret_cast<const uint64_t*>(q.in);
    float* dst = reinterpret_cast<float*>(uniform64(q.out));
    if (q.rate == 8)
      decode_tile<8, false, true>(geo, in, dst, 8, lane, wlds, b0, nact, vspan);
    else if (q.rate == 16)
      decode_tile<16, false, true>(geo, in, dst, 16, lane, wlds, b0, nact, vspan);
    else if (q.rate == 32)
      decode_tile<32, false, true>(geo, in, dst, 32, lane, wlds, b0, nact, vspan);
    else
      decode_tile<0, false, true>(geo, in, dst, q.rate, lane, wlds, b0, nact, vspan);
  }
}

constexpr int kDescWords = sizeof(ServeDesc) / sizeof(uint64_t);
static_assert(offsetof(ServeDesc, seq) == 0, "seq is descriptor word 0");
static_assert(sizeof(ServeDesc) % sizeof(uint64_t) == 0, "descriptor is whole words");
static_assert(kDescWords <= 64, "one descriptor word per lane");

// The dispatcher wavefront.
__device__ __forceinline__ void serve_dispatch(const ServeDev d, int lane, uint64_t t_start) {
  uint64_t seen = dev_load(&d.dctl->published);
  uint64_t t_work = t_start;
  // the claimers start their walk from the device copy of the host's hint
  // (one read of host memory here, not one per claimer)
  if (lane == 0)
    __hip_atomic_store(&d.dctl->oldest, sys_load(&d.ctl->oldest), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const uint64_t now = __builtin_amdgcn_s_memrealtime();
    if (now - t_start > d.max_ticks) break;
    // both host words read in one round trip over PCIe
    const uint32_t stop = sys_load32(&d.ctl->stop);
    const uint64_t hpub = sys_load(&d.ctl->published);
    if (stop) {
      if (lane == 0)
        __hip_atomic_store(&d.dctl->stop, uint64_t(1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    if (hpub > seen) {
      // A slot is rewritten once its previous request has completed, but a
      // worker that claimed past the end of that request may still be reading
      // it.  So seq (word 0) is first marked invalid, then the other words are
      // copied, then seq, each step complete before the next: a reader that
      // finds the same seq before and after reading the other words has read
      // one whole descriptor.  (The requests seen .. hpub-1 lie in distinct
      // slots: a slot is reused only after its request completed.)
      for (uint64_t sq = seen; sq < hpub; sq++) {
        const int slot = (int)(sq % (uint64_t)d.cap);
        if (lane == 0)
          __hip_atomic_store(&d.ring_dev[slot].seq, ~uint64_t(0), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_SYSTEM);
      }
      wait_memory();
      for (int pass = 0; pass < 2; pass++) {
        // pass 0: every word but seq (one word per lane); pass 1: seq
        for (uint64_t sq = seen; sq < hpub; sq++) {
          const int slot = (int)(sq % (uint64_t)d.cap);
          const uint64_t* from = reinterpret_cast<const uint64_t*>(d.ring + slot);
          uint64_t* to = reinterpret_cast<uint64_t*>(d.ring_dev + slot);
          if (pass == 0 ? lane >= 1 && lane < kDescWords : lane == 0)
            __hip_atomic_store(to + lane,
                               __hip_atomic_load(from + lane, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_SYSTEM),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        wait_memory();  // complete before seq is written / before publishing
      }
      if (lane == 0) {
        __hip_atomic_store(&d.dctl->published, hpub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&d.dctl->oldest, sys_load(&d.ctl->oldest), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      seen = hpub;
      t_work = now;
      continue;
    }
    if (now - t_work > d.idle_ticks) break;
    __builtin_amdgcn_s_sleep(16);
  }
}

// What wavefront 0 of a worker workgroup hands to the others in LDS: a run
// of tiles [t0, t1) of request q (slot `slot`), or the order to leave.
struct ServeRun {
  ServeDesc q;
  int32_t t0, t1, slot, leave;
};

// Wavefront 0 of a worker workgroup: find the workgroup's next run of tiles.
// It walks the device ring in order (cursor = request number) and claims a
// run with a fetch-add on the slot's counter, whose high half names the
// request it counts for.  The run belongs to that request, which is the one
// at the cursor or (the slot reused after that one finished) a later one,
// and is processed for it.  A counter still naming an older request is moved
// on with an atomic max (tags only grow, so the max neither loses a later tag
// nor fights the fetch-adds of other workgroups); the done counter first, so
// that no tile of the request can complete before its done counter is reset.
// Returns false when the workgroup is to leave (stop asked, idle too long, or
// out of time).
struct ServeCursor {
  uint64_t cursor, pub, t_work;
  uint32_t qtag;
  bool have_q;
  ServeDesc q;  // of the last request claimed (valid while have_q)
};

__device__ __forceinline__ bool serve_find_run(const ServeDev& d, int lane, uint64_t t_start,
                                               ServeCursor& c, int32_t& t0, int32_t& t1,
                                               int32_t& slot_out) {
  for (;;) {
    const uint64_t now = __builtin_amdgcn_s_memrealtime();
    if (now - t_start > d.max_ticks) return false;
    if (c.cursor >= c.pub) {
      // idle means nothing published for idle_ticks, not no work for this
      // workgroup: otherwise workgroups that small requests leave without
      // tiles would leave, and a large request find the loop thinned out
      const uint64_t p = dev_load(&d.dctl->published);
      if (p != c.pub) c.t_work = now;
      c.pub = p;
      if (c.cursor >= c.pub) {
        if (dev_load(&d.dctl->stop) || now - c.t_work > d.idle_ticks) return false;
        // Idle workgroups poll the published counter about every 14 us: many
        // pollers of one word every microsecond slow every coherent access of
        // the loop, and with hundreds of pollers at random phases some wake
        // within a microsecond.  Right after a launch, which happens because
        // requests are waiting, all of them are in phase and nothing runs yet:
        // for the first 1/40 of the idle spell they poll every 0.5 us.
        if (now - t_start < d.idle_ticks / 40) {
          __builtin_amdgcn_s_sleep(16);
        } else {
          for (int i = 0; i < 4; i++) __builtin_amdgcn_s_sleep(127);
        }
        continue;
      }
    }
    const int slot = (int)(c.cursor % (uint64_t)d.cap);
    const uint32_t want = (uint32_t)c.cursor;
    // one run per wavefront of the workgroup; before the descriptor is known,
    // one tile per wavefront
    const int32_t take = kServeWaves * (c.have_q && c.qtag == want ? c.q.per_claim : 1);
    uint64_t got = 0;  // (request tag << 32) | first tile
    if (lane == 0) {
      for (;;) {
        const uint64_t prev = __hip_atomic_fetch_add(d.claim + slot, (uint64_t)take,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t pseq = (uint32_t)(prev >> 32);
        if ((int32_t)(pseq - want) >= 0) {
          got = prev;
          break;
        }
        __hip_atomic_fetch_max(d.done + slot, (uint64_t)want << 32, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        wait_memory();
        __hip_atomic_fetch_max(d.claim + slot, (uint64_t)want << 32, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        wait_memory();
      }
    }
    got = __shfl(got, 0, 64);
    const uint32_t gtag = (uint32_t)(got >> 32);
    const int32_t tile = (int32_t)(uint32_t)got;
    if (!c.have_q || c.qtag != gtag) {
      const ServeDesc* r = d.ring_dev + slot;
      // coherent vector loads, kept in scalar registers (every lane read the
      // same words).  seq is read before and after the other words: if the
      // claimed request has completed, the dispatcher may be rewriting the
      // slot for a later one, and only a descriptor whose seq did not change
      // across the reads is whole.
      ServeDesc& q = c.q;
      const uint64_t seq0 = uniform64(dev_load(&r->seq));
      wait_memory();
      q.ntiles = __builtin_amdgcn_readfirstlane(dev_load32(&r->ntiles));
      q.op = __builtin_amdgcn_readfirstlane(dev_load32(&r->op));
      q.rate = __builtin_amdgcn_readfirstlane(dev_load32(&r->rate));
      q.nblocks = __builtin_amdgcn_readfirstlane(dev_load32(&r->nblocks));
      q.vspan = (uint32_t)__builtin_amdgcn_readfirstlane(
          dev_load32(reinterpret_cast<const int32_t*>(&r->vspan)));
      q.per_claim = __builtin_amdgcn_readfirstlane(dev_load32(&r->per_claim));
      q.geo.nx = (int64_t)uniform64((uint64_t)dev_load64i(&r->geo.nx));
      q.geo.ny = (int64_t)uniform64((uint64_t)dev_load64i(&r->geo.ny));
      q.geo.nz = (int64_t)uniform64((uint64_t)dev_load64i(&r->geo.nz));
      q.geo.sx = (int64_t)uniform64((uint64_t)dev_load64i(&r->geo.sx));
      q.geo.sy = (int64_t)uniform64((uint64_t)dev_load64i(&r->geo.sy));
      q.geo.sz = (int64_t)uniform64((uint64_t)dev_load64i(&r->geo.sz));
      q.geo.nbx = __builtin_amdgcn_readfirstlane(dev_load32(&r->geo.nbx));
      q.geo.nby = __builtin_amdgcn_readfirstlane(dev_load32(&r->geo.nby));
      q.in = uniform64(dev_load(&r->in));
      q.out = uniform64(dev_load(&r->out));
      wait_memory();
      q.seq = uniform64(dev_load(&r->seq));
      c.qtag = gtag;
      c.have_q = q.seq == seq0 && (uint32_t)q.seq == gtag;
      if (!c.have_q) {
        // the claimed request finished and the slot holds (or is being
        // rewritten for) a later one whose claim counter is not moved on
        // yet: nothing to do here
        c.cursor++;
        continue;
      }
    }
    if (tile >= c.q.ntiles) {
      // every tile of the slot's request is claimed (and the cursor's request
      // with it): move on
      c.cursor++;
      continue;
    }
    t0 = tile;
    t1 = c.q.ntiles - tile < take ? c.q.ntiles : tile + take;
    slot_out = slot;
    return true;
  }
}

// Workgroup 0's first wavefront is the dispatcher (the workgroup takes no
// tiles and meets no barrier).  Every other workgroup is a worker: its first
// wavefront finds a run of tiles for the whole workgroup and hands it over in
// LDS; each wavefront codes every kServeWaves-th tile of the run; after a
// barrier the first wavefront counts the run done.  Claims per workgroup, not
// per wavefront, keep the claim and descriptor traffic of walking every
// request at one claimer per workgroup (one per compute unit) while two
// wavefronts per SIMD share the coding.
__global__ __launch_bounds__(64 * kServeWaves) __attribute__((amdgpu_waves_per_eu(2)))
void k_serve(ServeDev d) {
  extern __shared__ uint64_t lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
  if (blockIdx.x == 0) {
    if (wave == 0) serve_dispatch(d, lane, t_start);
    return;
  }
  uint64_t* wlds = lds + (size_t)wave * 64 * lds_stride(32);
  ServeRun* run = reinterpret_cast<ServeRun*>(lds + (size_t)kServeWaves * 64 * lds_stride(32));
  // the claimer's walk state (only the first wavefront uses it).  It starts
  // from the device copy of the host's oldest-request hint: a launch that
  // began with one read of host memory per wavefront (thousands of reads of
  // one word over PCIe) took 70-120 us to start serving.  The copy may be the
  // previous launch's until the dispatcher refreshes it; a lagging start only
  // walks requests that are already done.
  ServeCursor c;
  c.cursor = wave == 0 ? dev_load(&d.dctl->oldest) : 0;
  c.pub = 0;
  c.t_work = t_start;
  c.qtag = 0;
  c.have_q = false;
  for (;;) {
    if (wave == 0) {
      int32_t t0 = 0, t1 = 0, slot = 0;
      const bool go = serve_find_run(d, lane, t_start, c, t0, t1, slot);
      if (lane == 0) {
        run->leave = go ? 0 : 1;
        if (go) {
          run->q = c.q;
          run->t0 = t0;
          run->t1 = t1;
          run->slot = slot;
        }
      }
    }
    __syncthreads();  // the run is in LDS
    if (__builtin_amdgcn_readfirstlane(run->leave)) break;
    ServeDesc q;
    q.seq = uniform64(run->q.seq);
    q.op = __builtin_amdgcn_readfirstlane(run->q.op);
    q.rate = __builtin_amdgcn_readfirstlane(run->q.rate);
    q.nblocks = __builtin_amdgcn_readfirstlane(run->q.nblocks);
    q.ntiles = __builtin_amdgcn_readfirstlane(run->q.ntiles);
    q.vspan = (uint32_t)__builtin_amdgcn_readfirstlane(run->q.vspan);
    q.per_claim = 0;
    q.geo.nx = (int64_t)uniform64((uint64_t)run->q.geo.nx);
    q.geo.ny = (int64_t)uniform64((uint64_t)run->q.geo.ny);
    q.geo.nz = (int64_t)uniform64((uint64_t)run->q.geo.nz);
    q.geo.sx = (int64_t)uniform64((uint64_t)run->q.geo.sx);
    q.geo.sy = (int64_t)uniform64((uint64_t)run->q.geo.sy);
    q.geo.sz = (int64_t)uniform64((uint64_t)run->q.geo.sz);
    q.geo.nbx = __builtin_amdgcn_readfirstlane(run->q.geo.nbx);
    q.geo.nby = __builtin_amdgcn_readfirstlane(run->q.geo.nby);
    q.in = uniform64(run->q.in);
    q.out = uniform64(run->q.out);
    const int32_t t0 = __builtin_amdgcn_readfirstlane(run->t0);
    const int32_t t1 = __builtin_amdgcn_readfirstlane(run->t1);
    const int32_t slot = __builtin_amdgcn_readfirstlane(run->slot);
    for (int32_t t = t0 + wave; t < t1; t += kServeWaves) {
      serve_tile(q, opaque(lane), wlds, t);
      wave_sync_lds();
    }
    // the tiles' output was written through to memory (system-coherent
    // stores): every wavefront waits until its stores have completed, and
    // after the barrier (which also frees the run record for the next
    // write) the run is counted done, so no cache write-back is needed
    wait_memory();
    __syncthreads();
    if (wave == 0) {
      if (lane == 0) {
        const int32_t n = t1 - t0;
        const uint64_t prev = __hip_atomic_fetch_add(d.done + slot, (uint64_t)n,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int32_t)(uint32_t)prev + n == q.ntiles)
          __hip_atomic_store(d.done_flag + slot, q.seq + 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_SYSTEM);
      }
      c.t_work = __builtin_amdgcn_s_memrealtime();
    }
  }
}

// float16 comparator; unaligned buffers take one value per thread.
// Truncate: a wavefront converts 128 consecutive groups of 4 values; lane l
// takes groups l and l + 64, so each 16-byte load reads 1 KB and each 8-byte
// store writes 512 B contiguously.  Both loads are issued (clamped in range)
// before either conversion, and loads and stores carry the non-temporal hint
// (every byte is touched once): on a 9.47 GB buffer this runs at 80% of the
// HBM peak against 72-74% with ordinary accesses.  The grid covers the buffer
// (the loop only runs more than once beyond kElementwiseMaxBlocks
// workgroups).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_f16_truncate_w2(const f32x4* __restrict__ in, size_t n4,
                                                         u32x2* __restrict__ out) {
  auto h = [](float f) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f); };
  const int lane = threadIdx.x & 63;
  const size_t nw = (n4 + 127) / 128;
  const size_t wstep = (size_t)gridDim.x * (blockDim.x / 64);
  for (size_t w = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); w < nw;
       w += wstep) {
    const size_t i0 = w * 128 + lane, i1 = i0 + 64;
    const f32x4 a = __builtin_nontemporal_load(in + (i0 < n4 ? i0 : n4 - 1));
    const f32x4 b = __builtin_nontemporal_load(in + (i1 < n4 ? i1 : n4 - 1));
    if (i0 < n4)
      __builtin_nontemporal_store(u32x2{h(a.x) | (h(a.y) << 16), h(a.z) | (h(a.w) << 16)},
                                  out + i0);
    if (i1 < n4)
      __builtin_nontemporal_store(u32x2{h(b.x) | (h(b.y) << 16), h(b.z) | (h(b.w) << 16)},
                                  out + i1);
  }
}

__global__ __launch_bounds__(256) void k_f16_truncate_s(const float* __restrict__ in, size_t n,
                                                        uint16_t* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = __builtin_bit_cast(uint16_t, (_Float16)in[i]);
}

// Restore: groups of 4 values (one 8-byte load, one 16-byte store), one
// group per thread on a covering grid, with non-temporal loads and stores as
// in truncate (81% of the HBM peak on a 9.47 GB output against 78%).
__global__ __launch_bounds__(256) void k_f16_restore_v4(const u32x2* __restrict__ in, size_t n4,
                                                        f32x4* __restrict__ out) {
  const size_t T = (size_t)gridDim.x * blockDim.x;
  auto f = [](uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)w); };
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += T) {
    const u32x2 r = __builtin_nontemporal_load(in + i);
    __builtin_nontemporal_store(f32x4{f(r.x), f(r.x >> 16), f(r.y), f(r.y >> 16)}, out + i);
  }
}

__global__ __launch_bounds__(256) void k_f16_restore_s(const uint16_t* __restrict__ in, size_t n,
                                                       float* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)__builtin_bit_cast(_Float16, in[i]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

size_t lds_bytes(int wg, int rate) {
  return (size_t)(wg / 64) * 64 * lds_stride(rate) * sizeof(uint64_t);
}

static int g_cus = -1;
static size_t g_max_lds = 0;

static void query_device() {
  if (g_cus >= 0) return;
  int dev = 0, cus = 0, lds = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  }
  g_cus = cus > 0 ? cus : 256;
  g_max_lds = lds > 0 ? (size_t)lds : 65536;
}

size_t device_max_lds() {
  query_device();
  return g_max_lds;
}

int device_cu_count() {
  query_device();
  return g_cus;
}

static dim3 grid_for(int32_t nblocks, LaunchCfg cfg, bool* persistent) {
  int waves = cfg.wg / 64;
  int64_t ntiles = ((int64_t)nblocks + 63) / 64;
  int64_t full = (ntiles + waves - 1) / waves;
  *persistent = cfg.grid > 0 && cfg.grid < full;
  int64_t g = *persistent ? cfg.grid : full;
  return dim3((unsigned)(g > 0 ? g : 1));
}

#define ZFPX_RATE_SWITCH2(KERNEL, GEO, VEC4, PERSIST, ...)                                \
  switch (rate) {                                                                          \
    case 8:                                                                                \
      hipLaunchKernelGGL((KERNEL<8, VEC4, PERSIST, GEO>), grid, block, shm, s, __VA_ARGS__); \
      break;                                                                               \
    case 16:                                                                               \
      hipLaunchKernelGGL((KERNEL<16, VEC4, PERSIST, GEO>), grid, block, shm, s, __VA_ARGS__); \
      break;                                                                               \
    case 32:                                                                               \
      hipLaunchKernelGGL((KERNEL<32, VEC4, PERSIST, GEO>), grid, block, shm, s, __VA_ARGS__); \
      break;                                                                               \
    default:                                                                               \
      hipLaunchKernelGGL((KERNEL<0, VEC4, PERSIST, GEO>), grid, block, shm, s, __VA_ARGS__); \
      break;                                                                               \
  }

// One tile per wavefront unless the configuration asks for a persistent grid.
#define ZFPX_RATE_SWITCH(KERNEL, GEO, VEC4, ...)                                         \
  if (persistent) {                                                                        \
    ZFPX_RATE_SWITCH2(KERNEL, GEO, VEC4, true, __VA_ARGS__)                                \
  } else {                                                                                 \
    ZFPX_RATE_SWITCH2(KERNEL, GEO, VEC4, false, __VA_ARGS__)                               \
  }

hipError_t launch_plan_encode(const PlanDev& p, bool vec4, const float* src, uint64_t* out,
                              int rate, int32_t b_begin, int32_t b_end, LaunchCfg cfg,
                              hipStream_t s) {
  if (b_end <= b_begin) return hipSuccess;
  bool persistent;
  dim3 grid = grid_for(b_end - b_begin, cfg, &persistent), block(cfg.wg);
  size_t shm = lds_bytes(cfg.wg, rate);
  PlanGeo geo{p};
  if (vec4) {
    ZFPX_RATE_SWITCH(k_encode, PlanGeo, true, geo, src, out, rate, b_begin, b_end);
  } else {
    ZFPX_RATE_SWITCH(k_encode, PlanGeo, false, geo, src, out, rate, b_begin, b_end);
  }
  return hipGetLastError();
}

hipError_t launch_plan_decode(const PlanDev& p, bool vec4, const uint64_t* in, float* dst,
                              int rate, int32_t b_begin, int32_t b_end, LaunchCfg cfg,
                              hipStream_t s) {
  if (b_end <= b_begin) return hipSuccess;
  bool persistent;
  dim3 grid = grid_for(b_end - b_begin, cfg, &persistent), block(cfg.wg);
  size_t shm = lds_bytes(cfg.wg, rate);
  PlanGeo geo{p};
  if (vec4) {
    ZFPX_RATE_SWITCH(k_decode, PlanGeo, true, geo, in, dst, rate, b_begin, b_end);
  } else {
    ZFPX_RATE_SWITCH(k_decode, PlanGeo, false, geo, in, dst, rate, b_begin, b_end);
  }
  return hipGetLastError();
}

hipError_t launch_regular_encode(const RegularDev& g, bool vec4, const float* src,
                                 uint64_t* out, int rate, int32_t nblocks, LaunchCfg cfg,
                                 hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  bool persistent;
  dim3 grid = grid_for(nblocks, cfg, &persistent), block(cfg.wg);
  size_t shm = lds_bytes(cfg.wg, rate);
  RegularGeo geo{g};
  int32_t b0 = 0;
  if (vec4) {
    ZFPX_RATE_SWITCH(k_encode, RegularGeo, true, geo, src, out, rate, b0, nblocks);
  } else {
    ZFPX_RATE_SWITCH(k_encode, RegularGeo, false, geo, src, out, rate, b0, nblocks);
  }
  return hipGetLastError();
}

hipError_t launch_regular_decode(const RegularDev& g, bool vec4, const uint64_t* in, float* dst,
                                 int rate, int32_t nblocks, LaunchCfg cfg, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  bool persistent;
  dim3 grid = grid_for(nblocks, cfg, &persistent), block(cfg.wg);
  size_t shm = lds_bytes(cfg.wg, rate);
  RegularGeo geo{g};
  int32_t b0 = 0;
  if (vec4) {
    ZFPX_RATE_SWITCH(k_decode, RegularGeo, true, geo, in, dst, rate, b0, nblocks);
  } else {
    ZFPX_RATE_SWITCH(k_decode, RegularGeo, false, geo, in, dst, rate, b0, nblocks);
  }
  return hipGetLastError();
}

static unsigned elementwise_grid(size_t work) {
  query_device();
  size_t g = (work + 255) / 256;
  size_t cap = (size_t)g_cus * 16;
  if (g > cap) g = cap;
  return (unsigned)(g > 0 ? g : 1);
}

// One thread per work item, up to kElementwiseMaxBlocks workgroups of 256
// (2^31 threads; the kernels loop beyond that).
constexpr size_t kElementwiseMaxBlocks = size_t(1) << 23;
static unsigned covering_grid(size_t work) {
  size_t g = (work + 255) / 256;
  if (g > kElementwiseMaxBlocks) g = kElementwiseMaxBlocks;
  return (unsigned)(g > 0 ? g : 1);
}

hipError_t launch_serve(const ServeDev& d, int workgroups, hipStream_t s) {
  size_t shm = (size_t)kServeWaves * 64 * lds_stride(32) * sizeof(uint64_t) + sizeof(ServeRun);
  hipLaunchKernelGGL(k_serve, dim3(workgroups > 0 ? workgroups : 1), dim3(64 * kServeWaves), shm,
                     s, d);
  return hipGetLastError();
}

hipError_t launch_f16_truncate(const float* in, size_t n, uint16_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t done = 0;
  if (((uintptr_t)in & 15) == 0 && ((uintptr_t)out & 7) == 0 && n >= 4) {
    size_t n4 = n / 4;
    hipLaunchKernelGGL(k_f16_truncate_w2, dim3(covering_grid((n4 + 1) / 2)), dim3(256), 0, s,
                       reinterpret_cast<const f32x4*>(in), n4, reinterpret_cast<u32x2*>(out));
    done = n4 * 4;
  }
  if (done < n)
    hipLaunchKernelGGL(k_f16_truncate_s, dim3(elementwise_grid(n - done)), dim3(256), 0, s,
                       in + done, n - done, out + done);
  return hipGetLastError();
}

hipError_t launch_f16_restore(const uint16_t* in, size_t n, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t done = 0;
  if (((uintptr_t)in & 7) == 0 && ((uintptr_t)out & 15) == 0 && n >= 4) {
    size_t n4 = n / 4;
    hipLaunchKernelGGL(k_f16_restore_v4, dim3(covering_grid(n4)), dim3(256), 0, s,
                       reinterpret_cast<const u32x2*>(in), n4, reinterpret_cast<f32x4*>(out));
    done = n4 * 4;
  }
  if (done < n)
    hipLaunchKernelGGL(k_f16_restore_s, dim3(elementwise_grid(n - done)), dim3(256), 0, s,
                       in + done, n - done, out + done);
  return hipGetLastError();
}

#define ZFPX_CAP_SWITCH(KERNEL, GEO, VEC4, ...)                                     \
  switch (cap) {                                                                   \
    case 8:                                                                        \
      hipLaunchKernelGGL((KERNEL<8, VEC4, GEO>), grid, block, shm, s, __VA_ARGS__);  \
      break;                                                                       \
    case 16:                                                                       \
      hipLaunchKernelGGL((KERNEL<16, VEC4, GEO>), grid, block, shm, s, __VA_ARGS__); \
      break;                                                                       \
    case 32:                                                                       \
      hipLaunchKernelGGL((KERNEL<32, VEC4, GEO>), grid, block, shm, s, __VA_ARGS__); \
      break;                                                                       \
    default:                                                                       \
      hipLaunchKernelGGL((KERNEL<0, VEC4, GEO>), grid, block, shm, s, __VA_ARGS__);  \
      break;                                                                       \
  }

size_t var_stage_words(int64_t nblocks, int cap) {
  return (size_t)((nblocks + 63) >> 6) * 64 * 2 * (size_t)cap;
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)(g < 1024 ? g : 1024)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_plan_encode_var(const PlanDev& p, bool vec4, const float* src, uint32_t* out,
                                  uint64_t out_words, uint8_t* nd, int64_t* tile_off,
                                  uint32_t* stage, uint32_t* tile_count, int cap,
                                  int32_t nblocks, int maxprec, int minexp, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  constexpr int wg = 128;
  const int ntiles = tiles_of(nblocks);
  dim3 grid((ntiles + wg / 64 - 1) / (wg / 64)), block(wg);
  size_t shm = lds_bytes(wg, cap);
  PlanGeo geo{p};
  if (vec4) {
    ZFPX_CAP_SWITCH(k_encode_var, PlanGeo, true, geo, src, stage, tile_count, nd, cap, nblocks,
                    maxprec, minexp);
  } else {
    ZFPX_CAP_SWITCH(k_encode_var, PlanGeo, false, geo, src, stage, tile_count, nd, cap, nblocks,
                    maxprec, minexp);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int32_t nchunks = (int32_t)(((int64_t)ntiles + kScanChunk - 1) / kScanChunk);
  if (nchunks > 0)
    hipLaunchKernelGGL(k_var_scan_sums, dim3(nchunks), dim3(1024), 0, s, tile_count, ntiles,
                       tile_off);
  hipLaunchKernelGGL(k_var_scan_bases, dim3(1), dim3(1024), 0, s, nchunks, ntiles, tile_off);
  if (nchunks > 0)
    hipLaunchKernelGGL(k_var_scan_chunks, dim3(nchunks), dim3(1024), 0, s, tile_count, ntiles,
                       tile_off);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_var_place, dim3((ntiles + 3) / 4), dim3(256), 0, s, stage, tile_count,
                     tile_off, ntiles, cap, out, out_words);
  return hipGetLastError();
}

hipError_t launch_plan_decode_var(const PlanDev& p, bool vec4, const uint32_t* in,
                                  uint64_t in_words, const uint8_t* nd, const int64_t* tile_off,
                                  float* dst, int cap, int32_t nblocks, int maxprec, int minexp,
                                  hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  constexpr int wg = 128;
  const int ntiles = tiles_of(nblocks);
  dim3 grid((ntiles + wg / 64 - 1) / (wg / 64)), block(wg);
  size_t shm = lds_bytes(wg, cap);
  PlanGeo geo{p};
  if (vec4) {
    ZFPX_CAP_SWITCH(k_decode_var, PlanGeo, true, geo, in, in_words, nd, tile_off, dst, cap,
                    nblocks, maxprec, minexp);
  } else {
    ZFPX_CAP_SWITCH(k_decode_var, PlanGeo, false, geo, in, in_words, nd, tile_off, dst, cap,
                    nblocks, maxprec, minexp);
  }
  return hipGetLastError();
}

hipError_t launch_var_chunk_offsets(const int64_t* chunk_first, int32_t nchunks,
                                    const uint8_t* nd, const int64_t* tile_off,
                                    int64_t* chunk_off, hipStream_t s) {
  hipLaunchKernelGGL(k_var_chunk_offsets, dim3((nchunks + 1 + 255) / 256), dim3(256), 0, s,
                     chunk_first, nchunks, nd, tile_off, chunk_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free variable-size encoder
// ---------------------------------------------------------------------------
// The staging slots and tile counts of one variable-size encode, for callers
// that cannot allocate.  Every GPU the library runs on holds its own copy of
// the array until the process ends.  In host code the array's name is not a
// device address: host code uses only the address hipGetSymbolAddress gives
// for the current device.
static __device__ __align__(256) uint32_t scratch[kNoAllocScratchBytes / sizeof(uint32_t)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace zfpx
